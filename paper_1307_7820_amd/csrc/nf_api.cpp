// extern "C" entry points of include/nf.h.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "nf.h"
#include "nf_runtime.h"
#include "nf_test.h"

using namespace nf;

namespace {
std::recursive_mutex g_api;

}

// A prepared batch: one plan per group width q among its folds (q = 0 gives
// each fold the q tuned for its length bucket).  Plan k > 0 runs on a stream
// of its own, forked from and joined back into the caller's stream.
struct nf_batch {
    std::vector<std::unique_ptr<Plan>> plans;
    std::vector<int> ns;
    std::vector<std::pair<int, int>> where;  // fold i -> (plan, index in that plan)
    std::vector<hipStream_t> side;           // side[k - 1] runs plan k
    std::vector<hipEvent_t> joins;           // joins[k - 1] marks the end of plan k
    hipEvent_t fork = nullptr, done = nullptr;
    DevBuf S, tb;  // expand target for table copies; traceback scratch
    bool ran = false;
    ~nf_batch()
    {
        if (done) (void)hipEventDestroy(done);
        if (fork) (void)hipEventDestroy(fork);
        for (auto e : joins) (void)hipEventDestroy(e);
        for (auto st : side) (void)hipStreamDestroy(st);
    }
    Plan& plan_of(int i) { return *plans[where[i].first]; }
    int index_in(int i) const { return where[i].second; }
};

extern "C" {

const char* nf_last_error(void) { return last_error(); }

int nf_init(int device)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    Context& c = ctx();
    if (!c.ready) c.requested_device = device;
    return ensure_device();
}

void nf_shutdown(void)
{
    serve_shutdown();
    std::lock_guard<std::recursive_mutex> lk(g_api);
    Context& c = ctx();
    if (!c.ready) return;
    (void)hipSetDevice(c.device);
    (void)hipDeviceSynchronize();
    c.plans.clear();
    for (auto& r : c.R) r.reset();
    if (c.stream) (void)hipStreamDestroy(c.stream);
    if (c.capture_stream) (void)hipStreamDestroy(c.capture_stream);
    if (c.side_stream) (void)hipStreamDestroy(c.side_stream);
    if (c.ev_tile) (void)hipEventDestroy(c.ev_tile);
    if (c.ev_btw) (void)hipEventDestroy(c.ev_btw);
    c.stream = c.capture_stream = c.side_stream = nullptr;
    c.ev_tile = c.ev_btw = nullptr;
    c.ready = false;
}

int nf_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx)
{
    clear_error();
    AllocHook h;
    h.alloc = alloc;
    h.free_ = free_;
    h.ctx = alloc ? ctx : nullptr;
    return set_allocator(h);
}

int nf_encode(const char* seq, int n, uint8_t* codes_out)
{
    clear_error();
    int rc = check_length(n);
    if (rc) return rc;
    if (n > 0 && (!seq || !codes_out)) return fail(NF_E_INVAL, "NULL argument");
    std::vector<uint8_t> tmp(n);
    if ((rc = encode_sequence(seq, n, tmp.data()))) return rc;
    std::copy(tmp.begin(), tmp.end(), codes_out);
    return NF_OK;
}

int nf_precompute_R(int q)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (q < NF_Q_MIN || q > NF_Q_MAX) return fail(NF_E_INVAL, "q = %d outside %d..%d", q, NF_Q_MIN, NF_Q_MAX);
    int rc = ensure_device();
    if (rc) return rc;
    const uint8_t* R = nullptr;
    return get_R(q, &R);
}

int nf_copy_R(int q, uint8_t* out, size_t cap)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (q < NF_Q_MIN || q > NF_Q_MAX) return fail(NF_E_INVAL, "q = %d outside %d..%d", q, NF_Q_MIN, NF_Q_MAX);
    const size_t bytes = (size_t)1 << (2 * (q - 1));
    if (!out || cap < bytes) return fail(NF_E_INVAL, "R for q = %d needs %zu bytes", q, bytes);
    int rc = ensure_device();
    if (rc) return rc;
    const uint8_t* R = nullptr;
    if ((rc = get_R(q, &R))) return rc;
    HIPCHK(hipMemcpy(out, R, bytes, hipMemcpyDeviceToHost));
    return NF_OK;
}

// Encode seq, fill its table on the library stream and leave the plan in *out
// (the copies and the fill are enqueued, not waited for; `padded` must live
// until the stream is synchronised, which `fence`, armed here once the device
// is up, sees to on every return).
static int fill_single(const char* seq, int n, int q, Plan** out, std::vector<uint8_t>& padded, StreamFence& fence)
{
    int rc = check_length(n);
    if (rc) return rc;
    if ((rc = check_q(q))) return rc;
    if (!seq && n > 0) return fail(NF_E_INVAL, "seq is NULL");
    std::vector<uint8_t> codes(n);
    if ((rc = encode_sequence(seq, n, codes.data()))) return rc;
    if ((rc = ensure_device())) return rc;
    fence.s = ctx().stream;
    q = resolve_q(q, n);
    Plan* p = nullptr;
    if ((rc = single_plan(n, q, &p))) return rc;
    const Geom& g = p->geom[0];
    padded.assign(g.codes_bytes, 0);
    std::copy(codes.begin(), codes.end(), padded.begin());
    hipStream_t s = ctx().stream;
    HIPCHK(hipMemcpyAsync((void*)p->h_folds[0].codes, padded.data(), g.codes_bytes, hipMemcpyHostToDevice, s));
    if ((rc = plan_enqueue(*p, s))) return rc;
    *out = p;
    return NF_OK;
}

int nf_fold(const char* seq, int n, int q, int16_t* S_out)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    Plan* p = nullptr;
    std::vector<uint8_t> padded;
    int32_t score = 0;
    StreamFence fence;
    int rc = fill_single(seq, n, q, &p, padded, fence);
    if (rc) return rc;
    const Geom& g = p->geom[0];
    hipStream_t s = ctx().stream;
    HIPCHK(hipMemcpyAsync(&score, p->d_scores.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (S_out && n > 0) {
        const size_t bytes = (size_t)n * n * sizeof(int16_t);
        if (p->d_S.bytes < bytes && (rc = p->d_S.alloc(bytes))) return rc;
        HIPCHK(launch_expand(p->h_folds[0].F, g.ld, n, (int16_t*)p->d_S.p, s));
        HIPCHK(hipMemcpyAsync(S_out, p->d_S.p, bytes, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return score;
}

int nf_test_set_perturb(unsigned seed)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    perturb_seed() = seed;
    return NF_OK;
}

int nf_test_packed_state(const char* seq, int n, int q, uint32_t* rs_out, uint32_t* cs_out, size_t cap_words,
                         int* nt_out)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (q < 1 || q > NF_Q_MAX) return fail(NF_E_INVAL, "q = %d outside 1..%d", q, NF_Q_MAX);
    if (n < 2 || !rs_out || !cs_out) return fail(NF_E_INVAL, "needs n >= 2 and both output buffers");
    int rc = check_length(n);
    if (rc) return rc;
    const Geom g0 = make_geom(n, q);
    if (nt_out) *nt_out = g0.NT;
    const size_t words = (size_t)tile_count(g0.NT) * state_words(q);
    if (cap_words < words) return fail(NF_E_INVAL, "packed state needs %zu words per block", words);
    Plan* p = nullptr;
    std::vector<uint8_t> padded;
    int32_t score = 0;
    StreamFence fence;
    if ((rc = fill_single(seq, n, q, &p, padded, fence))) return rc;
    hipStream_t s = ctx().stream;
    const FoldDesc& f = p->h_folds[0];
    const size_t skip = (size_t)f.NT * state_words(q);  // the main-diagonal tiles' blocks
    HIPCHK(hipMemcpyAsync(&score, p->d_scores.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rs_out + skip, f.RS + skip, (words - skip) * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(cs_out + skip, f.CS + skip, (words - skip) * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return score;
}

int nf_fold_structure(const char* seq, int n, int q, char* db_out)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (!db_out && n > 0) return fail(NF_E_INVAL, "db_out is NULL");
    Plan* p = nullptr;
    std::vector<uint8_t> padded;
    int32_t score = 0;
    int32_t status = 0;
    std::vector<char> db(n);
    StreamFence fence;
    int rc = fill_single(seq, n, q, &p, padded, fence);
    if (rc) return rc;
    const Geom& g = p->geom[0];
    hipStream_t s = ctx().stream;
    HIPCHK(hipMemcpyAsync(&score, p->d_scores.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (n > 0) {
        // [status: 256 B][structure: n B, rounded up to 256][spill: 2 (n/2 + 1) int2]
        const int cap = n / 2 + 1;
        const size_t db_off = 256, st_off = db_off + (((size_t)n + 255) & ~(size_t)255);
        const size_t bytes = st_off + 2 * (size_t)cap * sizeof(int2);
        if (p->d_tb.bytes < bytes && (rc = p->d_tb.alloc(bytes))) return rc;
        char* base = (char*)p->d_tb.p;
        HIPCHK(launch_traceback(p->h_folds[0].F, g.ld, p->h_folds[0].codes, n, (int2*)(base + st_off), cap,
                                base + db_off, (int*)base, s));
        HIPCHK(hipMemcpyAsync(&status, base, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(db.data(), base + db_off, n, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (status != 0) return fail(NF_E_DEVICE, "traceback stopped (status %d): no term of Eq. 1 attains a table entry", status);
    if (n > 0) std::copy(db.begin(), db.end(), db_out);
    return score;
}

int nf_fold_dev(const uint8_t* d_codes, int n, int q, int32_t* d_score, int16_t* d_S, void* stream)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    int rc = check_length(n);
    if (rc) return rc;
    if ((rc = check_q(q))) return rc;
    if (!d_codes && n > 0) return fail(NF_E_INVAL, "d_codes is NULL");
    if ((rc = ensure_device())) return rc;
    q = resolve_q(q, n);
    Plan* p = nullptr;
    if ((rc = single_plan(n, q, &p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Geom& g = p->geom[0];
    HIPCHK(launch_copy_codes(d_codes, n, (uint8_t*)p->h_folds[0].codes, (int)g.codes_bytes, s));
    if ((rc = plan_enqueue(*p, s))) return rc;
    if (d_score) HIPCHK(hipMemcpyAsync(d_score, p->d_scores.p, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (d_S && n > 0) HIPCHK(launch_expand(p->h_folds[0].F, g.ld, n, d_S, s));
    return NF_OK;
}

// ------------------------------------------------------------------ batches

int nf_batch_create(const char* const* seqs, const int* ns, int count, int q, nf_batch** out)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (!out) return fail(NF_E_INVAL, "out is NULL");
    *out = nullptr;
    if (count < 0 || (count > 0 && (!seqs || !ns))) return fail(NF_E_INVAL, "bad batch arguments");
    int rc = check_q(q);
    if (rc) return rc;
    for (int i = 0; i < count; ++i) {
        if ((rc = check_length(ns[i]))) return fail(rc, "sequence %d: %s", i, last_error());
        if (!seqs[i] && ns[i] > 0) return fail(NF_E_INVAL, "sequence %d is NULL", i);
    }
    std::vector<std::vector<uint8_t>> codes(count);
    for (int i = 0; i < count; ++i) {
        codes[i].resize(ns[i]);
        if ((rc = encode_sequence(seqs[i], ns[i], codes[i].data()))) return fail(rc, "sequence %d: %s", i, last_error());
    }
    if ((rc = ensure_device())) return rc;
    auto b = std::make_unique<nf_batch>();
    b->ns.assign(ns, ns + count);
    b->where.resize(count);
    // the group width of every fold, and one plan per width
    std::vector<int> qs(count), widths;
    for (int i = 0; i < count; ++i) {
        qs[i] = q ? q : resolve_q(0, ns[i]);
        if (std::find(widths.begin(), widths.end(), qs[i]) == widths.end()) widths.push_back(qs[i]);
    }
    std::sort(widths.begin(), widths.end(), [&](int x, int y) { return x > y; });
    for (size_t k = 0; k < widths.size(); ++k) {
        std::vector<int> group;
        for (int i = 0; i < count; ++i)
            if (qs[i] == widths[k]) {
                b->where[i] = {(int)k, (int)group.size()};
                group.push_back(ns[i]);
            }
        std::unique_ptr<Plan> p;
        if ((rc = make_plan(group, widths[k], p))) return rc;
        b->plans.push_back(std::move(p));
    }
    // zero-padded codes of every fold; the host buffers live until the copies finish
    hipStream_t s = ctx().stream;
    StreamFence fence{s};
    for (int i = 0; i < count; ++i) {
        Plan& p = b->plan_of(i);
        const int k = b->index_in(i);
        codes[i].resize(p.geom[k].codes_bytes, 0);
        HIPCHK(hipMemcpyAsync((void*)p.h_folds[k].codes, codes[i].data(), codes[i].size(), hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
    if (b->plans.size() > 1) {
        HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        for (size_t k = 1; k < b->plans.size(); ++k) {
            hipStream_t st = nullptr;
            hipEvent_t e = nullptr;
            HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            b->side.push_back(st);
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->joins.push_back(e);
        }
    }
    *out = b.release();
    return NF_OK;
}

int nf_batch_run(nf_batch* b, void* stream)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (!b) return fail(NF_E_INVAL, "batch is NULL");
    int rc = ensure_device();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (b->plans.size() > 1) HIPCHK(hipEventRecord(b->fork, s));
    for (size_t k = 1; k < b->plans.size(); ++k) {
        HIPCHK(hipStreamWaitEvent(b->side[k - 1], b->fork, 0));
        if ((rc = plan_enqueue(*b->plans[k], b->side[k - 1]))) return rc;
        HIPCHK(hipEventRecord(b->joins[k - 1], b->side[k - 1]));
    }
    if (!b->plans.empty() && (rc = plan_enqueue(*b->plans[0], s))) return rc;
    for (size_t k = 1; k < b->plans.size(); ++k) HIPCHK(hipStreamWaitEvent(s, b->joins[k - 1], 0));
    HIPCHK(hipEventRecord(b->done, s));
    b->ran = true;
    return NF_OK;
}

int nf_batch_scores(nf_batch* b, int32_t* scores_out)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (!b || !scores_out) return fail(NF_E_INVAL, "NULL argument");
    if (!b->ran) return fail(NF_E_INVAL, "batch has not been run");
    HIPCHK(hipEventSynchronize(b->done));
    std::vector<std::vector<int32_t>> per(b->plans.size());
    for (size_t k = 0; k < b->plans.size(); ++k) {
        per[k].resize(b->plans[k]->geom.size());
        if (!per[k].empty())
            HIPCHK(hipMemcpy(per[k].data(), b->plans[k]->d_scores.p, per[k].size() * sizeof(int32_t),
                             hipMemcpyDeviceToHost));
    }
    for (size_t i = 0; i < b->ns.size(); ++i) scores_out[i] = per[b->where[i].first][b->where[i].second];
    return NF_OK;
}

int nf_batch_table(nf_batch* b, int idx, int16_t* S_out)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (!b || !S_out) return fail(NF_E_INVAL, "NULL argument");
    if (idx < 0 || idx >= (int)b->ns.size()) return fail(NF_E_INVAL, "index %d out of range", idx);
    if (!b->ran) return fail(NF_E_INVAL, "batch has not been run");
    HIPCHK(hipEventSynchronize(b->done));
    const int n = b->ns[idx];
    if (n == 0) return NF_OK;
    const size_t bytes = (size_t)n * n * sizeof(int16_t);
    Plan& p = b->plan_of(idx);
    const int k = b->index_in(idx);
    int rc;
    if (b->S.bytes < bytes && (rc = b->S.alloc(bytes))) return rc;
    hipStream_t s = ctx().stream;
    StreamFence fence{s};
    HIPCHK(launch_expand(p.h_folds[k].F, p.geom[k].ld, n, (int16_t*)b->S.p, s));
    HIPCHK(hipMemcpyAsync(S_out, b->S.p, bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return NF_OK;
}

int nf_batch_structures(nf_batch* b, char* const* db_outs)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (!b || !db_outs) return fail(NF_E_INVAL, "NULL argument");
    if (!b->ran) return fail(NF_E_INVAL, "batch has not been run");
    HIPCHK(hipEventSynchronize(b->done));
    const int count = (int)b->ns.size();
    std::vector<int> idx;  // folds that get a structure
    size_t db_total = 0, sp_total = 0;
    for (int i = 0; i < count; ++i) {
        if (!db_outs[i] || b->ns[i] == 0) continue;
        idx.push_back(i);
        db_total += (size_t)b->ns[i];
        sp_total += 2 * (size_t)(b->ns[i] / 2 + 1);
    }
    if (idx.empty()) return NF_OK;
    // [work: one TracebackWork per fold][status: one int per fold][structures][spill]
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nw = idx.size();
    const size_t st_off = up(nw * sizeof(TracebackWork));
    const size_t db_off = st_off + up(nw * sizeof(int));
    const size_t sp_off = db_off + up(db_total);
    const size_t bytes = sp_off + sp_total * sizeof(int2);
    int rc;
    if (b->tb.bytes < bytes && (rc = b->tb.alloc(bytes))) return rc;
    char* base = (char*)b->tb.p;
    std::vector<TracebackWork> work(nw);
    size_t dbo = 0, spo = 0;
    for (size_t k = 0; k < nw; ++k) {
        const int i = idx[k], n = b->ns[i];
        const Plan& p = b->plan_of(i);
        const int f = b->index_in(i);
        TracebackWork& w = work[k];
        w.F = p.h_folds[f].F;
        w.codes = p.h_folds[f].codes;
        w.ld = p.geom[f].ld;
        w.n = n;
        w.spill_cap = n / 2 + 1;
        w.spill = (int2*)(base + sp_off) + spo;
        w.db = base + db_off + dbo;
        w.status = (int*)(base + st_off) + k;
        dbo += (size_t)n;
        spo += 2 * (size_t)w.spill_cap;
    }
    hipStream_t s = ctx().stream;
    std::vector<int> status(nw, 0);
    std::vector<char> db(db_total);
    StreamFence fence{s};
    HIPCHK(hipMemcpyAsync(base, work.data(), nw * sizeof(TracebackWork), hipMemcpyHostToDevice, s));
    HIPCHK(launch_traceback_many((const TracebackWork*)base, (int)nw, s));
    HIPCHK(hipMemcpyAsync(status.data(), base + st_off, nw * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(db.data(), base + db_off, db_total, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t k = 0; k < nw; ++k)
        if (status[k] != 0)
            return fail(NF_E_DEVICE, "traceback of fold %d stopped (status %d)", idx[k], status[k]);
    dbo = 0;
    for (size_t k = 0; k < nw; ++k) {
        const int n = b->ns[idx[k]];
        std::copy(db.begin() + dbo, db.begin() + dbo + n, db_outs[idx[k]]);
        dbo += (size_t)n;
    }
    return NF_OK;
}

int nf_batch_info(const nf_batch* b, int* count, size_t* device_bytes)
{
    clear_error();
    if (!b) return fail(NF_E_INVAL, "batch is NULL");
    if (count) *count = (int)b->ns.size();
    if (device_bytes) {
        size_t t = b->S.bytes + b->tb.bytes;
        for (auto& p : b->plans) t += p->device_bytes;
        *device_bytes = t;
    }
    return NF_OK;
}

void nf_batch_destroy(nf_batch* b)
{
    if (!b) return;
    std::lock_guard<std::recursive_mutex> lk(g_api);
    if (b->ran) (void)hipEventSynchronize(b->done);
    delete b;
}

int nf_fold_batch(const char* const* seqs, const int* ns, int count, int q, int32_t* scores_out,
                  int16_t* const* S_outs)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (!scores_out && count > 0) return fail(NF_E_INVAL, "scores_out is NULL");
    nf_batch* b = nullptr;
    int rc = nf_batch_create(seqs, ns, count, q, &b);
    if (rc) return rc;
    std::unique_ptr<nf_batch> hold(b);
    if ((rc = nf_batch_run(b, ctx().stream))) return rc;
    if ((rc = nf_batch_scores(b, scores_out))) return rc;
    if (S_outs)
        for (int i = 0; i < count; ++i)
            if (S_outs[i] && (rc = nf_batch_table(b, i, S_outs[i]))) return rc;
    return NF_OK;
}

// ------------------------------------------------------------------ serving

int nf_serve_config(size_t hbm_budget_bytes, int max_slots, int max_queue)
{
    clear_error();
    return serve_config(hbm_budget_bytes, max_slots, max_queue);
}

size_t nf_fold_bytes(int n, int q)
{
    if (n < 0 || n > NF_MAX_N || q < 0 || q > NF_Q_MAX) return 0;
    if (q == 0) {
        std::lock_guard<std::recursive_mutex> lk(g_api);
        q = resolve_q(0, n);
    }
    return serve_fold_bytes(n, q);
}

int64_t nf_submit(const char* seq, int n, int q, int flags)
{
    clear_error();
    return serve_submit(seq, n, q, flags);
}

int nf_poll(int64_t ticket, int32_t* score_out, int16_t* S_out)
{
    clear_error();
    return serve_poll(ticket, score_out, S_out, nullptr, 0, false);
}

int nf_wait(int64_t ticket, int timeout_ms, int32_t* score_out, int16_t* S_out)
{
    clear_error();
    return serve_poll(ticket, score_out, S_out, nullptr, timeout_ms, true);
}

int nf_poll_ex(int64_t ticket, int timeout_ms, int32_t* score_out, int16_t* S_out, char* db_out)
{
    clear_error();
    return serve_poll(ticket, score_out, S_out, db_out, timeout_ms, timeout_ms != 0);
}

int nf_serve_stats(nf_serve_stats_t* out)
{
    clear_error();
    if (!out) return fail(NF_E_INVAL, "out is NULL");
    return serve_stats(out);
}

// ------------------------------------------------------------------ tuning

int nf_autotune_q(int n)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (n < 0 || n > NF_MAX_N) return fail(NF_E_INVAL, "length %d out of range", n);
    return resolve_q(0, n);
}

int nf_autotune_target(int n, int q)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (n < 0 || n > NF_MAX_N) return fail(NF_E_INVAL, "length %d out of range", n);
    int rc = check_q(q);
    if (rc) return rc;
    return between_target(n, q);
}

int nf_autotune_wide(int n, int q)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (n < 0 || n > NF_MAX_N) return fail(NF_E_INVAL, "length %d out of range", n);
    int rc = check_q(q);
    if (rc) return rc;
    return stage_wide(n, resolve_q(q, n)) ? 1 : 0;
}

int nf_autotune(int n, int qmin, int qmax, int reps)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    return autotune_run(n, qmin, qmax, reps);
}

int nf_profile_fold(const uint8_t* d_codes, int n, int q, int reps, void* stream, nf_kernel_profile_t* out)
{
    std::lock_guard<std::recursive_mutex> lk(g_api);
    clear_error();
    if (!out || reps < 1) return fail(NF_E_INVAL, "bad profile arguments");
    int rc = check_length(n);
    if (rc) return rc;
    if ((rc = check_q(q))) return rc;
    if (!d_codes && n > 0) return fail(NF_E_INVAL, "d_codes is NULL");
    if ((rc = ensure_device())) return rc;
    q = resolve_q(q, n);
    Plan* p = nullptr;
    if ((rc = single_plan(n, q, &p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Geom& g = p->geom[0];
    HIPCHK(launch_copy_codes(d_codes, n, (uint8_t*)p->h_folds[0].codes, (int)g.codes_bytes, s));
    memset(out, 0, sizeof *out);
    out->q = q;
    out->tile = tile_size(q);
    out->tiles_per_side = g.NT;
    out->stages = p->sc.stages;
    out->wide = p->wide ? 1 : 0;
    return plan_profile(*p, s, reps, out);
}

}  // extern "C"

namespace nf {
// The serving engine takes the API lock for everything that touches the
// shared context (plans, R tables).
std::recursive_mutex& api_mutex() { return g_api; }
}  // namespace nf
