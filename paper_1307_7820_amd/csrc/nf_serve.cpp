// Serving engine: continuous batching of folds on one GPU.
//
// A background thread owns a device arena of `budget` bytes.  Each device
// step advances every active fold by one tile diagonal: the finishes of its
// current diagonal (on stream s1) and the between-group work of its next
// diagonal (on stream s2, overlapping the finishes, as in a single fold).
// Requests that arrive while others run are admitted at the next step when a
// slot and enough arena bytes are free; their codes, table, packed words and
// accumulators stay in the arena until the fold completes.  A finished fold's
// score (and table, if asked for) is copied to pinned host memory and the
// ticket completes when that copy has landed.  Results never depend on which
// other folds share a step: every fold's kernels read and write only its own
// arena block, and max is order-free.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <string>
#include <vector>

#include "nf_runtime.h"

namespace nf {

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kInflightSteps = 2;  // device steps queued ahead of the host
constexpr int kBypassLimit = 64;   // steps a blocked queue head may be overtaken
constexpr size_t kAlign = 256;

struct Request {
    int64_t ticket = 0;
    std::vector<uint8_t> codes;  // padded to the fold's codes block
    int n = 0, q = 8;
    bool want_table = false;
    bool want_structure = false;
    size_t bytes = 0;
};

struct Result {
    int status = 1;  // 1 = done, < 0 = error code
    int32_t score = 0;
    std::vector<int16_t> table;
    std::string structure;  // dot-bracket (want_structure)
};

// First-fit allocator over offsets of one device allocation.
class Arena {
public:
    void reset(size_t cap)
    {
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t sz, size_t* off)
    {
        sz = (sz + kAlign - 1) & ~(kAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= sz) {
                *off = it->first;
                const size_t rest = it->second - sz, at = it->first + sz;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t sz)
    {
        sz = (sz + kAlign - 1) & ~(kAlign - 1);
        auto it = free_.emplace(off, sz).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

struct Active {
    Request req;
    Geom g;
    size_t off = 0;
    FoldDesc fd{};
    int32_t* acc = nullptr;  // 2 * NT accumulators, [diagonal parity][A]
    int16_t* S = nullptr;    // expanded table (want_table)
    char* tb = nullptr;      // traceback area (want_structure): status, structure, spill
    int stage = 0;           // next diagonal to finish
    int slot = 0;            // index into the pinned score array
    int16_t* h_table = nullptr;
    char* h_db = nullptr;  // pinned: traceback status (int), then the structure
};

struct StepRec {
    hipEvent_t ev = nullptr;
    std::vector<Active*> finishing;
    int ring = 0;
};

struct Engine {
    // `life` orders submit, config and shutdown against one another: it is
    // the outermost lock, and the engine thread never takes it.
    std::mutex life;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    size_t budget = 0;
    int max_slots = 256;
    int max_queue = 65536;
    bool configured = false, running = false, stop = false;
    std::thread th;
    std::deque<Request> pending;
    std::unordered_map<int64_t, Result> done;
    std::unordered_set<int64_t> live;
    int64_t next_ticket = 1;
    nf_serve_stats_t st{};
    size_t held = 0;
    int head_bypassed = 0;
};

Engine& eng()
{
    static Engine e;
    return e;
}

// Traceback area of one fold: [status: kAlign][structure: n, rounded][spill]
size_t tb_bytes(int n)
{
    return kAlign + (((size_t)n + kAlign - 1) & ~(kAlign - 1)) + 2 * (size_t)(n / 2 + 1) * sizeof(int2);
}

size_t serve_bytes(const Geom& g, bool want_table, bool want_structure)
{
    size_t b = g.bytes + (size_t)2 * g.NT * kTileCells * sizeof(int32_t);
    if (want_table) b += (size_t)g.n * g.n * sizeof(int16_t) + kAlign;
    if (want_structure) b += tb_bytes(g.n) + kAlign;
    return b;
}

size_t default_budget()
{
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return (size_t)8 << 30;
    }
    return std::min((size_t)(fr * 0.8), (size_t)32 << 30);
}

// ---------------------------------------------------------------- engine thread

struct Device {
    DevBuf arena_mem;
    Arena arena;
    hipStream_t s1 = nullptr, s2 = nullptr;
    hipStream_t s3 = nullptr;  // tracebacks of finished folds, beside the steps
    // uploads of the steps' work lists: a step's copy runs while the steps
    // before it compute, so its launch does not wait for a copy on s1
    hipStream_t s0 = nullptr;
    hipEvent_t ev_tile = nullptr, ev_btw = nullptr;
    hipEvent_t ev_fin = nullptr, ev_end = nullptr;
    const uint8_t* R[NF_Q_MAX + 1] = {nullptr};
    // ring of item buffers (pinned staging + device copy)
    struct Ring {
        char* host = nullptr;
        DevBuf dev;
        size_t cap = 0;
        // completion of the step that uses this slot; reused, since a slot is
        // taken again only after that step has retired (at a launch at most
        // kInflightSteps - 1 steps are in flight, and there is one slot more)
        hipEvent_t step_ev = nullptr;
        hipEvent_t up_ev = nullptr;  // this slot's upload (on s0) is done
        bool used = false;
    } ring[kInflightSteps + 1];
    int32_t* h_scores = nullptr;  // pinned and mapped, one per slot: k_scores_to_slots writes here
    int32_t* h_scores_dev = nullptr;  // its device address
    std::vector<int> free_slots;
};

// The engine thread is ending: fail what it holds and mark it stopped in the
// same critical section, so that a later submit starts a new thread rather
// than queueing behind one that will never serve it.  The thread takes no
// lock after this, so a submit may join it while holding E.mu.
void fail_all(Engine& E, std::vector<Active*>& active, int code)
{
    std::lock_guard<std::mutex> lk(E.mu);
    E.running = false;
    E.held = 0;  // the thread's arena goes with it
    E.head_bypassed = 0;
    for (auto* a : active) {
        E.done[a->req.ticket] = Result{code, 0, {}};
        E.live.erase(a->req.ticket);
    }
    for (auto& r : E.pending) {
        E.done[r.ticket] = Result{code, 0, {}};
        E.live.erase(r.ticket);
    }
    E.pending.clear();
    E.cv_done.notify_all();
}

int engine_init(Engine& E, Device& D)
{
    {
        std::lock_guard<std::recursive_mutex> lk(api_mutex());
        int rc = ensure_device();
        if (rc) return rc;
    }
    HIPCHK(hipStreamCreateWithFlags(&D.s1, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&D.s2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&D.ev_tile, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&D.ev_btw, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&D.s3, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&D.s0, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&D.ev_fin, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&D.ev_end, hipEventDisableTiming));
    int rc = D.arena_mem.alloc(E.budget);
    if (rc) return rc;
    D.arena.reset(E.budget);
    HIPCHK(hipHostMalloc((void**)&D.h_scores, sizeof(int32_t) * E.max_slots, hipHostMallocMapped));
    HIPCHK(hipHostGetDevicePointer((void**)&D.h_scores_dev, D.h_scores, 0));
    for (int i = E.max_slots - 1; i >= 0; --i) D.free_slots.push_back(i);
    for (auto& r : D.ring) {
        HIPCHK(hipEventCreateWithFlags(&r.step_ev, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&r.up_ev, hipEventDisableTiming));
    }
    return NF_OK;
}

void engine_release(Device& D)
{
    if (D.s1) (void)hipStreamSynchronize(D.s1);
    if (D.s2) (void)hipStreamSynchronize(D.s2);
    if (D.s3) (void)hipStreamSynchronize(D.s3);
    if (D.s0) (void)hipStreamSynchronize(D.s0);
    for (auto& r : D.ring) {
        if (r.host) (void)hipHostFree(r.host);
        if (r.step_ev) (void)hipEventDestroy(r.step_ev);
        if (r.up_ev) (void)hipEventDestroy(r.up_ev);
        r.dev.reset();
    }
    if (D.h_scores) (void)hipHostFree(D.h_scores);
    D.h_scores = D.h_scores_dev = nullptr;
    D.arena_mem.reset();
    if (D.ev_tile) (void)hipEventDestroy(D.ev_tile);
    if (D.ev_btw) (void)hipEventDestroy(D.ev_btw);
    if (D.s1) (void)hipStreamDestroy(D.s1);
    if (D.s2) (void)hipStreamDestroy(D.s2);
    if (D.s0) (void)hipStreamDestroy(D.s0);
    if (D.ev_fin) (void)hipEventDestroy(D.ev_fin);
    if (D.ev_end) (void)hipEventDestroy(D.ev_end);
    if (D.s3) (void)hipStreamDestroy(D.s3);
}

int ensure_ring(Device::Ring& r, size_t bytes)
{
    if (r.cap >= bytes) return NF_OK;
    size_t cap = std::max(bytes, r.cap * 2);
    if (r.host) (void)hipHostFree(r.host);
    r.host = nullptr;
    HIPCHK(hipHostMalloc((void**)&r.host, cap, hipHostMallocDefault));
    int rc = r.dev.alloc(cap);
    if (rc) return rc;
    r.cap = cap;
    return NF_OK;
}

// Admit pending requests that fit (FIFO, with bounded overtaking of a head
// that does not fit).  Called with E.mu held.
void admit(Engine& E, Device& D, std::vector<Active*>& active, std::vector<Active*>& fresh)
{
    const int scan = 32;
    for (int idx = 0; idx < (int)E.pending.size() && idx < scan && (int)active.size() < E.max_slots;) {
        Request& r = E.pending[idx];
        size_t off = 0;
        if (D.free_slots.empty() || !D.arena.alloc(r.bytes, &off)) {
            if (idx == 0) {
                if (++E.head_bypassed > kBypassLimit) break;  // let the head in first
            }
            ++idx;
            continue;
        }
        if (idx == 0) E.head_bypassed = 0;
        auto* a = new Active();
        a->req = std::move(r);
        E.pending.erase(E.pending.begin() + idx);
        a->g = make_geom(a->req.n, a->req.q);
        a->off = off;
        char* base = (char*)D.arena_mem.p + off;
        const Geom& g = a->g;
        a->fd.codes = (const uint8_t*)base;
        a->fd.F = (int16_t*)(base + g.codes_bytes);
        a->fd.RS = (uint32_t*)(base + g.codes_bytes + g.F_bytes);
        a->fd.CS = (uint32_t*)(base + g.codes_bytes + g.F_bytes + g.rs_bytes);
        a->fd.n = g.n;
        a->fd.NT = g.NT;
        a->fd.ld = g.ld;
        a->acc = (int32_t*)(base + g.bytes);
        size_t tail = (g.bytes + (size_t)2 * g.NT * kTileCells * sizeof(int32_t) + kAlign - 1) & ~(kAlign - 1);
        if (a->req.want_table) {
            a->S = (int16_t*)(base + tail);
            tail = (tail + (size_t)g.n * g.n * sizeof(int16_t) + kAlign - 1) & ~(kAlign - 1);
        }
        if (a->req.want_structure) a->tb = base + tail;
        a->slot = D.free_slots.back();
        D.free_slots.pop_back();
        E.held += a->req.bytes;
        E.st.peak_bytes = std::max(E.st.peak_bytes, E.held);
        E.st.admitted++;
        active.push_back(a);
        fresh.push_back(a);
    }
}

// Complete the folds of a finished step.  Called without E.mu.
void complete(Engine& E, Device& D, StepRec& rec)
{
    std::vector<std::pair<int64_t, Result>> out;
    for (Active* a : rec.finishing) {
        Result res;
        res.score = D.h_scores[a->slot];
        if (a->req.want_table) {
            const size_t cnt = (size_t)a->req.n * a->req.n;
            res.table.assign(a->h_table, a->h_table + cnt);
            (void)hipHostFree(a->h_table);
        }
        if (a->req.want_structure) {
            int status = 0;
            std::memcpy(&status, a->h_db, sizeof status);
            if (status != 0)
                res.status = NF_E_DEVICE;  // the traceback found a table that is not Eq. 1's
            else
                res.structure.assign(a->h_db + sizeof(int), (size_t)a->req.n);
            (void)hipHostFree(a->h_db);
        }
        out.push_back({a->req.ticket, std::move(res)});
    }
    std::lock_guard<std::mutex> lk(E.mu);
    for (Active* a : rec.finishing) {
        D.arena.release(a->off, a->req.bytes);
        E.held -= a->req.bytes;
        D.free_slots.push_back(a->slot);
        delete a;
    }
    for (auto& kv : out) {
        E.live.erase(kv.first);
        E.done[kv.first] = std::move(kv.second);
        E.st.completed++;
    }
    E.cv_done.notify_all();
}

void engine_main()
{
    Engine& E = eng();
    Device D;
    int rc = engine_init(E, D);
    std::vector<Active*> active;
    if (rc) {
        fail_all(E, active, rc);
        engine_release(D);
        return;
    }
    std::deque<StepRec> inflight;
    int ring_next = 0;
    std::vector<TileWork> wdiag, wtile;
    std::vector<BetweenWork> wbtw;
    std::vector<FoldDesc> wfin;
    // between chunks per step over all active folds (NF_BETWEEN_TARGET overrides)
    const int target = between_target(-1, 0);
    // Engine steps are fused (one launch per q, no cross-stream waits) unless
    // NF_MODE = staged.  Unlike a batch, the engine holds at most max_slots
    // folds, and with up to 256 of them fused steps served the 2000-request
    // workload (mean n 1168, 2 GiB) at 7,930 folds/s on MI355X against 7,710
    // staged and 7,730 when steps above kFusedMaxTilesPerSide tiles were
    // staged.
    int force_mode = -1;
    if (const char* e = getenv("NF_MODE")) {
        if (strcmp(e, "fused") == 0) force_mode = kModeFused;
        if (strcmp(e, "staged") == 0) force_mode = kModeStaged;
    }

    for (;;) {
        std::vector<Active*> fresh;
        {
            std::unique_lock<std::mutex> lk(E.mu);
            if (E.stop) break;
            admit(E, D, active, fresh);
            E.st.active = (int64_t)active.size();
            E.st.pending = (int64_t)E.pending.size();
            bool steppable = false;
            for (auto* a : active)
                if (a->stage < a->g.NT) steppable = true;
            if (!steppable && inflight.empty()) {
                E.cv_work.wait_for(lk, std::chrono::milliseconds(50));
                continue;
            }
            if (!steppable) {  // nothing to launch: retire the oldest step
                lk.unlock();
                if (hipEventSynchronize(inflight.front().ev) != hipSuccess) {
                    rc = NF_E_DEVICE;
                    break;
                }
                complete(E, D, inflight.front());
                D.ring[inflight.front().ring].used = false;
                inflight.pop_front();
                continue;
            }
        }
        // R tables for any new q
        for (auto* a : fresh) {
            if (!D.R[a->req.q]) {
                std::lock_guard<std::recursive_mutex> lk(api_mutex());
                if ((rc = get_R(a->req.q, &D.R[a->req.q]))) break;
            }
        }
        if (rc) break;
        // bound the host's lead over the device
        while ((int)inflight.size() >= kInflightSteps) {
            if (hipEventSynchronize(inflight.front().ev) != hipSuccess) { rc = NF_E_DEVICE; break; }
            complete(E, D, inflight.front());
            D.ring[inflight.front().ring].used = false;
            inflight.pop_front();
        }
        if (rc) break;
        // Newly admitted folds: their padded codes go up with this step's
        // work lists, and their main-diagonal tiles copy them into place and
        // clear the fold's accumulators (launch_diag_admit), so admission
        // takes no copy or fill per fold.
        size_t nb_c = 0;
        for (auto* a : fresh) nb_c += (a->req.codes.size() + 15) & ~(size_t)15;

        // ---- work lists of this step
        wdiag.clear();
        wtile.clear();
        wbtw.clear();
        wfin.clear();
        StepRec rec;
        bool fused = false;
        long long W = 0;
        for (auto* a : active) {
            const int dd = a->stage + 1;
            if (a->stage < a->g.NT && dd >= 4 && dd < a->g.NT) W += (long long)(a->g.NT - dd) * (dd - 3);
        }
        const long long chunk = std::max<long long>(1, (W + target - 1) / target);
        std::vector<int> qs;
        for (auto* a : active) {
            if (a->stage >= a->g.NT) continue;
            const int s = a->stage, NT = a->g.NT;
            if (std::find(qs.begin(), qs.end(), a->req.q) == qs.end()) qs.push_back(a->req.q);
            if (s == 0) {
                for (int A = 0; A < NT; ++A) {
                    TileWork w{};
                    w.f = a->fd;
                    w.acc = a->acc;
                    w.A = A;
                    w.d = 0;
                    w.pad0 = a->req.q;
                    w.pad2 = 1;  // admission; pad1 (the staged codes) is set at the upload
                    wdiag.push_back(w);
                }
            } else {
                for (int A = 0; A < NT - s; ++A) {
                    TileWork w{};
                    w.f = a->fd;
                    w.acc = a->acc + ((size_t)((s & 1) * NT + A)) * kTileCells;
                    w.A = A;
                    w.d = s;
                    w.nslot = s >= 4 ? 1 : 0;
                    w.pad0 = a->req.q;
                    wtile.push_back(w);
                }
            }
            const int dd = s + 1;
            if (dd >= 4 && dd < NT) {
                const int nC = dd - 3;
                const int ns = (int)((nC + chunk - 1) / chunk);
                for (int A = 0; A < NT - dd; ++A)
                    for (int k = 0; k < ns; ++k) {
                        BetweenWork w{};
                        w.f = a->fd;
                        w.acc = a->acc + ((size_t)((dd & 1) * NT + A)) * kTileCells;
                        w.A = A;
                        w.d = dd;
                        w.c0 = A + 2 + (int)((long long)k * nC / ns);
                        w.c1 = A + 2 + (int)((long long)(k + 1) * nC / ns);
                        w.atomic = ns > 1 ? 1 : 0;
                        w.pad0 = a->req.q;
                        wbtw.push_back(w);
                    }
            }
            if (s + 1 == NT) {
                rec.finishing.push_back(a);
                wfin.push_back(a->fd);
                wfin.back().pad = a->slot;  // the score goes to h_scores[slot]
            }
        }
        // group each list by q (kernels are specialised per q); a list of one
        // q, the usual case, is already in order
        auto by_q = [](auto& v) {
            auto lt = [](const auto& x, const auto& y) { return x.pad0 < y.pad0; };
            if (!std::is_sorted(v.begin(), v.end(), lt)) std::stable_sort(v.begin(), v.end(), lt);
        };
        by_q(wdiag);
        by_q(wtile);
        by_q(wbtw);
        // ---- upload through the ring
        Device::Ring& rg = D.ring[ring_next];
        rec.ring = ring_next;
        ring_next = (ring_next + 1) % (kInflightSteps + 1);
        const size_t nb_d = wdiag.size() * sizeof(TileWork), nb_t = wtile.size() * sizeof(TileWork);
        const size_t nb_b = wbtw.size() * sizeof(BetweenWork), nb_f = wfin.size() * sizeof(FoldDesc);
        const size_t off_c = nb_d + nb_t + nb_b + nb_f;  // staged codes of the fresh folds (16-byte aligned)
        const size_t total = off_c + nb_c + 64;
        if (rg.used) (void)hipEventSynchronize(rg.step_ev);  // never taken: see Ring::step_ev
        if ((rc = ensure_ring(rg, total))) break;
        char* h = rg.host;
        {
            // each diagonal item (a fold at stage 0, admitted in this step)
            // reads its fold's codes at that fold's offset in the staged area
            std::vector<std::pair<const uint8_t*, size_t>> where;
            size_t c = off_c;
            for (auto* a : fresh) {
                std::memcpy(h + c, a->req.codes.data(), a->req.codes.size());
                where.push_back({a->fd.codes, c});
                c += (a->req.codes.size() + 15) & ~(size_t)15;
            }
            for (auto& w : wdiag) {
                auto it = std::find_if(where.begin(), where.end(), [&](const auto& x) { return x.first == w.f.codes; });
                if (it == where.end()) {
                    rc = fail(NF_E_DEVICE, "engine: a stage-0 fold was not admitted in this step");
                    break;
                }
                w.pad1 = (int)it->second;
            }
            if (rc) break;
        }
        std::memcpy(h, wdiag.data(), nb_d);
        std::memcpy(h + nb_d, wtile.data(), nb_t);
        std::memcpy(h + nb_d + nb_t, wbtw.data(), nb_b);
        std::memcpy(h + nb_d + nb_t + nb_b, wfin.data(), nb_f);
        char* dv = (char*)rg.dev.p;
        const TileWork* d_diag = (const TileWork*)dv;
        const TileWork* d_tile = (const TileWork*)(dv + nb_d);
        const BetweenWork* d_btw = (const BetweenWork*)(dv + nb_d + nb_t);
        const FoldDesc* d_fin = (const FoldDesc*)(dv + nb_d + nb_t + nb_b);
        bool ok = hipMemcpyAsync(dv, h, off_c + nb_c, hipMemcpyHostToDevice, D.s0) == hipSuccess &&
                  hipEventRecord(rg.up_ev, D.s0) == hipSuccess && hipStreamWaitEvent(D.s1, rg.up_ev, 0) == hipSuccess;
        // ---- launches
        // s1 already follows the previous step's between work: a staged step
        // ends with s1 waiting for s2, a fused one runs it on s1.  A fused
        // step uses s1 alone; a staged one runs its between work on s2 after
        // the previous finishes and this step's items are in place.
        fused = force_mode != kModeStaged;
        if (!fused) ok = ok && hipEventRecord(D.ev_tile, D.s1) == hipSuccess;
        auto launch_groups = [&](auto* dptr, auto& v, int which, hipStream_t st) {
            size_t b = 0;
            while (ok && b < v.size()) {
                size_t e = b;
                while (e < v.size() && v[e].pad0 == v[b].pad0) ++e;
                const int q = v[b].pad0;
                hipError_t he;
                if (which == 0) he = launch_diag_admit(q, (const TileWork*)dptr + b, (int)(e - b), (const uint8_t*)dv, st);
                else if (which == 1)
                    he = launch_tile(q, (const TileWork*)dptr + b, (int)(e - b), D.R[q], st, nullptr, nullptr, true);
                else he = launch_between(q, (const BetweenWork*)dptr + b, (int)(e - b), D.R[q], st);
                ok = he == hipSuccess;
                b = e;
            }
        };
        launch_groups(d_diag, wdiag, 0, D.s1);
        if (fused) {
            // one launch per q on s1 holding the finishes of this step and the
            // between work of the next diagonals: that work reads only tiles
            // finished in earlier steps (the previous step's between work on
            // s2, if any, was waited for above)
            size_t bt = 0, bb = 0;
            while (ok && (bt < wtile.size() || bb < wbtw.size())) {
                const int q = std::min(bt < wtile.size() ? wtile[bt].pad0 : NF_Q_MAX + 1,
                                       bb < wbtw.size() ? wbtw[bb].pad0 : NF_Q_MAX + 1);
                size_t et = bt, eb = bb;
                while (et < wtile.size() && wtile[et].pad0 == q) ++et;
                while (eb < wbtw.size() && wbtw[eb].pad0 == q) ++eb;
                ok = launch_stage(q, false, d_tile + bt, (int)(et - bt), d_btw + bb, (int)(eb - bb), D.R[q],
                                  D.s1) == hipSuccess;
                bt = et;
                bb = eb;
            }
        } else {
            launch_groups(d_tile, wtile, 1, D.s1);
            ok = ok && hipStreamWaitEvent(D.s2, D.ev_tile, 0) == hipSuccess;
            launch_groups(d_btw, wbtw, 2, D.s2);
            ok = ok && hipEventRecord(D.ev_btw, D.s2) == hipSuccess;
        }
        // finished folds: score (and table) to pinned memory; structures are
        // traced back on s3 once this step's finishes are done, so the next
        // steps on s1 do not wait for them
        bool any_tb = false;
        if (ok && !rec.finishing.empty()) {
            ok = launch_scores_to_slots(d_fin, (int)wfin.size(), D.h_scores_dev, D.s1) == hipSuccess;
            for (size_t k = 0; ok && k < rec.finishing.size(); ++k) {
                Active* a = rec.finishing[k];
                if (a->req.want_table && a->req.n > 0) {
                    const size_t cnt = (size_t)a->req.n * a->req.n;
                    ok = hipHostMalloc((void**)&a->h_table, cnt * sizeof(int16_t), hipHostMallocDefault) ==
                         hipSuccess;
                    ok = ok && launch_expand(a->fd.F, a->g.ld, a->req.n, a->S, D.s1) == hipSuccess;
                    ok = ok && hipMemcpyAsync(a->h_table, a->S, cnt * sizeof(int16_t), hipMemcpyDeviceToHost,
                                              D.s1) == hipSuccess;
                } else if (ok && a->req.want_table) {
                    ok = hipHostMalloc((void**)&a->h_table, 16, hipHostMallocDefault) == hipSuccess;
                }
                if (ok && a->req.want_structure) {
                    // one optimal structure, read back on the device before the
                    // fold's memory is released
                    const int n = a->req.n;
                    ok = hipHostMalloc((void**)&a->h_db, sizeof(int) + (size_t)n + 16, hipHostMallocDefault) ==
                         hipSuccess;
                    if (ok && n > 0) {
                        if (!any_tb) {
                            ok = hipEventRecord(D.ev_fin, D.s1) == hipSuccess &&
                                 hipStreamWaitEvent(D.s3, D.ev_fin, 0) == hipSuccess;
                            any_tb = true;
                        }
                        char* db = a->tb + kAlign;
                        int2* spill = (int2*)(db + (((size_t)n + kAlign - 1) & ~(kAlign - 1)));
                        ok = ok && launch_traceback(a->fd.F, a->g.ld, a->fd.codes, n, spill, n / 2 + 1, db,
                                                    (int*)a->tb, D.s3) == hipSuccess;
                        ok = ok && hipMemcpyAsync(a->h_db, a->tb, sizeof(int), hipMemcpyDeviceToHost, D.s3) ==
                                       hipSuccess;
                        ok = ok && hipMemcpyAsync(a->h_db + sizeof(int), db, (size_t)n, hipMemcpyDeviceToHost,
                                                  D.s3) == hipSuccess;
                    } else if (ok) {
                        std::memset(a->h_db, 0, sizeof(int));
                    }
                }
            }
        }
        // the step is complete when both streams are through it
        if (!fused) ok = ok && hipStreamWaitEvent(D.s1, D.ev_btw, 0) == hipSuccess;
        rec.ev = rg.step_ev;
        if (any_tb) {  // ... and the tracebacks on s3
            ok = ok && hipEventRecord(D.ev_end, D.s1) == hipSuccess;
            ok = ok && hipStreamWaitEvent(D.s3, D.ev_end, 0) == hipSuccess;
            ok = ok && hipEventRecord(rec.ev, D.s3) == hipSuccess;
        } else {
            ok = ok && hipEventRecord(rec.ev, D.s1) == hipSuccess;
        }
        if (!ok) {
            (void)hipGetLastError();
            rc = NF_E_DEVICE;
            break;
        }
        rg.used = true;
        for (auto* a : active)
            if (a->stage < a->g.NT) a->stage++;
        {
            std::lock_guard<std::mutex> lk(E.mu);
            E.st.steps++;
            if (fused) E.st.steps_fused++;
        }
        // finished folds leave the active set now; they complete with rec
        active.erase(std::remove_if(active.begin(), active.end(),
                                    [&](Active* a) {
                                        return std::find(rec.finishing.begin(), rec.finishing.end(), a) !=
                                               rec.finishing.end();
                                    }),
                     active.end());
        inflight.push_back(std::move(rec));
        // opportunistic completion of steps the device has already finished
        while (!inflight.empty() && hipEventQuery(inflight.front().ev) == hipSuccess) {
            complete(E, D, inflight.front());
            D.ring[inflight.front().ring].used = false;
            inflight.pop_front();
        }
    }
    // drain what is in flight, then fail or abort the rest
    for (auto& r : inflight) {
        if (rc == NF_OK && hipEventSynchronize(r.ev) == hipSuccess) {
            complete(E, D, r);
        } else {
            for (auto* a : r.finishing) active.push_back(a);
        }
    }
    inflight.clear();
    const int code = rc ? rc : NF_E_ABORTED;
    fail_all(E, active, code);
    for (auto* a : active) {
        if (a->h_table) (void)hipHostFree(a->h_table);
        if (a->h_db) (void)hipHostFree(a->h_db);
        delete a;
    }
    engine_release(D);
}

}  // namespace

// ---------------------------------------------------------------- API side

int serve_config(size_t budget, int max_slots, int max_queue)
{
    Engine& E = eng();
    std::lock_guard<std::mutex> life(E.life);
    std::lock_guard<std::mutex> lk(E.mu);
    if (E.running) return fail(NF_E_BUSY, "serving engine already running; call nf_shutdown first");
    if (max_slots < 0 || max_queue < 0) return fail(NF_E_INVAL, "negative limits");
    E.budget = budget;
    E.max_slots = max_slots ? max_slots : 256;
    E.max_queue = max_queue ? max_queue : 65536;
    E.configured = true;
    E.st = nf_serve_stats_t{};
    return NF_OK;
}

size_t serve_fold_bytes(int n, int q) { return serve_bytes(make_geom(n, q), false, false); }

int64_t serve_submit(const char* seq, int n, int q, int flags)
{
    int rc = check_length(n);
    if (rc) return rc;
    if ((rc = check_q(q))) return rc;
    if (!seq && n > 0) return fail(NF_E_INVAL, "seq is NULL");
    Request r;
    {
        std::lock_guard<std::recursive_mutex> lk(api_mutex());
        q = resolve_q(q, n);
    }
    Geom g = make_geom(n, q);
    r.codes.assign(g.codes_bytes, 0);
    if ((rc = encode_sequence(seq, n, r.codes.data()))) return rc;
    r.n = n;
    r.q = q;
    if (flags & ~(NF_WANT_TABLE | NF_WANT_STRUCTURE)) return fail(NF_E_INVAL, "unknown flags 0x%x", flags);
    r.want_table = (flags & NF_WANT_TABLE) != 0;
    r.want_structure = (flags & NF_WANT_STRUCTURE) != 0;
    r.bytes = serve_bytes(g, r.want_table, r.want_structure);
    Engine& E = eng();
    std::lock_guard<std::mutex> life(E.life);
    std::unique_lock<std::mutex> lk(E.mu);
    if (!E.running) {
        if (!E.configured) {
            E.max_slots = 256;
            E.max_queue = 65536;
            E.configured = true;
            E.st = nf_serve_stats_t{};
        }
        if (E.budget == 0) {
            lk.unlock();
            size_t b;
            {
                std::lock_guard<std::recursive_mutex> alk(api_mutex());
                rc = ensure_device();
                b = rc ? 0 : default_budget();
            }
            if (rc) return rc;
            lk.lock();
            if (E.budget == 0) E.budget = b;
        }
    }
    if (r.bytes > E.budget) {
        E.st.rejected++;
        return fail(NF_E_NOMEM, "fold needs %zu device bytes; the serving budget is %zu", r.bytes, E.budget);
    }
    if ((int)E.pending.size() >= E.max_queue) {
        E.st.rejected++;
        return fail(NF_E_BUSY, "serving queue full (%d requests)", E.max_queue);
    }
    if (!E.running) {
        if (E.th.joinable()) E.th.join();  // a thread that has ended: it no longer takes E.mu
        E.stop = false;
        E.running = true;
        E.st.budget_bytes = E.budget;
        E.th = std::thread(engine_main);
    }
    r.ticket = E.next_ticket++;
    const int64_t t = r.ticket;
    E.live.insert(t);
    E.pending.push_back(std::move(r));
    E.st.submitted++;
    E.cv_work.notify_one();
    return t;
}

int serve_poll(int64_t ticket, int32_t* score_out, int16_t* S_out, char* db_out, int timeout_ms, bool blocking)
{
    Engine& E = eng();
    std::unique_lock<std::mutex> lk(E.mu);
    const auto deadline = Clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    for (;;) {
        auto it = E.done.find(ticket);
        if (it != E.done.end()) {
            Result res = std::move(it->second);
            E.done.erase(it);
            if (res.status < 0) return fail(res.status, "ticket %lld did not complete", (long long)ticket);
            if (score_out) *score_out = res.score;
            if (S_out && !res.table.empty()) std::memcpy(S_out, res.table.data(), res.table.size() * sizeof(int16_t));
            if (db_out && !res.structure.empty()) std::memcpy(db_out, res.structure.data(), res.structure.size());
            return 1;
        }
        if (!E.live.count(ticket)) return fail(NF_E_NOTFOUND, "unknown or released ticket %lld", (long long)ticket);
        if (!blocking) return 0;
        if (timeout_ms < 0) {
            E.cv_done.wait(lk);
        } else if (E.cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            if (E.done.count(ticket)) continue;
            return fail(NF_E_TIMEOUT, "ticket %lld still pending after %d ms", (long long)ticket, timeout_ms);
        }
    }
}

int serve_stats(nf_serve_stats_t* out)
{
    Engine& E = eng();
    std::lock_guard<std::mutex> lk(E.mu);
    *out = E.st;
    out->pending = (int64_t)E.pending.size();
    out->budget_bytes = E.budget;
    return NF_OK;
}

void serve_shutdown()
{
    Engine& E = eng();
    std::lock_guard<std::mutex> life(E.life);
    {
        std::lock_guard<std::mutex> lk(E.mu);
        if (!E.running && !E.th.joinable()) return;
        E.stop = true;
        E.cv_work.notify_all();
    }
    if (E.th.joinable()) E.th.join();
    std::lock_guard<std::mutex> lk(E.mu);
    E.running = false;
    E.stop = false;
    E.configured = false;
    E.budget = 0;
    E.held = 0;
    E.head_bypassed = 0;
    E.st = nf_serve_stats_t{};
}

}  // namespace nf
