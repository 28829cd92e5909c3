// Host runtime behind the C ABI of include/nf.h: device context, R cache,
// fold plans (workspace + packed wavefront schedule + captured HIP graph),
// prepared batches, the serving engine and the q autotuner.
#include "nf.h"
#include "nf_test.h"
#include "nf_internal.h"
#include "nf_runtime.h"

#include <algorithm>
#include <random>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

namespace nf {

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char* last_error() { return g_err.c_str(); }
void clear_error() { g_err.clear(); }

// ------------------------------------------------------------------ device memory

static std::mutex g_hook_mu;
static AllocHook g_hook;

int set_allocator(const AllocHook& h)
{
    if ((h.alloc == nullptr) != (h.free_ == nullptr))
        return fail(NF_E_INVAL, "nf_set_allocator needs both functions, or neither");
    std::lock_guard<std::mutex> lk(g_hook_mu);
    g_hook = h;
    return NF_OK;
}

static AllocHook current_hook()
{
    std::lock_guard<std::mutex> lk(g_hook_mu);
    return g_hook;
}

DevBuf::~DevBuf() { reset(); }
void DevBuf::reset()
{
    if (p) {
        if (from.free_) {
            // the owner of a hooked allocator may hand the block out again at
            // once (a caching allocator does): no kernel may still use it
            (void)hipDeviceSynchronize();
            from.free_(p, from.ctx);
        } else {
            (void)hipFree(p);
        }
    }
    p = nullptr;
    bytes = 0;
    from = AllocHook{};
}
int DevBuf::alloc(size_t nbytes)
{
    reset();
    if (nbytes == 0) return NF_OK;
    const AllocHook h = current_hook();
    if (h.alloc) {
        p = h.alloc(nbytes, h.ctx);
        if (!p) return fail(NF_E_NOMEM, "allocator hook returned NULL for %zu bytes", nbytes);
        if ((uintptr_t)p & 255) {
            h.free_(p, h.ctx);
            p = nullptr;
            return fail(NF_E_INVAL, "allocator hook returned an address not aligned to 256 bytes");
        }
        from = h;
        bytes = nbytes;
        return NF_OK;
    }
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return fail(NF_E_NOMEM, "hipMalloc(%zu bytes): %s", nbytes, hipGetErrorString(e));
    }
    bytes = nbytes;
    return NF_OK;
}

// ------------------------------------------------------------------ encoding

int encode_sequence(const char* seq, int n, uint8_t* out)
{
    for (int i = 0; i < n; ++i) {
        switch (seq[i]) {
        case 'A': case 'a': out[i] = 0; break;
        case 'C': case 'c': out[i] = 1; break;
        case 'G': case 'g': out[i] = 2; break;
        case 'U': case 'u': out[i] = 3; break;
        default:
            return fail(NF_E_INVAL, "base %d is 0x%02x, not one of A, C, G, U", i, (unsigned char)seq[i]);
        }
    }
    return NF_OK;
}

int check_length(int n)
{
    if (n < 0) return fail(NF_E_INVAL, "negative length %d", n);
    if (n > NF_MAX_N) return fail(NF_E_TOOLONG, "length %d exceeds NF_MAX_N (%d)", n, NF_MAX_N);
    return NF_OK;
}

// ------------------------------------------------------------------ context

Context& ctx()
{
    static Context c;
    return c;
}

int ensure_device()
{
    Context& c = ctx();
    if (c.ready) {
        HIPCHK(hipSetDevice(c.device));
        return NF_OK;
    }
    int dev = c.requested_device;
    if (const char* env = getenv("NF_DEVICE")) dev = atoi(env);
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(NF_E_DEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    }
    if (dev < 0 || dev >= count) return fail(NF_E_DEVICE, "device %d out of range (count %d)", dev, count);
    HIPCHK(hipSetDevice(dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(NF_E_DEVICE, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
    // the static scratch of the allocation-free entry point; a failed lookup
    // only disables that entry point, which reports it
    if (scratch_setup(dev) != NF_OK) clear_error();
    c.device = dev;
    c.num_cu = prop.multiProcessorCount;
    HIPCHK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&c.capture_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&c.side_stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c.ev_tile, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c.ev_btw, hipEventDisableTiming));
    c.ready = true;
    return NF_OK;
}

int get_R(int q, const uint8_t** out)
{
    Context& c = ctx();
    if (q < NF_Q_MIN || q > NF_Q_MAX) return fail(NF_E_INVAL, "q = %d outside %d..%d", q, NF_Q_MIN, NF_Q_MAX);
    DevBuf& b = c.R[q];
    if (!b.p) {
        const size_t bytes = (size_t)1 << (2 * (q - 1));
        int rc = b.alloc(bytes < 16 ? 16 : bytes);
        if (rc) return rc;
        HIPCHK(launch_precompute_R(q, (uint8_t*)b.p, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
    }
    *out = (const uint8_t*)b.p;
    return NF_OK;
}

// ------------------------------------------------------------------ geometry & schedule

Geom make_geom(int n, int q)
{
    Geom g;
    const int T = tile_size(q);
    g.n = n;
    g.NT = (n + 1 + T - 1) / T;
    g.ld = g.NT * T;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    g.codes_bytes = up((size_t)g.NT * T + 64);
    g.F_bytes = up((size_t)g.ld * g.ld * sizeof(int16_t));
    g.rs_bytes = up((size_t)tile_count(g.NT) * row_words(q) * sizeof(uint32_t));
    g.cs_bytes = up((size_t)tile_count(g.NT) * state_words(q) * sizeof(uint32_t));
    g.bytes = g.codes_bytes + g.F_bytes + g.rs_bytes + g.cs_bytes;
    return g;
}

static int bucket_of(int n);
static void load_tune_file();

// Between chunks per wavefront step: NF_BETWEEN_TARGET if set; else, for a
// single fold (n_single >= 0) at the q tuned for its length bucket (or q = 0,
// which resolves to it), the target tuned with that q; else enough
// workgroups to fill the device.  A target is tuned for one q only: another
// q has another amount of between work per step.
int between_target(int n_single, int q)
{
    const char* e = getenv("NF_BETWEEN_TARGET");
    const int env = e ? atoi(e) : 0;
    if (env > 0) return env;
    if (n_single >= 0) {
        load_tune_file();
        const int b = bucket_of(n_single);
        const int t = ctx().tuned_target[b];
        if (t > 0 && (q == 0 || q == ctx().tuned_q[b])) return t;
    }
    return kDefaultTarget;
}

bool stage_wide(int n_single, int q)
{
    if (q != 8 || n_single < 0) return false;
    if (const char* e = getenv("NF_STAGE_WIDE")) return atoi(e) != 0;
    load_tune_file();
    const int b = bucket_of(n_single);
    if (ctx().tuned_wide[b] && ctx().tuned_q[b] == q) return ctx().tuned_wide[b] == 2;
    return n_single >= 8192;
}

// Append the between-group items of diagonal dd for the listed folds.  The
// intermediate tiles C in [A+2, A+dd-2] of every tile are cut into chunks of
// about equal work so that the step has roughly `target` workgroups.  Every
// tile owns one accumulator slot (numbered from *next_slot); when a tile is
// split its chunks combine there with atomic max, otherwise the single item
// stores.  The tile finish reads the slot and clears it for its next use.
void append_between(const std::vector<std::pair<int, int>>& folds_nt, int dd, int target,
                    std::vector<BetweenItem>& out, int* next_slot,
                    std::vector<std::vector<std::pair<int, int>>>& pending)
{
    if (dd < 4) return;
    long long W = 0;
    for (auto& fn : folds_nt)
        if (fn.second > dd) W += (long long)(fn.second - dd) * (dd - 3);
    if (W == 0) return;
    const long long chunk = std::max<long long>(kMinChunkTiles, (W + target - 1) / target);
    const int nC = dd - 3;
    const int ns = (int)((nC + chunk - 1) / chunk);
    for (auto& fn : folds_nt) {
        const int f = fn.first, NT = fn.second;
        if (NT <= dd) continue;
        auto& pend = pending[f];
        pend.assign(NT - dd, {0, 0});
        for (int A = 0; A < NT - dd; ++A) {
            const int slot = (*next_slot)++;
            for (int s = 0; s < ns; ++s) {
                BetweenItem it{};
                it.fold = f;
                it.A = A;
                it.d = dd;
                it.c0 = A + 2 + (int)((long long)s * nC / ns);
                it.c1 = A + 2 + (int)((long long)(s + 1) * nC / ns);
                it.slot = slot;
                it.pad0 = ns > 1 ? 1 : 0;
                out.push_back(it);
            }
            pend[A] = {slot, 1};
        }
    }
}

void build_schedule(const std::vector<int>& NTs, int target, Schedule& sc)
{
    const int nf = (int)NTs.size();
    int stages = 0;
    for (int v : NTs) stages = std::max(stages, v);
    sc = Schedule{};
    sc.stages = stages;
    sc.tile_off.assign(stages, 0);
    sc.tile_cnt.assign(stages, 0);
    sc.btw_off.assign(stages, 0);
    sc.btw_cnt.assign(stages, 0);
    std::vector<std::vector<std::pair<int, int>>> pending(nf);
    std::vector<int> btw_stage_local;  // local slot per between item
    std::vector<int> btw_stage;        // stage of each between item
    std::vector<int> tile_stage;
    std::vector<std::pair<int, int>> folds_nt;
    folds_nt.reserve(nf);
    for (int f = 0; f < nf; ++f) folds_nt.push_back({f, NTs[f]});
    int max_slots = 0;
    for (int sg = 0; sg < stages; ++sg) {
        if (sg == 0) {
            for (int f = 0; f < nf; ++f)
                for (int A = 0; A < NTs[f]; ++A) sc.diag.push_back(TileItem{f, A, 0, 0, 0, 0, 0, 0});
        } else {
            sc.tile_off[sg] = (int)sc.tile.size();
            for (int f = 0; f < nf; ++f) {
                if (NTs[f] <= sg) continue;
                for (int A = 0; A < NTs[f] - sg; ++A) {
                    TileItem it{f, A, sg, 0, 0, 0, 0, 0};
                    if (sg >= 4) {
                        it.slot0 = pending[f][A].first;
                        it.nslot = pending[f][A].second;
                    }
                    sc.tile.push_back(it);
                    tile_stage.push_back(sg);
                }
            }
            sc.tile_cnt[sg] = (int)sc.tile.size() - sc.tile_off[sg];
        }
        sc.btw_off[sg] = (int)sc.btw.size();
        int local = 0;
        append_between(folds_nt, sg + 1, target, sc.btw, &local, pending);
        sc.btw_cnt[sg] = (int)sc.btw.size() - sc.btw_off[sg];
        for (int k = 0; k < sc.btw_cnt[sg]; ++k) btw_stage.push_back(sg);
        max_slots = std::max(max_slots, local);
    }
    // Accumulator slots are double-buffered by stage parity: the items of
    // stage s write half (s & 1) while the tiles of stage s read (and clear)
    // what stage s-1 wrote.
    sc.max_slots = max_slots;
    for (size_t k = 0; k < sc.btw.size(); ++k) sc.btw[k].slot += (btw_stage[k] & 1) * max_slots;
    for (size_t k = 0; k < sc.tile.size(); ++k)
        if (sc.tile[k].nslot > 0) sc.tile[k].slot0 += ((tile_stage[k] - 1) & 1) * max_slots;
}

// Execution of a new plan.  NF_MODE = "staged" or "fused" forces one (see
// PlanMode); otherwise fused steps for one fold and for batches whose steps
// hold few tiles (kFusedMaxTilesPerSide).

bool plain_between_for(int q)
{
    const char* e = getenv("NF_BETWEEN");
    return e && strcmp(e, "plain") == 0 && tile_size(q) == 64;
}

// The between launch of a staged step: the lookup kernel, or the plain one.
static hipError_t launch_btw(const Plan& p, const BetweenWork* items, int nitems, const uint8_t* R, hipStream_t s,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    return p.plain ? launch_between_plain(p.q, items, nitems, s, e0, e1)
                   : launch_between(p.q, items, nitems, R, s, e0, e1);
}

int plan_mode_for(const std::vector<int>& NTs)
{
    if (const char* e = getenv("NF_MODE")) {  // read per plan: cached plans keep their mode
        if (strcmp(e, "fused") == 0) return kModeFused;
        if (strcmp(e, "staged") == 0) return kModeStaged;
    }
    if (NTs.size() == 1) return kModeFused;
    long long sum = 0;
    for (int nt : NTs) sum += nt;
    return sum <= kFusedMaxTilesPerSide ? (int)kModeFused : (int)kModeStaged;
}

// ------------------------------------------------------------------ plans

Plan::~Plan() { release_graph(); }

void Plan::release_graph()
{
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
}

static bool use_graphs()
{
    static bool g = [] {
        const char* e = getenv("NF_GRAPH");
        return !(e && e[0] == '0');
    }();
    return g;
}

TileWork to_work(const TileItem& it, const std::vector<FoldDesc>& fd, int32_t* acc_base)
{
    TileWork w{};
    w.f = fd[it.fold];
    w.acc = acc_base + (size_t)it.slot0 * kTileCells;
    w.A = it.A;
    w.d = it.d;
    w.nslot = it.nslot;
    return w;
}

BetweenWork to_work(const BetweenItem& it, const std::vector<FoldDesc>& fd, int32_t* acc_base)
{
    BetweenWork w{};
    w.f = fd[it.fold];
    w.acc = acc_base + (size_t)it.slot * kTileCells;
    w.A = it.A;
    w.d = it.d;
    w.c0 = it.c0;
    w.c1 = it.c1;
    w.atomic = it.pad0;
    return w;
}

// Allocate the device side of a plan whose geoms and schedule are set.
int plan_allocate(Plan& p)
{
    size_t arena = 0;
    for (auto& g : p.geom) arena += g.bytes;
    int rc = p.arena.alloc(arena);
    if (rc) return rc;
    std::vector<FoldDesc> fd(p.geom.size());
    size_t off = 0;
    char* base = (char*)p.arena.p;
    for (size_t f = 0; f < p.geom.size(); ++f) {
        const Geom& g = p.geom[f];
        fd[f].codes = (const uint8_t*)(base + off);
        fd[f].F = (int16_t*)(base + off + g.codes_bytes);
        fd[f].RS = (uint32_t*)(base + off + g.codes_bytes + g.F_bytes);
        fd[f].CS = (uint32_t*)(base + off + g.codes_bytes + g.F_bytes + g.rs_bytes);
        fd[f].n = g.n;
        fd[f].NT = g.NT;
        fd[f].ld = g.ld;
        p.geom[f].codes_off = off;
        off += g.bytes;
    }
    p.h_folds = fd;
    const Schedule& sc = p.sc;
    if ((rc = p.d_folds.alloc(fd.size() * sizeof(FoldDesc)))) return rc;
    if ((rc = p.d_part.alloc(std::max<size_t>(1, (size_t)2 * sc.max_slots) * kTileCells * sizeof(int32_t))))
        return rc;
    // device work lists with the fold descriptors and accumulator addresses folded in
    int32_t* acc_base = (int32_t*)p.d_part.p;
    std::vector<TileWork> wd(sc.diag.size()), wt(sc.tile.size());
    std::vector<BetweenWork> wb(sc.btw.size());
    for (size_t k = 0; k < sc.diag.size(); ++k) wd[k] = to_work(sc.diag[k], fd, acc_base);
    for (size_t k = 0; k < sc.tile.size(); ++k) wt[k] = to_work(sc.tile[k], fd, acc_base);
    for (size_t k = 0; k < sc.btw.size(); ++k) wb[k] = to_work(sc.btw[k], fd, acc_base);
    if ((rc = p.d_diag.alloc(std::max<size_t>(1, wd.size()) * sizeof(TileWork)))) return rc;
    if ((rc = p.d_tile.alloc(std::max<size_t>(1, wt.size()) * sizeof(TileWork)))) return rc;
    if ((rc = p.d_btw.alloc(std::max<size_t>(1, wb.size()) * sizeof(BetweenWork)))) return rc;
    if ((rc = p.d_scores.alloc(std::max<size_t>(1, fd.size()) * sizeof(int32_t)))) return rc;
    hipStream_t s = ctx().stream;
    StreamFence fence{s};  // fd, wd, wt and wb are read by the copies below
    // accumulators start at zero (max with 0 is neutral: every score is >= 0)
    HIPCHK(hipMemsetAsync(p.d_part.p, 0, p.d_part.bytes, s));
    HIPCHK(hipMemcpyAsync(p.d_folds.p, fd.data(), fd.size() * sizeof(FoldDesc), hipMemcpyHostToDevice, s));
    if (!wd.empty())
        HIPCHK(hipMemcpyAsync(p.d_diag.p, wd.data(), wd.size() * sizeof(TileWork), hipMemcpyHostToDevice, s));
    if (!wt.empty())
        HIPCHK(hipMemcpyAsync(p.d_tile.p, wt.data(), wt.size() * sizeof(TileWork), hipMemcpyHostToDevice, s));
    if (!wb.empty())
        HIPCHK(hipMemcpyAsync(p.d_btw.p, wb.data(), wb.size() * sizeof(BetweenWork), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    p.device_bytes = p.arena.bytes + p.d_folds.bytes + p.d_diag.bytes + p.d_tile.bytes + p.d_btw.bytes +
                     p.d_part.bytes + p.d_scores.bytes;
    return NF_OK;
}

// Fused steps: one launch per step on one stream.  Kernel order alone gives
//     finish(s)  after between(s)  (in launch s-1)
//     between(s+1) after finish(s-1) (launch s-1)
static int plan_enqueue_fused(Plan& p, hipStream_t s)
{
    const uint8_t* R = nullptr;
    int rc = get_R(p.q, &R);
    if (rc) return rc;
    const Schedule& sc = p.sc;
    for (int sg = 0; sg < sc.stages; ++sg) {
        if (sg == 0) {
            HIPCHK(launch_diag(p.q, (const TileWork*)p.d_diag.p, (int)sc.diag.size(), s));
            if (sc.btw_cnt[0] > 0)
                HIPCHK(launch_between(p.q, (const BetweenWork*)p.d_btw.p + sc.btw_off[0], sc.btw_cnt[0], R, s));
        } else {
            HIPCHK(launch_stage(p.q, p.wide, (const TileWork*)p.d_tile.p + sc.tile_off[sg], sc.tile_cnt[sg],
                                (const BetweenWork*)p.d_btw.p + sc.btw_off[sg], sc.btw_cnt[sg], R, s));
        }
    }
    HIPCHK(launch_scores((const FoldDesc*)p.d_folds.p, (int)p.geom.size(), (int32_t*)p.d_scores.p, s));
    return NF_OK;
}

int plan_enqueue_direct(Plan& p, hipStream_t s)
{
    if (p.mode == kModeFused) return plan_enqueue_fused(p, s);
    const uint8_t* R = nullptr;
    int rc = get_R(p.q, &R);
    if (rc) return rc;
    Context& c = ctx();
    const FoldDesc* folds = (const FoldDesc*)p.d_folds.p;
    const Schedule& sc = p.sc;
    hipStream_t s2 = c.side_stream;
    hipEvent_t ev_tile = c.ev_tile, ev_btw = c.ev_btw;
    HIPCHK(hipEventRecord(ev_tile, s));  // fork: s2 starts after the work already on s
    for (int sg = 0; sg < sc.stages; ++sg) {
        // a perturbed plan delays either stream's launch of this stage by 0..5 sleeps
        const unsigned h = p.perturb ? (p.perturb * 2654435761u) ^ ((unsigned)sg * 40503u) : 0;
        const int delay_tile = p.perturb ? (int)((h >> 8) % 6) : 0, delay_btw = p.perturb ? (int)((h >> 16) % 6) : 0;
        if (sg == 0) {
            HIPCHK(launch_diag(p.q, (const TileWork*)p.d_diag.p, (int)sc.diag.size(), s));
        } else {
            HIPCHK(hipStreamWaitEvent(s, ev_btw, 0));  // between(sg-1) done
            HIPCHK(hipEventRecord(ev_tile, s));         // marks finish(sg-1) done
            HIPCHK(launch_delay(delay_tile, s));
            if (sc.tile_cnt[sg] > 0)
                HIPCHK(launch_tile(p.q, (const TileWork*)p.d_tile.p + sc.tile_off[sg], sc.tile_cnt[sg], R, s,
                                   nullptr, nullptr, p.tile_wide));
        }
        HIPCHK(hipStreamWaitEvent(s2, ev_tile, 0));  // finish(sg-1) done
        HIPCHK(launch_delay(delay_btw, s2));
        if (sc.btw_cnt[sg] > 0)
            HIPCHK(launch_btw(p, (const BetweenWork*)p.d_btw.p + sc.btw_off[sg], sc.btw_cnt[sg], R, s2));
        HIPCHK(hipEventRecord(ev_btw, s2));
    }
    // join the side stream back into s
    HIPCHK(hipEventRecord(ev_btw, s2));
    HIPCHK(hipStreamWaitEvent(s, ev_btw, 0));
    HIPCHK(launch_scores(folds, (int)p.geom.size(), (int32_t*)p.d_scores.p, s));
    return NF_OK;
}

// Valid (non-padding) columns of tile column B of a fold.
static int valid_cols(const Geom& g, int T, int B) { return std::max(0, std::min(T, g.n + 1 - B * T)); }

// Work of the finish of an off-diagonal tile with vb valid columns, as the
// finish runs it.  Split points inside the tile's own columns (tile B): j for
// cell (i, j), one by one in the row closure.  Split points inside its own
// rows (tile A): when q divides 8 the rows are finished in 8-row blocks, a
// row goes into the rows above it in its block one split at a time, and each
// finished block's q-groups reach every row above the block by one lookup
// (Eq. 3); otherwise every row goes into every row above it one split at a
// time.  Plus the pairing term of every cell.
static double tile_terms(int q, int T, int vb)
{
    const double own_cols = (double)T * vb * (vb - 1) / 2;
    const double own_rows = (8 % q == 0) ? (double)vb * 8 * 28 : (double)vb * T * (T - 1) / 2;
    return own_cols + own_rows + (double)T * vb;
}
static double tile_block_lookups(int q, int vb)
{
    return (8 % q == 0) ? (double)vb * 8 * 28 * (8 / q) : 0.0;  // 8 rows x groups of the blocks below
}
// The same for a main-diagonal tile of v valid posts: cell (i, i+t) has t-1
// split points and one pairing term (t >= 1).
static double diag_terms(int v)
{
    double s = 0;
    for (int t = 1; t < v; ++t) s += (double)(v - t) * t;
    return s;
}

int plan_profile(Plan& p, hipStream_t s, int reps, nf_kernel_profile_t* out)
{
    const uint8_t* R = nullptr;
    int rc = get_R(p.q, &R);
    if (rc) return rc;
    const int T = tile_size(p.q), G = groups_per_tile(p.q);
    const FoldDesc* folds = (const FoldDesc*)p.d_folds.p;
    const Schedule& sc = p.sc;
    // algorithmic work per launch, from the work lists
    std::vector<double> tile_lk(sc.stages, 0), tile_sp(sc.stages, 0), tile_cells(sc.stages, 0),
        btw_lk(sc.stages, 0);
    for (int sg = 0; sg < sc.stages; ++sg) {
        for (int k = 0; k < sc.tile_cnt[sg]; ++k) {
            const TileItem& it = sc.tile[sc.tile_off[sg] + k];
            const int vb = valid_cols(p.geom[it.fold], T, it.A + it.d);
            tile_lk[sg] += (double)std::min(std::max(it.d - 1, 0), 2) * G * T * vb + tile_block_lookups(p.q, vb);
            tile_sp[sg] += tile_terms(p.q, T, vb);
            tile_cells[sg] += (double)T * vb;
        }
        for (int k = 0; k < sc.btw_cnt[sg]; ++k) {
            const BetweenItem& it = sc.btw[sc.btw_off[sg] + k];
            const int vb = valid_cols(p.geom[it.fold], T, it.A + it.d);
            btw_lk[sg] += (double)(it.c1 - it.c0) * G * T * vb;
        }
    }
    double diag_cells = 0, diag_sp = 0;
    for (auto& it : sc.diag) {
        const int v = valid_cols(p.geom[it.fold], T, it.A);
        diag_cells += (double)v * (v + 1) / 2;
        diag_sp += diag_terms(v);
    }
    std::vector<hipEvent_t> ev;
    auto fresh = [&]() {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return (hipEvent_t) nullptr;
        ev.push_back(e);
        return e;
    };
    struct Rec { int kind; hipEvent_t a, b; double lk, sp, cells; };
    std::vector<Rec> recs;
    // every timed launch gets its own event pair, recorded by the dispatch
    // itself at kernel start and end
    auto pair = [&](hipEvent_t& e0, hipEvent_t& e1) {
        e0 = fresh();
        e1 = fresh();
        return e0 && e1;
    };
    hipEvent_t a = nullptr, b = nullptr;
    {
        const bool fused = p.mode == kModeFused;
        for (int r = 0; r < reps; ++r) {
            if (!pair(a, b)) return fail(NF_E_DEVICE, "event creation failed");
            HIPCHK(launch_diag(p.q, (const TileWork*)p.d_diag.p, (int)sc.diag.size(), s, a, b));
            recs.push_back({0, a, b, 0.0, diag_sp, diag_cells});
            for (int sg = 0; sg < sc.stages; ++sg) {
                const TileWork* tw = (const TileWork*)p.d_tile.p + sc.tile_off[sg];
                const BetweenWork* bw = (const BetweenWork*)p.d_btw.p + sc.btw_off[sg];
                if (fused && sg >= 1) {
                    if (sc.tile_cnt[sg] + sc.btw_cnt[sg] == 0) continue;
                    if (!pair(a, b)) return fail(NF_E_DEVICE, "event creation failed");
                    HIPCHK(launch_stage(p.q, p.wide, tw, sc.tile_cnt[sg], bw, sc.btw_cnt[sg], R, s, a, b));
                    recs.push_back({3, a, b, tile_lk[sg] + btw_lk[sg], tile_sp[sg], tile_cells[sg]});
                    continue;
                }
                if (sg >= 1 && sc.tile_cnt[sg] > 0) {
                    if (!pair(a, b)) return fail(NF_E_DEVICE, "event creation failed");
                    HIPCHK(launch_tile(p.q, tw, sc.tile_cnt[sg], R, s, a, b, p.tile_wide));
                    recs.push_back({1, a, b, tile_lk[sg], tile_sp[sg], tile_cells[sg]});
                }
                if (sc.btw_cnt[sg] > 0) {
                    if (!pair(a, b)) return fail(NF_E_DEVICE, "event creation failed");
                    HIPCHK(launch_btw(p, bw, sc.btw_cnt[sg], R, s, a, b));
                    recs.push_back({2, a, b, btw_lk[sg], 0.0, 0.0});
                }
            }
            HIPCHK(launch_scores(folds, (int)p.geom.size(), (int32_t*)p.d_scores.p, s));
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    for (auto& rc2 : recs) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, rc2.a, rc2.b));
        out->launches[rc2.kind] += 1;
        out->ms[rc2.kind] += ms;
        out->lookups[rc2.kind] += rc2.lk;
        out->splits[rc2.kind] += rc2.sp;
        out->cells[rc2.kind] += rc2.cells;
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    return NF_OK;
}

int plan_enqueue(Plan& p, hipStream_t s)
{
    if (!use_graphs()) return plan_enqueue_direct(p, s);
    if (!p.exec) {
        const uint8_t* R = nullptr;
        int rc = get_R(p.q, &R);  // outside the capture
        if (rc) return rc;
        hipStream_t cs = ctx().capture_stream;
        HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        rc = plan_enqueue_direct(p, cs);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(NF_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        p.graph = g;
        e = hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            p.release_graph();
            return fail(NF_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        }
    }
    HIPCHK(hipGraphLaunch(p.exec, s));
    return NF_OK;
}

int make_plan(const std::vector<int>& ns, int q, std::unique_ptr<Plan>& out, int target, int wide)
{
    auto p = std::make_unique<Plan>();
    p->q = q;
    std::vector<int> NTs;
    for (int n : ns) {
        p->geom.push_back(make_geom(n, q));
        NTs.push_back(p->geom.back().NT);
    }
    p->mode = plan_mode_for(NTs);
    p->plain = plain_between_for(q);
    if (p->plain) p->mode = kModeStaged;  // the fused step has the lookup built in
    p->target = target > 0 ? target : between_target(ns.size() == 1 ? ns[0] : -1, q);
    p->wide = ns.size() == 1 && q == 8 && (wide >= 0 ? wide > 0 : stage_wide(ns[0], q));
    // staged finishes in the lean shape at q = 8: three per CU (MI355X, the
    // 4096-fold batch 20.35 -> 19.1 ms; staged single folds unchanged);
    // NF_TILE_WIDE=0 keeps the default shape
    p->tile_wide = q == 8;
    if (const char* e = getenv("NF_TILE_WIDE")) p->tile_wide = q == 8 && atoi(e) != 0;
    build_schedule(NTs, p->target, p->sc);
    if ((p->perturb = perturb_seed())) perturb_schedule(p->sc, p->perturb);
    int rc = plan_allocate(*p);
    if (rc) return rc;
    out = std::move(p);
    return NF_OK;
}

// Single-fold plans are cached by (n, q) and the chunk target, least recently
// used first out.
int single_plan(int n, int q, Plan** out, int target, int wide)
{
    Context& c = ctx();
    if (target <= 0) target = between_target(n, q);
    if (wide < 0) wide = (q == 8 && stage_wide(n, q)) ? 1 : 0;
    // NF_MODE and NF_BETWEEN are read when a plan is made, so they are part of the key
    const char* me = getenv("NF_MODE");
    const int mode_env = !me ? 0 : strcmp(me, "fused") == 0 ? 1 : strcmp(me, "staged") == 0 ? 2 : 0;
    const long long key = (((long long)n * 16 + q) * 2 + (plain_between_for(q) ? 1 : 0)) * 3 + mode_env;
    for (auto it = c.plans.begin(); it != c.plans.end(); ++it) {
        if (it->first == key && it->second->target == target && it->second->wide == (wide > 0) &&
            it->second->perturb == perturb_seed()) {
            auto ent = std::move(*it);
            c.plans.erase(it);
            c.plans.push_back(std::move(ent));
            *out = c.plans.back().second.get();
            return NF_OK;
        }
    }
    size_t cap = (size_t)8 << 30;
    if (const char* e = getenv("NF_PLAN_CACHE_BYTES")) cap = strtoull(e, nullptr, 10);
    const size_t need = make_geom(n, q).bytes;
    size_t held = 0;
    for (auto& e : c.plans) held += e.second->device_bytes;
    while (!c.plans.empty() && held + need > cap) {
        held -= c.plans.front().second->device_bytes;
        c.plans.erase(c.plans.begin());
    }
    std::unique_ptr<Plan> p;
    int rc = make_plan({n}, q, p, target, wide);
    if (rc == NF_E_NOMEM && !c.plans.empty()) {  // drop every cached plan and retry once
        c.plans.clear();
        rc = make_plan({n}, q, p, target, wide);
    }
    if (rc) return rc;
    c.plans.push_back({key, std::move(p)});
    *out = c.plans.back().second.get();
    return NF_OK;
}

unsigned& perturb_seed()
{
    static unsigned seed = 0;
    return seed;
}

// Shuffle the finishes and the between chunks of every wavefront step, and
// the main-diagonal tiles, in an order drawn from `seed`.  The items of one
// step touch disjoint cells and packed words, and chunks that share an
// accumulator slot combine by atomic max, so no order may change a result.
void perturb_schedule(Schedule& sc, unsigned seed)
{
    std::mt19937 rng(seed);
    std::shuffle(sc.diag.begin(), sc.diag.end(), rng);
    for (int sg = 0; sg < sc.stages; ++sg) {
        const auto t0 = sc.tile.begin() + sc.tile_off[sg];
        const auto b0 = sc.btw.begin() + sc.btw_off[sg];
        std::shuffle(t0, t0 + sc.tile_cnt[sg], rng);
        std::shuffle(b0, b0 + sc.btw_cnt[sg], rng);
    }
}

int resolve_q(int q, int n)
{
    if (q == 0) return autotune_lookup(n);
    return q;
}

int check_q(int q)
{
    if (q < 0 || q > NF_Q_MAX) return fail(NF_E_INVAL, "q = %d outside 0..%d", q, NF_Q_MAX);
    return NF_OK;
}

// ------------------------------------------------------------------ autotune cache

static int bucket_of(int n)
{
    int b = 0;
    while (b < kTuneBuckets - 1 && n >= (256 << b)) ++b;
    return b;
}

static void load_tune_file()
{
    Context& c = ctx();
    if (c.tune_loaded) return;
    c.tune_loaded = true;
    const char* path = getenv("NF_AUTOTUNE_CACHE");
    if (!path) return;
    // one line per length bucket: "bucket q [target [wide]]"
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        int b = -1, q = 0, t = 0, w = -1;
        const int got = sscanf(line.c_str(), "%d %d %d %d", &b, &q, &t, &w);
        if (got < 2 || b < 0 || b >= kTuneBuckets || q < NF_Q_MIN || q > NF_Q_MAX) continue;
        c.tuned_q[b] = q;
        if (got >= 3 && t > 0 && t <= (1 << 20)) c.tuned_target[b] = t;
        if (got == 4 && (w == 0 || w == 1)) c.tuned_wide[b] = 1 + w;
    }
}

static void save_tune_file()
{
    const char* path = getenv("NF_AUTOTUNE_CACHE");
    if (!path) return;
    std::ofstream out(path);
    for (int b = 0; b < kTuneBuckets; ++b)
        if (ctx().tuned_q[b]) {
            out << b << " " << ctx().tuned_q[b] << " " << ctx().tuned_target[b];
            if (ctx().tuned_wide[b]) out << " " << ctx().tuned_wide[b] - 1;
            out << "\n";
        }
}

int autotune_lookup(int n)
{
    load_tune_file();
    const int q = ctx().tuned_q[bucket_of(n)];
    return q ? q : kDefaultQ;
}

int autotune_run(int n, int qmin, int qmax, int reps)
{
    if (n < 2 || n > NF_MAX_N) return fail(NF_E_INVAL, "autotune length %d out of range", n);
    qmin = std::max(qmin, NF_Q_MIN);
    qmax = std::min(qmax, NF_Q_MAX);
    if (qmin > qmax || reps < 1) return fail(NF_E_INVAL, "empty autotune range");
    int rc = ensure_device();
    if (rc) return rc;
    Context& c = ctx();
    // a fixed pseudo-random sequence (64-bit LCG), iid over the 4 bases
    std::vector<uint8_t> codes(n);
    uint64_t x = 0x9E3779B97F4A7C15ull ^ (uint64_t)n;
    for (int i = 0; i < n; ++i) {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        codes[i] = (uint8_t)(x >> 62);
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    StreamFence fence{c.stream};  // the uploads read `codes`
    // time `reps` fills of the plan for (q, target, fused-step shape) after
    // one warm-up fill
    auto time_plan = [&](int q, int target, int wide, float* ms) -> int {
        Plan* p = nullptr;
        int r = single_plan(n, q, &p, target, wide);
        if (r) return r;
        const Geom& g = p->geom[0];
        if (hipMemcpyAsync((char*)p->arena.p + g.codes_off, codes.data(), n, hipMemcpyHostToDevice, c.stream) !=
            hipSuccess)
            return fail(NF_E_DEVICE, "autotune upload failed");
        if ((r = plan_enqueue(*p, c.stream))) return r;  // warm-up (and graph capture)
        (void)hipEventRecord(e0, c.stream);
        for (int k = 0; k < reps && !r; ++k) r = plan_enqueue(*p, c.stream);
        (void)hipEventRecord(e1, c.stream);
        (void)hipEventSynchronize(e1);
        *ms = 0;
        (void)hipEventElapsedTime(ms, e0, e1);
        return r;
    };
    // q at the default chunk target and step shape, then the chunk target at
    // that q, then (q = 8) the other fused-step shape; the default comes
    // first, so a tie keeps it
    auto default_wide = [&](int q) { return (q == 8 && n >= 8192) ? 1 : 0; };
    int best_q = kDefaultQ, best_t = kDefaultTarget;
    float best_ms = 1e30f, ms = 0;
    for (int q = qmin; q <= qmax && !rc; ++q) {
        if ((rc = time_plan(q, kDefaultTarget, default_wide(q), &ms))) break;
        if (ms < best_ms) {
            best_ms = ms;
            best_q = q;
        }
    }
    best_ms = 1e30f;
    int best_w = default_wide(best_q);
    for (int t : {kDefaultTarget, 256, 512, 2048, 2560}) {
        if (rc) break;
        if ((rc = time_plan(best_q, t, best_w, &ms))) break;
        if (ms < best_ms) {
            best_ms = ms;
            best_t = t;
        }
    }
    if (!rc && best_q == 8) {
        if (!(rc = time_plan(best_q, best_t, 1 - best_w, &ms)) && ms < best_ms) best_w = 1 - best_w;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    load_tune_file();
    c.tuned_q[bucket_of(n)] = best_q;
    c.tuned_target[bucket_of(n)] = best_t;
    c.tuned_wide[bucket_of(n)] = best_q == 8 ? 1 + best_w : 0;
    save_tune_file();
    return best_q;
}

}  // namespace nf

// ------------------------------------------------------------------ test hook

namespace nf {
namespace {

// Check the invariants of build_schedule for folds of NT[f] tiles per side;
// "" when they hold, else the first violation.
std::string check_schedule(const std::vector<int>& NTs, int target)
{
    Schedule sc;
    build_schedule(NTs, target, sc);
    if (perturb_seed()) perturb_schedule(sc, perturb_seed());  // the invariants hold in any item order
    char buf[256];
    auto bad = [&](const char* fmt, long long a, long long b, long long c) {
        snprintf(buf, sizeof buf, fmt, a, b, c);
        return std::string(buf);
    };
    int stages = 0;
    for (int v : NTs) stages = std::max(stages, v);
    if (sc.stages != stages) return bad("stages %lld, expected %lld%.0lld", sc.stages, stages, 0);
    const int nf = (int)NTs.size();
    // main-diagonal tiles: each (f, A) once
    std::vector<std::vector<int>> seen(nf);
    for (int f = 0; f < nf; ++f) seen[f].assign(NTs[f], 0);
    for (const TileItem& it : sc.diag) {
        if (it.fold < 0 || it.fold >= nf || it.A < 0 || it.A >= NTs[it.fold] || it.d != 0)
            return bad("bad diagonal item fold %lld A %lld d %lld", it.fold, it.A, it.d);
        if (seen[it.fold][it.A]++) return bad("diagonal tile (%lld, %lld) twice%.0lld", it.fold, it.A, 0);
    }
    for (int f = 0; f < nf; ++f)
        for (int A = 0; A < NTs[f]; ++A)
            if (!seen[f][A]) return bad("diagonal tile (%lld, %lld) missing%.0lld", f, A, 0);
    // between items, by (fold, A, d): the groups C in [A+2, A+d-1) exactly once,
    // in the stage d-1, one slot per tile, atomic iff several items
    std::map<std::tuple<int, int, int>, std::vector<const BetweenItem*>> btw;
    for (int sg = 0; sg < stages; ++sg) {
        std::set<int> slots_of_stage;
        std::map<int, std::tuple<int, int, int>> owner;
        for (int k = sc.btw_off[sg]; k < sc.btw_off[sg] + sc.btw_cnt[sg]; ++k) {
            const BetweenItem& it = sc.btw[k];
            if (it.d != sg + 1) return bad("between item of stage %lld has d = %lld%.0lld", sg, it.d, 0);
            const int half = (sg & 1) * sc.max_slots;
            if (it.slot < half || it.slot >= half + sc.max_slots)
                return bad("stage %lld slot %lld outside its half (max_slots %lld)", sg, it.slot, sc.max_slots);
            auto key = std::make_tuple(it.fold, it.A, it.d);
            auto o = owner.find(it.slot);
            if (o != owner.end() && o->second != key) return bad("stage %lld: slot %lld shared by two tiles%.0lld", sg, it.slot, 0);
            owner[it.slot] = key;
            btw[key].push_back(&it);
        }
    }
    for (int f = 0; f < nf; ++f)
        for (int d = 1; d < NTs[f]; ++d)
            for (int A = 0; A + d < NTs[f]; ++A) {
                auto itv = btw.find(std::make_tuple(f, A, d));
                if (d < 4) {
                    if (itv != btw.end()) return bad("tile d = %lld (fold %lld) has between items%.0lld", d, f, 0);
                    continue;
                }
                if (itv == btw.end()) return bad("tile (%lld, %lld, d = %lld) has no between items", f, A, d);
                std::vector<int> cover(NTs[f], 0);
                const int slot = itv->second[0]->slot;
                for (const BetweenItem* it : itv->second) {
                    if (it->slot != slot) return bad("tile (%lld, %lld): items in two slots%.0lld", f, A, 0);
                    if (it->pad0 != (itv->second.size() > 1 ? 1 : 0))
                        return bad("tile (%lld, %lld): atomic flag %lld", f, A, it->pad0);
                    for (int C = it->c0; C < it->c1; ++C) {
                        if (C < A + 2 || C > A + d - 2) return bad("tile (%lld, %lld): group tile C = %lld outside (A+1, B-1)", f, A, C);
                        cover[C]++;
                    }
                }
                for (int C = A + 2; C <= A + d - 2; ++C)
                    if (cover[C] != 1) return bad("tile (%lld, %lld): C = %lld not covered exactly once", f, A, C);
            }
    // tile finishes: every (f, A, d >= 1) once, at stage d, reading its slot
    for (int f = 0; f < nf; ++f) seen[f].assign(NTs[f] * (size_t)NTs[f], 0);
    for (int sg = 1; sg < stages; ++sg) {
        std::set<int> slots;
        for (int k = sc.tile_off[sg]; k < sc.tile_off[sg] + sc.tile_cnt[sg]; ++k) {
            const TileItem& it = sc.tile[k];
            if (it.d != sg || it.fold < 0 || it.fold >= nf || it.A < 0 || it.A + it.d >= NTs[it.fold])
                return bad("bad tile item at stage %lld (A %lld, d %lld)", sg, it.A, it.d);
            if (seen[it.fold][(size_t)it.A * NTs[it.fold] + it.d]++) return bad("tile (%lld, %lld, %lld) twice", it.fold, it.A, it.d);
            if (it.d < 4) {
                if (it.nslot != 0) return bad("tile d = %lld reads a slot%.0lld%.0lld", it.d, 0, 0);
                continue;
            }
            auto itv = btw.find(std::make_tuple(it.fold, it.A, it.d));
            if (it.nslot != 1 || itv == btw.end() || it.slot0 != itv->second[0]->slot)
                return bad("tile (%lld, %lld, %lld) reads the wrong slot", it.fold, it.A, it.d);
            if (!slots.insert(it.slot0).second) return bad("stage %lld: two tiles read slot %lld%.0lld", sg, it.slot0, 0);
        }
    }
    for (int f = 0; f < nf; ++f)
        for (int A = 0; A < NTs[f]; ++A)
            for (int d = 1; A + d < NTs[f]; ++d)
                if (!seen[f][(size_t)A * NTs[f] + d]) return bad("tile (%lld, %lld, %lld) missing", f, A, d);
    return "";
}

// The closed form SingleSchedule, which the allocation-free entry point
// evaluates on the device, against build_schedule for one fold: the same
// items in the same order, and the same slot count.
std::string check_single_schedule(int NT, int target)
{
    Schedule sc;
    build_schedule({NT}, target, sc);
    SingleSchedule S;
    S.NT = NT;
    S.target = target;
    char buf[256];
    auto bad = [&](const char* what, int sg, long long k) {
        snprintf(buf, sizeof buf, "single schedule NT %d target %d: %s at stage %d item %lld", NT, target, what, sg, k);
        return std::string(buf);
    };
    if (sc.max_slots != S.max_slots()) return bad("max_slots", -1, sc.max_slots);
    if ((int)sc.diag.size() != NT) return bad("diagonal count", 0, (long long)sc.diag.size());
    for (int sg = 0; sg < sc.stages; ++sg) {
        if (sc.tile_cnt[sg] != S.finishes(sg)) return bad("finish count", sg, sc.tile_cnt[sg]);
        if (sg >= 1 && sc.tile_off[sg] != S.finish_offset(sg)) return bad("finish offset", sg, sc.tile_off[sg]);
        for (int A = 0; A < sc.tile_cnt[sg]; ++A) {
            const TileItem a = sc.tile[sc.tile_off[sg] + A], b = S.finish(sg, A);
            if (a.fold != b.fold || a.A != b.A || a.d != b.d || a.nslot != b.nslot || (a.nslot && a.slot0 != b.slot0))
                return bad("finish item", sg, A);
        }
        if (sc.btw_cnt[sg] != S.between_count(sg)) return bad("between count", sg, sc.btw_cnt[sg]);
        if (sc.btw_off[sg] != S.between_offset(sg)) return bad("between offset", sg, sc.btw_off[sg]);
        for (int k = 0; k < sc.btw_cnt[sg]; ++k) {
            const BetweenItem a = sc.btw[sc.btw_off[sg] + k], b = S.between(sg, k);
            if (a.fold != b.fold || a.A != b.A || a.d != b.d || a.c0 != b.c0 || a.c1 != b.c1 || a.slot != b.slot ||
                a.pad0 != b.pad0)
                return bad("between item", sg, k);
        }
    }
    return "";
}

}  // namespace
}  // namespace nf

// Test hook (include/nf_test.h): host-only check of the wavefront schedule.
extern "C" int nf_test_schedule(const int* NTs, int count, int target, char* msg, int cap)
{
    if (count < 0 || (count > 0 && !NTs) || target < 1) return NF_E_INVAL;
    std::vector<int> v(NTs, NTs + count);
    for (int x : v)
        if (x < 1) return NF_E_INVAL;
    std::string err = nf::check_schedule(v, target);
    if (err.empty() && count == 1 && !nf::perturb_seed()) err = nf::check_single_schedule(v[0], target);
    if (msg && cap > 0) snprintf(msg, (size_t)cap, "%s", err.c_str());
    return err.empty() ? NF_OK : 1;
}
