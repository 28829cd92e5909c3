// Host-side internals of libnf (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "nf.h"
#include "nf_internal.h"

namespace nf {

int fail(int code, const char* fmt, ...);
const char* last_error();
void clear_error();

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            (void)hipGetLastError();                                                              \
            return ::nf::fail(NF_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
        }                                                                                         \
    } while (0)

// Waits for a stream when a function returns, so that no copy still in
// flight on an early error return reads or writes host memory of the
// caller's or of the returning frame.  Declare it after the host buffers it
// guards, so it runs before they are freed; a null stream is not waited on.
struct StreamFence {
    hipStream_t s = nullptr;
    ~StreamFence()
    {
        if (s) (void)hipStreamSynchronize(s);
    }
};

// Device memory hook (nf_set_allocator): null members mean hipMalloc/hipFree.
struct AllocHook {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*free_)(void*, void*) = nullptr;
    void* ctx = nullptr;
};
int set_allocator(const AllocHook& h);

// Owned device allocation, taken from the hook in force when it is
// allocated and given back through that same hook.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    AllocHook from;  // the hook p came from
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    int alloc(size_t nbytes);
    void reset();
};

// Device layout of one fold (see nf_internal.h).
struct Geom {
    int n = 0, NT = 0, ld = 0;
    size_t codes_bytes = 0, F_bytes = 0, rs_bytes = 0, cs_bytes = 0, bytes = 0;
    size_t codes_off = 0;  // offset of this fold's block in its arena
};

// Packed wavefront schedule of a group of folds that start together: stage s
// finishes the tiles of diagonal s of every fold that has one and does the
// between-group work of diagonal s+1.
struct Schedule {
    int stages = 0;
    int max_slots = 0;  // partial slots per parity half
    std::vector<TileItem> diag;
    std::vector<TileItem> tile;
    std::vector<BetweenItem> btw;
    std::vector<int> tile_off, tile_cnt, btw_off, btw_cnt;
};

// How a plan's fill runs:
//   staged: per wavefront step, the tile finishes of diagonal s on one stream
//           and the between chunks of diagonal s+1 on a second one;
//   fused:  per step one launch holding both (one stream, no cross-stream
//           waits).
enum PlanMode { kModeStaged = 0, kModeFused = 1 };

// Fused steps while a step holds at most this many tiles to finish (for a
// batch: the folds' tiles per side summed, the size of its first step):
// one launch and no cross-stream wait per step is cheapest there; above it
// staged steps fill the device on two streams with many folds' tiles and
// chunks.  Measured on MI355X: fused is faster for one fold at n = 6000,
// 12000 and 16000 (2.19 / 6.94 / 13.6 ms against 3.07 / 8.19 / 14.6 ms),
// staged for a batch of 4096 folds (21.2 against 22.6 ms).
constexpr int kFusedMaxTilesPerSide = 208;

struct Plan {
    int q = 8;
    int mode = kModeStaged;
    bool plain = false;  // between-group work by the plain recurrence (NF_BETWEEN=plain)
    int target = 0;      // between chunks per wavefront step the schedule was built for
    bool wide = false;   // fused steps in the wide shape (three workgroups per CU at q = 8)
    unsigned perturb = 0;  // test: seed of the shuffled item order and staged delays (0: none)
    bool tile_wide = false;  // staged finishes in the lean shape (three workgroups per CU at q = 8)
    std::vector<Geom> geom;
    std::vector<FoldDesc> h_folds;
    Schedule sc;
    DevBuf arena, d_folds, d_diag, d_tile, d_btw, d_part, d_scores;
    DevBuf d_S;  // expand target for host copies of tables
    DevBuf d_tb;  // traceback: status, structure, stack
    size_t device_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Plan();
    void release_graph();
};

constexpr int kTuneBuckets = 10;  // n < 256, < 512, ..., >= 65536
constexpr int kDefaultQ = 8;
constexpr int kDefaultTarget = 1024;  // between chunks per step: 4 workgroups per CU

struct Context {
    bool ready = false;
    int requested_device = 0;
    int device = 0;
    int num_cu = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    hipStream_t side_stream = nullptr;  // between-group kernels overlap the tile finishes here
    hipEvent_t ev_tile = nullptr, ev_btw = nullptr;
    DevBuf R[NF_Q_MAX + 1];
    std::vector<std::pair<long long, std::unique_ptr<Plan>>> plans;  // LRU, most recent last
    int tuned_q[kTuneBuckets] = {0};
    int tuned_target[kTuneBuckets] = {0};
    int tuned_wide[kTuneBuckets] = {0};  // 0: not tuned, 1: default fused step, 2: wide fused step
    bool tune_loaded = false;
};

Context& ctx();
int ensure_device();
std::recursive_mutex& api_mutex();  // serialises the host entry points
// Device address of the allocation-free entry point's static scratch array,
// looked up once per device at set-up (nf_noalloc.hip).
int scratch_setup(int device);
int get_R(int q, const uint8_t** out);
int encode_sequence(const char* seq, int n, uint8_t* out);
int check_length(int n);
int check_q(int q);
int resolve_q(int q, int n);
// Test hook state: the seed plans made from now on perturb their schedule with
// (nf_test_set_perturb; 0 = none).
unsigned& perturb_seed();
void perturb_schedule(Schedule& sc, unsigned seed);
Geom make_geom(int n, int q);
void append_between(const std::vector<std::pair<int, int>>& folds_nt, int dd, int target,
                    std::vector<BetweenItem>& out, int* next_slot,
                    std::vector<std::vector<std::pair<int, int>>>& pending);
void build_schedule(const std::vector<int>& NTs, int target, Schedule& sc);
int between_target(int n_single, int q);
int plan_allocate(Plan& p);
TileWork to_work(const TileItem& it, const std::vector<FoldDesc>& fd, int32_t* acc_base);
BetweenWork to_work(const BetweenItem& it, const std::vector<FoldDesc>& fd, int32_t* acc_base);
int plan_enqueue(Plan& p, hipStream_t s);
int plan_enqueue_direct(Plan& p, hipStream_t s);
int plan_mode_for(const std::vector<int>& NTs);
// NF_BETWEEN=plain: the between-group work of new plans runs the plain
// recurrence (k_between_plain, the ablation of the lookup) on staged steps;
// only for 64-post tiles (q = 1, 2, 4, 8), ignored otherwise.
bool plain_between_for(int q);
int plan_profile(Plan& p, hipStream_t s, int reps, nf_kernel_profile_t* out);
// target > 0 fixes the between chunks per step; wide < 0 takes stage_wide's
// choice for a single fold (batches always run the default fused step).
int make_plan(const std::vector<int>& ns, int q, std::unique_ptr<Plan>& out, int target = 0, int wide = -1);
int single_plan(int n, int q, Plan** out, int target = 0, int wide = -1);
int autotune_lookup(int n);
int autotune_run(int n, int qmin, int qmax, int reps);

// serving engine (nf_serve.cpp)
int serve_config(size_t budget, int max_slots, int max_queue);
int64_t serve_submit(const char* seq, int n, int q, int flags);
int serve_poll(int64_t ticket, int32_t* score_out, int16_t* S_out, char* db_out, int timeout_ms, bool blocking);
int serve_stats(nf_serve_stats_t* out);
void serve_shutdown();
size_t serve_fold_bytes(int n, int q);

}  // namespace nf
