/*
 * nf.h -- C ABI of libnf.so: the two-vector Four-Russians fill of the Nussinov
 * base-pair maximisation table on one AMD MI355X (gfx950) GPU.
 *
 * Problem (Section 2, Eq. 1): for S_1..S_n over {A,C,G,U},
 *     D(i,i-1) = D(i,i) = 0,
 *     D(i,j) = max{ b(S_i,S_j) + D(i+1,j-1), max_{i+1<=k<=j} D(i,k-1) + D(k,j) },
 * b = 1 for A-U, U-A, C-G, G-C and 0 otherwise (G-U is not a pair, there is no
 * minimum hairpin loop).  The score is D(1,n).
 *
 * Method (Section 3.1, Eq. 2 -> Eq. 3, Lemma 1, and the tiled parallel form
 * of Sections 4-5): rows and columns of the table are cut into groups of q
 * split points; q consecutive table cells are a base value plus a 0/1
 * difference vector, and the best of q splits is the two bases plus one
 * lookup R[v][v-bar] into a table built once per q.  Tiles are swept as an
 * anti-diagonal wavefront.  The table the GPU returns is identical to Eq. 1's.
 *
 * General conventions
 *  - Every function returns NF_OK (0) or a negative NF_E_* code (nf_fold also
 *    returns the score >= 0).  On error nothing is written to the outputs and
 *    nf_last_error() describes the failure (thread-local string, valid until
 *    the next call on that thread).
 *  - Sequences: n bytes of 'A','C','G','U' (lower case accepted); any other
 *    byte (including 'T' and 'N') is NF_E_INVAL.  0 <= n <= NF_MAX_N.
 *  - q: 1..9, or 0 to let the library choose (autotuned value, else 8).
 *  - Table layout (S_out, row-major n*n int16, caller-owned):
 *        S_out[i*n + j] = D(i+1, j+1) for i <= j, and 0 for i > j.
 *  - Inputs are borrowed for the duration of the call (nf_submit copies);
 *    outputs are caller-allocated.  Device memory the library needs is
 *    allocated and owned by the library (through nf_set_allocator's hook if
 *    one is set, else hipMalloc) and released by nf_shutdown().
 *  - Host functions are thread-safe; calls are serialised internally.
 *  - No GPU fallback: without a usable gfx950 device every call that needs
 *    the GPU returns NF_E_DEVICE.
 */
#ifndef NF_H
#define NF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NF_OK = 0,
    NF_E_INVAL = -1,     /* bad argument or bad base */
    NF_E_NOMEM = -2,     /* device memory exhausted, or request above the serving budget */
    NF_E_DEVICE = -3,    /* no GPU, HIP error, or wrong architecture */
    NF_E_BUSY = -4,      /* serving queue full */
    NF_E_NOTFOUND = -5,  /* unknown or already released ticket */
    NF_E_TOOLONG = -6,   /* n > NF_MAX_N */
    NF_E_TIMEOUT = -7,   /* nf_wait deadline passed */
    NF_E_ABORTED = -8    /* serving engine shut down before the request finished */
};

/* Scores are at most n/2 and are stored in int16 tables. */
#define NF_MAX_N 65534
#define NF_Q_MIN 1
#define NF_Q_MAX 9

/* Message for the last negative return on the calling thread ("" if none). */
const char* nf_last_error(void);

/* Select and initialise the GPU (default device 0; the environment variable
 * NF_DEVICE overrides).  Idempotent; called implicitly by every GPU entry
 * point.  NF_E_DEVICE when no gfx950 device is present. */
int nf_init(int device);

/* Release every device buffer, cached plan and graph, and stop the serving
 * engine (pending tickets then report NF_E_ABORTED).  The library can be used
 * again afterwards. */
void nf_shutdown(void);

/* Device memory hook.  Every device buffer the library holds (fold and batch
 * workspaces, R, the serving arena, traceback scratch) is taken from
 * alloc(bytes, ctx), which must return device memory of the library's device
 * aligned to 256 bytes, or NULL (the call that needed it then fails with
 * NF_E_NOMEM).  A buffer goes back through the free_(ptr, ctx) of the hook it
 * came from, after the library has waited for the device to be idle, so the
 * owner may reuse the block at once.  Both NULL restores hipMalloc/hipFree for
 * later allocations.  Buffers already held keep their own hook, so the hook
 * may be changed at any time; the functions must stay callable until
 * nf_shutdown() has returned and every batch is destroyed.  They may be
 * called from the serving engine's thread.  NF_E_INVAL when exactly one of
 * the two is NULL.  Host code only: no device is needed to set it. */
int nf_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_)(void* ptr, void* ctx), void* ctx);

/* Base codes of Section 2's alphabet: codes_out[i] = 0, 1, 2, 3 for seq[i] =
 * A, C, G, U (lower case accepted), the encoding nf_fold_dev takes; a pair
 * is complementary exactly when its two codes add up to 3.  NF_E_INVAL at the
 * first other byte (its position is in nf_last_error()), and then codes_out
 * is left untouched.  Host code only. */
int nf_encode(const char* seq, int n, uint8_t* codes_out);

/* ---- Four-Russians table R (Section 3.1, preprocessing listing; Eq. 3) ----
 * Builds R for vectors of length q on the device, once per q (cached;
 * idempotent).  Encoding: v_0 = v-bar_0 = 0 carry no information, so
 * h has bit p-1 = v_p and c has bit p-1 = -v-bar_p for p = 1..q-1, and
 *     R[h][c] = max_{k=0..q-1} sum_{p<=k} (v_p + v-bar_p)   (values 0..q-1).
 * Stored as uint8, row-major [2^(q-1)][2^(q-1)]. */
int nf_precompute_R(int q);

/* Copy R for q (building it if needed) into out: 2^(2(q-1)) bytes, row h,
 * column c.  NF_E_INVAL if cap is smaller. */
int nf_copy_R(int q, uint8_t* out, size_t cap);

/* ---- Single fold (host buffers) ----
 * Fold seq[0..n) and return D(1,n) >= 0.  If S_out is not NULL, the full table
 * (layout above) is written to it.  Synchronous.
 *
 * Execution (Sections 4-5: the wavefront over tile diagonals), chosen per
 * workspace: for one fold, and for batches whose steps hold few tiles, each
 * step is one launch holding the finishes of diagonal s and the
 * between-group chunks of diagonal s+1; for larger batches the two kinds run
 * as separate launches on two streams.  NF_MODE=staged|fused forces one.
 * NF_BETWEEN=plain (ablation only, q = 1, 2, 4, 8) computes the between-group
 * maxima by Eq. 1's splits from the dense table instead of by R lookups, on
 * staged steps; the table is the same.  Both are read when a workspace for
 * (n, q) is first made and are part of its cache key. */
int nf_fold(const char* seq, int n, int q, int16_t* S_out);

/* nf_fold_structure
 * Fold seq[0..n) and write one optimal secondary structure to db_out: n
 * characters '(' ')' '.' (no terminator; caller-owned, at least n bytes),
 * base i+1 pairs with base j+1 when db_out[i] = '(' matches db_out[j] = ')'.
 * Returns D(1,n) >= 0, the number of pairs.  Synchronous.
 *
 * The structure is the traceback of Section 2 through D*, the argmax of
 * Eq. 1, taken as a strict '>' scan takes it: on D(i,j) the pairing term
 * b(S_i,S_j) + D(i+1,j-1) first (a pair when b = 1; with b = 0 both ends stay
 * unpaired), else the split D(i,k-1) + D(k,j) with the smallest k.  So among
 * the optimal structures one fixed one is returned.  It runs on the GPU from
 * the finished table (one wavefront; D* is recomputed, not stored).
 * NF_E_DEVICE if the traceback cannot complete (a table that is not Eq. 1's). */
int nf_fold_structure(const char* seq, int n, int q, char* db_out);

/* ---- Single fold (device buffers, asynchronous on a HIP stream) ----
 * d_codes: n device bytes, base codes A=0, C=1, G=2, U=3 (other values give
 *          unspecified scores but never access memory out of bounds).
 * d_score: device int32 that receives D(1,n) (may be NULL).
 * d_S:     device int16 n*n table, layout above (may be NULL; when set the
 *          lower triangle is written as 0).
 * stream:  hipStream_t passed as void* (NULL = the null stream).
 * Work is enqueued on stream and the call returns without waiting.  The
 * library keeps a per-(n,q) workspace; concurrent calls with the same (n,q)
 * on different streams must be ordered by the caller. */
int nf_fold_dev(const uint8_t* d_codes, int n, int q, int32_t* d_score, int16_t* d_S, void* stream);

/* ---- Single fold on device buffers, allocating nothing ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result and stream semantics as nf_fold_dev, and the same
 * kernels, but every buffer beyond the caller's inputs and outputs (R, the
 * padded codes, the dense table, the packed words, the accumulators, the
 * work lists) lives in one static device array of NF_NOALLOC_SCRATCH_BYTES
 * that each GPU the library runs on holds until the process ends.  The call
 * makes kernel launches on `stream` only: no allocation, no host copy, no
 * memset, so it can be captured into a graph.  It always runs the fused
 * wavefront steps with R lookups (NF_MODE and NF_BETWEEN do not apply).
 * A fold whose buffers do not fit the array (n > 3519 at q = 8, n > 3199
 * at q = 4, at the default chunk target) is NF_E_NOMEM, with the bytes it needs in
 * nf_last_error(), before any device work.  Every call on a GPU shares that
 * GPU's array and overwrites what the last call left there: calls that
 * overlap on one GPU (on different streams, or a graph replayed while
 * another call runs) race, and the caller must order them. */
#define NF_NOALLOC_SCRATCH_BYTES (32u << 20)
int nf_fold_dev_noalloc(const uint8_t* d_codes, int n, int q, int32_t* d_score, int16_t* d_S, void* stream);

/* ---- Batched folds: one packed wavefront over many sequences ----
 * A prepared batch uploads the codes of all sequences once, builds the packed
 * per-diagonal work lists of all of them and captures the whole fill as one
 * HIP graph (execution as for nf_fold).
 * Handles are opaque; a handle must only be used from one thread at a time. */
typedef struct nf_batch nf_batch;

/* seqs[i] holds ns[i] bases (i < count).  q as above; with q = 0 every fold
 * takes the q tuned for its own length bucket (nf_autotune_q), and the folds
 * of each q form one packed wavefront of their own: the groups run at once,
 * on streams forked from and joined back into the stream of nf_batch_run. */
int nf_batch_create(const char* const* seqs, const int* ns, int count, int q, nf_batch** out);
/* Enqueue one complete fill of every sequence in the batch on stream. */
int nf_batch_run(nf_batch* b, void* stream);
/* Wait for the last run and copy the count scores to host memory. */
int nf_batch_scores(nf_batch* b, int32_t* scores_out);
/* Wait for the last run and copy the table of sequence idx (ns[idx]^2 int16). */
int nf_batch_table(nf_batch* b, int idx, int16_t* S_out);
/* One optimal structure per fold of a run batch, as nf_fold_structure gives
 * it (Section 2, the traceback through D* with the same tie rule), all folds
 * traced back at once (one workgroup per fold).  db_outs[i] receives n_i
 * characters (no terminator); a NULL entry skips that fold.  NF_E_INVAL if
 * the batch has not been run. */
int nf_batch_structures(nf_batch* b, char* const* db_outs);
/* Number of sequences and total device bytes the batch holds. */
int nf_batch_info(const nf_batch* b, int* count, size_t* device_bytes);
void nf_batch_destroy(nf_batch* b);

/* Convenience: create, run, copy scores (and the tables for every non-NULL
 * S_outs[i] when S_outs is not NULL), destroy.  Synchronous. */
int nf_fold_batch(const char* const* seqs, const int* ns, int count, int q,
                  int32_t* scores_out, int16_t* const* S_outs);

/* ---- Serving: continuous batching ----
 * A background engine keeps admitted folds resident on the device and
 * advances every active fold by one tile diagonal per device step; requests
 * that arrive while others run join at the next step when a slot and enough
 * of the device-memory budget are free.  If a device call of the engine
 * fails, every request it holds or has queued completes with that error
 * (NF_E_DEVICE, NF_E_NOMEM), and the next nf_submit starts a new engine.
 * nf_serve_config, nf_submit and nf_shutdown may be called from any thread;
 * a request submitted while nf_shutdown runs completes with NF_E_ABORTED or
 * is served by the next engine. */

/* Configure before the first nf_submit (or after nf_shutdown):
 * hbm_budget_bytes = device bytes the active folds may hold together
 * (0 = 80% of free device memory); max_slots = folds active at once (0 = 256);
 * max_queue = pending requests before NF_E_BUSY (0 = 65536). */
int nf_serve_config(size_t hbm_budget_bytes, int max_slots, int max_queue);

/* Device bytes a fold of length n holds while active in the serving engine
 * under q (table, packed words, accumulators; a request with NF_WANT_TABLE
 * holds n*n*2 more, one with NF_WANT_STRUCTURE about 9n more).  0 for
 * arguments out of range. */
size_t nf_fold_bytes(int n, int q);

/* What a served fold keeps for its result, beside the score (flags of
 * nf_submit): the full table (nf_poll / nf_wait / nf_poll_ex S_out), and one
 * optimal structure as nf_fold_structure gives it (nf_poll_ex db_out), read
 * back on the device when the fold finishes. */
#define NF_WANT_TABLE 1
#define NF_WANT_STRUCTURE 2

/* Queue a fold (the sequence is copied).  Returns a ticket >= 0 or a negative
 * code: NF_E_INVAL/NF_E_TOOLONG for bad input or unknown flags, NF_E_NOMEM if
 * the fold alone is larger than the budget, NF_E_BUSY if the queue is full.
 * Never waits on the GPU.  flags: 0, or NF_WANT_TABLE and/or
 * NF_WANT_STRUCTURE. */
int64_t nf_submit(const char* seq, int n, int q, int flags);

/* 1 = done (outputs written, ticket released), 0 = still pending, < 0 error.
 * score_out may be NULL; S_out (n*n int16) may be NULL, and is ignored unless
 * the ticket was submitted with want_table. */
int nf_poll(int64_t ticket, int32_t* score_out, int16_t* S_out);

/* Like nf_poll but blocks up to timeout_ms (< 0: no limit); NF_E_TIMEOUT when
 * the deadline passes first (the ticket stays valid). */
int nf_wait(int64_t ticket, int timeout_ms, int32_t* score_out, int16_t* S_out);

/* nf_poll and nf_wait in one, with the structure: timeout_ms = 0 polls,
 * > 0 waits up to that long, < 0 waits without limit.  db_out (n characters,
 * no terminator) may be NULL, and is ignored unless the ticket was submitted
 * with NF_WANT_STRUCTURE; S_out as for nf_poll.  Same returns as nf_wait
 * (0 only when polling). */
int nf_poll_ex(int64_t ticket, int timeout_ms, int32_t* score_out, int16_t* S_out, char* db_out);

/* Engine counters: admitted, completed, rejected requests, device steps run,
 * the largest number of budget bytes ever held by active folds, and how many
 * steps ran fused (one launch per q holding the step's finishes and between
 * work, as nf_fold does; the others ran staged, on two streams).  A step is
 * fused while it holds at most 208 tiles to finish, unless NF_MODE (read when
 * the engine starts) forces one form. */
typedef struct {
    int64_t submitted, admitted, completed, rejected, steps;
    int64_t active, pending;
    size_t budget_bytes, peak_bytes;
    int64_t steps_fused;
} nf_serve_stats_t;
int nf_serve_stats(nf_serve_stats_t* out);

/* ---- Tuning ----
 * Choices are kept per length bucket (n < 256, < 512, ..., >= 65536).  They
 * come from the autotune cache file named by NF_AUTOTUNE_CACHE if set and
 * readable (one line per bucket: "bucket q target"; a line without the
 * target leaves it at its default), from nf_autotune, else from built-in
 * defaults.  Neither changes a result: every q and every target fills the
 * same table.
 *
 * The q that q = 0 resolves to for sequences of length n (group width of
 * Eq. 3; default 8). */
int nf_autotune_q(int n);
/* The launch shape of a single fold of length n at group width q (0 = what
 * q = 0 resolves to): the number of between-group chunks (workgroups) each
 * wavefront step is cut into.  The tuned target of n's bucket applies only
 * to the q tuned with it; otherwise, and for batches and the serving
 * engine's steps, the default 1024.  The environment variable
 * NF_BETWEEN_TARGET, if set, overrides every value.  NF_E_INVAL for n or q
 * out of range. */
int nf_autotune_target(int n, int q);
/* Whether a single fold of length n at group width q (0 = what q = 0
 * resolves to) runs its fused wavefront steps in the wide shape: the same
 * kernel code held to fewer registers so that a CU takes three workgroups
 * instead of two, which speeds the between-group lookups of long folds and
 * slows each tile finish.  Only at q = 8.  The tuned choice of n's bucket
 * (fourth column of the cache file: 1 wide, 0 not) if it was tuned at this q,
 * else wide for n >= 8192; NF_STAGE_WIDE=0|1 overrides.  Returns 1 or 0, or
 * NF_E_INVAL for n or q out of range. */
int nf_autotune_wide(int n, int q);
/* Time the fill at length n (reps folds each, after one warm-up fold): first
 * q in qmin..qmax at the default target, then the targets 1024, 256, 512,
 * 2048 and 2560 at the fastest q, then (q = 8) the other fused-step shape.  Records
 * all three in the in-memory cache (and in the cache file if set).  Returns
 * the chosen q. */
int nf_autotune(int n, int qmin, int qmax, int reps);

/* ---- Diagnostics ----
 * Per-kernel timing of the fill of one sequence given as device codes (as in
 * nf_fold_dev).  Runs the fill reps times on stream without a graph; each
 * launch is timed by a pair of HIP events that its own dispatch records when
 * the kernel starts and ends (hipExtLaunchKernelGGL), and the durations are
 * summed per kernel class k:
 * 0 = main-diagonal tiles, 1 = tile finish, 2 = between-group lookups (the
 * launches of the staged execution), 3 = one fused step (finishes of a
 * diagonal and the between-group chunks of the next); the fill runs in the
 * execution its workspace uses (see nf_fold).  For every class:
 * lookups[k] counts the Four-Russians steps of Eq. 3 on table cells (padding
 * excluded): the groups between the end tiles, those of the two end tiles,
 * and, when q divides 8, the groups of each finished 8-row block of a tile
 * for the rows above it; splits[k] the terms of Eq. 1 evaluated one by one
 * (split points within a tile's own columns, those within its own rows that
 * are not looked up, plus the pairing term); cells[k] the table cells
 * finished.  Synchronous. */
typedef struct {
    int64_t launches[4];
    double ms[4];
    double lookups[4];
    double splits[4];
    double cells[4];
    int q, tile, tiles_per_side, stages;
    int wide; /* 1 when the fused steps ran in the wide shape (nf_autotune_wide) */
} nf_kernel_profile_t;
int nf_profile_fold(const uint8_t* d_codes, int n, int q, int reps, void* stream, nf_kernel_profile_t* out);

/* The device's LDS byte-gather ceiling, the second unit a lookup of Eq. 3
 * uses besides VALU issue (one 1-byte read of R from LDS per lookup): every
 * lane of 8 workgroups per CU repeatedly reads 16 fixed offsets of a
 * table_bytes table in LDS with 1-byte loads.  row_bytes = 0 draws the
 * offsets uniformly over the table; row_bytes > 0 gives each load of a
 * wavefront one row of row_bytes bytes with a random byte per lane, the
 * pattern of R[h][c] with a wave-uniform h (row_bytes = 2^(q-1)).  Writes
 * lane-gathers per second.  table_bytes: a power of two in 64..65536;
 * row_bytes: 0 or a divisor of it.  Synchronous. */
int nf_lds_gather_rate(int table_bytes, int row_bytes, double* lane_gathers_per_s);

#ifdef __cplusplus
}
#endif
#endif /* NF_H */
