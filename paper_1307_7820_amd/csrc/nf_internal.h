// Internal declarations shared by the kernels (nf_kernels.hip) and the host
// runtime (nf_runtime.cpp).  Not part of the public ABI.
//
// Coordinates.  The kernels index the table of Eq. 1 by fence posts: post a
// sits before base a+1, and F(a, b) = D(a+1, b) for 0 <= a <= b <= n.  Then
// F(a, a) = F(a, a+1) = 0 and, for b >= a+2,
//     F(a, b) = max{ b(S_{a+1}, S_b) + F(a+1, b-1), max_{a<m<b} F(a, m) + F(m, b) }.
// The split point m = k-1 of Eq. 1 indexes both the row cell F(a, m) and the
// column cell F(m, b), so the row grouping and the column grouping of
// Section 3.1 (columns from 0, rows from 1, i.e. offset by one) become the
// same grouping of posts: group K = posts [Kq, Kq+q-1].
//
// Tiles.  Posts 0..n are cut into NT tiles of T = G*q posts (G = 64/q groups,
// T <= 64).  Tile (A, B), A <= B, holds F(a, b) for a in [AT, AT+T) and b in
// [BT, BT+T); its diagonal is d = B - A.  Tiles are numbered diagonal-major:
// tile_index(NT, A, d) = d*NT - d(d-1)/2 + A, so the tiles a wavefront step
// writes are contiguous.
//
// Packed state of a finished off-diagonal tile (A, B) (Lemma 1: neighbours
// differ by 0 or 1), one 32-bit word per row and group and per column and
// group:
//   row word (group k of the tile's columns, row i):
//       bits 31..16 = h << (q-1), bit p-1 of h = F(a, BT+kq+p) - F(a, BT+kq+p-1)
//       bits 15..0  = F(a, BT+kq)                (Eq. 3 "D(i,l)")
//   column word (group k of the tile's rows, column j):
//       bits 31..16 = c, bit p-1 of c = F(AT+kq+p-1, b) - F(AT+kq+p, b)
//       bits 15..0  = F(AT+kq, b)                (Eq. 3 "D(l+1,j)")
// Scores are below 2^15 and h << (q-1) | c below 2^16 for q <= 9.  Per tile
// the row block and the column block are each [k][64] (rows/columns >= T
// unused), so one group of one tile is one 256-byte line.  The Four-Russians
// step of Eq. 3 for cell (a, b) and group K is then
//     (rw & 0xffff) + (cw & 0xffff) + R[(rw >> 16) + (cw >> 16)]
// with the row word rw read wave-uniformly.  Every such term is one split of
// Eq. 1, so it is at most F(a, b) < 2^15: the low half of rw + cw + R holds
// it without a carry, whatever the high halves hold.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nf {

constexpr int kThreads = 512;  // main-diagonal tiles: 8 wavefronts, 64 groups of 8 lanes (one pass per diagonal)
// between-group chunks: 8 wavefronts.  A wavefront owns 16 rows (8 rows
// measured slower: twice the column-word loads for the same lookups); two
// wavefronts share each block of rows and take alternate groups of split
// points.
constexpr int kBetweenThreads = 512;
constexpr int kRowsPerWave = 16;
constexpr int kBetweenSplit = kBetweenThreads / 64 / (64 / kRowsPerWave);
static_assert(kBetweenSplit == 1 || kBetweenSplit == 2, "one or two wavefronts per row block");
constexpr int kTileCells = 64 * 64;
// A between chunk spans at least this many group tiles C when the step's work
// allows: a chunk has fixed costs (R into LDS, the merge of its row blocks,
// its atomic maxima), and MI355X folds of n = 10000 and 16000 ran 0.4-0.7%
// faster with 4 than with 1 (the smallest chunks come in the early steps).
constexpr int kMinChunkTiles = 4;

__host__ __device__ constexpr int groups_per_tile(int q) { return 64 / q; }
__host__ __device__ constexpr int tile_size(int q) { return (64 / q) * q; }
__host__ __device__ constexpr int state_words(int q) { return (64 / q) * 64; }  // column block
__host__ __device__ constexpr int row_words(int q) { return state_words(q); }      // row block
__host__ __device__ inline long long tile_index(int NT, int A, int d)
{
    return (long long)d * NT - (long long)d * (d - 1) / 2 + A;
}
__host__ __device__ inline long long tile_count(int NT) { return (long long)NT * (NT + 1) / 2; }

// One sequence being folded.  All pointers are device pointers.
struct FoldDesc {
    const uint8_t* codes;  // NT*T + 64 bytes: base codes A0 C1 G2 U3, zero padding
    int16_t* F;            // ld x ld table of F(a, b), ld = NT*T
    uint32_t* RS;          // row blocks, tile_count(NT) * row_words(q)
    uint32_t* CS;          // column blocks, tile_count(NT) * state_words(q)
    int n, NT, ld, pad;
};

// Between-group work (host form): tile (A, A+d) of fold `fold`, the groups
// of the tiles C in [c0, c1) (A < c0 <= C < c1 < A+d).  The 64x64 maxima go
// to the tile's accumulator slot `slot`; pad0 != 0 when several items share
// that slot (combined with atomic max).
struct BetweenItem {
    int fold, A, d, c0, c1, slot, pad0, pad1;
};

// Tile finish (host form): tile (A, A+d) of fold `fold`; when nslot > 0 the
// accumulator slot slot0 holds between-group maxima to fold in (and is
// cleared after reading).
struct TileItem {
    int fold, A, d, slot0, nslot, pad0, pad1, pad2;
};

// The packed wavefront schedule of one fold alone, in closed form: the same
// items, in the same order and slots, as the host's schedule builder makes
// for a single fold of NT tiles per side at `target` between chunks per step
// (a host test checks the two against each other).  Stage sg finishes the
// tiles of diagonal sg and runs the between chunks of diagonal sg+1; the
// between work of tile (A, A+d), d >= 4, is cut into chunks(d) pieces of its
// group tiles C in [A+2, A+d-2], combined in accumulator slot
// A + (stage parity) * max_slots.
struct SingleSchedule {
    int NT = 0, target = 1;

    __host__ __device__ int max_slots() const { return NT >= 5 ? NT - 4 : 0; }
    // chunks per tile of diagonal dd (0 when the diagonal has no between work)
    __host__ __device__ int chunks(int dd) const
    {
        if (dd < 4 || NT <= dd) return 0;
        const long long W = (long long)(NT - dd) * (dd - 3);
        long long chunk = (W + target - 1) / target;
        if (chunk < kMinChunkTiles) chunk = kMinChunkTiles;
        return (int)((dd - 3 + chunk - 1) / chunk);
    }
    __host__ __device__ int finishes(int sg) const { return (sg >= 1 && sg < NT) ? NT - sg : 0; }
    __host__ __device__ long long finish_offset(int sg) const
    {
        return sg <= 1 ? 0 : (long long)(sg - 1) * NT - (long long)(sg - 1) * sg / 2;
    }
    __host__ __device__ int between_count(int sg) const { return (NT - sg - 1) * chunks(sg + 1); }
    __host__ __device__ long long between_offset(int sg) const
    {
        long long off = 0;
        for (int s = 0; s < sg; ++s) off += between_count(s);
        return off;
    }
    __host__ __device__ TileItem finish(int sg, int A) const
    {
        TileItem it{0, A, sg, 0, 0, 0, 0, 0};
        if (sg >= 4) {
            it.slot0 = A + ((sg - 1) & 1) * max_slots();
            it.nslot = 1;
        }
        return it;
    }
    // item k of stage sg: tile A = k / ns, chunk k % ns
    __host__ __device__ BetweenItem between(int sg, int k) const
    {
        const int dd = sg + 1, ns = chunks(dd), nC = dd - 3;
        const int A = k / ns, c = k - A * ns;
        BetweenItem it{};
        it.fold = 0;
        it.A = A;
        it.d = dd;
        it.c0 = A + 2 + (int)((long long)c * nC / ns);
        it.c1 = A + 2 + (int)((long long)(c + 1) * nC / ns);
        it.slot = A + (sg & 1) * max_slots();
        it.pad0 = ns > 1 ? 1 : 0;
        return it;
    }
};

// Device-side work items: the fold's descriptor travels inside the item, so a
// workgroup reaches its data with a single dependent load.
// acc points at the tile's 64x64 int32 accumulator (between-group maxima).
struct TileWork {
    FoldDesc f;
    int32_t* acc;  // read and cleared when nslot > 0 (admission: the fold's accumulators)
    int A, d, nslot, pad0, pad1, pad2;  // pad1, pad2: admission (launch_diag_admit)
};
struct BetweenWork {
    FoldDesc f;
    int32_t* acc;  // combined with atomic max when atomic != 0, else stored
    int A, d, c0, c1, atomic, pad0;
};
static_assert(sizeof(TileWork) == 80, "TileWork layout");
static_assert(sizeof(BetweenWork) == 80, "BetweenWork layout");

// One fused wavefront step: ntile tile finishes and nbtw between chunks of
// the next diagonal in one launch of kTileThreads-thread workgroups.  wide
// (q = 8 only; ignored otherwise) selects the shape that fits three
// workgroups per CU instead of two.
hipError_t launch_stage(int q, bool wide, const TileWork* titems, int ntile, const BetweenWork* bitems, int nbtw,
                        const uint8_t* R, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Whether a single fold of length n at q runs the wide fused step: the tuned
// choice of n's length bucket if one was tuned at this q, else n >= 8192 at
// q = 8 (NF_STAGE_WIDE=0|1 overrides).
bool stage_wide(int n_single, int q);

// Plain between-group maxima from the dense table (no R): the ablation of the
// lookup.  q must give 64-post tiles (1, 2, 4, 8).
hipError_t launch_between_plain(int q, const BetweenWork* items, int nitems, hipStream_t s, hipEvent_t e0 = nullptr,
                                hipEvent_t e1 = nullptr);
hipError_t launch_precompute_R(int q, uint8_t* R, hipStream_t s);
hipError_t launch_copy_codes(const uint8_t* src, int n, uint8_t* dst, int padded, hipStream_t s);
// With events e0/e1 the dispatch records the kernel's own start and end.
hipError_t launch_diag(int q, const TileWork* items, int nitems, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
// wide (q = 8 only): the lean finish, three workgroups per CU
hipError_t launch_tile(int q, const TileWork* items, int nitems, const uint8_t* R, hipStream_t s,
                       hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, bool wide = false);
hipError_t launch_between(int q, const BetweenWork* items, int nitems, const uint8_t* R, hipStream_t s,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// The main-diagonal tiles of newly admitted folds (items with pad2 = 1 read
// their fold's padded codes at staged + pad1, copy them into the fold's block
// and clear the fold's 2 NT accumulator blocks at acc).
hipError_t launch_diag_admit(int q, const TileWork* items, int nitems, const uint8_t* staged, hipStream_t s);
// scores[f] = F(0, n_f)
hipError_t launch_scores(const FoldDesc* folds, int nfolds, int32_t* scores, hipStream_t s);
// scores[folds[f].pad] = F(0, n_f)
hipError_t launch_scores_to_slots(const FoldDesc* folds, int nfolds, int32_t* scores, hipStream_t s);
// A bounded delay of about iters x 3.4 us (at most 16) on stream s: one wavefront
// that sleeps (perturbed schedules, nf_test_set_perturb).
hipError_t launch_delay(int iters, hipStream_t s);
hipError_t launch_expand(const int16_t* F, int ld, int n, int16_t* S, hipStream_t s);
// One optimal structure of the fold whose table F (leading dimension ld) and
// codes are given, as n dot-bracket characters in db; *status = 0 on success.
// spill: 2 * spill_cap entries of device scratch, spill_cap >= n/2 + 1.
hipError_t launch_traceback(const int16_t* F, int ld, const uint8_t* codes, int n, int2* spill, int spill_cap,
                            char* db, int* status, hipStream_t s);
// The same for many folds at once, one workgroup per entry of work (device).
struct TracebackWork {
    const int16_t* F;
    const uint8_t* codes;
    int2* spill;   // 2 * spill_cap entries, spill_cap >= n/2 + 1
    char* db;      // n bytes
    int* status;
    long long ld;
    int n, spill_cap;
};
hipError_t launch_traceback_many(const TracebackWork* work, int count, hipStream_t s);

}  // namespace nf
