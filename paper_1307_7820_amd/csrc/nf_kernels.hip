// HIP kernels for gfx950: the two-vector Four-Russians fill of the Nussinov
// table (Section 3.1, Eq. 3) swept as a tile wavefront (Sections 4-5).
//
// Work of one wavefront step (tile diagonal d):
//   * k_between: for a tile (A, B = A+d) and a range of intermediate tiles C,
//     the best split over every q-group of posts inside those tiles, one R
//     lookup per group (Eq. 3).  Only tiles of diagonals < d are read.
//   * k_tile: the finish of tile (A, B): folds in the partial maxima, the
//     groups of the two tiles next to the diagonal ends (C = A+1, C = B-1),
//     the pairing term and the splits that fall inside tiles A and B
//     (the "residual" split points of Section 3.1), cell by cell along the
//     tile's own anti-diagonals; then writes the dense int16 cells and the
//     packed row/column words.
//   * k_diag: the tiles (A, A) on the main diagonal, where every split point
//     is inside the tile.
// Max is idempotent and order-free, so the result does not depend on how the
// between-group work is split into partial slots.
#include "nf_internal.h"

#include <hip/hip_ext.h>

#include <type_traits>

namespace nf {

namespace {

// Address-space views of generic pointers.  The between-group lookups read
// row words wave-uniformly through the scalar cache (constant address
// space); column words are per-lane global loads.  The scalar cache is not
// kept coherent with vector stores inside a launch, so the invariant is: no
// row word that a launch reads through the scalar cache is written by that
// same launch.  It holds because a between chunk of tile (A, A+d) reads only
// tiles of diagonals 2 .. d-2, a staged between launch writes no packed
// words (the finishes of diagonal d-1 that may run beside it on another
// stream write only that diagonal), and the fused step that runs it
// (d = s+1) writes only the words of diagonal s.  Packed blocks of different
// tiles never share a cache line (each block is a multiple of 256 bytes).
// The tile finish reads every packed word through vector loads.
#define NF_GLOBAL __attribute__((address_space(1)))
#define NF_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const NF_GLOBAL T* as_global(const T* p)
{
    return (const NF_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const NF_CONST T* as_const(const T* p)
{
    return (const NF_CONST T*)p;
}

// R index of a row word held in a scalar register and a column word: bits
// 31..16 of each, one VALU instruction (SDWA selects both high halves; an
// ALU operation, not a load).
__device__ __forceinline__ uint32_t r_index_s(uint32_t rw, uint32_t cw)
{
    uint32_t idx;
    __asm__("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:WORD_1"
            : "=v"(idx)
            : "s"(rw), "v"(cw));
    return idx;
}

// The same with both words in vector registers.
__device__ __forceinline__ uint32_t r_index_v(uint32_t rw, uint32_t cw)
{
    uint32_t idx;
    __asm__("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:WORD_1"
            : "=v"(idx)
            : "v"(rw), "v"(cw));
    return idx;
}

// max of a and the low 16 bits of b (as an unsigned number), one VALU
// instruction (SDWA selects the low half of b).
__device__ __forceinline__ int max_lo16(int a, uint32_t b)
{
    int d;
    __asm__("v_max_i32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
            : "=v"(d)
            : "v"(a), "v"(b));
    return d;
}

// max of the low 16 bits of a, b and c as unsigned numbers, one VALU
// instruction (the high halves of the operands are ignored).
__device__ __forceinline__ uint32_t max3_u16(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t d;
    __asm__("v_max3_u16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Copy the q-dependent R table (RSZ bytes) into LDS.  From 1 KB on by DMA
// (global -> LDS, no registers and no LDS store; a wave moves 1 KB and RSZ is
// a multiple of it, so no lane reads past R or writes past Rl), waited for
// here; below that through registers.  The caller's barrier follows.
template <int RSZ>
__device__ __forceinline__ void load_R(uint8_t* Rl, const uint8_t* __restrict__ Rg, int nthr)
{
    if constexpr (RSZ >= 1024) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
        for (int base = wave * 1024; base < RSZ; base += nthr * 16)  // wave-uniform
            __builtin_amdgcn_global_load_lds((const NF_GLOBAL void*)(Rg + base + lane * 16),
                                             (__attribute__((address_space(3))) void*)(Rl + base), 16, 0, 0);
        __builtin_amdgcn_s_waitcnt(0);
    } else if constexpr (RSZ >= 16) {
        for (int x = threadIdx.x * 16; x < RSZ; x += nthr * 16)
            *reinterpret_cast<uint4*>(Rl + x) = *reinterpret_cast<const uint4*>(Rg + x);
    } else {
        if (threadIdx.x < RSZ) Rl[threadIdx.x] = Rg[threadIdx.x];
    }
}

// Between-group maxima for the RPW rows r0..r0+RPW-1 (wave-uniform) and column j
// (the lane) of tile (A, B), over the groups of tiles C in [c0, c1).
// For group k of tile C the row word comes from tile (A, C) and the column
// word from tile (C, B); Eq. 3 turns the q split points of the group into
//     F(a, Cq') + F(Cq', b) + R[h][c].
// With NS > 1 the caller's share is every NS-th group of the flattened
// (C, k) sequence, starting at group h.
//
// A lookup is two and a half VALU instructions: the R index (one SDWA add of
// the high halves of the scalar row word and the column word), one 3-input
// add of the whole row word, the whole column word and R (the low halves
// hold the two bases, so the low half of the sum is the split's value, see
// the packed words), and half of a 16-bit 3-input max over two groups.  acc
// holds its maxima in the low 16 bits.
template <int Q, int RPW, int NS>
__device__ __forceinline__ void between_accumulate(int (&acc)[RPW], const uint8_t* Rl,
                                                   const uint32_t* __restrict__ RS,
                                                   const uint32_t* __restrict__ CS, int NT, int A,
                                                   int B, int c0, int c1, int r0, int j, int h)
{
    constexpr int G = groups_per_tile(Q);
    constexpr int SW = state_words(Q);
    constexpr int RW = row_words(Q);
    if constexpr (G % NS == 0) {
        // every tile gives this wave the same KPT groups k = h, h+NS, ...,
        // taken KB at a time (KB * RPW row words fit the scalar registers):
        // all the row words (scalar loads) and column words of a batch are
        // loaded before its first lookup, so the wait for the scalar loads,
        // which also waits for the LDS gathers in flight, comes once per
        // batch; the next batch's column words are loaded while this batch's
        // lookups run
        constexpr int KPT = G / NS;
        constexpr int KB = KPT % 4 == 0 ? 4 : (KPT % 2 == 0 ? 2 : 1);
        constexpr int NBT = KPT / KB;  // batches per tile
        uint32_t cwn[KB];
        auto load_cw = [&](int C, int u0) {
            const NF_GLOBAL uint32_t* cs = as_global(CS + tile_index(NT, C, B - C) * SW + j);
#pragma unroll
            for (int v = 0; v < KB; ++v) cwn[v] = cs[(h + (u0 + v) * NS) * 64];
        };
        if (c0 < c1) load_cw(c0, 0);
        for (int C = c0; C < c1; ++C) {
            const NF_CONST uint32_t* rs = as_const(RS + tile_index(NT, A, C - A) * RW + r0);
#pragma unroll
            for (int bt = 0; bt < NBT; ++bt) {
                const int u0 = bt * KB;
                uint32_t cw[KB], rw[KB][RPW];
#pragma unroll
                for (int v = 0; v < KB; ++v) cw[v] = cwn[v];
#pragma unroll
                for (int v = 0; v < KB; ++v)
#pragma unroll
                    for (int r = 0; r < RPW; ++r) rw[v][r] = rs[(h + (u0 + v) * NS) * 64 + r];
                if (bt + 1 < NBT)
                    load_cw(C, u0 + KB);
                else if (C + 1 < c1)
                    load_cw(C + 1, 0);
#pragma unroll
                for (int v = 0; v < KB; v += 2) {
#pragma unroll
                    for (int r = 0; r < RPW; ++r) {
                        const uint32_t t0 = rw[v][r] + cw[v] + Rl[r_index_s(rw[v][r], cw[v])];
                        const uint32_t t1 =
                            v + 1 < KB ? rw[v + 1][r] + cw[v + 1] + Rl[r_index_s(rw[v + 1][r], cw[v + 1])] : 0u;
                        acc[r] = (int)max3_u16((uint32_t)acc[r], t0, t1);
                    }
                }
            }
        }
    } else {
        for (int C = c0; C < c1; ++C) {
            const NF_CONST uint32_t* rs = as_const(RS + tile_index(NT, A, C - A) * RW + r0);
            const NF_GLOBAL uint32_t* cs = as_global(CS + tile_index(NT, C, B - C) * SW + j);
            const int k0 = ((h - (C - c0) * G) % NS + NS) % NS;
#pragma unroll 2
            for (int k = k0; k < G; k += NS) {
                const uint32_t cw = cs[k * 64];
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const uint32_t rw = rs[k * 64 + r];
                    const uint32_t t = rw + cw + Rl[r_index_s(rw, cw)];
                    acc[r] = (int)max3_u16((uint32_t)acc[r], t, 0u);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] &= 0xffff;
}

__global__ void k_precompute_R(int q, uint8_t* __restrict__ R)
{
    const int m = q - 1;
    const int size = 1 << m;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= size * size) return;
    const int h = e >> m;
    const int c = e & (size - 1);
    int tot = 0, best = 0;  // running total of v + v-bar, starting at k = 0 with 0
    for (int p = 1; p <= m; ++p) {
        tot += ((h >> (p - 1)) & 1) - ((c >> (p - 1)) & 1);
        best = max(best, tot);
    }
    R[e] = (uint8_t)best;
}

__global__ void k_copy_codes(const uint8_t* __restrict__ src, int n, uint8_t* __restrict__ dst, int padded)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < padded) dst[e] = e < n ? (src[e] & 3) : 0;
}

// Main-diagonal tiles (A, A): every split point lies inside the tile, so the
// tile is filled by its own diagonals t = b - a = 2..T-1 (Eq. 1 directly).
struct DiagLds {
    int32_t X[64 * 65];  // padded stride 65: rows of a column are in distinct banks
    uint8_t ca[64], cb[64];
};

//
// Admission (staged != null and it.pad2 != 0, the serving engine's newly
// admitted folds): the fold's padded codes are read from staged + it.pad1
// instead of its own block, and the tile also does the fold's set-up: it
// copies its T codes (the last tile also the padding after them) into the
// fold's block and clears its two accumulator blocks (it.acc, one per
// diagonal parity), so that admitting a fold takes no copy or fill of its
// own.  Nothing else reads the fold's block before this launch has ended.
template <int Q>
__device__ __forceinline__ void diag_body(const TileWork& it, DiagLds& s, int tid, int nthr, const uint8_t* staged)
{
    constexpr int T = tile_size(Q);
    constexpr int XS = 65;
    int32_t* X = s.X;
    const FoldDesc& f = it.f;
    const int aT = it.A * T;
    const bool admit = staged != nullptr && it.pad2 != 0;
    const uint8_t* src = admit ? staged + it.pad1 : f.codes;

    for (int e = tid; e < 64 * XS; e += nthr) X[e] = 0;
    if (tid < 64) {
        s.ca[tid] = src[aT + tid];                              // S_{a+1} for a = aT + i
        s.cb[tid] = (aT + tid - 1 >= 0) ? src[aT + tid - 1] : 0;  // S_b for b = aT + j
    }
    if (admit) {
        uint8_t* dst = const_cast<uint8_t*>(f.codes);
        const int hi = it.A == f.NT - 1 ? f.NT * T + 64 : aT + T;
        for (int e = aT + tid; e < hi; e += nthr) dst[e] = src[e];
        int4* a0 = reinterpret_cast<int4*>(it.acc + (size_t)it.A * kTileCells);
        int4* a1 = reinterpret_cast<int4*>(it.acc + (size_t)(f.NT + it.A) * kTileCells);
        for (int e = tid; e < kTileCells / 4; e += nthr) a0[e] = a1[e] = make_int4(0, 0, 0, 0);
    }
    __syncthreads();

    // diagonal t: cell (i, i+t) takes max over its split points m; eight
    // lanes share a cell (lane k of the group takes m = i+1+k, i+9+k, ...)
    // and combine their maxima inside the group with DPP (mirror within 8
    // lanes, then two quad permutations).  Every value is >= 0, so 0 is the
    // identity of max here.
    const int grp = tid >> 3, sub = tid & 7, ngrp = nthr >> 3;
    for (int t = 2; t < T; ++t) {
        for (int i0 = 0; i0 < T - t; i0 += ngrp) {
            const int i = i0 + grp;
            const int j = i + t;
            const bool live = i < T - t;
            int v = 0;
            if (live) {
                for (int m = i + 1 + sub; m < j; m += 8) v = max(v, X[i * XS + m] + X[m * XS + j]);
            }
            v = max(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));  // row_half_mirror
            v = max(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));   // quad_perm [1,0,3,2]
            v = max(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));   // quad_perm [2,3,0,1]
            if (live && sub == 0) X[i * XS + j] = max(v, (s.ca[i] + s.cb[j] == 3) + X[(i + 1) * XS + (j - 1)]);
        }
        __syncthreads();
    }

    int16_t* F = f.F;
    const long long ld = f.ld;
    for (int e = tid; e < 64 * 64; e += nthr) {
        const int i = e >> 6, j = e & 63;
        if (i < T && j < T) F[(aT + i) * ld + aT + j] = (int16_t)X[i * XS + j];
    }
}

template <int Q>
__global__ __launch_bounds__(kThreads) void k_diag(const TileWork* __restrict__ items, const uint8_t* staged)
{
    __shared__ DiagLds s;
    diag_body<Q>(items[blockIdx.x], s, threadIdx.x, kThreads, staged);
}

// One between item: rows r0 .. r0+RPW-1 and column j (the lane) of the tile's
// 64x64 maxima, written to its accumulator.  Wavefront w takes the row block
// w % (64/RPW); with NS = 2 the two wavefronts of a row block split the
// groups and merge their maxima through red (64x64 ints of LDS).  Every
// thread of the workgroup must call this.
template <int Q, int RPW, int NS>
__device__ __forceinline__ void between_body(const BetweenWork& it, const uint8_t* Rl,
                                             const uint32_t* RS, const uint32_t* CS, int wave, int j,
                                             uint16_t* red)
{
    constexpr int NB = 64 / RPW;
    static_assert(NS == 1 || NS == 2, "one or two wavefronts per row block");
    const int h = wave / NB;
    const int r0 = (wave - h * NB) * RPW;
    int acc[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = 0;
    between_accumulate<Q, RPW, NS>(acc, Rl, RS, CS, it.f.NT, it.A, it.A + it.d, it.c0, it.c1, r0, j, h);
    if constexpr (NS == 2) {
        if (h == 1) {
#pragma unroll
            for (int r = 0; r < RPW; ++r) red[(r0 + r) * 64 + j] = (uint16_t)acc[r];  // maxima < 2^15
        }
        __syncthreads();
        if (h == 1) return;
#pragma unroll
        for (int r = 0; r < RPW; ++r) acc[r] = max(acc[r], (int)red[(r0 + r) * 64 + j]);
    }

    int32_t* out = it.acc + r0 * 64 + j;
    if (it.atomic) {  // several items share the tile's accumulator
#pragma unroll
        for (int r = 0; r < RPW; ++r) atomicMax(out + r * 64, acc[r]);
    } else {
#pragma unroll
        for (int r = 0; r < RPW; ++r) out[r * 64] = acc[r];
    }
}

template <int Q>
__global__ __launch_bounds__(kBetweenThreads) void k_between(const BetweenWork* __restrict__ items,
                                                      const uint8_t* __restrict__ Rg)
{
    constexpr int RSZ = 1 << (2 * (Q - 1));
    __shared__ __align__(16) uint8_t Rl[RSZ < 16 ? 16 : RSZ];
    __shared__ uint16_t red[kBetweenSplit == 2 ? 64 * 64 : 1];

    const BetweenWork& it = items[blockIdx.x];
    load_R<RSZ>(Rl, Rg, kBetweenThreads);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    between_body<Q, kRowsPerWave, kBetweenSplit>(it, Rl, it.f.RS, it.f.CS, wave, threadIdx.x & 63, red);
}

// Finish of an off-diagonal tile (A, B), B > A, by 8 wavefronts (512 threads).
//
// Inside the tile, with L(i, i') = F(AT+i, AT+i') (tile (A, A)) and
// U(j', j) = F(BT+j', BT+j) (tile (B, B)), cell X(i, j) = F(AT+i, BT+j) is
//     max{ P(i, j),                                 between groups, in acc
//          b(S_{a+1}, S_b) + X(i+1, j-1),            pairing
//          max_{i < i' < T} L(i, i') + X(i', j),     splits inside tile A
//          max_{0 <= j' < j} X(i, j') + U(j', j) }   splits inside tile B.
// The last term only involves row i.  Eq. 1 makes F superadditive
// (F(m1, m3) >= F(m1, m2) + F(m2, m3), since m2 is one of its split points),
// so chains of U terms never beat a single one and the row recurrence has the
// closed form  X(i, .) = Q(i, .) (max,+) (I + U),  Q = the first three terms.
// Rows are finished bottom-up, one max-plus vector-matrix product per row.
//
// Work split: wave w owns the 8 columns J_w = [8w, 8w+8) of every row.  Lane
// l = 8g + c holds column j = 8w + c and the accumulators of the rows
// i = 8b + g (b = 0..7: one row in each 8-row block), and for the closure it
// reduces the split points j' in [8g, 8g+8) (its 8 entries of U sit in
// registers); the 8 lanes of a column then combine their partial maxima with
// a butterfly inside the wavefront (DPP row rotation and the gfx950 16/32-lane
// swaps).  Each row costs one workgroup barrier: the row's Q is published in
// LDS before it, the row's cells and the next row's Q after it.  The pairing
// partner of the first column of a slice lives in the wavefront to the left,
// so that one term is added by the readers of Q instead.
//
// A finished row is pushed (its L terms) into the rows above it in its 8-row
// block, one split each, by the lanes that hold those rows; when a whole
// block is finished and q divides 8 its q-groups reach every row above the
// block through one R lookup per group (Eq. 3: row words of tile (A, A),
// column words of this tile).  For other q every row is pushed into every row
// above it one split at a time.  The groups of the two end tiles (C = A+1,
// C = B-1) for the rows of block b-1 are looked up while block b is closed,
// a few per row, in the slack of the row steps.
constexpr int kTileThreads = 512;
static_assert(kTileThreads == 512, "the tile finish maps 8 wavefronts onto 8 column slices");
constexpr int kNeg = -(1 << 20);  // stands for minus infinity; sums stay far from overflow

template <int Q>
__device__ __forceinline__ int rlookup(const uint8_t* Rl, uint32_t rw, uint32_t cw)
{
    return (int)((rw & 0xffffu) + (cw & 0xffffu)) + (int)Rl[(rw >> 16) + (cw >> 16)];
}

// The Eq. 3 term of a row word and a column word in the low 16 bits of the
// result (the whole words are added: the term is one split of a cell, so it
// stays below 2^15 and nothing carries out of the low half; the high half is
// not meaningful).  Both words in vector registers.
__device__ __forceinline__ uint32_t rterm(const uint8_t* Rl, uint32_t rw, uint32_t cw)
{
    return rw + cw + (uint32_t)Rl[r_index_v(rw, cw)];
}

// max of v over the 8 lanes l ^ {8, 16, 32} (lanes 8g + c, g = 0..7)
__device__ __forceinline__ int max_over_groups(int v)
{
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true));  // row_ror:8 = lane ^ 8 (every lane valid)
    // the swaps return unsigned words: compare them as signed (-inf is negative)
    auto p16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);           // {v[l], v[l ^ 16]}
    v = max((int)p16[0], (int)p16[1]);
    auto p32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);           // {v[l], v[l ^ 32]}
    return max((int)p32[0], (int)p32[1]);
}

// kLean: the finish's lean form for the wide fused step (fewer registers and
// less LDS): finished cells kept as 16-bit values and the end tiles' column
// words read from LDS a row step ahead instead of held in registers.
// The 7 difference bits of 8 values that fall by 0 or 1 from each to the
// next (a column of the table going down, Lemma 1): bit p-1 is
// x[p-1] - x[p].  As integers that is the sum over p of
// (x[p-1] - x[p]) 2^(p-1) = x0 + x1 + 2 x2 + 4 x3 + 8 x4 + 16 x5 + 32 x6 - 64 x7,
// formed here as a tree of shift-adds three deep (7 instructions instead of
// a compare, a select and an or per bit).
__device__ __forceinline__ uint32_t drop_bits8(const int (&x)[8])
{
    const int t0123 = (x[0] + x[1]) + ((x[2] + (x[3] << 1)) << 1);
    const int t4567 = (x[4] + (x[5] << 1)) + ((x[6] - (x[7] << 1)) << 2);
    return (uint32_t)(t0123 + (t4567 << 3));
}

template <int Q, bool kLean>
struct TileLds {
    static constexpr int G = groups_per_tile(Q);
    static constexpr bool kBlockFR = (8 % Q) == 0;  // q-groups tile the 8-row blocks
    static constexpr bool kStageEdges = G <= 16;    // end-tile words fit in LDS
    using Cell = typename std::conditional<kLean, int16_t, int32_t>::type;
    Cell Xs[64 * 64];  // finished cells, row-major (values < 2^15)
    // Lp[i*kLS + 8g + b] = L(8b+g, i) for 8b+g < i < T, else -inf; the row
    // stride keeps 16-byte rows and spreads the transposed writes over the
    // banks.  The lean form keeps 16-bit values (-2^15 for -inf: a push of
    // it stays below every cell) to make room for its Q slots.
    using LCell = typename std::conditional<kLean, int16_t, int32_t>::type;
    static constexpr int kLS = kLean ? 72 : 68;
    LCell Lp[64 * kLS];
    uint32_t LW[kBlockFR ? G * 64 : 4];  // LW[k*64 + 8g + b]: row word of row 8b+g, group k, tile (A, A)
    uint32_t EB[kStageEdges ? 2 * G * 64 : 1];  // EB[(e*G + k)*64 + row] = row word, end tile e
    uint32_t EC[kStageEdges ? 2 * G * 64 : 1];  // EC[(e*G + k)*64 + col] = column word, end tile e
    // Q of the row being closed (double-buffered).  16-bit where every
    // column of the tile is a cell (T = 64): the closure then runs on packed
    // pairs.  With fewer posts the padding columns' values are not bounded
    // by a cell, so those q keep 32-bit values.
    static constexpr bool kPacked = tile_size(Q) == 64;
    using QCell = typename std::conditional<kPacked, int16_t, int32_t>::type;
    // Each of the 8 lane groups has a slot, so that every lane writes its
    // candidate and the row's chain has no masked write (the readers take the
    // slot of the row's group).
    // (slots 144 or 272 bytes apart: the 8 lanes that write one column's
    // slots hit 8 different banks, and rows stay 16-byte aligned)
    static constexpr int kQS = kPacked ? 72 : 68;
    alignas(16) QCell Qs[2][8][kQS];
    int32_t hrow[64];
    alignas(16) int32_t hcT[64];  // hcT[8g + b] = halo partner of column 0 in row 8b + g
    alignas(16) uint8_t caT[64];  // caT[8g + b] = S_{a+1} of row 8b + g
    uint8_t ca[64], cb[64];
    unsigned long long GM[8];  // GM[g] bit i: pairing of (row i, column 8g)
};

// The finish of one tile by kTileThreads threads.  With kLoadR the finish
// copies R from Rg (global) into Rl itself; otherwise Rl already holds it.
// wait_pre() runs before
// the loads that need the main-diagonal tiles (A, A) and (B, B); wait_main()
// before the loads that need the tiles of diagonal d-1 and the between-group
// maxima.  Both are collective (every thread calls them).
template <int Q, bool kLoadR, bool kLean, class Pre, class Main>
__device__ __forceinline__ void tile_body(const TileWork& it, uint8_t* Rl, const uint8_t* Rg, TileLds<Q, kLean>& s,
                                          Pre&& wait_pre, Main&& wait_main)
{
    constexpr int M = Q - 1;
    constexpr int G = groups_per_tile(Q);
    constexpr int T = tile_size(Q);
    constexpr int SW = state_words(Q);
    constexpr int RW = row_words(Q);
    using Lds = TileLds<Q, kLean>;
    using Cell = typename Lds::Cell;
    constexpr bool kBlockFR = Lds::kBlockFR;
    constexpr int GPB = kBlockFR ? 8 / Q : 1;  // groups per block
    constexpr bool kStageEdges = Lds::kStageEdges;
    constexpr int NE = kStageEdges ? 2 * G : 1;  // end-tile lookups per row (both edges)
    static_assert(!kStageEdges || NE > 8, "every row's share of the end-tile groups is at least one");
    constexpr int LS = Lds::kLS;
    Cell* Xs = s.Xs;
    typename Lds::LCell* Lp = s.Lp;
    uint32_t* LW = s.LW;
    uint32_t* EB = s.EB;
    uint32_t* EC = s.EC;
    using QCell = typename Lds::QCell;
    QCell (*Qs)[8][Lds::kQS] = s.Qs;
    int32_t* hrow = s.hrow;
    int32_t* hcT = s.hcT;
    uint8_t* caT = s.caT;
    uint8_t* ca = s.ca;
    uint8_t* cb = s.cb;
    unsigned long long* GM = s.GM;

    const FoldDesc& f = it.f;
    const int A = it.A, d = it.d, B = A + d;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int g = lane >> 3, c = lane & 7;
    const int j = wave * 8 + c;  // this lane's column; its rows are 8b + g
    const long long ld = f.ld;
    const int aT = A * T, bT = B * T;
    const NF_GLOBAL int16_t* F = (const NF_GLOBAL int16_t*)f.F;  // global loads: see the output pointers
    const NF_GLOBAL uint8_t* codes = (const NF_GLOBAL uint8_t*)f.codes;
    const NF_GLOBAL uint32_t* RSr = (const NF_GLOBAL uint32_t*)f.RS;
    const NF_GLOBAL uint32_t* CSr = (const NF_GLOBAL uint32_t*)f.CS;
    const int nedge = d >= 3 ? 2 : (d == 2 ? 1 : 0);

    // ---- prologue.  Every global load is issued before the first LDS store
    // (an LDS store of loaded data waits on the load counter, which drains in
    // order), so the tile pays about one memory round trip here.
    // part 1: R (when loading it), L, U and the codes
    wait_pre();
    constexpr int RSZ = 1 << (2 * M);
    uint8_t rbyte = 0;
    uint4 rvec = make_uint4(0u, 0u, 0u, 0u);
    if constexpr (kLoadR) {
        if constexpr (RSZ >= 1024) {
            // R goes global -> LDS by DMA (no registers, no LDS store): lane l
            // of a wave lands at the wave's base + 16 l.  One wave moves 1 KB,
            // and RSZ is a multiple of 1 KB here, so no lane reads past R or
            // writes past Rl.
#pragma unroll
            for (int u = 0; u < (RSZ + kTileThreads * 16 - 1) / (kTileThreads * 16); ++u) {
                const int base = (u * kTileThreads + wave * 64) * 16;  // wave-uniform
                if (base < RSZ)
                    __builtin_amdgcn_global_load_lds((const NF_GLOBAL void*)(Rg + base + lane * 16),
                                                     (__attribute__((address_space(3))) void*)(Rl + base), 16, 0, 0);
            }
        } else if constexpr (RSZ >= 16) {
            // 16 .. 256 bytes: one 16-byte load per lane that holds a piece,
            // stored to LDS with the other prologue stores
            if (tid * 16 < RSZ) {
                const NF_GLOBAL uint32_t* src = (const NF_GLOBAL uint32_t*)(Rg + tid * 16);
                rvec = make_uint4(src[0], src[1], src[2], src[3]);
            }
        } else {
            rbyte = ((const NF_GLOBAL uint8_t*)Rg)[min(tid, RSZ - 1)];
        }
    }
    // Addresses below are a wave-uniform base (scalar arithmetic) plus a
    // 32-bit lane offset, so the loads need almost no vector instructions.
    int lv[8];  // L(ip, lane) for the row ip = wave + 8u of tile (A, A), read coalesced
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int ip = wave + 8 * u;
        const NF_GLOBAL int16_t* Lrow = F + (long long)(aT + ip) * ld + aT;
        lv[u] = (ip < lane && lane < T) ? (int)Lrow[(unsigned)lane] : kNeg;
    }
    int ureg[8];  // U(8g + t, j); -inf where the split point is not left of column j
    const unsigned uoff = (unsigned)(8 * g) * (unsigned)ld + (unsigned)j;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int jp = 8 * g + t;
        const NF_GLOBAL int16_t* Urow = F + (long long)(bT + t) * ld + bT;
        ureg[t] = (jp <= j && j < T) ? (int)Urow[uoff] : kNeg;
    }
    uint8_t cda = 0, cdb = 0;
    if (tid < 64) {
        cda = codes[aT + tid];      // S_{a+1}, a = AT + i
        cdb = codes[bT + tid - 1];  // S_b,     b = BT + j  (BT >= 1)
    }

    // part 2: the between maxima, the end tiles and the halo
    wait_main();
    int acc[8];  // acc[b]: row 8b + g, column j
    NF_GLOBAL int32_t* accb = (NF_GLOBAL int32_t*)it.acc;
    const unsigned aoff = (unsigned)(g * 64 + j);
    if (it.nslot > 0) {
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[b] = (accb + b * 512)[aoff];
    } else {
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[b] = 0;
    }
    // edge e: C = A+1 (e = 0) and C = B-1 (e = 1); {base, bits} per row of
    // tile (A, C), column words of tile (C, B).  An end tile that does not
    // exist (e >= nedge) gets zero words: its lookups then give 0, which no
    // accumulator is below, so every lookup can run unguarded.  (The loads
    // stay inside the fold's tile arrays either way.)
    constexpr int kIter = kStageEdges ? (2 * G * 64 + kTileThreads - 1) / kTileThreads : 1;
    uint32_t rb[kIter], cw[kIter];
    if constexpr (kStageEdges) {
#pragma unroll
        for (int u = 0; u < kIter; ++u) {
            const int eg = wave + u * (kTileThreads / 64);  // (tid + u * kTileThreads) >> 6, wave-uniform
            const int e = eg / G, k = eg - e * G;
            const int C = e == 0 ? A + 1 : B - 1;
            rb[u] = cw[u] = 0;
            if (eg < 2 * G) {
                rb[u] = (RSr + tile_index(f.NT, A, C - A) * RW + k * 64)[(unsigned)lane];
                cw[u] = (CSr + tile_index(f.NT, C, B - C) * SW + k * 64)[(unsigned)lane];
            }
        }
    }
    int hrv = 0, hcv = 0;
    if (tid < T) {
        const int hr_r = aT + T, hr_c = bT - 1 + tid;  // F((A+1)T, BT-1+j)
        if (hr_c >= hr_r) hrv = F[hr_r * ld + hr_c];
        const int hc_r = aT + 1 + tid, hc_c = bT - 1;  // F(AT+1+i, BT-1)
        if (hc_c >= hc_r) hcv = F[hc_r * ld + hc_c];
    }

    // stores
    if constexpr (kLoadR && RSZ < 16) {
        if (tid < RSZ) Rl[tid] = rbyte;
    } else if constexpr (kLoadR && RSZ < 1024) {
        if (tid * 16 < RSZ) *reinterpret_cast<uint4*>(Rl + tid * 16) = rvec;
    }
    if (tid < 64) {
        ca[tid] = cda;
        cb[tid] = cdb;
        caT[(tid & 7) * 8 + (tid >> 3)] = cda;  // transposed: one 8-byte read per lane
    }
    if constexpr (kStageEdges) {
#pragma unroll
        for (int u = 0; u < kIter; ++u) {
            const int x = tid + u * kTileThreads;
            if (x < 2 * G * 64) {
                const bool live = (x >> 6) < nedge * G;
                EB[x] = live ? rb[u] : 0u;
                EC[x] = live ? cw[u] : 0u;
            }
        }
    }
    if (tid < T) hrow[tid] = hrv;
    if (tid < 64) hcT[(tid & 7) * 8 + (tid >> 3)] = hcv;  // hcv = 0 for rows >= T
    // this thread holds L(8u + wave, lane), u = 0..7: eight consecutive words
    if constexpr (kLean) {
        auto h16 = [](int v) { return (uint32_t)(uint16_t)(int16_t)max(v, -32768); };
        *reinterpret_cast<int4*>(&Lp[lane * LS + 8 * wave]) =
            make_int4((int)(h16(lv[0]) | (h16(lv[1]) << 16)), (int)(h16(lv[2]) | (h16(lv[3]) << 16)),
                      (int)(h16(lv[4]) | (h16(lv[5]) << 16)), (int)(h16(lv[6]) | (h16(lv[7]) << 16)));
    } else {
        *reinterpret_cast<int4*>(&Lp[lane * LS + 8 * wave]) = make_int4(lv[0], lv[1], lv[2], lv[3]);
        *reinterpret_cast<int4*>(&Lp[lane * LS + 8 * wave + 4]) = make_int4(lv[4], lv[5], lv[6], lv[7]);
    }
    if (it.nslot > 0) {  // hand the accumulator back zeroed for its next use
#pragma unroll
        for (int b = 0; b < 8; ++b) (accb + b * 512)[aoff] = 0;
    }
    if constexpr (kLoadR && RSZ >= 1024) __builtin_amdgcn_s_waitcnt(0);  // the R transfer (vector memory counter) is done
    __syncthreads();

    // ---- row words of tile (A, A) for the block pushes
    if constexpr (kBlockFR) {
        for (int x = tid; x < G * 64; x += kTileThreads) {
            const int k = x >> 6, pos = x & 63;       // pos = 8g' + b'
            const int r = (pos & 7) * 8 + (pos >> 3);  // row 8b' + g'
            const int top = k * Q;
            uint32_t h = 0;
            int base = 0;
            if (top > r && top < T) {
                base = Lp[top * LS + pos];
                if constexpr (Q == 8) {
                    // along a row the values rise by 0 or 1 (Lemma 1)
                    int v[8];
#pragma unroll
                    for (int p = 0; p < 8; ++p) v[p] = Lp[(top + p) * LS + pos];
                    h = 0u - drop_bits8(v);
                } else {
#pragma unroll
                    for (int p = 1; p <= M; ++p)
                        h |= (uint32_t)(Lp[(top + p) * LS + pos] > Lp[(top + p - 1) * LS + pos]) << (p - 1);
                }
            }
            LW[x] = ((h << M) << 16) | (uint32_t)base;
        }
    }

    // column words of the end tiles at this lane's column (fixed for the
    // tile): in registers, or in the lean form read from LDS where used
    constexpr int NEC = (kStageEdges && !kLean) ? NE : 1;
    uint32_t ecw[NEC];
    if constexpr (kStageEdges && !kLean) {
#pragma unroll
        for (int x = 0; x < NE; ++x) ecw[x] = EC[x * 64 + j];
    }
    auto col_word = [&](int x) -> uint32_t {
        if constexpr (kStageEdges && !kLean) return ecw[x];
        else return EC[x * 64 + j];
    };
    // one end-tile lookup (edge e, group k: x = e*G + k) for row 8b + g and
    // this lane's column
    // (low 16 bits of the result, see rterm)
    auto edge = [&](int x, int b) { return rterm(Rl, EB[x * 64 + 8 * b + g], col_word(x)); };

    if constexpr (kStageEdges) {
        // rows of block 7 take their end-tile groups here, the other blocks
        // inside the row loop (NE = 2G is even)
        const uint32_t e0 = edge(0, 7);
        uint32_t e16 = max3_u16(e0, edge(1, 7), e0);
#pragma unroll
        for (int x = 2; x < NE; x += 2) e16 = max3_u16(e16, edge(x, 7), edge(x + 1, 7));
        acc[7] = max_lo16(acc[7], e16);
    } else {
        // q < 4: the end tiles' words are read straight from memory
        for (int e = 0; e < nedge; ++e) {
            const int C = e == 0 ? A + 1 : B - 1;
            const NF_GLOBAL uint32_t* rs = RSr + tile_index(f.NT, A, C - A) * RW;
            const NF_GLOBAL uint32_t* cs = CSr + tile_index(f.NT, C, B - C) * SW;
            for (int k = 0; k < G; ++k) {
                const uint32_t cw = cs[k * 64 + j];
#pragma unroll
                for (int b = 0; b < 8; ++b) acc[b] = max(acc[b], rlookup<Q>(Rl, rs[k * 64 + 8 * b + g], cw));
            }
        }
    }

    // pairing bits of this lane's rows; pairing terms whose partner lies
    // outside the tile (last row, first column) come from the halo
    const int cbj = cb[j];
    uint32_t pmask = 0;
    {  // pairing mask of slice-start column 8*wave, by ballot over rows
        const unsigned long long m = __ballot(ca[lane] + (int)cb[wave * 8] == 3);
        if (lane == 0) GM[wave] = m;
    }
    const int hrj = hrow[j];
    int cai[8], hci[8];
    {
        const unsigned long long cw8 = *reinterpret_cast<const unsigned long long*>(&caT[8 * g]);
        const int4 ha = *reinterpret_cast<const int4*>(&hcT[8 * g]);
        const int4 hb = *reinterpret_cast<const int4*>(&hcT[8 * g + 4]);
#pragma unroll
        for (int b = 0; b < 8; ++b) cai[b] = (int)((cw8 >> (8 * b)) & 0xffu);
        hci[0] = ha.x; hci[1] = ha.y; hci[2] = ha.z; hci[3] = ha.w;
        hci[4] = hb.x; hci[5] = hb.y; hci[6] = hb.z; hci[7] = hb.w;
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int i = 8 * b + g;
        const int bp = (i < T && j < T && cai[b] + cbj == 3) ? 1 : 0;
        pmask |= (uint32_t)bp << b;
        const int halo = (i == T - 1) ? hrj : hci[b];  // the last row's partner first, then column 0's
        if (i < T && j < T && (i == T - 1 || j == 0)) acc[b] = max(acc[b], bp + halo);
    }
    // the pairing bias of row 8b + g at column j for its Q: the bit, or
    // -inf where the partner X(i, j-1) is in another wavefront (c = 0: the
    // readers add that term)
    int pbv[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) pbv[b] = c > 0 ? (int)((pmask >> b) & 1u) : kNeg;

    // outputs: dense cells, row words, column words, written after the row
    // loop (global address space: generic
    // accesses also count against the LDS counter that barriers wait on)
    const long long t_idx = tile_index(f.NT, A, d);
    NF_GLOBAL int16_t* Fw = (NF_GLOBAL int16_t*)f.F;
    NF_GLOBAL uint32_t* RSw = (NF_GLOBAL uint32_t*)(f.RS + t_idx * RW);
    NF_GLOBAL uint32_t* CSw = (NF_GLOBAL uint32_t*)(f.CS + t_idx * SW);

    // ---- rows bottom-up.  Rows >= T (only when T < 64) are inert: their
    // pushes are -inf in Lp and their pairing into row T-1 is skipped.
    // row 63: Q complete (no row below)
    Qs[1][g][j] = (QCell)acc[7];  // (slot 7 is row 63's)
    // U as pairs of 16-bit values for the packed closure, with -2^15 for
    // minus infinity.  Every real sum Q(i, j') + U(j', j) is at most
    // X(i, j) < 2^15 and Q >= 0, so no sum leaves the 16-bit range.  u0p is
    // U(8g, j) for the pairing term, minus infinity also where g = 0 (that
    // lane's term then stays <= 0, which no cell is below, and needs no
    // select per row).
    constexpr bool kPacked = Lds::kPacked;
    uint32_t up[4] = {0u, 0u, 0u, 0u};
    if constexpr (kPacked) {
        auto h16 = [](int v) { return (uint32_t)(v < 0 ? 0x8000 : v); };
#pragma unroll
        for (int t = 0; t < 4; ++t) up[t] = h16(ureg[2 * t]) | (h16(ureg[2 * t + 1]) << 16);
    }
    const int u0p = (g > 0 && ureg[0] >= 0) ? ureg[0] : (kPacked ? -32768 : kNeg);
    const int xlc = g > 0 ? 8 * g - 1 : 0;
    // end-tile row and column words of the share of row (bb, r): groups
    // x = r + 8m of block bb-1, loaded one row step ahead of their use
    // (erw/erc: this row's, ern/ecn: the next row's, fetched while this row
    // is closed)
    constexpr int kEPer = (NE + 7) / 8;
    uint32_t erw[kEPer], erc[kEPer], ern[kEPer], ecn[kEPer];
    auto fetch_edges = [&](int bb, int r, uint32_t (&rw)[kEPer], uint32_t (&cw)[kEPer]) {
#pragma unroll
        for (int m = 0; m < kEPer; ++m) {
            const int x = r + 8 * m;
            const bool live = bb >= 1 && x < NE;
            rw[m] = live ? EB[x * 64 + 8 * (bb - 1) + g] : 0u;
            if constexpr (kLean) cw[m] = live ? EC[x * 64 + j] : 0u;
        }
    };
    if constexpr (kStageEdges) fetch_edges(7, 7, erw, erc);
    __syncthreads();
    const unsigned long long gmask = GM[g];

    uint32_t evb = 0;  // see edge_terms
#pragma unroll
    for (int blk = 7; blk >= 0; --blk) {
#pragma unroll
        for (int rr = 7; rr >= 0; --rr) {
            const int i = blk * 8 + rr;
            // ---- LDS loads of the row, issued together after the barrier:
            // Q(i, 8g..8g+7), the pairing partner of column 8g, L(., i) for
            // the pushes, and the end-tile words of this row's share of
            // block blk-1
            const int qslot = i & 7;  // the slot of row i's lane group (a constant once unrolled)
            const int4 qa = *reinterpret_cast<const int4*>(&Qs[i & 1][qslot][8 * g]);  // 8 values (packed) or 4
            int4 qb = make_int4(0, 0, 0, 0);
            if constexpr (!kPacked) qb = *reinterpret_cast<const int4*>(&Qs[i & 1][qslot][8 * g + 4]);
            int xl = kNeg;
            // X(i+1, 8g-1); lanes of slice 0 read the finished X(i+1, 0)
            // instead, so that their pairing term stays finite and, with
            // u0p, below every cell
            if (i < T - 1) xl = Xs[(i + 1) * 64 + xlc];
            int lp[8];
            if constexpr (kBlockFR) {
                lp[blk] = Lp[i * LS + 8 * g + blk];
            } else {
                const int4 la = *reinterpret_cast<const int4*>(&Lp[i * LS + 8 * g]);
                const int4 lb = *reinterpret_cast<const int4*>(&Lp[i * LS + 8 * g + 4]);
                lp[0] = la.x; lp[1] = la.y; lp[2] = la.z; lp[3] = la.w;
                lp[4] = lb.x; lp[5] = lb.y; lp[6] = lb.z; lp[7] = lb.w;
            }
            // The row's chain waits on Q: nothing below is issued before
            // these reads, the end-tile gathers of this row's share (words
            // fetched a row ahead) go out next with the next row's words, and
            // their sums come after the closure (see edge_terms)
            __builtin_amdgcn_sched_barrier(0);
            uint32_t rg[kEPer];
            if constexpr (kStageEdges) {
                if (blk >= 1) {
#pragma unroll
                    for (int m = 0; m < kEPer; ++m) {
                        const int x = rr + 8 * m;
                        rg[m] = x < NE ? (uint32_t)Rl[r_index_v(erw[m], kLean ? erc[m] : col_word(x))] : 0u;
                    }
                }
                fetch_edges(rr > 0 ? blk : blk - 1, rr > 0 ? rr - 1 : 7, ern, ecn);
            }
            // pairing of (i-1, j) with partner X(i, j-1), for the next row's
            // Q: its bit, or -inf where there is no partner (formed here,
            // off the chain)
            const int pb = (i >= 1 && i < T) ? pbv[(i - 1) >> 3] : kNeg;
            __builtin_amdgcn_sched_barrier(0);
            // the end-tile terms of this row's share into the rows of block
            // blk-1 (Eq. 3; the term's value in the low 16 bits, see rterm)
            // The block's 8 row steps keep their terms in a running 16-bit
            // maximum (evb), which goes into acc[blk-1] once, at the block's
            // last row: nothing reads acc[blk-1] before that.
            auto edge_terms = [&] {
                if constexpr (kStageEdges) {
                    if (blk >= 1) {
                        uint32_t ev = evb;
#pragma unroll
                        for (int m = 0; m < kEPer; m += 2) {
                            const int m1 = m + 1 < kEPer ? m + 1 : m;
                            const int x0 = rr + 8 * m, x1 = rr + 8 * (m + 1);
                            if (x0 >= NE) continue;  // x0 = rr < 8 < NE when m = 0
                            const uint32_t t0 = erw[m] + (kLean ? erc[m] : col_word(x0)) + rg[m];
                            const uint32_t t1 = (m + 1 < kEPer && x1 < NE)
                                                    ? erw[m1] + (kLean ? erc[m1] : col_word(x1)) + rg[m1]
                                                    : t0;
                            ev = max3_u16((m == 0 && rr == 7) ? t0 : ev, t0, t1);  // rr = 7: the block's first row
                        }
                        if (rr == 0) acc[blk - 1] = max_lo16(acc[blk - 1], ev);
                        else evb = ev;
                    }
                }
            };
            // the pairing term of cell (i, 8g) (partner X(i+1, 8g-1)) is a
            // candidate for Q(i, 8g): it joins the closure at split point 8g
            // as one more term, formed before Q arrives
            // (X(i, j) >= 0, so 0 stands for no candidate)
            int pt = 0;
            if (i < T - 1) pt = (int)((gmask >> i) & 1u) + xl + u0p;
            // closure over j' in [8g, 8g+8), then across the 8 lane groups:
            // packed 16-bit adds and maxima over the pairs, then the two
            // halves and the pairing candidate (the row step is bound by
            // instruction issue on its SIMD as much as by its chain, so
            // fewer instructions win here over a shallower 32-bit tree)
            // (with 32-bit values, a tree of 3-input maxima)
            int xc;
            if constexpr (kPacked) {
                typedef short s16x2 __attribute__((ext_vector_type(2)));
                const s16x2 a0 = __builtin_bit_cast(s16x2, qa.x) + __builtin_bit_cast(s16x2, up[0]);
                const s16x2 a1 = __builtin_bit_cast(s16x2, qa.y) + __builtin_bit_cast(s16x2, up[1]);
                const s16x2 a2 = __builtin_bit_cast(s16x2, qa.z) + __builtin_bit_cast(s16x2, up[2]);
                const s16x2 a3 = __builtin_bit_cast(s16x2, qa.w) + __builtin_bit_cast(s16x2, up[3]);
                const s16x2 mm = __builtin_elementwise_max(__builtin_elementwise_max(a0, a1),
                                                           __builtin_elementwise_max(a2, a3));
                xc = max(max((int)mm.x, (int)mm.y), pt);
            } else {
                const int m0 = max(max(qa.x + ureg[0], qa.y + ureg[1]), qa.z + ureg[2]);
                const int m1 = max(max(qa.w + ureg[3], qb.x + ureg[4]), qb.y + ureg[5]);
                const int m2 = max(max(qb.z + ureg[6], qb.w + ureg[7]), pt);
                xc = max(max(m0, m1), m2);
            }
            const int xi = max_over_groups(xc);  // X(i, j)
            __builtin_amdgcn_sched_barrier(0);
            // pushes of row i: into row 8*blk+g (one split; -inf unless the row
            // is above i), or for other q into every row above
            if constexpr (kBlockFR) {
                acc[blk] = max(acc[blk], lp[blk] + xi);
            } else {
#pragma unroll
                for (int b = 0; b <= blk; ++b) acc[b] = max(acc[b], lp[b] + xi);
            }
            // the last row of a block: the next row (in block blk-1) takes
            // its Q from acc[blk-1] now, so its end-tile terms go in first.
            // The lean form sums them here at every row: it is bound by
            // instruction issue, not by the row's chain, which the default
            // form keeps them off by summing after the writes below
            if (kLean || rr == 0) edge_terms();
            if constexpr (kBlockFR) {
                if (rr == 0 && blk >= 1) {
                    // block blk finished: its q-groups into every row above it
#pragma unroll
                    for (int gg = 0; gg < GPB; ++gg) {
                        const int k = blk * GPB + gg;
                        const int top = k * Q;
                        // column word of group k at column j from rows top..top+q-1
                        int xs[Q];
#pragma unroll
                        for (int p2 = 0; p2 < Q; ++p2) xs[p2] = (top + p2 == i) ? xi : Xs[(top + p2) * 64 + j];
                        uint32_t cbits = 0;
                        if constexpr (Q == 8) {
                            cbits = drop_bits8(xs);
                        } else {
#pragma unroll
                            for (int p2 = 1; p2 <= M; ++p2) cbits |= (uint32_t)(xs[p2 - 1] > xs[p2]) << (p2 - 1);
                        }
                        const uint32_t cw = (cbits << 16) | (uint32_t)xs[0];
                        const uint4 wa = *reinterpret_cast<const uint4*>(&LW[k * 64 + 8 * g]);
                        const uint4 wb = *reinterpret_cast<const uint4*>(&LW[k * 64 + 8 * g + 4]);
                        const uint32_t ws[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
#pragma unroll
                        for (int b = 0; b < blk; ++b) acc[b] = max_lo16(acc[b], rterm(Rl, ws[b], cw));
                    }
                }
            }
            // Q of row i-1 for this lane's column (pairing partner X(i, j-1)
            // is the lane to the left; column 8w gets it from its readers)
            if (i >= 1) {
                // row_shr:1.  Lanes with c = 0 take no left partner, so what
                // they read does not matter (lanes 0, 16, 32, 48 read 0)
                const int left = __builtin_amdgcn_mov_dpp(xi, 0x111, 0xF, 0xF, true);
                const int bo = (i - 1) >> 3;
                // every lane writes its own row's candidate: slot (i-1) & 7
                // holds row i-1's
                Qs[(i - 1) & 1][g][j] = (QCell)max(acc[bo], left + pb);
            }
            // (the 8 lanes of a column hold the same X; all of them store
            // it, so that the store is not masked)
            Xs[i * 64 + j] = (Cell)xi;
            if (!kLean && rr > 0) edge_terms();
            if constexpr (kStageEdges) {
#pragma unroll
                for (int m = 0; m < kEPer; ++m) {
                    erw[m] = ern[m];
                    if constexpr (kLean) erc[m] = ecn[m];
                }
            }
            __syncthreads();
        }
    }

    // ---- emit: dense cells, row words (ballot), column words
    int xcol[8];  // X(8 * wave + r, lane)
    {
        const int wv = wave, ln = lane;  // row-major view: wave -> 8 rows, lane -> column
        int xv[8], xlft[8];  // every LDS read first: X(i, ln) and X(i, ln-1)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = wv * 8 + r;
            xv[r] = Xs[i * 64 + ln];
            xlft[r] = Xs[i * 64 + max(ln - 1, 0)];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) xcol[r] = xv[r];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = wv * 8 + r;
            const int v = xv[r];
            if (i < T) {
                if (ln < T) (Fw + (long long)(aT + i) * ld + bT)[(unsigned)ln] = (int16_t)v;
                const unsigned long long diff = __ballot(ln > 0 && ln < T && v > xlft[r]);
                if (ln < T && (ln % Q) == 0) {
                    uint32_t h = 0;
                    if constexpr (M > 0) h = (uint32_t)(diff >> (ln + 1)) & ((1u << M) - 1u);
                    RSw[(ln / Q) * 64 + i] = ((h << M) << 16) | (uint32_t)v;
                }
            } else if (ln < G) {
                // padding row (T < 64): readers load whole 64-row lines, so
                // give it words that keep their sums bounded and R in range
                RSw[ln * 64 + i] = 0;
            }
        }
    }
    if constexpr (Q == 8) {
        // q = 8: group k = wave holds rows 8k..8k+7, this lane's xv[], so
        // the column word of (group wave, column lane) needs no LDS reads
        CSw[wave * 64 + lane] = (drop_bits8(xcol) << 16) | (uint32_t)(uint16_t)xcol[0];
    } else
    for (int e = tid; e < G * 64; e += kTileThreads) {
        const int k = e >> 6, jj = e & 63;
        if (jj < T) {
            const int top = k * Q;
            uint32_t cbits = 0;
#pragma unroll
            for (int p = 1; p <= M; ++p)
                cbits |= (uint32_t)(Xs[(top + p - 1) * 64 + jj] > Xs[(top + p) * 64 + jj]) << (p - 1);
            CSw[k * 64 + jj] = (cbits << 16) | (uint32_t)(uint16_t)Xs[top * 64 + jj];
        } else {
            CSw[k * 64 + jj] = 0;  // padding column, as for padding rows
        }
    }
}

template <int Q, bool kWide>
constexpr int kStageWavesPerSimd = (Q == 8 && kWide) ? 6 : 1;

// Tile finishes alone (staged steps).  kWide: the lean finish at six
// wavefronts per SIMD, three workgroups per CU (q = 8), as in the fused step.
template <int Q, bool kWide>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(kStageWavesPerSimd<Q, kWide>)))
void k_tile(const TileWork* __restrict__ items, const uint8_t* __restrict__ Rg)
{
    constexpr int RSZ = 1 << (2 * (Q - 1));
    __shared__ __align__(16) uint8_t Rl[RSZ < 16 ? 16 : RSZ];
    __shared__ __align__(16) TileLds<Q, kWide> s;
    tile_body<Q, true, kWide>(items[blockIdx.x], Rl, Rg, s, [] {}, [] {});
}

// One wavefront step in one launch: workgroups [0, ntile) finish the tiles
// of diagonal s, the rest run the between chunks of diagonal s+1 (which only
// read diagonals <= s-1 and write the other half of the accumulators).
//
// Two shapes of the same code.  The default leaves the register count to the
// compiler (two workgroups per CU at q = 8: the finish's registers and LDS
// bound it), which keeps the finish, the fold's critical path, fastest.  The
// wide shape (q = 8 only) holds each workgroup to 80 VGPRs (the compiler
// spills a few registers to scratch) so that a CU takes three, six
// wavefronts per SIMD: the between chunks, which bound long folds, then run
// faster while each finish runs slower.  (Measured on MI355X: n = 16000
// 13.2 -> 12.2 ms, n = 6000 2.21 -> 2.34 ms.)
template <int Q, bool kWide>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(kStageWavesPerSimd<Q, kWide>)))
void k_stage(const TileWork* __restrict__ titems, int ntile,
                                                        const BetweenWork* __restrict__ bitems,
                                                        const uint8_t* __restrict__ Rg)
{
    constexpr int RSZ = 1 << (2 * (Q - 1));
    __shared__ __align__(16) uint8_t Rl[RSZ < 16 ? 16 : RSZ];
    __shared__ __align__(16) TileLds<Q, kWide> s;
    const int b = blockIdx.x;
    if (b < ntile) {
        tile_body<Q, true, kWide>(titems[b], Rl, Rg, s, [] {}, [] {});
    } else {
        load_R<RSZ>(Rl, Rg, kTileThreads);
        __syncthreads();
        const BetweenWork& it = bitems[b - ntile];
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        between_body<Q, 16, kTileThreads / 64 / 4>(it, Rl, it.f.RS, it.f.CS, wave, threadIdx.x & 63,
                                                   reinterpret_cast<uint16_t*>(s.Xs));
    }
}

__global__ void k_scores(const FoldDesc* __restrict__ folds, int nfolds, int32_t* __restrict__ scores)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nfolds) scores[e] = folds[e].F[folds[e].n];  // F(0, n) = D(1, n)
}

// The same, each score to scores[fold.pad] (the serving engine's slots in
// mapped host memory).
__global__ void k_scores_to_slots(const FoldDesc* __restrict__ folds, int nfolds, int32_t* __restrict__ scores)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nfolds) scores[folds[e].pad] = folds[e].F[folds[e].n];
}

// S[i*n + j] = D(i+1, j+1) = F(i, j+1) for i <= j, 0 below the diagonal.
__global__ void k_expand(const int16_t* __restrict__ F, int ld, int n, int16_t* __restrict__ S)
{
    const int i = blockIdx.y;
    const int j0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    const int16_t* src = F + (long long)i * ld + 1;
    int16_t* dst = S + (long long)i * n;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int j = j0 + u;
        if (j < n) dst[j] = j >= i ? src[j] : (int16_t)0;
    }
}

// Launch on stream s; with events, the dispatch itself records e0 when the
// kernel starts and e1 when it ends (kernel-only durations for profiling).
template <class K, class... Args>
hipError_t launch_k(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args)
{
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    return hipGetLastError();
}

template <int Q>
hipError_t launch_q(int which, const void* items, int nitems, const uint8_t* R, hipStream_t s, hipEvent_t e0,
                    hipEvent_t e1)
{
    if (nitems <= 0) return hipSuccess;
    dim3 grid(nitems);
    // (for the main-diagonal tiles R carries the staged codes of admission, or null)
    if (which == 0) return launch_k(k_diag<Q>, grid, dim3(kThreads), s, e0, e1, (const TileWork*)items, R);
    if (which == 1) return launch_k(k_tile<Q, false>, grid, dim3(kTileThreads), s, e0, e1, (const TileWork*)items, R);
    return launch_k(k_between<Q>, grid, dim3(kBetweenThreads), s, e0, e1, (const BetweenWork*)items, R);
}

hipError_t dispatch(int q, int which, const void* items, int nitems, const uint8_t* R, hipStream_t s, hipEvent_t e0,
                    hipEvent_t e1)
{
    switch (q) {
    case 1: return launch_q<1>(which, items, nitems, R, s, e0, e1);
    case 2: return launch_q<2>(which, items, nitems, R, s, e0, e1);
    case 3: return launch_q<3>(which, items, nitems, R, s, e0, e1);
    case 4: return launch_q<4>(which, items, nitems, R, s, e0, e1);
    case 5: return launch_q<5>(which, items, nitems, R, s, e0, e1);
    case 6: return launch_q<6>(which, items, nitems, R, s, e0, e1);
    case 7: return launch_q<7>(which, items, nitems, R, s, e0, e1);
    case 8: return launch_q<8>(which, items, nitems, R, s, e0, e1);
    case 9: return launch_q<9>(which, items, nitems, R, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_precompute_R(int q, uint8_t* R, hipStream_t s)
{
    if (q < 1 || q > 9) return hipErrorInvalidValue;
    const int entries = 1 << (2 * (q - 1));
    hipLaunchKernelGGL(k_precompute_R, dim3((entries + 255) / 256), dim3(256), 0, s, q, R);
    return hipGetLastError();
}

hipError_t launch_copy_codes(const uint8_t* src, int n, uint8_t* dst, int padded, hipStream_t s)
{
    if (padded <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_codes, dim3((padded + 255) / 256), dim3(256), 0, s, src, n, dst, padded);
    return hipGetLastError();
}

hipError_t launch_diag(int q, const TileWork* items, int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    return dispatch(q, 0, items, nitems, nullptr, s, e0, e1);
}

hipError_t launch_diag_admit(int q, const TileWork* items, int nitems, const uint8_t* staged, hipStream_t s)
{
    return dispatch(q, 0, items, nitems, staged, s, nullptr, nullptr);
}

hipError_t launch_tile(int q, const TileWork* items, int nitems, const uint8_t* R, hipStream_t s, hipEvent_t e0,
                       hipEvent_t e1, bool wide)
{
    if (wide && q == 8 && nitems > 0)
        return launch_k(k_tile<8, true>, dim3(nitems), dim3(kTileThreads), s, e0, e1, items, R);
    return dispatch(q, 1, items, nitems, R, s, e0, e1);
}

hipError_t launch_between(int q, const BetweenWork* items, int nitems, const uint8_t* R, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1)
{
    return dispatch(q, 2, items, nitems, R, s, e0, e1);
}

hipError_t launch_scores(const FoldDesc* folds, int nfolds, int32_t* scores, hipStream_t s)
{
    if (nfolds <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scores, dim3((nfolds + 255) / 256), dim3(256), 0, s, folds, nfolds, scores);
    return hipGetLastError();
}

hipError_t launch_scores_to_slots(const FoldDesc* folds, int nfolds, int32_t* scores, hipStream_t s)
{
    if (nfolds <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scores_to_slots, dim3((nfolds + 255) / 256), dim3(256), 0, s, folds, nfolds, scores);
    return hipGetLastError();
}

namespace {
template <int Q>
hipError_t stage_q(const TileWork* t, int nt, const BetweenWork* b, int nb, const uint8_t* R, hipStream_t s,
                   hipEvent_t e0, hipEvent_t e1)
{
    return launch_k(k_stage<Q, false>, dim3(nt + nb), dim3(kTileThreads), s, e0, e1, t, nt, b, R);
}
}  // namespace

hipError_t launch_stage(int q, bool wide, const TileWork* titems, int ntile, const BetweenWork* bitems, int nbtw,
                        const uint8_t* R, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (ntile + nbtw <= 0) return hipSuccess;
    if (wide && q == 8)
        return launch_k(k_stage<8, true>, dim3(ntile + nbtw), dim3(kTileThreads), s, e0, e1, titems, ntile, bitems, R);
    switch (q) {
    case 1: return stage_q<1>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    case 2: return stage_q<2>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    case 3: return stage_q<3>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    case 4: return stage_q<4>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    case 5: return stage_q<5>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    case 6: return stage_q<6>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    case 7: return stage_q<7>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    case 8: return stage_q<8>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    case 9: return stage_q<9>(titems, ntile, bitems, nbtw, R, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_expand(const int16_t* F, int ld, int n, int16_t* S, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((n + 1023) / 1024, n);
    hipLaunchKernelGGL(k_expand, grid, dim3(256), 0, s, F, ld, n, S);
    return hipGetLastError();
}

}  // namespace nf
