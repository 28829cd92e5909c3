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

namespace nf {

namespace {

// Address-space views of generic pointers: row words are wave-uniform and
// read-only while a kernel runs, so they go through the scalar cache
// (constant address space); column words are per-lane global loads.
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

// Copy the q-dependent R table (RSZ bytes) into LDS.
template <int RSZ>
__device__ __forceinline__ void load_R(uint8_t* Rl, const uint8_t* __restrict__ Rg)
{
    if constexpr (RSZ >= 16) {
        for (int x = threadIdx.x * 16; x < RSZ; x += kThreads * 16)
            *reinterpret_cast<uint4*>(Rl + x) = *reinterpret_cast<const uint4*>(Rg + x);
    } else {
        if (threadIdx.x < RSZ) Rl[threadIdx.x] = Rg[threadIdx.x];
    }
}

// Between-group maxima for the 16 rows r0..r0+15 (wave-uniform) and column j
// (the lane) of tile (A, B), over the groups of tiles C in [c0, c1).
// For group k of tile C the row word comes from tile (A, C) and the column
// word from tile (C, B); Eq. 3 turns the q split points of the group into
//     F(a, Cq') + F(Cq', b) + R[h][c].
template <int Q, int RPW>
__device__ __forceinline__ void between_accumulate(int (&acc)[RPW], const uint8_t* Rl,
                                                   const uint32_t* __restrict__ RS,
                                                   const uint32_t* __restrict__ CS, int NT, int A,
                                                   int B, int c0, int c1, int r0, int j)
{
    constexpr int G = groups_per_tile(Q);
    constexpr int SW = state_words(Q);
    for (int C = c0; C < c1; ++C) {
        const NF_CONST uint32_t* rs = as_const(RS + tile_index(NT, A, C - A) * SW + r0);
        const NF_GLOBAL uint32_t* cs = as_global(CS + tile_index(NT, C, B - C) * SW + j);
#pragma unroll 2
        for (int k = 0; k < G; ++k) {
            const uint32_t cw = cs[k * 64];
            const uint32_t clo = cw & 0xffffu;
            const uint32_t chi = cw >> 16;
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const uint32_t rw = rs[k * 64 + r];
                const int v = Rl[(rw & 0xffffu) + clo];
                acc[r] = max(acc[r], (int)((rw >> 16) + chi) + v);
            }
        }
    }
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
template <int Q>
__global__ __launch_bounds__(kThreads) void k_diag(const TileWork* __restrict__ items)
{
    constexpr int T = tile_size(Q);
    constexpr int XS = 65;  // padded stride: rows of a column are in distinct banks
    __shared__ int32_t X[64 * XS];
    __shared__ uint8_t ca[64], cb[64];

    const TileWork it = items[blockIdx.x];
    const FoldDesc& f = it.f;
    const int aT = it.A * T;
    const int tid = threadIdx.x;

    for (int e = tid; e < 64 * XS; e += kThreads) X[e] = 0;
    if (tid < 64) {
        ca[tid] = f.codes[aT + tid];                        // S_{a+1} for a = aT + i
        cb[tid] = (aT + tid - 1 >= 0) ? f.codes[aT + tid - 1] : 0;  // S_b for b = aT + j
    }
    __syncthreads();

    for (int t = 2; t < T; ++t) {
        for (int i = tid; i < T - t; i += kThreads) {
            const int j = i + t;
            int v = (ca[i] + cb[j] == 3) + X[(i + 1) * XS + (j - 1)];
            for (int m = i + 1; m < j; ++m) v = max(v, X[i * XS + m] + X[m * XS + j]);
            X[i * XS + j] = v;
        }
        __syncthreads();
    }

    int16_t* F = f.F;
    const long long ld = f.ld;
    for (int e = tid; e < 64 * 64; e += kThreads) {
        const int i = e >> 6, j = e & 63;
        if (i < T && j < T) F[(aT + i) * ld + aT + j] = (int16_t)X[i * XS + j];
    }
}

template <int Q>
__global__ __launch_bounds__(kThreads) void k_between(const BetweenWork* __restrict__ items,
                                                      const uint8_t* __restrict__ Rg)
{
    constexpr int M = Q - 1;
    constexpr int RSZ = 1 << (2 * M);
    __shared__ __align__(16) uint8_t Rl[RSZ < 16 ? 16 : RSZ];

    const BetweenWork it = items[blockIdx.x];
    const FoldDesc& f = it.f;
    load_R<RSZ>(Rl, Rg);
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = threadIdx.x & 63;
    const int r0 = wave * kRowsPerWave;
    int acc[kRowsPerWave];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) acc[r] = 0;
    between_accumulate<Q, kRowsPerWave>(acc, Rl, f.RS, f.CS, f.NT, it.A, it.A + it.d, it.c0, it.c1, r0, j);

    int32_t* out = it.acc + r0 * 64 + j;
    if (it.atomic) {  // several items share the tile's accumulator
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) atomicMax(out + r * 64, acc[r]);
    } else {
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) out[r * 64] = acc[r];
    }
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
// Rows are finished bottom-up, one max-plus vector-matrix product per row:
// wave w reduces the split points j' in [8w, 8w+8) (its slice of U sits in
// registers) and the eight partial maxima are combined in LDS.
//
// Wave w owns the accumulators of the 8-row block [8w, 8w+8); lane j is
// column j.  A finished row is pushed (its L terms) into the rows above it in
// its own block one split at a time; when a whole block is finished and q
// divides 8, its q-groups are pushed into every row above the block with one
// R lookup per group (Eq. 3, row words of tile (A, A), column words of this
// tile).  For other q every row is pushed one split at a time.
constexpr int kTileThreads = 512;
constexpr int kNeg = -(1 << 20);  // stands for minus infinity; sums stay far from overflow

template <int Q>
__device__ __forceinline__ int rlookup(const uint8_t* Rl, uint32_t rw, uint32_t cw)
{
    return (int)((rw >> 16) + (cw >> 16)) + (int)Rl[(rw & 0xffffu) + (cw & 0xffffu)];
}

__device__ __forceinline__ int max8(const int4 a, const int4 b)
{
    return max(max(max(a.x, a.y), max(a.z, a.w)), max(max(b.x, b.y), max(b.z, b.w)));
}

template <int Q>
__global__ __launch_bounds__(kTileThreads) void k_tile(const TileWork* __restrict__ items,
                                                       const uint8_t* __restrict__ Rg)
{
    constexpr int M = Q - 1;
    constexpr int G = groups_per_tile(Q);
    constexpr int T = tile_size(Q);
    constexpr int RSZ = 1 << (2 * M);
    constexpr int SW = state_words(Q);
    constexpr int RPW = 8;                      // rows per wavefront
    constexpr bool kBlockFR = (8 % Q) == 0;     // q-groups tile the 8-row blocks
    constexpr int GPB = kBlockFR ? 8 / Q : 1;   // groups per block
    constexpr bool kStageEdges = G <= 16;       // end-tile words fit in LDS
    __shared__ __align__(16) uint8_t Rl[RSZ < 16 ? 16 : RSZ];
    __shared__ __align__(16) int32_t Xs[64 * 64];  // finished cells
    __shared__ __align__(16) int32_t Lt[64 * 64];  // Lt[i*64 + i''] = L(i'', i) for i'' < i < T, else -inf
    __shared__ __align__(16) uint32_t LW[kBlockFR ? G * 64 : 4];  // row words of tile (A, A), [k][row]
    __shared__ __align__(16) uint32_t EW[kStageEdges ? 4 * G * 64 : 4];  // [edge][row|col][k][64]
    __shared__ __align__(16) int32_t Qs[2][64];    // Q of the row being closed (double-buffered)
    __shared__ __align__(16) int32_t Ps[64 * 8];   // closure partials, Ps[j*8 + w]
    __shared__ int32_t hrow[64], hcol[64];
    __shared__ uint8_t ca[64], cb[64];

    const TileWork it = items[blockIdx.x];
    const FoldDesc& f = it.f;
    const int A = it.A, d = it.d, B = A + d;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = tid & 63;
    const int r0 = wave * RPW;
    const long long ld = f.ld;
    const int aT = A * T, bT = B * T;
    const int16_t* F = f.F;
    const int nedge = d >= 3 ? 2 : (d == 2 ? 1 : 0);

    // ---- prologue: every load issued before the first wait
    int lv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = tid + u * kTileThreads;
        const int ip = e >> 6, i = e & 63;  // row ip of L, read coalesced
        lv[u] = (ip < i && i < T) ? (int)F[(aT + ip) * ld + aT + i] : kNeg;
    }
    int ureg[8];  // U(8w + c, j); -inf where the split point is not left of column j
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int jp = r0 + c;
        ureg[c] = (jp <= j && j < T) ? (int)F[(bT + jp) * ld + bT + j] : kNeg;
    }
    int acc[RPW];
    int32_t* accp = it.acc + r0 * 64 + j;
    if (it.nslot > 0) {
#pragma unroll
        for (int r = 0; r < RPW; ++r) acc[r] = accp[r * 64];
    } else {
#pragma unroll
        for (int r = 0; r < RPW; ++r) acc[r] = 0;
    }
    if constexpr (RSZ >= 16) {
        for (int x = tid * 16; x < RSZ; x += kTileThreads * 16)
            *reinterpret_cast<uint4*>(Rl + x) = *reinterpret_cast<const uint4*>(Rg + x);
    } else {
        if (tid < RSZ) Rl[tid] = Rg[tid];
    }
    if constexpr (kStageEdges) {
        // edge e: C = A+1 (e = 0) and C = B-1 (e = 1); row words of (A, C), column words of (C, B)
        for (int x = tid; x < nedge * 2 * G * 16; x += kTileThreads) {
            const int e = x / (2 * G * 16), rem = x % (2 * G * 16);
            const int rc = rem / (G * 16), o = rem % (G * 16);
            const int C = e == 0 ? A + 1 : B - 1;
            const uint32_t* src = rc == 0 ? f.RS + tile_index(f.NT, A, C - A) * SW
                                          : f.CS + tile_index(f.NT, C, B - C) * SW;
            *reinterpret_cast<uint4*>(&EW[(e * 2 + rc) * G * 64 + o * 4]) =
                *reinterpret_cast<const uint4*>(src + o * 4);
        }
    }
    if (tid < 64) {
        if (tid < T) {
            const int hr_r = aT + T, hr_c = bT - 1 + tid;  // F((A+1)T, BT-1+j)
            hrow[tid] = hr_c >= hr_r ? F[hr_r * ld + hr_c] : 0;
            const int hc_r = aT + 1 + tid, hc_c = bT - 1;  // F(AT+1+i, BT-1)
            hcol[tid] = hc_c >= hc_r ? F[hc_r * ld + hc_c] : 0;
        }
        ca[tid] = f.codes[aT + tid];      // S_{a+1}, a = AT + i
        cb[tid] = f.codes[bT + tid - 1];  // S_b,     b = BT + j  (BT >= 1)
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = tid + u * kTileThreads;
        Lt[(e & 63) * 64 + (e >> 6)] = lv[u];
    }
    if (it.nslot > 0) {  // hand the accumulator back zeroed for its next use
#pragma unroll
        for (int r = 0; r < RPW; ++r) accp[r * 64] = 0;
    }
    __syncthreads();

    // ---- row words of tile (A, A) for the block pushes
    if constexpr (kBlockFR) {
        for (int x = tid; x < G * 64; x += kTileThreads) {
            const int k = x >> 6, i = x & 63;
            const int top = k * Q;
            uint32_t h = 0;
            int base = 0;
            if (top > i && top < T) {
                base = Lt[top * 64 + i];
#pragma unroll
                for (int p = 1; p <= M; ++p)
                    h |= (uint32_t)(Lt[(top + p) * 64 + i] > Lt[(top + p - 1) * 64 + i]) << (p - 1);
            }
            LW[x] = ((uint32_t)base << 16) | (h << M);
        }
    }

    // ---- groups of the two end tiles C = A+1 and C = B-1
    if constexpr (kStageEdges) {
        for (int e = 0; e < nedge; ++e) {
            const uint32_t* er = &EW[(e * 2 + 0) * G * 64];
            const uint32_t* ec = &EW[(e * 2 + 1) * G * 64];
#pragma unroll 2
            for (int k = 0; k < G; ++k) {
                const uint32_t cw = ec[k * 64 + j];
                const uint4 ra = *reinterpret_cast<const uint4*>(&er[k * 64 + r0]);
                const uint4 rb = *reinterpret_cast<const uint4*>(&er[k * 64 + r0 + 4]);
                acc[0] = max(acc[0], rlookup<Q>(Rl, ra.x, cw));
                acc[1] = max(acc[1], rlookup<Q>(Rl, ra.y, cw));
                acc[2] = max(acc[2], rlookup<Q>(Rl, ra.z, cw));
                acc[3] = max(acc[3], rlookup<Q>(Rl, ra.w, cw));
                acc[4] = max(acc[4], rlookup<Q>(Rl, rb.x, cw));
                acc[5] = max(acc[5], rlookup<Q>(Rl, rb.y, cw));
                acc[6] = max(acc[6], rlookup<Q>(Rl, rb.z, cw));
                acc[7] = max(acc[7], rlookup<Q>(Rl, rb.w, cw));
            }
        }
    } else {
        if (d >= 2) between_accumulate<Q, RPW>(acc, Rl, f.RS, f.CS, f.NT, A, B, A + 1, A + 2, r0, j);
        if (d >= 3) between_accumulate<Q, RPW>(acc, Rl, f.RS, f.CS, f.NT, A, B, B - 1, B, r0, j);
    }

    // pairing bits of this lane's rows; pairing terms whose partner lies
    // outside the tile (last row, first column) come from the halo
    const int cbj = cb[j];
    uint32_t pmask = 0;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int i = r0 + r;
        if (i < T && j < T) {
            const int bp = (ca[i] + cbj == 3) ? 1 : 0;
            pmask |= (uint32_t)bp << r;
            if (i == T - 1) acc[r] = max(acc[r], bp + hrow[j]);
            else if (j == 0) acc[r] = max(acc[r], bp + hcol[i]);
        }
    }

    // ---- rows bottom-up.  Rows >= T (only when T < 64) are inert: their
    // pushes are -inf in Lt and their pairing into row T-1 is skipped.
    if (wave == 7) Qs[1][j] = acc[7];  // row 63 has no row below it
    __syncthreads();
    const int jl = j > 0 ? j - 1 : 0;

#pragma unroll 1
    for (int blk = 7; blk >= 0; --blk) {
#pragma unroll
        for (int rr = 7; rr >= 0; --rr) {
            const int i = blk * 8 + rr;
            {   // closure partial over j' in [8w, 8w+8)
                const int4 qa = *reinterpret_cast<const int4*>(&Qs[i & 1][r0]);
                const int4 qb = *reinterpret_cast<const int4*>(&Qs[i & 1][r0 + 4]);
                int p = max(max(qa.x + ureg[0], qa.y + ureg[1]), max(qa.z + ureg[2], qa.w + ureg[3]));
                p = max(p, max(max(qb.x + ureg[4], qb.y + ureg[5]), max(qb.z + ureg[6], qb.w + ureg[7])));
                Ps[j * 8 + wave] = p;
            }
            __syncthreads();
            if constexpr (kBlockFR) {
                if (wave == blk) {
                    // issue every read of this phase before the first wait
                    const int4 pa = *reinterpret_cast<const int4*>(&Ps[j * 8]);
                    const int4 pb = *reinterpret_cast<const int4*>(&Ps[j * 8 + 4]);
                    int4 pla, plb, la, lb;
                    if (rr > 0) {
                        pla = *reinterpret_cast<const int4*>(&Ps[jl * 8]);
                        plb = *reinterpret_cast<const int4*>(&Ps[jl * 8 + 4]);
                        la = *reinterpret_cast<const int4*>(&Lt[i * 64 + r0]);
                        lb = *reinterpret_cast<const int4*>(&Lt[i * 64 + r0 + 4]);
                    }
                    const int xi = max8(pa, pb);
                    Xs[i * 64 + j] = xi;
                    if (rr > 0) {
                        const int left = max8(pla, plb);
                        const int lt[8] = {la.x, la.y, la.z, la.w, lb.x, lb.y, lb.z, lb.w};
#pragma unroll
                        for (int r = 0; r < 8; ++r)
                            if (r < rr) acc[r] = max(acc[r], lt[r] + xi);
                        int qv = acc[rr - 1];
                        if (i < T && j > 0) qv = max(qv, (int)((pmask >> (rr - 1)) & 1u) + left);
                        Qs[(i - 1) & 1][j] = qv;
                    }
                }
                if (rr == 0 && blk > 0) {
                    __syncthreads();  // the block's rows are in Xs
                    if (wave < blk) {
#pragma unroll
                        for (int g = 0; g < GPB; ++g) {
                            const int k = blk * GPB + g;
                            const int top = k * Q;
                            uint32_t c = 0;
#pragma unroll
                            for (int p = 1; p <= M; ++p)
                                c |= (uint32_t)(Xs[(top + p - 1) * 64 + j] > Xs[(top + p) * 64 + j]) << (p - 1);
                            const uint32_t cw = ((uint32_t)Xs[top * 64 + j] << 16) | c;
                            const uint4 wa = *reinterpret_cast<const uint4*>(&LW[k * 64 + r0]);
                            const uint4 wb = *reinterpret_cast<const uint4*>(&LW[k * 64 + r0 + 4]);
                            acc[0] = max(acc[0], rlookup<Q>(Rl, wa.x, cw));
                            acc[1] = max(acc[1], rlookup<Q>(Rl, wa.y, cw));
                            acc[2] = max(acc[2], rlookup<Q>(Rl, wa.z, cw));
                            acc[3] = max(acc[3], rlookup<Q>(Rl, wa.w, cw));
                            acc[4] = max(acc[4], rlookup<Q>(Rl, wb.x, cw));
                            acc[5] = max(acc[5], rlookup<Q>(Rl, wb.y, cw));
                            acc[6] = max(acc[6], rlookup<Q>(Rl, wb.z, cw));
                            acc[7] = max(acc[7], rlookup<Q>(Rl, wb.w, cw));
                        }
                        if (wave == blk - 1) {
                            const int left = Xs[i * 64 + jl];
                            int qv = acc[7];
                            if (i < T && j > 0) qv = max(qv, (int)((pmask >> 7) & 1u) + left);
                            Qs[(i - 1) & 1][j] = qv;
                        }
                    }
                }
            } else {
                const int xi = max8(*reinterpret_cast<const int4*>(&Ps[j * 8]),
                                    *reinterpret_cast<const int4*>(&Ps[j * 8 + 4]));
                const int left = max8(*reinterpret_cast<const int4*>(&Ps[jl * 8]),
                                      *reinterpret_cast<const int4*>(&Ps[jl * 8 + 4]));
                if (wave == blk) Xs[i * 64 + j] = xi;
                const int4 la = *reinterpret_cast<const int4*>(&Lt[i * 64 + r0]);
                const int4 lb = *reinterpret_cast<const int4*>(&Lt[i * 64 + r0 + 4]);
                acc[0] = max(acc[0], la.x + xi);
                acc[1] = max(acc[1], la.y + xi);
                acc[2] = max(acc[2], la.z + xi);
                acc[3] = max(acc[3], la.w + xi);
                acc[4] = max(acc[4], lb.x + xi);
                acc[5] = max(acc[5], lb.y + xi);
                acc[6] = max(acc[6], lb.z + xi);
                acc[7] = max(acc[7], lb.w + xi);
                if (i >= 1) {
                    const int owner = (rr > 0) ? blk : blk - 1;
                    const int slot = (rr > 0) ? rr - 1 : 7;
                    if (wave == owner) {
                        int qv = acc[slot];
                        if (i < T && j > 0) qv = max(qv, (int)((pmask >> slot) & 1u) + left);
                        Qs[(i - 1) & 1][j] = qv;
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- emit: dense cells, row words (ballot), column words
    int16_t* Fw = f.F;
    const long long t_idx = tile_index(f.NT, A, d);
    uint32_t* RSw = f.RS + t_idx * SW;
    uint32_t* CSw = f.CS + t_idx * SW;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int i = r0 + r;
        if (i < T) {
            const int v = Xs[i * 64 + j];
            if (j < T) Fw[(aT + i) * ld + bT + j] = (int16_t)v;
            const int left = __shfl_up(v, 1);
            const unsigned long long diff = __ballot(j > 0 && j < T && v > left);
            if (j < T && (j % Q) == 0) {
                uint32_t h = 0;
                if constexpr (M > 0) h = (uint32_t)(diff >> (j + 1)) & ((1u << M) - 1u);
                RSw[(j / Q) * 64 + i] = ((uint32_t)v << 16) | (h << M);
            }
        }
    }
    for (int e = tid; e < G * 64; e += kTileThreads) {
        const int k = e >> 6, jj = e & 63;
        if (jj < T) {
            const int top = k * Q;
            uint32_t c = 0;
#pragma unroll
            for (int p = 1; p <= M; ++p)
                c |= (uint32_t)(Xs[(top + p - 1) * 64 + jj] > Xs[(top + p) * 64 + jj]) << (p - 1);
            CSw[k * 64 + jj] = ((uint32_t)Xs[top * 64 + jj] << 16) | c;
        }
    }
}

__global__ void k_scores(const FoldDesc* __restrict__ folds, int nfolds, int32_t* __restrict__ scores)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nfolds) scores[e] = folds[e].F[folds[e].n];  // F(0, n) = D(1, n)
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

template <int Q>
hipError_t launch_q(int which, const void* items, int nitems, const uint8_t* R, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    dim3 grid(nitems), block(kThreads);
    if (which == 0)
        hipLaunchKernelGGL(k_diag<Q>, grid, block, 0, s, (const TileWork*)items);
    else if (which == 1)
        hipLaunchKernelGGL(k_tile<Q>, grid, dim3(kTileThreads), 0, s, (const TileWork*)items, R);
    else
        hipLaunchKernelGGL(k_between<Q>, grid, block, 0, s, (const BetweenWork*)items, R);
    return hipGetLastError();
}

hipError_t dispatch(int q, int which, const void* items, int nitems, const uint8_t* R, hipStream_t s)
{
    switch (q) {
    case 1: return launch_q<1>(which, items, nitems, R, s);
    case 2: return launch_q<2>(which, items, nitems, R, s);
    case 3: return launch_q<3>(which, items, nitems, R, s);
    case 4: return launch_q<4>(which, items, nitems, R, s);
    case 5: return launch_q<5>(which, items, nitems, R, s);
    case 6: return launch_q<6>(which, items, nitems, R, s);
    case 7: return launch_q<7>(which, items, nitems, R, s);
    case 8: return launch_q<8>(which, items, nitems, R, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_precompute_R(int q, uint8_t* R, hipStream_t s)
{
    if (q < 1 || q > 8) return hipErrorInvalidValue;
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

hipError_t launch_diag(int q, const TileWork* items, int nitems, hipStream_t s)
{
    return dispatch(q, 0, items, nitems, nullptr, s);
}

hipError_t launch_tile(int q, const TileWork* items, int nitems, const uint8_t* R, hipStream_t s)
{
    return dispatch(q, 1, items, nitems, R, s);
}

hipError_t launch_between(int q, const BetweenWork* items, int nitems, const uint8_t* R, hipStream_t s)
{
    return dispatch(q, 2, items, nitems, R, s);
}

hipError_t launch_scores(const FoldDesc* folds, int nfolds, int32_t* scores, hipStream_t s)
{
    if (nfolds <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scores, dim3((nfolds + 255) / 256), dim3(256), 0, s, folds, nfolds, scores);
    return hipGetLastError();
}

hipError_t launch_expand(const int16_t* F, int ld, int n, int16_t* S, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((n + 1023) / 1024, n);
    hipLaunchKernelGGL(k_expand, grid, dim3(256), 0, s, F, ld, n, S);
    return hipGetLastError();
}

}  // namespace nf
