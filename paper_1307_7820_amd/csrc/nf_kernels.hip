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
template <int Q>
__device__ __forceinline__ void between_accumulate(int (&acc)[kRowsPerWave], const uint8_t* Rl,
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
            for (int r = 0; r < kRowsPerWave; ++r) {
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
__global__ __launch_bounds__(kThreads) void k_diag(const FoldDesc* __restrict__ folds,
                                                   const TileItem* __restrict__ items)
{
    constexpr int T = tile_size(Q);
    constexpr int XS = 65;  // padded stride: rows of a column are in distinct banks
    __shared__ int32_t X[64 * XS];
    __shared__ uint8_t ca[64], cb[64];

    const TileItem it = items[blockIdx.x];
    const FoldDesc f = folds[it.fold];
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
__global__ __launch_bounds__(kThreads) void k_between(const FoldDesc* __restrict__ folds,
                                                      const BetweenItem* __restrict__ items,
                                                      const uint8_t* __restrict__ Rg,
                                                      int32_t* __restrict__ part)
{
    constexpr int M = Q - 1;
    constexpr int RSZ = 1 << (2 * M);
    __shared__ __align__(16) uint8_t Rl[RSZ < 16 ? 16 : RSZ];

    const BetweenItem it = items[blockIdx.x];
    const FoldDesc f = folds[it.fold];
    load_R<RSZ>(Rl, Rg);
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = threadIdx.x & 63;
    const int r0 = wave * kRowsPerWave;
    int acc[kRowsPerWave];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) acc[r] = 0;
    between_accumulate<Q>(acc, Rl, f.RS, f.CS, f.NT, it.A, it.A + it.d, it.c0, it.c1, r0, j);

    int32_t* out = part + (size_t)it.slot * kTileCells;
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) out[(r0 + r) * 64 + j] = acc[r];
}

// Finish of an off-diagonal tile (A, B), B > A.  Lane j owns column j; wave w
// owns rows 16w..16w+15 and keeps their accumulators in registers.
//
// Inside the tile, with L(i, i') = F(AT+i, AT+i') (tile (A, A)) and
// U(j', j) = F(BT+j', BT+j) (tile (B, B)), cell (i, j) still needs
//     splits in tile A:  L(i, i') + X(i', j)   for i < i' < T,
//     splits in tile B:  X(i, j') + U(j', j)   for 0 <= j' < j,
//     pairing:           b(S_{a+1}, S_b) + F(a+1, b-1).
// X(i, j) depends only on cells with a smaller step t = j + (T-1-i); at
// iteration s every open cell takes the (at most one) row and (at most one)
// column term whose source lies on step s-1, then the cells of step s are
// final and are published in LDS.
template <int Q>
__global__ __launch_bounds__(kThreads) void k_tile(const FoldDesc* __restrict__ folds,
                                                   const TileItem* __restrict__ items,
                                                   const uint8_t* __restrict__ Rg,
                                                   const int32_t* __restrict__ part)
{
    constexpr int M = Q - 1;
    constexpr int G = groups_per_tile(Q);
    constexpr int T = tile_size(Q);
    constexpr int RSZ = 1 << (2 * M);
    constexpr int SW = state_words(Q);
    __shared__ __align__(16) uint8_t Rl[RSZ < 16 ? 16 : RSZ];
    __shared__ __align__(16) int32_t X[64 * 64];
    __shared__ __align__(16) int16_t Ls[64 * 64];
    __shared__ __align__(16) int16_t Us[64 * 64];
    __shared__ int32_t hrow[64], hcol[64];
    __shared__ uint8_t ca[64], cb[64];

    const TileItem it = items[blockIdx.x];
    const FoldDesc f = folds[it.fold];
    const int A = it.A, d = it.d, B = A + d;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = tid & 63;
    const int r0 = wave * kRowsPerWave;
    const long long ld = f.ld;
    const int aT = A * T, bT = B * T;
    const int16_t* F = f.F;

    load_R<RSZ>(Rl, Rg);
    for (int e = tid; e < 64 * 64; e += kThreads) {
        const int i = e >> 6, jj = e & 63;
        if (i < T && jj < T) {
            Ls[e] = F[(aT + i) * ld + aT + jj];
            Us[e] = F[(bT + i) * ld + bT + jj];
        }
    }
    if (tid < 64) {
        if (tid < T) {
            // halo: F((A+1)T, BT-1+j) and F(AT+1+i, BT-1); below the diagonal = 0
            const int hr_r = aT + T, hr_c = bT - 1 + tid;
            hrow[tid] = hr_c >= hr_r ? F[hr_r * ld + hr_c] : 0;
            const int hc_r = aT + 1 + tid, hc_c = bT - 1;
            hcol[tid] = hc_c >= hc_r ? F[hc_r * ld + hc_c] : 0;
        }
        ca[tid] = f.codes[aT + tid];      // S_{a+1}, a = AT + i
        cb[tid] = f.codes[bT + tid - 1];  // S_b,     b = BT + j   (BT >= 1)
    }

    int acc[kRowsPerWave];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) acc[r] = 0;
    for (int s = 0; s < it.nslot; ++s) {
        const int32_t* p = part + (size_t)(it.slot0 + s) * kTileCells + r0 * 64 + j;
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) acc[r] = max(acc[r], p[r * 64]);
    }
    __syncthreads();

    // groups of the intermediate tiles next to the ends: C = A+1 and C = B-1
    if (d >= 2) between_accumulate<Q>(acc, Rl, f.RS, f.CS, f.NT, A, B, A + 1, A + 2, r0, j);
    if (d >= 3) between_accumulate<Q>(acc, Rl, f.RS, f.CS, f.NT, A, B, B - 1, B, r0, j);

    // pairing bits of this lane's cells; pairing terms whose partner cell
    // lies outside the tile (last row, first column) come from the halo
    const int cbj = cb[j];
    uint32_t pmask = 0;
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int i = r0 + r;
        if (i < T && j < T) {
            const int bp = (ca[i] + cbj == 3) ? 1 : 0;
            pmask |= (uint32_t)bp << r;
            if (i == T - 1) acc[r] = max(acc[r], bp + hrow[j]);
            else if (j == 0) acc[r] = max(acc[r], bp + hcol[i]);
        }
    }

    for (int s = 0; s <= 2 * T - 2; ++s) {
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) {
            const int i = r0 + r;
            if (i < T && j < T) {
                if (s >= 1) {
                    const int jp = s - T + i;   // row source (i, jp) on step s-1
                    if (jp >= 0 && jp < j) acc[r] = max(acc[r], X[i * 64 + jp] + (int)Us[jp * 64 + j]);
                    const int ip = j + T - s;   // column source (ip, j) on step s-1
                    if (ip > i && ip <= T - 1) acc[r] = max(acc[r], (int)Ls[i * 64 + ip] + X[ip * 64 + j]);
                }
                if (j + (T - 1) - i == s) {
                    if (i < T - 1 && j > 0)
                        acc[r] = max(acc[r], (int)((pmask >> r) & 1) + X[(i + 1) * 64 + j - 1]);
                    X[i * 64 + j] = acc[r];
                }
            }
        }
        __syncthreads();
    }

    // dense cells, straight from the registers
    int16_t* Fw = f.F;
    const long long t_idx = tile_index(f.NT, A, d);
    uint32_t* RSw = f.RS + t_idx * SW;
    uint32_t* CSw = f.CS + t_idx * SW;
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int i = r0 + r;
        if (i < T) {
            const int v = acc[r];
            if (j < T) Fw[(aT + i) * ld + bT + j] = (int16_t)v;
            // row words: difference bits of the row by a wave ballot
            const int left = __shfl_up(v, 1);
            const unsigned long long diff = __ballot(j > 0 && j < T && v > left);
            if (j < T && (j % Q) == 0) {
                const uint32_t h = (uint32_t)(diff >> (j + 1)) & ((1u << M) - 1u);
                RSw[(j / Q) * 64 + i] = ((uint32_t)v << 16) | (h << M);
            }
        }
    }
    // column words from the published cells
    for (int e = tid; e < G * 64; e += kThreads) {
        const int k = e >> 6, jj = e & 63;
        if (jj < T) {
            const int top = k * Q;
            uint32_t c = 0;
#pragma unroll
            for (int p = 1; p <= M; ++p)
                c |= (uint32_t)(X[(top + p - 1) * 64 + jj] > X[(top + p) * 64 + jj]) << (p - 1);
            CSw[k * 64 + jj] = ((uint32_t)X[top * 64 + jj] << 16) | c;
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
hipError_t launch_q(int which, const FoldDesc* folds, const void* items, int nitems, const uint8_t* R,
                    int32_t* part, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    dim3 grid(nitems), block(kThreads);
    if (which == 0)
        hipLaunchKernelGGL(k_diag<Q>, grid, block, 0, s, folds, (const TileItem*)items);
    else if (which == 1)
        hipLaunchKernelGGL(k_tile<Q>, grid, block, 0, s, folds, (const TileItem*)items, R, part);
    else
        hipLaunchKernelGGL(k_between<Q>, grid, block, 0, s, folds, (const BetweenItem*)items, R, part);
    return hipGetLastError();
}

hipError_t dispatch(int q, int which, const FoldDesc* folds, const void* items, int nitems,
                    const uint8_t* R, int32_t* part, hipStream_t s)
{
    switch (q) {
    case 1: return launch_q<1>(which, folds, items, nitems, R, part, s);
    case 2: return launch_q<2>(which, folds, items, nitems, R, part, s);
    case 3: return launch_q<3>(which, folds, items, nitems, R, part, s);
    case 4: return launch_q<4>(which, folds, items, nitems, R, part, s);
    case 5: return launch_q<5>(which, folds, items, nitems, R, part, s);
    case 6: return launch_q<6>(which, folds, items, nitems, R, part, s);
    case 7: return launch_q<7>(which, folds, items, nitems, R, part, s);
    case 8: return launch_q<8>(which, folds, items, nitems, R, part, s);
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

hipError_t launch_diag(int q, const FoldDesc* folds, const TileItem* items, int nitems, hipStream_t s)
{
    return dispatch(q, 0, folds, items, nitems, nullptr, nullptr, s);
}

hipError_t launch_tile(int q, const FoldDesc* folds, const TileItem* items, int nitems, const uint8_t* R,
                       const int32_t* part, hipStream_t s)
{
    return dispatch(q, 1, folds, items, nitems, R, const_cast<int32_t*>(part), s);
}

hipError_t launch_between(int q, const FoldDesc* folds, const BetweenItem* items, int nitems,
                          const uint8_t* R, int32_t* part, hipStream_t s)
{
    return dispatch(q, 2, folds, items, nitems, R, part, s);
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
