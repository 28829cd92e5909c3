// Plain between-group maxima: the ablation of the Four-Russians lookup.
#include <hip/hip_ext.h>

#include "nf_internal.h"

namespace nf {
namespace {

#define NF_GLOBAL __attribute__((address_space(1)))

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kPlainThreads = 256;
constexpr int kLR = 64 + 8;  // row stride (16-bit entries) of the staged tiles: 144-byte rows

// Between-group maxima of tile (A, B) over tiles C in [c0, c1) straight from
// Eq. 1, with no R: acc(i, j) = max over the T split points m of tile C of
//     F(AT+i, CT+m) + F(CT+m, BT+j),
// the same set of split points one Four-Russians lookup per group covers.
// The two 64x64 tiles of dense table entries go through LDS (the row tile
// transposed); thread (ty, tx) holds rows 4ty..4ty+3 and columns 4tx..4tx+3,
// two columns per 32-bit register, with packed unsigned 16-bit adds and
// maxima: every entry is at most n/2 < 2^15, so sums stay below 2^16.
template <int Q>
__global__ __launch_bounds__(kPlainThreads) void k_between_plain(const BetweenWork* __restrict__ items)
{
    static_assert(tile_size(Q) == 64, "64-post tiles only");
    __shared__ __align__(16) uint16_t Lr[64 * kLR];  // Lr[m*kLR + i] = F(AT+i, CT+m)
    __shared__ __align__(16) uint16_t Lc[64 * kLR];  // Lc[m*kLR + j] = F(CT+m, BT+j)
    const BetweenWork& it = items[blockIdx.x];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int lr = tid >> 2, lc = (tid & 3) * 16;  // staging: row lr, entries lc..lc+15
    const long long ld = it.f.ld;
    const long long aT = (long long)it.A * 64, bT = (long long)(it.A + it.d) * 64;
    const NF_GLOBAL int16_t* F = (const NF_GLOBAL int16_t*)it.f.F;

    u16x2 acc[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r][0] = acc[r][1] = (u16x2)(0);

    for (int C = it.c0; C < it.c1; ++C) {
        const long long cT = (long long)C * 64;
        const NF_GLOBAL u32x4* pr = (const NF_GLOBAL u32x4*)(F + (aT + lr) * ld + cT + lc);
        const NF_GLOBAL u32x4* pc = (const NF_GLOBAL u32x4*)(F + (cT + lr) * ld + bT + lc);
        const u32x4 r0 = pr[0], r1 = pr[1], c0 = pc[0], c1 = pc[1];
        __syncthreads();  // the previous pair of tiles is consumed
        const uint32_t rw[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            Lr[(lc + 2 * k) * kLR + lr] = (uint16_t)(rw[k] & 0xffffu);
            Lr[(lc + 2 * k + 1) * kLR + lr] = (uint16_t)(rw[k] >> 16);
        }
        *reinterpret_cast<u32x4*>(&Lc[lr * kLR + lc]) = c0;
        *reinterpret_cast<u32x4*>(&Lc[lr * kLR + lc + 8]) = c1;
        __syncthreads();
#pragma unroll 8
        for (int m = 0; m < 64; ++m) {
            const uint2 rv = *reinterpret_cast<const uint2*>(&Lr[m * kLR + 4 * ty]);
            const uint2 cv = *reinterpret_cast<const uint2*>(&Lc[m * kLR + 4 * tx]);
            const u16x2 cp0 = __builtin_bit_cast(u16x2, cv.x), cp1 = __builtin_bit_cast(u16x2, cv.y);
            const unsigned short rr[4] = {(unsigned short)(rv.x & 0xffffu), (unsigned short)(rv.x >> 16),
                                          (unsigned short)(rv.y & 0xffffu), (unsigned short)(rv.y >> 16)};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                acc[r][0] = __builtin_elementwise_max(acc[r][0], cp0 + (u16x2)(rr[r]));
                acc[r][1] = __builtin_elementwise_max(acc[r][1], cp1 + (u16x2)(rr[r]));
            }
        }
    }

    int32_t* out = it.acc + (4 * ty) * 64 + 4 * tx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int v[4] = {acc[r][0].x, acc[r][0].y, acc[r][1].x, acc[r][1].y};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (it.atomic)
                atomicMax(out + r * 64 + c, v[c]);
            else
                out[r * 64 + c] = v[c];
        }
    }
}

template <int Q>
hipError_t launch_q(const BetweenWork* items, int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (e0 || e1)
        hipExtLaunchKernelGGL(k_between_plain<Q>, dim3(nitems), dim3(kPlainThreads), 0, s, e0, e1, 0, items);
    else
        hipLaunchKernelGGL(k_between_plain<Q>, dim3(nitems), dim3(kPlainThreads), 0, s, items);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_between_plain(int q, const BetweenWork* items, int nitems, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1)
{
    if (nitems <= 0) return hipSuccess;
    switch (q) {
        case 1: return launch_q<1>(items, nitems, s, e0, e1);
        case 2: return launch_q<2>(items, nitems, s, e0, e1);
        case 4: return launch_q<4>(items, nitems, s, e0, e1);
        case 8: return launch_q<8>(items, nitems, s, e0, e1);
        default: return hipErrorInvalidValue;  // tiles of fewer than 64 posts
    }
}

}  // namespace nf
