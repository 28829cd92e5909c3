// Measurement and test kernels outside the fill.
//
// nf_lds_gather_rate: the LDS byte-gather ceiling of the device, the unit
// that bounds a Four-Russians lookup besides VALU issue (one random 1-byte
// read of R from LDS per lookup, Eq. 3).
//
// Every lane holds 16 table offsets in registers and reads them again and
// again with ds_read_u8; two bytes are consumed per 3-input add, so VALU
// issue stays well below the LDS's rate and the gathers set the time.
// Offsets are either uniformly random over the table or, as the lookups of
// the between-group kernel make them, one wave-uniform row of `row_bytes`
// bytes with a random byte inside it per lane.
#include <hip/hip_runtime.h>

#include "nf.h"
#include "nf_runtime.h"

namespace nf {
namespace {

constexpr int kGatherThreads = 512;
constexpr int kGatherPerRound = 16;

__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(kGatherThreads) void k_lds_gather(int table_bytes, int row_bytes, int rounds,
                                                                uint32_t* __restrict__ sink)
{
    extern __shared__ __align__(16) uint8_t tab[];  // table_bytes of dynamic LDS
    for (int e = threadIdx.x; e < table_bytes; e += blockDim.x) tab[e] = (uint8_t)mix((uint32_t)e);
    __syncthreads();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t off[kGatherPerRound];
#pragma unroll
    for (int k = 0; k < kGatherPerRound; ++k) {
        const uint32_t r = mix((blockIdx.x * kGatherThreads + threadIdx.x) * kGatherPerRound + k + 1u);
        if (row_bytes > 0) {
            const uint32_t rows = (uint32_t)(table_bytes / row_bytes);
            const uint32_t row = mix(blockIdx.x * 64u + wave * kGatherPerRound + k) % rows;  // wave-uniform
            off[k] = row * row_bytes + r % (uint32_t)row_bytes;
        } else {
            off[k] = r % (uint32_t)table_bytes;
        }
    }
    uint32_t acc = 0;
    for (int it = 0; it < rounds; ++it) {
        __asm__ volatile("" ::: "memory");  // the table may change: read it again every round
#pragma unroll
        for (int k = 0; k < kGatherPerRound; k += 2) acc = acc + tab[off[k]] + tab[off[k + 1]];
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the reads; practically never true
}

// One wavefront that sleeps `iters` times for about 8K clocks each: a
// bounded delay put between the launches of a perturbed schedule.
__global__ __launch_bounds__(64) void k_delay(int iters)
{
    for (int i = 0; i < iters; ++i) __builtin_amdgcn_s_sleep(127);
}

}  // namespace

hipError_t launch_delay(int iters, hipStream_t s)
{
    if (iters <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_delay, dim3(1), dim3(64), 0, s, iters < 16 ? iters : 16);
    return hipGetLastError();
}

}  // namespace nf

using namespace nf;

extern "C" int nf_lds_gather_rate(int table_bytes, int row_bytes, double* lane_gathers_per_s)
{
    std::lock_guard<std::recursive_mutex> lk(api_mutex());
    clear_error();
    if (!lane_gathers_per_s || table_bytes < 64 || table_bytes > 65536 || (table_bytes & (table_bytes - 1)))
        return fail(NF_E_INVAL, "table_bytes must be a power of two in 64..65536");
    if (row_bytes < 0 || row_bytes > table_bytes || (row_bytes && table_bytes % row_bytes))
        return fail(NF_E_INVAL, "row_bytes must be 0 or divide table_bytes");
    int rc = ensure_device();
    if (rc) return rc;
    HIPCHK(hipFuncSetAttribute((const void*)k_lds_gather, hipFuncAttributeMaxDynamicSharedMemorySize, 65536));
    DevBuf sink;
    if ((rc = sink.alloc(256))) return rc;
    hipStream_t s = ctx().stream;
    const int blocks = 8 * ctx().num_cu;  // several workgroups per CU
    const int rounds = 4096;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_lds_gather, dim3(blocks), dim3(kGatherThreads), table_bytes, s, table_bytes, row_bytes, 16,
                       (uint32_t*)sink.p);  // warm-up
    (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL(k_lds_gather, dim3(blocks), dim3(kGatherThreads), table_bytes, s, table_bytes, row_bytes,
                       rounds, (uint32_t*)sink.p);
    (void)hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(NF_E_DEVICE, "gather timing failed: %s", hipGetErrorString(e));
    const double gathers = (double)blocks * kGatherThreads * rounds * kGatherPerRound;
    *lane_gathers_per_s = gathers / (ms * 1e-3);
    return NF_OK;
}
