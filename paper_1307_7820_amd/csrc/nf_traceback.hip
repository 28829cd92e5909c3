// Traceback of Section 2 on the GPU: one optimal structure read back from the
// finished table through D*, the argmax of Eq. 1.
#include "nf_internal.h"

namespace nf {
namespace {

// The argmax is taken as a strict '>' scan takes it: the first term of Eq. 1
// that attains the maximum, in the order pairing term, then splits by
// increasing k.  In fence posts (F(a, b) = D(a+1, b)), on (a, b) with
// b - a >= 2:
//   - if F(a, b) = b(S_{a+1}, S_b) + F(a+1, b-1): the pairing term; bases a+1
//     and b pair when complementary (else both stay unpaired); go on with
//     (a+1, b-1);
//   - else split at the smallest m in (a, b) with F(a, m) + F(m, b) = F(a, b)
//     and go on with (a, m) and (m, b), which are independent.
// D* is not stored: every decision is recomputed from F on the way back.
//
// One workgroup walks the tree of splits level by level: the intervals of a
// level are shared among kTbWaves wavefronts, each follows its interval's run
// of pairing terms to the next split and appends the two halves to the next
// level; a barrier closes the level.  Inside a wavefront, lane k tries the
// k-th step of the run, on (a+k, b-k), so one round trip to memory covers up
// to 64 steps of a helix; a split tests 256 split points (four per lane) per
// round trip and takes the first hit by ballot.  The first 64 split points are
// loaded together with the run, for when the run is empty.  A level holds
// disjoint intervals of at least two bases, so at most n/2 of them: the first
// kFront in LDS, the rest in `spill` (spill_cap entries per level buffer).
// Each child is shorter than its parent, so there are at most n levels.
constexpr int kTbWaves = 16;
constexpr int kFront = 2048;

__device__ __forceinline__ void traceback_body(const int16_t* __restrict__ F, long long ld,
                                               const uint8_t* __restrict__ codes, int n, int2* __restrict__ spill,
                                               int spill_cap, char* __restrict__ db, int* __restrict__ status)
{
    __shared__ int2 front[2][kFront];
    __shared__ int count[2];
    __shared__ int fail;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int x = tid; x < n; x += kTbWaves * 64) db[x] = '.';
    if (tid == 0) {
        count[0] = n >= 2 ? 1 : 0;
        count[1] = 0;
        fail = 0;
        front[0][0] = make_int2(0, n);
    }
    __syncthreads();

    auto get = [&](int buf, int idx) {
        return idx < kFront ? front[buf][idx] : spill[(long long)buf * spill_cap + idx - kFront];
    };
    auto put = [&](int buf, int2 iv) {  // lane 0 only
        const int pos = atomicAdd(&count[buf], 1);
        if (pos < kFront)
            front[buf][pos] = iv;
        else if (pos - kFront < spill_cap)
            spill[(long long)buf * spill_cap + pos - kFront] = iv;
        else
            fail = 3;
    };

    int cur = 0, levels = 0;
    for (; levels <= n; ++levels) {
        const int cnt = count[cur];
        if (cnt == 0 || fail) break;
        for (int idx = wave; idx < cnt; idx += kTbWaves) {
            int2 t = make_int2(0, 0);
            if (lane == 0) t = get(cur, idx);
            int a = __builtin_amdgcn_readfirstlane(t.x);
            int b = __builtin_amdgcn_readfirstlane(t.y);
            while (b - a >= 2) {
                // a run of pairing terms, and the first window of split points
                const int ak = a + lane, bk = b - lane;
                const bool live = bk - ak >= 2;
                int v = 0, inner = 0, bp = 0;
                if (live) {
                    v = F[ak * ld + bk];
                    inner = F[(ak + 1) * ld + bk - 1];
                    bp = (codes[ak] + codes[bk - 1] == 3) ? 1 : 0;
                }
                const int m1 = a + 1 + lane;
                int w1 = -1;
                if (m1 < b) w1 = (int)F[a * ld + m1] + (int)F[m1 * ld + b];
                const bool take = live && v == bp + inner;
                const unsigned long long stop = __ballot(!take);
                const int s = stop ? __builtin_ctzll(stop) : 64;  // steps taken (wave-uniform)
                if (take && lane < s && bp) {
                    db[ak] = '(';
                    db[bk - 1] = ')';
                }
                const int vab = __builtin_amdgcn_readlane(v, s < 64 ? s : 0);  // F(a+s, b-s)
                a += s;
                b -= s;
                if (s == 64) continue;
                if (b - a < 2) break;
                // split: the smallest m in (a, b) with F(a, m) + F(m, b) = F(a, b)
                int m = -1;
                int m0 = a + 1;
                if (s == 0) {  // the window loaded with the run is this interval's
                    const unsigned long long hm = __ballot(w1 == vab);
                    if (hm) m = m0 + __builtin_ctzll(hm);
                    m0 += 64;
                }
                for (; m < 0 && m0 < b; m0 += 256) {
                    int w[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int mm = m0 + 64 * u + lane;
                        w[u] = mm < b ? (int)F[a * ld + mm] + (int)F[mm * ld + b] : -1;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const unsigned long long hm = __ballot(w[u] == vab);
                        if (hm) {
                            m = m0 + 64 * u + __builtin_ctzll(hm);
                            break;
                        }
                    }
                }
                if (lane == 0) {
                    if (m < 0) {
                        fail = 2;
                    } else {
                        if (m - a >= 2) put(cur ^ 1, make_int2(a, m));
                        if (b - m >= 2) put(cur ^ 1, make_int2(m, b));
                    }
                }
                break;
            }
        }
        __syncthreads();  // the level is done and its children are written
        if (tid == 0) count[cur] = 0;
        cur ^= 1;
        __syncthreads();
    }
    if (tid == 0) *status = fail ? fail : (levels > n ? 1 : 0);
}

__global__ __launch_bounds__(kTbWaves * 64) void k_traceback(const int16_t* __restrict__ F, long long ld,
                                                             const uint8_t* __restrict__ codes, int n,
                                                             int2* __restrict__ spill, int spill_cap,
                                                             char* __restrict__ db, int* __restrict__ status)
{
    traceback_body(F, ld, codes, n, spill, spill_cap, db, status);
}

// One workgroup per fold of a batch.
__global__ __launch_bounds__(kTbWaves * 64) void k_traceback_many(const TracebackWork* __restrict__ work)
{
    const TracebackWork& w = work[blockIdx.x];
    traceback_body(w.F, w.ld, w.codes, w.n, w.spill, w.spill_cap, w.db, w.status);
}

}  // namespace

hipError_t launch_traceback(const int16_t* F, int ld, const uint8_t* codes, int n, int2* spill, int spill_cap,
                            char* db, int* status, hipStream_t s)
{
    if (n < 0 || ld < n + 1 || spill_cap < n / 2 + 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_traceback, dim3(1), dim3(kTbWaves * 64), 0, s, F, (long long)ld, codes, n, spill,
                       spill_cap, db, status);
    return hipGetLastError();
}

hipError_t launch_traceback_many(const TracebackWork* work, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_traceback_many, dim3(count), dim3(kTbWaves * 64), 0, s, work);
    return hipGetLastError();
}

}  // namespace nf
