// nf_fold_dev_noalloc: the single-fold fill of nf_fold_dev with every
// buffer beyond the caller's inputs and outputs in one static device array,
// for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array `scratch` holds, for one call: R, the fold descriptor, the padded
// codes, the dense table F, the packed row and column words, the
// accumulators and the work lists.  The work lists are written on the device
// from the closed-form single-fold schedule (SingleSchedule), so a call makes
// only kernel launches on the caller's stream: no allocation, no host copy,
// no memset (the accumulators are cleared by a fill kernel).
//
// Host code never passes `scratch` itself to a kernel (in host code the name
// is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returned for the device at set-up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "nf.h"
#include "nf_internal.h"
#include "nf_runtime.h"

namespace nf {

namespace {

static __device__ __align__(256) uint8_t scratch[NF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {nullptr};  // device address of `scratch`, per device
std::mutex g_scratch_mu;

// Every work item of one fold, one workgroup per stage: stage 0 also writes
// the main-diagonal items and the fold descriptor.
__global__ void k_single_items(SingleSchedule S, FoldDesc fd, int32_t* acc, TileWork* diag, TileWork* tiles,
                               BetweenWork* btw, FoldDesc* fd_out)
{
    const int sg = blockIdx.x;
    const int tid = threadIdx.x;
    if (sg == 0) {
        if (tid == 0) *fd_out = fd;
        for (int A = tid; A < S.NT; A += blockDim.x) {
            TileWork w{};
            w.f = fd;
            w.acc = acc;
            w.A = A;
            diag[A] = w;
        }
    } else {
        const long long off = S.finish_offset(sg);
        for (int A = tid; A < S.finishes(sg); A += blockDim.x) {
            const TileItem it = S.finish(sg, A);
            TileWork w{};
            w.f = fd;
            w.acc = acc + (size_t)it.slot0 * kTileCells;
            w.A = it.A;
            w.d = it.d;
            w.nslot = it.nslot;
            tiles[off + A] = w;
        }
    }
    const long long off = S.between_offset(sg);
    const int cnt = S.between_count(sg);
    for (int k = tid; k < cnt; k += blockDim.x) {
        const BetweenItem it = S.between(sg, k);
        BetweenWork w{};
        w.f = fd;
        w.acc = acc + (size_t)it.slot * kTileCells;
        w.A = it.A;
        w.d = it.d;
        w.c0 = it.c0;
        w.c1 = it.c1;
        w.atomic = it.pad0;
        btw[off + k] = w;
    }
}

__global__ void k_zero(uint4* p, size_t n16)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n16) p[e] = make_uint4(0u, 0u, 0u, 0u);
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Offsets of one call's buffers inside the scratch array.
struct Layout {
    size_t R = 0, fd = 0, fold = 0, acc = 0, diag = 0, tiles = 0, btw = 0, total = 0;
    size_t acc_bytes = 0;
    long long ntiles = 0, nbtw = 0;
};

Layout layout(const Geom& g, const SingleSchedule& S, int q)
{
    Layout L;
    L.R = 0;
    L.fd = up256((size_t)1 << (2 * (q - 1)));
    L.fold = L.fd + up256(sizeof(FoldDesc));
    L.acc = L.fold + g.bytes;
    L.acc_bytes = (size_t)std::max(1, 2 * S.max_slots()) * kTileCells * sizeof(int32_t);
    L.diag = L.acc + up256(L.acc_bytes);
    L.ntiles = S.finish_offset(S.NT);  // finishes of every stage 1 .. NT-1
    L.nbtw = S.between_offset(S.NT);
    L.tiles = L.diag + up256((size_t)S.NT * sizeof(TileWork));
    L.btw = L.tiles + up256((size_t)std::max<long long>(1, L.ntiles) * sizeof(TileWork));
    L.total = L.btw + up256((size_t)std::max<long long>(1, L.nbtw) * sizeof(BetweenWork));
    return L;
}

}  // namespace

// Called at device set-up (ensure_device), with that device current: the
// device address of this device's copy of `scratch`.
int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(NF_E_DEVICE, "device %d beyond the %d the library tracks", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return NF_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(NF_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    }
    g_scratch[device] = ptr;
    return NF_OK;
}

}  // namespace nf

using namespace nf;

extern "C" int nf_fold_dev_noalloc(const uint8_t* d_codes, int n, int q, int32_t* d_score, int16_t* d_S,
                                   void* stream)
{
    std::lock_guard<std::recursive_mutex> lk(api_mutex());
    clear_error();
    int rc = check_length(n);
    if (rc) return rc;
    if ((rc = check_q(q))) return rc;
    if (!d_codes && n > 0) return fail(NF_E_INVAL, "d_codes is NULL");
    q = resolve_q(q, n);
    const Geom g = make_geom(n, q);
    SingleSchedule S;
    S.NT = g.NT;
    S.target = between_target(n, q);
    const Layout L = layout(g, S, q);
    if (L.total > (size_t)NF_NOALLOC_SCRATCH_BYTES)
        return fail(NF_E_NOMEM,
                    "n = %d at q = %d needs %zu bytes of scratch; the static scratch holds %zu; use nf_fold_dev",
                    n, q, L.total, (size_t)NF_NOALLOC_SCRATCH_BYTES);
    if ((rc = ensure_device())) return rc;
    if ((rc = scratch_setup(ctx().device))) return rc;  // done at set-up; repeated here only to report a failure
    uint8_t* base = nullptr;
    {
        std::lock_guard<std::mutex> lk2(g_scratch_mu);
        base = (uint8_t*)g_scratch[ctx().device];
    }
    hipStream_t s = (hipStream_t)stream;

    FoldDesc fd{};
    uint8_t* fold = base + L.fold;
    fd.codes = fold;
    fd.F = (int16_t*)(fold + g.codes_bytes);
    fd.RS = (uint32_t*)(fold + g.codes_bytes + g.F_bytes);
    fd.CS = (uint32_t*)(fold + g.codes_bytes + g.F_bytes + g.rs_bytes);
    fd.n = n;
    fd.NT = g.NT;
    fd.ld = g.ld;
    uint8_t* R = base + L.R;
    int32_t* acc = (int32_t*)(base + L.acc);
    TileWork* diag = (TileWork*)(base + L.diag);
    TileWork* tiles = (TileWork*)(base + L.tiles);
    BetweenWork* btw = (BetweenWork*)(base + L.btw);
    FoldDesc* fdp = (FoldDesc*)(base + L.fd);

    // R, the codes, cleared accumulators and the work lists, then the fill
    HIPCHK(launch_precompute_R(q, R, s));
    HIPCHK(launch_copy_codes(d_codes, n, fold, (int)g.codes_bytes, s));
    const size_t n16 = L.acc_bytes / 16;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s, (uint4*)acc, n16);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_single_items, dim3(S.NT), dim3(256), 0, s, S, fd, acc, diag, tiles, btw, fdp);
    HIPCHK(hipGetLastError());
    HIPCHK(launch_diag(q, diag, S.NT, s));
    const bool wide = stage_wide(n, q);
    for (int sg = 1; sg < S.NT; ++sg)
        HIPCHK(launch_stage(q, wide, tiles + S.finish_offset(sg), S.finishes(sg), btw + S.between_offset(sg),
                            S.between_count(sg), R, s));
    if (d_score) HIPCHK(launch_scores(fdp, 1, d_score, s));
    if (d_S && n > 0) HIPCHK(launch_expand(fd.F, g.ld, n, d_S, s));
    return NF_OK;
}
