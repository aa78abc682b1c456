// Allocation-free FP64 residual: the variant of lx_sim_debug_residual for
// callers that cannot allocate device memory (code under stream or graph
// capture, tight serving loops).  Its inputs and outputs are the caller's device
// arrays; every other buffer it needs lives in one file-scope device array of
// fixed size, resolved to a device address once per device when the first
// simulation is created there.
#include <mutex>

#include "lx_device.h"
#include "lx_sim.h"

namespace lx {

namespace {

// Work space of lx_sim_residual_noalloc: the iterate, the residual and the
// right-hand side [nv][4] each, and the element contributions [kRRec nt].
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// internal vertex i (library order) <- caller vertex perm[i]: x [nv][4] from u [nv][3], p [nv]
__global__ void k_na_gather(int64_t nv, const int32_t *perm, const double *u, const double *p, double *x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const int64_t o = perm[i];
    x[4 * i + 0] = u[3 * o + 0];
    x[4 * i + 1] = u[3 * o + 1];
    x[4 * i + 2] = u[3 * o + 2];
    x[4 * i + 3] = p[o];
}

// caller vertex perm[i] <- internal vertex i: out [nv][4]
__global__ void k_na_scatter(int64_t nv, const int32_t *perm, const double *r, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const int64_t o = perm[i];
    for (int c = 0; c < 4; ++c) out[4 * o + c] = r[4 * i + c];
}

}  // namespace

lx_status noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(LX_EINVAL, "device ordinal %d out of range", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return LX_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(LX_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
    g_scratch[device] = (unsigned char *)p;
    return LX_OK;
}

int64_t noalloc_scratch_bytes(int64_t nv, int64_t nt) { return 3 * 4 * nv * 8 + (int64_t)kRRec * nt * 8; }

}  // namespace lx

using lx::fail;

extern "C" lx_status lx_sim_residual_noalloc(lx_sim *s, const double *u, const double *p, double *r)
{
    if (!s) return fail(LX_EINVAL, "simulation handle is NULL");
    if (!u || !p || !r) return fail(LX_EINVAL, "u, p and r must be device pointers");
    if (s->p2) return fail(LX_EINVAL, "the matrix-free residual is built for the P1-P1 pair");
    const int64_t need = lx::noalloc_scratch_bytes(s->nv, s->nt);
    if (need > (int64_t)lx::kScratchBytes)
        return fail(LX_EINVAL, "mesh of %lld vertices and %lld tets needs %lld bytes of scratch, above the %lld-byte "
                    "limit of the allocation-free residual (at most about 160k tets)", (long long)s->nv,
                    (long long)s->nt, (long long)need, (long long)lx::kScratchBytes);
    LX_HIP(hipSetDevice(s->device));
    unsigned char *base;
    {
        std::lock_guard<std::mutex> lk(lx::g_mu);
        base = (s->device >= 0 && s->device < lx::kMaxDevices) ? lx::g_scratch[s->device] : nullptr;
    }
    if (!base) return fail(LX_ESTATE, "scratch of device %d was not resolved", s->device);
    const int64_t n4 = 4 * s->nv;
    double *x = (double *)base, *rr = x + n4, *b = rr + n4, *rec = b + n4;
    lx::StepCoef C;
    lx_status st = s->prepare(s->t + s->prob.dt, C);
    if (st != LX_OK) return st;
    const unsigned g = (unsigned)((s->nv + 255) / 256);
    hipLaunchKernelGGL(lx::k_na_gather, dim3(g), dim3(256), 0, s->stream, s->nv, s->d_perm, u, p, x);
    st = s->residual64_into(C, x, true, s->t + s->prob.dt, rec, rr, b, false);
    if (st != LX_OK) return st;
    hipLaunchKernelGGL(lx::k_na_scatter, dim3(g), dim3(256), 0, s->stream, s->nv, s->d_perm, rr, r);
    LX_HIP(hipGetLastError());
    return LX_OK;
}
