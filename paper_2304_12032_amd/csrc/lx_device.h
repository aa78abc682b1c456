// Device-side helpers shared by the kernel translation units.
#pragma once

#include <type_traits>

#include "lx_common.h"

namespace lx {

struct __align__(32) v4d { double v[4]; };
struct __align__(16) v4f { float v[4]; };
template <typename T> struct V4;
template <> struct V4<double> { using type = v4d; };
template <> struct V4<float> { using type = v4f; };

__device__ inline double lx_cos(double x) { return cos(x); }
__device__ inline float lx_cos(float x) { return cosf(x); }
__device__ inline double lx_sqrt(double x) { return sqrt(x); }
__device__ inline float lx_sqrt(float x) { return sqrtf(x); }

__device__ inline void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// True if the device's done flag is set.  dep is a value the caller has just
// loaded: testing it in the same expression keeps that load ahead of the
// branch, so the flag's memory latency overlaps the load's instead of adding to
// it at the start of every kernel.
__device__ __forceinline__ bool done_with(const int32_t *done, int32_t dep)
{
    return done != nullptr && ((done[0] != 0) & (dep != INT32_MIN));
}

// Bytes of one MI355X's last-level cache (the 256 MB MALL in front of HBM).  The
// SpMV's planes, when larger than that, are streamed from HBM by every product,
// and its loads are non-temporal (ld_mat<true>), leaving the caches to the
// gathered vector blocks: 65 -> 57 us per FP64 product on the 983k-tet tube (347
// MB of planes), no change on the 8M-tet chamber.  The other streamed passes keep
// ordinary loads, as measured: non-temporal loads slowed the velocity-block
// Chebyshev pass of the chamber (FP64 step 589 -> 640 ms) and, with the
// round-robin row order of P2-P1, its Chebyshev pass (234 -> 305 us) and SpMV.
// LXNS_STREAM_LOADS=0 turns them off.
constexpr int64_t kLastLevelCacheBytes = int64_t(256) << 20;
bool streamed(int64_t bytes);

template <bool NT, typename T>
__device__ __forceinline__ T ld_mat(const T *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Workgroup index with the grid split into 8 contiguous ranges, one per die
// (XCD): the dispatcher hands workgroups to the dies round-robin, so
// workgroup w runs on die w % 8, and range w % 8 keeps rows that share
// gathered data (element records, neighbouring x blocks) in one die's L2
// rather than fetching them once per die.  A bijection for any grid size.
__device__ inline int64_t xcd_block()
{
    const uint32_t n = gridDim.x, w = blockIdx.x;
    const uint32_t per = n >> 3, rem = n & 7, die = w & 7, local = w >> 3;
    return (int64_t)(die < rem ? die * (per + 1) : rem * (per + 1) + (die - rem) * per) + local;
}

// xcd_block() where rows are of similar cost; the plain round-robin order where
// they are not (contiguous die ranges would then give one die most of the work).
__device__ inline int64_t grid_block(int32_t remap) { return remap ? xcd_block() : (int64_t)blockIdx.x; }

template <typename T, int LPR>
__device__ inline T group_sum(T v)
{
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LPR);
    return v;
}

constexpr int kRedThreads = 256;

// Sums K per-thread values over the block; the result is valid in thread 0.
template <int K>
__device__ inline void block_sum(double (&acc)[K], double *lds)
{
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < K; ++j) lds[j * 4 + wid] = acc[j];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] = (lds[j * 4] + lds[j * 4 + 1]) + (lds[j * 4 + 2] + lds[j * 4 + 3]);
}

// Arrival protocol: every block publishes its partial sums, then the last block
// to arrive reduces all partials in a fixed order (deterministic) and resets
// the counter.
__device__ inline bool arrive_last(uint32_t *counter)
{
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t prev = atomicAdd(counter, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// Final reduction of partial[nb][K] (stride K) in the last block.
template <int K>
__device__ inline void reduce_partials(const double *partial, int nb, int count, double (&out)[K], double *lds)
{
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < count) out[j] += partial[(int64_t)b * K + j];
    block_sum<K>(out, lds);
}

// Chebyshev scalars of step i >= 1 for the interval [lmax/ratio, lmax] of the
// scaled operator M^{-1} A (M a diagonal or block-diagonal scaling):
// d_i = a d_{i-1} + b M^{-1} r_i; step 0 is d_0 = M^{-1} r_0 / theta.
__device__ inline void cheb_coef(double lmax, double ratio, int i, double &theta, double &a, double &b)
{
    const double lmin = lmax / ratio;
    theta = 0.5 * (lmax + lmin);
    const double delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    double rho = 1.0 / sigma, rho_prev = rho;
    for (int j = 1; j <= i; ++j) {
        rho_prev = rho;
        rho = 1.0 / (2.0 * sigma - rho);
    }
    a = rho * rho_prev;
    b = 2.0 * rho / delta;
}

// The same scalars rounded to the working precision T of the pass that uses them.
template <typename T>
__device__ inline void cheb_coef_t(double lmax, double ratio, int i, T &theta, T &a, T &b)
{
    double t, x, y;
    cheb_coef(lmax, ratio, i, t, x, y);
    theta = (T)t;
    a = (T)x;
    b = (T)y;
}

template <typename T>
__device__ inline double to_d(T v) { return (double)v; }

}  // namespace lx
