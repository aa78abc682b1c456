// Device side of the SIMPLE block approximations (Sec. 2.4 names AMG and block
// Jacobi among the block approximations of its SIMPLE preconditioner):
//  * the Schur block S~ = C - B D^{-1} G is formed explicitly each step, and
//    approximated by one cycle of unsmoothed-aggregation multigrid with
//    Chebyshev smoothing on diag(A_l)^{-1} A_l and a dense inverse on the
//    coarsest level;
//  * the velocity block F is approximated by a Chebyshev iteration on
//    F~^{-1} F, F~ its nodal 3x3 diagonal blocks, whose upper bound comes from
//    a few power iterations warm-started from the previous step.
// Row kernels use LPR lanes per row and accumulate in the working precision T
// (FP32 for the inner solves of FP32 + refinement); FP64 stays in the scalar
// bounds that place the Chebyshev intervals (Gershgorin maxima, power-iteration
// norms) and in the dense inverse of the coarsest level.  Every apply-phase
// kernel honours the GMRES done flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <utility>

#include "lx_amg.h"
#include "lx_device.h"

namespace lx {

// ================================================================== set-up

// Position of column k in the sorted CSR row [lo, hi), or -1.
__device__ inline int32_t find_col(const int32_t *col, int32_t lo, int32_t hi, int32_t k)
{
    if (lo >= hi) return -1;
    --hi;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return col[lo] == k ? lo : -1;
}

// S~_ik = C_ik - sum_{j, d} B_ij[d] D^{-1}_j[d] G_jk[d] over the velocity nodes j
// of B's row i.  One wavefront per row i.  The wave first stages, in LDS, C's
// row, S~'s columns and, for every G row j that B's row names (row after row,
// in B's order), the products sum_d B_ij[d] D^{-1}_j[d] G_jk[d] with the
// position of their column k in S~'s row (binary search in the staged row).
// The accumulator of each entry starts at C_ik; then the G rows are taken in
// B's order, each lane subtracting one product of the row from its entry (the
// columns of one G row are distinct, so no two lanes meet).  The sum runs over
// B's row in order, so the result does not depend on scheduling.  Rows whose
// rows do not fit the LDS share search C and G in global memory instead, with
// the same arithmetic.
// The LDS share per row is a template pair (B and C entries at most ROWS <= 128,
// staged products at most CAP, entries of S~'s row at most 2 ROWS + 32): a small
// one for P1-P1, whose rows are short, keeps more workgroups per compute unit;
// P2-P1 rows need the large one.
constexpr int kSfWaves = 4;      // waves (rows) per workgroup

__device__ inline int32_t find_col_lds(const int32_t *col, int32_t lo, int32_t hi, int32_t k)
{
    if (lo >= hi) return -1;
    --hi;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return col[lo] == k ? lo : -1;
}

template <typename T>
__device__ inline T schur_term(const SimpleView<T> &V, const T *__restrict__ Dinv, int32_t k1, int32_t j, int32_t kg)
{
    const int64_t nu = V.nu;
    return V.Bv[k1] * Dinv[j] * V.Gv[kg] + V.Bv[V.bs + k1] * Dinv[nu + j] * V.Gv[V.gs + kg] +
           V.Bv[2 * V.bs + k1] * Dinv[2 * nu + j] * V.Gv[2 * V.gs + kg];
}

template <typename T, int kSfRows, int kSfCap>
__global__ __launch_bounds__(256) void k_schur_form(SimpleView<T> V, const T *__restrict__ Dinv,
                                                    const int32_t *__restrict__ srow,
                                                    const int32_t *__restrict__ scol, T *__restrict__ sval,
                                                    const int32_t *__restrict__ soff)
{
    constexpr int kSfOut = 2 * kSfRows + 32;
    __shared__ int32_t s_off[kSfWaves][kSfRows + 1];
    __shared__ int32_t s_j[kSfWaves][kSfRows];
    __shared__ int32_t s_gb[kSfWaves][kSfRows];
    __shared__ int32_t s_cc[kSfWaves][kSfRows];
    __shared__ T s_cv[kSfWaves][kSfRows];
    __shared__ int32_t s_sc[kSfWaves][kSfOut];
    __shared__ T s_acc[kSfWaves][kSfOut];
    __shared__ int32_t s_tgt[kSfWaves][kSfCap];
    __shared__ T s_val[kSfWaves][kSfCap];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = xcd_block() * kSfWaves + wv;
    const bool live = i < V.np;
    const int32_t b0 = live ? V.bptr[i] : 0, b1 = live ? V.bptr[i + 1] : 0;
    const int32_t c0 = live ? V.cptr[i] : 0, c1 = live ? V.cptr[i + 1] : 0;
    const int32_t e0 = live ? srow[i] : 0, e1 = live ? srow[i + 1] : 0;
    const int nb = b1 - b0, nc = c1 - c0, ns = e1 - e0;
    bool staged = live && nb <= kSfRows && nc <= kSfRows && ns <= kSfOut;   // uniform over the wave
    int32_t *off = s_off[wv];
    if (staged) {
        // B entries: velocity node, start and length of its G row; inclusive scan of
        // the lengths over the wave (two entries per lane)
        int32_t len[2] = {0, 0};
        for (int h = 0; h < 2; ++h) {
            const int t = lane + 64 * h;
            if (t < nb) {
                const int32_t j = V.bcol[b0 + t], g0 = V.gptr[j];
                s_j[wv][t] = j;
                s_gb[wv][t] = g0;
                len[h] = V.gptr[j + 1] - g0;
            }
            if (t < nc) {
                s_cc[wv][t] = V.ccol[c0 + t];
                s_cv[wv][t] = V.Cv[c0 + t];
            }
        }
        for (int e = lane; e < ns; e += 64) s_sc[wv][e] = scol[e0 + e];
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t u0 = __shfl_up(len[0], d), u1 = __shfl_up(len[1], d);
            if (lane >= d) {
                len[0] += u0;
                len[1] += u1;
            }
        }
        const int32_t first = __shfl(len[0], 63);
        if (lane == 0) off[0] = 0;
        if (lane < nb) off[lane + 1] = len[0];
        if (lane + 64 < nb) off[lane + 65] = len[1] + first;
    }
    __syncthreads();
    staged = staged && off[nb] <= kSfCap;
    if (staged) {
        // every entry's accumulator starts at C_ik (0 where C has no entry)
        for (int e = lane; e < ns; e += 64) {
            const int32_t kc = find_col_lds(s_cc[wv], 0, nc, s_sc[wv][e]);
            s_acc[wv][e] = kc >= 0 ? s_cv[wv][kc] : 0.0;
        }
        // four products per lane at a time, so that their gathers are in flight together
        const int total = off[nb];
        for (int q0 = 0; q0 < total; q0 += 256) {
            int32_t kg[4], t[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + 64 * u + lane;
                int lo = 0, hi = nb - 1;     // the B entry t with off[t] <= q < off[t + 1]
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (off[mid] <= q)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                t[u] = lo;
                kg[u] = q < total ? s_gb[wv][lo] + (q - off[lo]) : -1;
            }
            int32_t col[4];
            T pv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (kg[u] >= 0) {
                    col[u] = V.gcol[kg[u]];
                    pv[u] = schur_term(V, Dinv, b0 + t[u], s_j[wv][t[u]], kg[u]);
                }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (kg[u] >= 0) {
                    // S~'s pattern holds every column of every G row that B's row names
                    s_tgt[wv][q0 + 64 * u + lane] = find_col_lds(s_sc[wv], 0, ns, col[u]);
                    s_val[wv][q0 + 64 * u + lane] = pv[u];
                }
        }
    }
    __syncthreads();
    if (!live) return;
    if (staged) {
        // G rows in B's order; within one row the targets are distinct.  The wave's
        // LDS accesses complete in program order, so row t + 1 sees row t's updates.
        for (int t = 0; t < nb; ++t) {
            for (int q = off[t] + lane; q < off[t + 1]; q += 64) {
                const int32_t e = s_tgt[wv][q];
                if (e >= 0) s_acc[wv][e] -= s_val[wv][q];
            }
            __builtin_amdgcn_wave_barrier();
        }
        __builtin_amdgcn_wave_barrier();
        for (int e = lane; e < ns; e += 64)
            sval[soff ? (int64_t)soff[i >> 6] + (int64_t)e * 64 + (i & 63) : (int64_t)(e0 + e)] = (T)s_acc[wv][e];
        return;
    }
    for (int32_t e = e0 + lane; e < e1; e += 64) {
        const int32_t k = scol[e];
        const int32_t kc = find_col(V.ccol, c0, c1, k);
        T acc = kc >= 0 ? V.Cv[kc] : 0.0;
        for (int32_t k1 = b0; k1 < b1; ++k1) {
            const int32_t j = V.bcol[k1];
            const int32_t kg = find_col(V.gcol, V.gptr[j], V.gptr[j + 1], k);
            if (kg >= 0) acc -= schur_term(V, Dinv, k1, j, kg);
        }
        sval[soff ? (int64_t)soff[i >> 6] + (int64_t)(e - e0) * 64 + (i & 63) : (int64_t)e] = (T)acc;
    }
}

// Block maximum of v (valid in thread 0); blockDim = 256.
__device__ inline double block_max(double v, double *lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    return fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
}

// dinv_i = 1 / A_ii and partial[block] = max over the block's rows of
// sum_k |A_ik| / |A_ii|; k_max_fin turns the block maxima into the Gershgorin
// bound of diag(A)^{-1} A.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_rowinfo(int64_t n, const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ diag, const T *__restrict__ val,
                                                     T *__restrict__ dinv, double *partial)
{
    __shared__ double lds[4];
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    T s = 0;
    if (row < n)
        for (int32_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += LPR) s += fabs(val[k]);
    s = group_sum<T, LPR>(s);
    double g = 0;
    if (row < n && lane == 0) {
        const int32_t dk = diag[row];
        const T a = dk >= 0 ? val[dk] : T(0);
        const T di = a != T(0) ? T(1) / a : T(0);
        dinv[row] = di;
        g = (double)(s * fabs(di));
    }
    const double m = block_max(g, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// *out = max of partial[0..nb) (one block of 256)
__global__ __launch_bounds__(256) void k_max_fin(int nb, const double *partial, double *out)
{
    __shared__ double lds[4];
    double m = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) m = fmax(m, partial[b]);
    m = block_max(m, lds);
    if (threadIdx.x == 0) *out = m;
}

// Galerkin sum with piecewise-constant prolongation: each coarse entry is the
// sum of the fine entries listed for it, LPR lanes per coarse entry reading the
// list with unit stride (each lane's partial sum in list order, then a fixed
// butterfly over the lanes).
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_coarsen(int64_t nnzc, const int32_t *__restrict__ cptr,
                                                     const int32_t *__restrict__ cidx, const T *__restrict__ fval,
                                                     T *__restrict__ cval)
{
    const int64_t c = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (c >= nnzc) return;
    T s = 0;
    for (int32_t q = cptr[c] + lane; q < cptr[c + 1]; q += LPR) s += fval[cidx[q]];
    s = group_sum<T, LPR>(s);
    if (lane == 0) cval[c] = (T)s;
}

// aug = [0 | I] (nc x 2nc, row-major)
__global__ void k_dense_init(int64_t nc, double *aug)
{
    const int64_t q = xcd_block() * blockDim.x + threadIdx.x;
    if (q >= 2 * nc * nc) return;
    const int64_t r = q / (2 * nc), c = q % (2 * nc);
    aug[q] = (c == nc + r) ? 1.0 : 0.0;
}

template <typename T>
__global__ void k_dense_scatter(int64_t nnz, int64_t nc, const int32_t *__restrict__ crow,
                                const int32_t *__restrict__ col, const T *__restrict__ val, double *aug)
{
    const int64_t k = xcd_block() * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    aug[(int64_t)crow[k] * 2 * nc + col[k]] = (double)val[k];
}

// Gauss-Jordan elimination with partial pivoting on [A | I] in one block: the
// right half becomes A^{-1}.  A pivot at or below 1e-14 max|A| zeroes its row
// (a singular coarse operator then yields a generalised inverse).
__global__ __launch_bounds__(1024) void k_dense_gj(int nc, double *aug)
{
    __shared__ double sv[1024];
    __shared__ int si[1024];
    __shared__ double fac[kAmgDenseMax];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int w = 2 * nc;
    double m = 0;
    for (int q = tid; q < nc * nc; q += nth) m = fmax(m, fabs(aug[(q / nc) * w + q % nc]));
    sv[tid] = m;
    __syncthreads();
    for (int s = nth / 2; s > 0; s >>= 1) {
        if (tid < s) sv[tid] = fmax(sv[tid], sv[tid + s]);
        __syncthreads();
    }
    const double tiny = 1e-14 * sv[0];
    __syncthreads();
    for (int p = 0; p < nc; ++p) {
        double bv = -1.0;
        int bi = p;
        for (int r = p + tid; r < nc; r += nth) {
            const double v = fabs(aug[r * w + p]);
            if (v > bv) {
                bv = v;
                bi = r;
            }
        }
        sv[tid] = bv;
        si[tid] = bi;
        __syncthreads();
        for (int s = nth / 2; s > 0; s >>= 1) {
            if (tid < s && (sv[tid + s] > sv[tid] || (sv[tid + s] == sv[tid] && si[tid + s] < si[tid]))) {
                sv[tid] = sv[tid + s];
                si[tid] = si[tid + s];
            }
            __syncthreads();
        }
        const int pr = si[0];
        const double pv = sv[0];
        __syncthreads();
        if (!(pv > tiny)) {
            for (int c = tid; c < w; c += nth) aug[p * w + c] = 0.0;
            __syncthreads();
            continue;
        }
        if (pr != p)
            for (int c = tid; c < w; c += nth) {
                const double t = aug[p * w + c];
                aug[p * w + c] = aug[pr * w + c];
                aug[pr * w + c] = t;
            }
        __syncthreads();
        const double inv = 1.0 / aug[p * w + p];
        __syncthreads();
        for (int c = tid; c < w; c += nth) aug[p * w + c] *= inv;
        for (int r = tid; r < nc; r += nth) fac[r] = (r == p) ? 0.0 : aug[r * w + p];
        __syncthreads();
        // columns left of p in the left half are already eliminated in row p
        const int c0 = p, wc = w - c0;
        for (int q = tid; q < nc * wc; q += nth) {
            const int r = q / wc, c = c0 + q % wc;
            if (r != p) aug[r * w + c] -= fac[r] * aug[p * w + c];
        }
        __syncthreads();
    }
}

// The same elimination for a small dense level (nc <= kGjLdsMax), held in LDS:
// wavefront 0 finds the pivot (largest magnitude, lowest row on ties) and the
// row factors by shuffles, then the block swaps and scales the pivot row and
// eliminates, with three barriers per column instead of a tree reduction and
// global-memory passes.  Same operations and order of each entry's update as
// k_dense_gj, so the inverse is the same.
constexpr int kGjLdsMax = 48;

__global__ __launch_bounds__(1024) void k_dense_gj_lds(int nc, double *aug)
{
    __shared__ double a[kGjLdsMax * 2 * kGjLdsMax];
    __shared__ double fac[kGjLdsMax];
    __shared__ double red[16];
    __shared__ int s_pr;
    __shared__ double s_inv;
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wid = tid >> 6;
    const int w = 2 * nc;
    double m = 0;
    for (int q = tid; q < nc * w; q += nth) {
        const double v = aug[q];
        a[q] = v;
        if (q % w < nc) m = fmax(m, fabs(v));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane == 0) red[wid] = m;
    __syncthreads();
    double mx = 0;
    for (int i = 0; i < (nth >> 6); ++i) mx = fmax(mx, red[i]);
    const double tiny = 1e-14 * mx;
    for (int p = 0; p < nc; ++p) {
        if (wid == 0) {
            // pivot: the largest |a[r][p]|, r >= p, lowest r on ties
            double bv = (lane >= p && lane < nc) ? fabs(a[lane * w + p]) : -1.0;
            int bi = (lane >= p && lane < nc) ? lane : nc;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            const int pr = bi;
            const bool ok = bv > tiny;
            // factors of the rows after the swap: row r holds old row (r == p ? pr : r == pr ? p : r)
            if (lane < nc) {
                const int src = lane == p ? pr : (lane == pr ? p : lane);
                fac[lane] = (lane == p || !ok) ? 0.0 : a[src * w + p];
            }
            if (lane == 0) {
                s_pr = ok ? pr : -1;
                s_inv = ok ? 1.0 / a[pr * w + p] : 0.0;
            }
        }
        __syncthreads();
        const int pr = s_pr;
        if (pr < 0) {
            for (int c = tid; c < w; c += nth) a[p * w + c] = 0.0;
            __syncthreads();
            continue;
        }
        const double inv = s_inv;
        for (int c = tid; c < w; c += nth) {
            const double vp = a[p * w + c], vr = a[pr * w + c];
            a[p * w + c] = vr * inv;
            if (pr != p) a[pr * w + c] = vp;
        }
        __syncthreads();
        // columns left of p in the left half are already eliminated in row p
        const int c0 = p, wc = w - c0;
        for (int q = tid; q < nc * wc; q += nth) {
            const int r = q / wc, c = c0 + q % wc;
            if (r != p) a[r * w + c] -= fac[r] * a[p * w + c];
        }
        __syncthreads();
    }
    for (int q = tid; q < nc * w; q += nth) aug[q] = a[q];
}

// One power step w = F~^{-1} F v / ||v|| (velocity block, [nv][4] vectors),
// ||v||^2 read from lam[slot_in]; partial[block] = the block's part of ||w||^2.
// v = null: the start vector of +-1 entries from a multiplicative hash of the
// index.
__device__ inline double pm_one(uint32_t q)
{
    return ((q * 2654435761u) >> 13) & 1u ? 1.0 : -1.0;
}

template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_fpow(RowPattern P, const T *__restrict__ val, const T *__restrict__ Finv,
                                              const T *__restrict__ v, T *__restrict__ w, const double *lam,
                                              int slot_in, double *partial)
{
    __shared__ double lds[16];
    const int64_t row = (grid_block(P.remap) * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    const int64_t nb = P.nblk, nv = P.nv;
    using V = typename V4<T>::type;
    const T nin = (T)(v ? sqrt(lam[slot_in]) : sqrt(3.0 * (double)nv));
    T t0 = 0, t1 = 0, t2 = 0;
    if (row < nv)
        for (int32_t k = P.rowptr[row] + lane; k < P.rowptr[row + 1]; k += LPR) {
            const int32_t j = P.col[k];
            T x0, x1, x2;
            if (v) {
                const V xv = reinterpret_cast<const V *>(v)[j];
                x0 = xv.v[0];
                x1 = xv.v[1];
                x2 = xv.v[2];
            } else {
                x0 = pm_one(3u * (uint32_t)j);
                x1 = pm_one(3u * (uint32_t)j + 1u);
                x2 = pm_one(3u * (uint32_t)j + 2u);
            }
            T a[9];
#pragma unroll
            for (int p = 0; p < 9; ++p) a[p] = val[p * nb + k];
            t0 += a[0] * x0 + a[1] * x1 + a[2] * x2;
            t1 += a[3] * x0 + a[4] * x1 + a[5] * x2;
            t2 += a[6] * x0 + a[7] * x1 + a[8] * x2;
        }
    t0 = group_sum<T, LPR>(t0);
    t1 = group_sum<T, LPR>(t1);
    t2 = group_sum<T, LPR>(t2);
    double acc[1] = {0.0};
    if (row < nv && lane == 0) {
        T fi[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) fi[p] = Finv[p * nv + row];
        V o;
        o.v[0] = (T)((fi[0] * t0 + fi[1] * t1 + fi[2] * t2) / nin);
        o.v[1] = (T)((fi[3] * t0 + fi[4] * t1 + fi[5] * t2) / nin);
        o.v[2] = (T)((fi[6] * t0 + fi[7] * t1 + fi[8] * t2) / nin);
        o.v[3] = T(0);
        reinterpret_cast<V *>(w)[row] = o;
        acc[0] = (double)o.v[0] * o.v[0] + (double)o.v[1] * o.v[1] + (double)o.v[2] * o.v[2];
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

// lam[slot_out] = sum of partial[0..nb) in a fixed order; factor > 0 also sets
// lam[kLamF] = factor * sqrt(that sum).
__global__ __launch_bounds__(256) void k_fpow_fin(int nb, const double *partial, double *lam, int slot_out,
                                                  double factor)
{
    __shared__ double lds[16];
    double a[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) a[0] += partial[b];
    block_sum<1>(a, lds);
    if (threadIdx.x == 0) {
        lam[slot_out] = a[0];
        if (factor > 0) lam[kLamF] = factor * sqrt(a[0]);
    }
}

// ================================================================== apply

// z.u = F~^{-1} (scale r.u) (f_degree 1), or the Chebyshev start on F (fr =
// scale r.u, fd = F~^{-1} fr / theta, z.u = fd); z.p = scale r.p.
template <typename T>
__global__ void k_fz_start(int64_t nv, const T *__restrict__ Finv, const T *__restrict__ r,
                           const double *scale_ptr, T *__restrict__ z, T *__restrict__ fr, T *__restrict__ fd,
                           const double *lamF, double ratio, int degree, const int32_t *done)
{
    if (done && *done) return;
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const T sc = scale_ptr ? *scale_ptr : 1.0;
    using V = typename V4<T>::type;
    const V rv = reinterpret_cast<const V *>(r)[i];
    const T r0 = rv.v[0] * sc, r1 = rv.v[1] * sc, r2 = rv.v[2] * sc;
    T fi[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) fi[p] = Finv[p * nv + i];
    T y0 = fi[0] * r0 + fi[1] * r1 + fi[2] * r2;
    T y1 = fi[3] * r0 + fi[4] * r1 + fi[5] * r2;
    T y2 = fi[6] * r0 + fi[7] * r1 + fi[8] * r2;
    V zv;
    if (degree > 1) {
        T theta, a, b;
        cheb_coef_t(*lamF, ratio, 0, theta, a, b);
        y0 /= theta;
        y1 /= theta;
        y2 /= theta;
        V f;
        f.v[0] = (T)r0;
        f.v[1] = (T)r1;
        f.v[2] = (T)r2;
        f.v[3] = T(0);
        reinterpret_cast<V *>(fr)[i] = f;
        V d;
        d.v[0] = (T)y0;
        d.v[1] = (T)y1;
        d.v[2] = (T)y2;
        d.v[3] = T(0);
        reinterpret_cast<V *>(fd)[i] = d;
        zv.v[0] = d.v[0];
        zv.v[1] = d.v[1];
        zv.v[2] = d.v[2];
    } else {
        zv.v[0] = (T)y0;
        zv.v[1] = (T)y1;
        zv.v[2] = (T)y2;
    }
    zv.v[3] = (T)(rv.v[3] * sc);
    reinterpret_cast<V *>(z)[i] = zv;
}

// Chebyshev step on F z.u = fr: res = fr - F d, dn = a d + b F~^{-1} res,
// z.u += dn, dnext = dn (fr keeps the running residual).
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_fcheb(RowPattern P, const T *__restrict__ val, const T *__restrict__ Finv,
                                               T *__restrict__ z, T *__restrict__ fr, const T *__restrict__ dcur,
                                               T *__restrict__ dnext, const double *lamF, double ratio, int step,
                                               const int32_t *done)
{
    const int64_t row = (grid_block(P.remap) * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int32_t beg = P.rowptr[row], end = P.rowptr[row + 1];
    if (done_with(done, end)) return;
    const int64_t nb = P.nblk, nv = P.nv;
    using V = typename V4<T>::type;
    T t0 = 0, t1 = 0, t2 = 0;
    for (int32_t k = beg + lane; k < end; k += LPR) {
        const V xv = reinterpret_cast<const V *>(dcur)[P.col[k]];
        const T x0 = xv.v[0], x1 = xv.v[1], x2 = xv.v[2];
        T a[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) a[p] = val[p * nb + k];
        t0 += a[0] * x0 + a[1] * x1 + a[2] * x2;
        t1 += a[3] * x0 + a[4] * x1 + a[5] * x2;
        t2 += a[6] * x0 + a[7] * x1 + a[8] * x2;
    }
    t0 = group_sum<T, LPR>(t0);
    t1 = group_sum<T, LPR>(t1);
    t2 = group_sum<T, LPR>(t2);
    if (lane != 0) return;
    T theta, a, b;
    cheb_coef_t(*lamF, ratio, step, theta, a, b);
    V f = reinterpret_cast<V *>(fr)[row];
    const T e0 = f.v[0] - t0, e1 = f.v[1] - t1, e2 = f.v[2] - t2;
    f.v[0] = (T)e0;
    f.v[1] = (T)e1;
    f.v[2] = (T)e2;
    reinterpret_cast<V *>(fr)[row] = f;
    T fi[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) fi[p] = Finv[p * nv + row];
    const V dc = reinterpret_cast<const V *>(dcur)[row];
    V dn;
    dn.v[0] = (T)(a * dc.v[0] + b * (fi[0] * e0 + fi[1] * e1 + fi[2] * e2));
    dn.v[1] = (T)(a * dc.v[1] + b * (fi[3] * e0 + fi[4] * e1 + fi[5] * e2));
    dn.v[2] = (T)(a * dc.v[2] + b * (fi[6] * e0 + fi[7] * e1 + fi[8] * e2));
    dn.v[3] = T(0);
    reinterpret_cast<V *>(dnext)[row] = dn;
    V zv = reinterpret_cast<V *>(z)[row];
    zv.v[0] = (T)(zv.v[0] + dn.v[0]);
    zv.v[1] = (T)(zv.v[1] + dn.v[1]);
    zv.v[2] = (T)(zv.v[2] + dn.v[2]);
    reinterpret_cast<V *>(z)[row] = zv;
}

// t = z.p - sum_j B_ij z.u_j (z.p holds scale r.p): the right-hand side of the
// Schur solve, stored in L0.r; with smoothed levels also the Chebyshev start
// x0 = d0 = dinv t / theta, res = t.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_zp_amg(SimpleView<T> V, const T *__restrict__ z, AmgLevel<T> L,
                                                const double *lam, double ratio, int smooth, const int32_t *done)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= V.np) return;
    const int32_t beg = V.bptr[row], end = V.bptr[row + 1];
    if (done_with(done, end)) return;
    using VT = typename V4<T>::type;
    T acc = 0;
    for (int32_t k = beg + lane; k < end; k += LPR) {
        const VT zj = reinterpret_cast<const VT *>(z)[V.bcol[k]];
        acc += V.Bv[k] * zj.v[0] + V.Bv[V.bs + k] * zj.v[1] + V.Bv[2 * V.bs + k] * zj.v[2];
    }
    acc = group_sum<T, LPR>(acc);
    if (lane != 0) return;
    const T t = z[4 * row + 3] - acc;
    L.r[row] = (T)t;
    if (smooth) {
        T theta, a, b;
        cheb_coef_t(*lam, ratio, 0, theta, a, b);
        const T x = (T)(L.dinv[row] * t / theta);
        L.res[row] = (T)t;
        L.x0[row] = x;
        L.d0[row] = x;
    }
}

// z.u -= D^{-1} sum_j G_ij p_j, z.p = p on the pressure rows (0 elsewhere)
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_xu_amg(SimpleView<T> V, const T *__restrict__ Dinv, T *__restrict__ z,
                                                const T *__restrict__ p, const int32_t *done)
{
    const int64_t row = (grid_block(V.Fp.remap) * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= V.nu) return;
    const int32_t beg = V.gptr[row], end = V.gptr[row + 1];
    if (done_with(done, end)) return;
    const int64_t nu = V.nu;
    T a0 = 0, a1 = 0, a2 = 0;
    for (int32_t k = beg + lane; k < end; k += LPR) {
        const T pj = p[V.gcol[k]];
        a0 += V.Gv[k] * pj;
        a1 += V.Gv[V.gs + k] * pj;
        a2 += V.Gv[2 * V.gs + k] * pj;
    }
    a0 = group_sum<T, LPR>(a0);
    a1 = group_sum<T, LPR>(a1);
    a2 = group_sum<T, LPR>(a2);
    if (lane != 0) return;
    using VT = typename V4<T>::type;
    VT zv = reinterpret_cast<VT *>(z)[row];
    zv.v[0] = (T)(zv.v[0] - Dinv[row] * a0);
    zv.v[1] = (T)(zv.v[1] - Dinv[nu + row] * a1);
    zv.v[2] = (T)(zv.v[2] - Dinv[2 * nu + row] * a2);
    zv.v[3] = row < V.np ? p[row] : T(0);
    reinterpret_cast<VT *>(z)[row] = zv;
}

// Level l > 0 start: r = restriction of the finer residual (sum over the
// aggregate's members), x0 = d0 = dinv r / theta, res = r.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_pre(AmgLevel<T> L, const T *__restrict__ fres,
                                                 const int32_t *__restrict__ mptr, const int32_t *__restrict__ mem,
                                                 const double *lam, double ratio, const int32_t *done)
{
    const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (i >= L.n) return;
    const int32_t beg = mptr[i], end = mptr[i + 1];
    if (done_with(done, end)) return;
    T s = 0;
    for (int32_t q = beg + lane; q < end; q += LPR) s += fres[mem[q]];
    s = group_sum<T, LPR>(s);
    if (lane != 0) return;
    T theta, a, b;
    cheb_coef_t(*lam, ratio, 0, theta, a, b);
    const T x = (T)(L.dinv[i] * s / theta);
    L.r[i] = (T)s;
    L.res[i] = (T)s;
    L.x0[i] = x;
    L.d0[i] = x;
}

// Chebyshev smoothing step: res -= A d, dn = a d + b dinv res, x += dn.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_cheb(AmgLevel<T> L, T *__restrict__ x, const T *__restrict__ dcur,
                                                  T *__restrict__ dnext, const double *lam, double ratio, int step,
                                                  const int32_t *done)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= L.n) return;
    const int32_t beg = L.rowptr[row], end = L.rowptr[row + 1];
    if (done_with(done, end)) return;
    T q = 0;
    for (int32_t k = beg + lane; k < end; k += LPR)
        q += L.val[k] * dcur[L.col[k]];
    q = group_sum<T, LPR>(q);
    if (lane != 0) return;
    T theta, a, b;
    cheb_coef_t(*lam, ratio, step, theta, a, b);
    const T r = L.res[row] - q;
    L.res[row] = (T)r;
    const T dn = a * dcur[row] + b * L.dinv[row] * r;
    dnext[row] = (T)dn;
    x[row] = (T)(x[row] + dn);
}

// The last Chebyshev step of a coarse level's visit, which also hands the finer
// level its corrected iterate: xp[m] = fx0[m] + x_new[row] for every member m
// of the row's aggregate (fx0: the finer level's iterate before the coarse
// correction), so that the finer level's first post-smoothing pass reads one
// vector instead of gathering the coarse correction entry by entry.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_cheb_prolong(AmgLevel<T> L, T *__restrict__ x, const T *__restrict__ dcur,
                                                          T *__restrict__ dnext, const double *lam, double ratio,
                                                          int step, const int32_t *done, const T *__restrict__ fx0,
                                                          T *__restrict__ xp, const int32_t *__restrict__ fmptr,
                                                          const int32_t *__restrict__ fmem)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= L.n) return;
    const int32_t beg = L.rowptr[row], end = L.rowptr[row + 1];
    if (done_with(done, end)) return;
    T q = 0;
    for (int32_t k = beg + lane; k < end; k += LPR)
        q += L.val[k] * dcur[L.col[k]];
    q = group_sum<T, LPR>(q);   // every lane of the group holds the sum
    T theta, a, b;
    cheb_coef_t(*lam, ratio, step, theta, a, b);
    const T r = L.res[row] - q;
    const T dn = a * dcur[row] + b * L.dinv[row] * r;
    const T xn = (T)(x[row] + dn);
    for (int32_t k = fmptr[row] + lane; k < fmptr[row + 1]; k += LPR) {
        const int32_t m = fmem[k];
        xp[m] = (T)(fx0[m] + xn);
    }
    if (lane != 0) return;
    L.res[row] = (T)r;
    dnext[row] = (T)dn;
    x[row] = xn;
}

// res = r - A x
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_resid(AmgLevel<T> L, const T *__restrict__ x, const int32_t *done)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= L.n) return;
    const int32_t beg = L.rowptr[row], end = L.rowptr[row + 1];
    if (done_with(done, end)) return;
    T q = 0;
    for (int32_t k = beg + lane; k < end; k += LPR)
        q += L.val[k] * x[L.col[k]];
    q = group_sum<T, LPR>(q);
    if (lane == 0) L.res[row] = (T)(L.r[row] - q);
}

// Coarse correction and first post-smoothing step: y = x0 + P e,
// res = r - A y, d0 = dinv res / theta, x1 = y + d0.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_post0(AmgLevel<T> L, const T *__restrict__ e, const double *lam,
                                                   double ratio, const int32_t *done)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= L.n) return;
    const int32_t beg = L.rowptr[row], end = L.rowptr[row + 1];
    if (done_with(done, end)) return;
    T q = 0;
    for (int32_t k = beg + lane; k < end; k += LPR) {
        const int32_t j = L.col[k];
        q += L.val[k] * (L.x0[j] + e[L.agg[j]]);
    }
    q = group_sum<T, LPR>(q);
    if (lane != 0) return;
    T theta, a, b;
    cheb_coef_t(*lam, ratio, 0, theta, a, b);
    const T r = L.r[row] - q;
    const T d = L.dinv[row] * r / theta;
    L.res[row] = (T)r;
    L.d0[row] = (T)d;
    L.x1[row] = (T)(L.x0[row] + e[L.agg[row]] + d);
}

// Dense coarsest solve out = A^{-1} rc, rc the restriction of the finer
// residual (mptr = null: rc = fres).  One block.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_solve(int nc, const double *__restrict__ aug,
                                                     const T *__restrict__ fres, const int32_t *__restrict__ mptr,
                                                     const int32_t *__restrict__ mem, T *__restrict__ out,
                                                     const int32_t *done)
{
    if (done && *done) return;
    __shared__ double rc[kAmgDenseMax];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        double s = 0;
        if (mptr)
            for (int32_t q = mptr[c]; q < mptr[c + 1]; ++q) s += (double)fres[mem[q]];
        else
            s = (double)fres[c];
        rc[c] = s;
    }
    __syncthreads();
    const int w = 2 * nc;
    for (int r = threadIdx.x; r < nc; r += blockDim.x) {
        double s = 0;
        for (int c = 0; c < nc; ++c) s += aug[(int64_t)r * w + nc + c] * rc[c];
        out[r] = (T)s;
    }
}

// ---- the finest level in sliced-ELL order: the entries of 64 consecutive rows
// side by side (entry j of the slice's rows is one contiguous run), so a
// wavefront's load of entry j over its 64 rows is one coalesced access.

template <typename T, bool D16>
__device__ __forceinline__ int32_t sell_col(const AmgLevel<T> &L, int64_t p, int64_t row)
{
    if constexpr (D16)
        return (int32_t)row + (int32_t)L.sdel[p];
    else
        return L.scol[p];
}

template <typename T>
__global__ __launch_bounds__(256) void k_amg_rowinfo_sell(AmgLevel<T> L, double *partial)
{
    __shared__ double lds[4];
    const int64_t row = xcd_block() * blockDim.x + threadIdx.x;
    double g = 0;
    if (row < L.n) {
        const int64_t base = L.soff[row >> 6] + (row & 63);
        const int w = L.swid[row >> 6];
        T s = 0;
        for (int j = 0; j < w; ++j) s += fabs(L.val[base + 64 * (int64_t)j]);
        const int32_t dk = L.diag[row];
        const T a = dk >= 0 ? L.val[base + 64 * (int64_t)(dk - L.rowptr[row])] : T(0);
        const T di = a != T(0) ? T(1) / a : T(0);
        L.dinv[row] = di;
        g = (double)(s * fabs(di));
    }
    const double m = block_max(g, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// The smoothing passes run SW = kSellWaves wavefronts per slice of 64 rows (one
// workgroup per slice): wavefront v takes the entries j = v, v + SW, ... of
// every row, and wavefront 0 adds the SW partial sums in order and finishes the
// row, so that several loads per row are in flight at once.
constexpr int kSellWaves = 4;

template <typename T, bool D16, int SW, typename X>
__device__ __forceinline__ T sell_slice_dot(const AmgLevel<T> &L, int64_t slice, int64_t sbase, int w, X xval,
                                            T (*part)[64])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row = slice * 64 + lane;
    T q = 0;
    if (row < L.n) {
        const int64_t base = sbase + lane;
#pragma unroll 4
        for (int j = wv; j < w; j += SW) {
            const int64_t p = base + 64 * (int64_t)j;
            q += L.val[p] * xval(sell_col<T, D16>(L, p, row));
        }
    }
    part[wv][lane] = q;
    __syncthreads();
    T t = part[0][lane];
#pragma unroll
    for (int v = 1; v < SW; ++v) t += part[v][lane];
    return t;
}

template <typename T, bool D16, int SW>
__global__ __launch_bounds__(64 * SW) void k_amg_cheb_sell(AmgLevel<T> L, T *__restrict__ x,
                                                            const T *__restrict__ dcur, T *__restrict__ dnext,
                                                            const double *lam, double ratio, int step,
                                                            const int32_t *done)
{
    __shared__ T part[SW][64];
    const int64_t slice = xcd_block();
    const int64_t sbase = L.soff[slice];
    const int sw = L.swid[slice];
    if (done_with(done, sw + (int32_t)sbase)) return;
    const T q =
        sell_slice_dot<T, D16, SW>(L, slice, sbase, sw, [&](int32_t c) { return dcur[c]; }, part);
    const int64_t row = slice * 64 + (threadIdx.x & 63);
    if (threadIdx.x >= 64 || row >= L.n) return;
    T theta, a, b;
    cheb_coef_t(*lam, ratio, step, theta, a, b);
    const T r = L.res[row] - q;
    L.res[row] = (T)r;
    const T dn = a * dcur[row] + b * L.dinv[row] * r;
    dnext[row] = (T)dn;
    x[row] = (T)(x[row] + dn);
}

template <typename T, bool D16, int SW>
__global__ __launch_bounds__(64 * SW) void k_amg_resid_sell(AmgLevel<T> L, const T *__restrict__ x,
                                                             const int32_t *done)
{
    __shared__ T part[SW][64];
    const int64_t slice = xcd_block();
    const int64_t sbase = L.soff[slice];
    const int sw = L.swid[slice];
    if (done_with(done, sw + (int32_t)sbase)) return;
    const T q = sell_slice_dot<T, D16, SW>(L, slice, sbase, sw, [&](int32_t c) { return x[c]; }, part);
    const int64_t row = slice * 64 + (threadIdx.x & 63);
    if (threadIdx.x >= 64 || row >= L.n) return;
    L.res[row] = (T)(L.r[row] - q);
}

template <typename T, bool D16, int SW>
__global__ __launch_bounds__(64 * SW) void k_amg_post0_sell(AmgLevel<T> L, const T *__restrict__ e,
                                                             const double *lam, double ratio, const int32_t *done)
{
    __shared__ T part[SW][64];
    const int64_t slice = xcd_block();
    const int64_t sbase = L.soff[slice];
    const int sw = L.swid[slice];
    if (done_with(done, sw + (int32_t)sbase)) return;
    const T *x0 = L.x0;
    const int32_t *agg = L.agg;
    const T q = sell_slice_dot<T, D16, SW>(
        L, slice, sbase, sw, [&](int32_t c) { return x0[c] + e[agg[c]]; }, part);
    const int64_t row = slice * 64 + (threadIdx.x & 63);
    if (threadIdx.x >= 64 || row >= L.n) return;
    T theta, a, b;
    cheb_coef_t(*lam, ratio, 0, theta, a, b);
    const T r = L.r[row] - q;
    const T d = L.dinv[row] * r / theta;
    L.res[row] = (T)r;
    L.d0[row] = (T)d;
    L.x1[row] = (T)(L.x0[row] + e[L.agg[row]] + d);
}

// The same with the corrected iterate xp = x0 + P e already formed by the
// coarser level's last pass.
template <typename T, bool D16, int SW>
__global__ __launch_bounds__(64 * SW) void k_amg_post0_sell_xp(AmgLevel<T> L, const T *__restrict__ xp,
                                                               const double *lam, double ratio, const int32_t *done)
{
    __shared__ T part[SW][64];
    const int64_t slice = xcd_block();
    const int64_t sbase = L.soff[slice];
    const int sw = L.swid[slice];
    if (done_with(done, sw + (int32_t)sbase)) return;
    const T q =
        sell_slice_dot<T, D16, SW>(L, slice, sbase, sw, [&](int32_t c) { return xp[c]; }, part);
    const int64_t row = slice * 64 + (threadIdx.x & 63);
    if (threadIdx.x >= 64 || row >= L.n) return;
    T theta, a, b;
    cheb_coef_t(*lam, ratio, 0, theta, a, b);
    const T r = L.r[row] - q;
    const T d = L.dinv[row] * r / theta;
    L.res[row] = (T)r;
    L.d0[row] = (T)d;
    L.x1[row] = (T)(xp[row] + d);
}

// ================================================================== one-workgroup coarse cycle

// The levels from `first` down to the dense one, cycled by one workgroup out of
// LDS: the same operations as the level kernels above (restriction and first
// Chebyshev step, Chebyshev steps, residual, coarse correction with the first
// post-smoothing step, dense solve), each a pass over the rows with a
// lane group per row, separated by workgroup barriers instead of launches.
template <typename T>
struct TailArgs {
    TailLayout lay;
    const unsigned char *img;
    const double *lam;
    double ratio;
    int degree, cycle;
    const T *fres;                       // residual of level first - 1 (global)
    const int32_t *fmptr, *fmem;         // its member lists (global; the image's copy when it has one)
    T *out;                              // result of level first (global)
    const int32_t *done;
    int32_t basis;                       // 1: workgroup j cycles the unit vector e_j into out + j n
};

template <typename T>
__device__ __forceinline__ T *lds_v(unsigned char *lds, int32_t o)
{
    return reinterpret_cast<T *>(lds + o);
}
__device__ __forceinline__ int32_t *lds_i(unsigned char *lds, int32_t o)
{
    return reinterpret_cast<int32_t *>(lds + o);
}

template <typename S>
__device__ __forceinline__ S lane_sum(S v, int lanes)
{
    for (int off = lanes >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, lanes);
    return v;
}

// sum_k val[k] x[col[k]] over the lane's share of row `row`
template <typename T>
__device__ __forceinline__ T tail_rowdot(const int32_t *rowptr, const int32_t *col, const T *val, const T *x, int row,
                                         int lane, int lanes)
{
    T q = 0;
    for (int32_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += lanes) q += val[k] * x[col[k]];
    return lane_sum(q, lanes);
}

// level start from the global residual of the finer level (its member lists in
// LDS, the residual gathered from global memory): r = restriction,
// x0 = d0 = dinv r / theta, res = r (members gathered eight at a time per lane)
template <typename T>
__device__ __forceinline__ void tail_pre_global(const TailArgs<T> &A, const TailLevelLds &L, unsigned char *lds,
                                                double lam)
{
    const int lanes = L.lanes, lane = threadIdx.x & (lanes - 1);
    T *r = lds_v<T>(lds, L.o_r), *res = lds_v<T>(lds, L.o_res), *x0 = lds_v<T>(lds, L.o_x0),
      *d0 = lds_v<T>(lds, L.o_d0);
    const T *dinv = lds_v<T>(lds, L.o_dinv);
    T theta, a, b;
    cheb_coef_t(lam, A.ratio, 0, theta, a, b);
    if (A.basis) {
        // tabulating the cycle's operator: the restricted residual is e_j, j the workgroup
        for (int i = threadIdx.x; i < L.n; i += kTailThreads) {
            const T s = i == (int)blockIdx.x ? T(1) : T(0);
            const T x = dinv[i] * s / theta;
            r[i] = s;
            res[i] = s;
            x0[i] = x;
            d0[i] = x;
        }
        return;
    }
    const bool in_lds = A.lay.o_fmem >= 0;
    const int32_t *fmptr = in_lds ? lds_i(lds, A.lay.o_fmptr) : A.fmptr;
    const int32_t *fmem = in_lds ? lds_i(lds, A.lay.o_fmem) : A.fmem;
    if (A.lay.o_fstage >= 0) {
        // the finer residual gathered in member order by all threads at once
        // (eight loads each in flight), then each row sums a contiguous range
        T *stage = lds_v<T>(lds, A.lay.o_fstage);
        const int32_t nf = fmptr[L.n];
        for (int32_t q0 = 0; q0 < nf; q0 += 8 * kTailThreads) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t q = q0 + u * kTailThreads + (int32_t)threadIdx.x;
                v[u] = q < nf ? A.fres[fmem[q]] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t q = q0 + u * kTailThreads + (int32_t)threadIdx.x;
                if (q < nf) stage[q] = v[u];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x / lanes; i < L.n; i += kTailThreads / lanes) {
            T s = 0;
            for (int32_t q = fmptr[i] + lane; q < fmptr[i + 1]; q += lanes) s += stage[q];
            s = lane_sum(s, lanes);
            if (lane == 0) {
                const T x = (T)(dinv[i] * s / theta);
                r[i] = (T)s;
                res[i] = (T)s;
                x0[i] = x;
                d0[i] = x;
            }
        }
        return;
    }
    for (int i = threadIdx.x / lanes; i < L.n; i += kTailThreads / lanes) {
        const int32_t q0 = fmptr[i], q1 = fmptr[i + 1];
        T s = 0;
        for (int32_t q = q0 + lane; q < q1; q += 8 * lanes) {
            int32_t idx[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) idx[u] = q + u * lanes < q1 ? fmem[q + u * lanes] : -1;
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = idx[u] >= 0 ? A.fres[idx[u]] : T(0);
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        s = lane_sum(s, lanes);
        if (lane == 0) {
            const T x = (T)(dinv[i] * s / theta);
            r[i] = (T)s;
            res[i] = (T)s;
            x0[i] = x;
            d0[i] = x;
        }
    }
}

// the same from the finer level's residual in LDS
template <typename T>
__device__ __forceinline__ void tail_pre_lds(const TailArgs<T> &A, const TailLevelLds &F, const TailLevelLds &L,
                                             unsigned char *lds, double lam)
{
    const int lanes = L.lanes, lane = threadIdx.x & (lanes - 1);
    const T *fres = lds_v<T>(lds, F.o_res);
    const int32_t *mptr = lds_i(lds, F.o_mptr), *mem = lds_i(lds, F.o_mem);
    T *r = lds_v<T>(lds, L.o_r), *res = lds_v<T>(lds, L.o_res), *x0 = lds_v<T>(lds, L.o_x0),
      *d0 = lds_v<T>(lds, L.o_d0);
    const T *dinv = lds_v<T>(lds, L.o_dinv);
    T theta, a, b;
    cheb_coef_t(lam, A.ratio, 0, theta, a, b);
    for (int i = threadIdx.x / lanes; i < L.n; i += kTailThreads / lanes) {
        T s = 0;
        for (int32_t q = mptr[i] + lane; q < mptr[i + 1]; q += lanes) s += fres[mem[q]];
        s = lane_sum(s, lanes);
        if (lane == 0) {
            const T x = (T)(dinv[i] * s / theta);
            r[i] = (T)s;
            res[i] = (T)s;
            x0[i] = x;
            d0[i] = x;
        }
    }
}

// Chebyshev step: res -= A dc, dn = a dc + b dinv res, x += dn
template <typename T>
__device__ __forceinline__ void tail_cheb(const TailArgs<T> &A, const TailLevelLds &L, unsigned char *lds, T *x,
                                          const T *dc, T *dn, double lam, int step)
{
    const int lanes = L.lanes, lane = threadIdx.x & (lanes - 1);
    const int32_t *rowptr = lds_i(lds, L.o_rowptr), *col = lds_i(lds, L.o_col);
    const T *val = lds_v<T>(lds, L.o_val), *dinv = lds_v<T>(lds, L.o_dinv);
    T *res = lds_v<T>(lds, L.o_res);
    T theta, a, b;
    cheb_coef_t(lam, A.ratio, step, theta, a, b);
    for (int row = threadIdx.x / lanes; row < L.n; row += kTailThreads / lanes) {
        const T q = tail_rowdot(rowptr, col, val, dc, row, lane, lanes);
        if (lane == 0) {
            const T rr = res[row] - q;
            res[row] = (T)rr;
            const T d = a * dc[row] + b * dinv[row] * rr;
            dn[row] = (T)d;
            x[row] = (T)(x[row] + d);
        }
    }
}

// res = r - A x
template <typename T>
__device__ __forceinline__ void tail_resid(const TailLevelLds &L, unsigned char *lds, const T *x)
{
    const int lanes = L.lanes, lane = threadIdx.x & (lanes - 1);
    const int32_t *rowptr = lds_i(lds, L.o_rowptr), *col = lds_i(lds, L.o_col);
    const T *val = lds_v<T>(lds, L.o_val), *r = lds_v<T>(lds, L.o_r);
    T *res = lds_v<T>(lds, L.o_res);
    for (int row = threadIdx.x / lanes; row < L.n; row += kTailThreads / lanes) {
        const T q = tail_rowdot(rowptr, col, val, x, row, lane, lanes);
        if (lane == 0) res[row] = (T)(r[row] - q);
    }
}

// y = xa + P e, res = r - A y, d0 = dinv res / theta, xb = y + d0
template <typename T>
__device__ __forceinline__ void tail_post0(const TailArgs<T> &A, const TailLevelLds &L, unsigned char *lds,
                                           const T *xa, T *xb, const T *e, double lam)
{
    const int lanes = L.lanes, lane = threadIdx.x & (lanes - 1);
    const int32_t *rowptr = lds_i(lds, L.o_rowptr), *col = lds_i(lds, L.o_col), *agg = lds_i(lds, L.o_agg);
    const T *val = lds_v<T>(lds, L.o_val), *dinv = lds_v<T>(lds, L.o_dinv), *r = lds_v<T>(lds, L.o_r);
    T *res = lds_v<T>(lds, L.o_res), *d0 = lds_v<T>(lds, L.o_d0);
    T theta, a, b;
    cheb_coef_t(lam, A.ratio, 0, theta, a, b);
    for (int row = threadIdx.x / lanes; row < L.n; row += kTailThreads / lanes) {
        T q = 0;
        for (int32_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += lanes) {
            const int32_t j = col[k];
            q += val[k] * (xa[j] + e[agg[j]]);
        }
        q = lane_sum(q, lanes);
        if (lane == 0) {
            const T rr = r[row] - q;
            const T d = dinv[row] * rr / theta;
            res[row] = (T)rr;
            d0[row] = (T)d;
            xb[row] = (T)(xa[row] + e[agg[row]] + d);
        }
    }
}

// dense coarsest solve: rc = restriction of the finer level's residual, xc = A^{-1} rc
template <typename T>
__device__ __forceinline__ T *tail_dense(const TailArgs<T> &A, const TailLevelLds &F, unsigned char *lds)
{
    const int nc = A.lay.nc;
    const T *fres = lds_v<T>(lds, F.o_res);
    const int32_t *mptr = lds_i(lds, F.o_mptr), *mem = lds_i(lds, F.o_mem);
    double *rc = lds_v<double>(lds, A.lay.o_rc);
    const double *aug = lds_v<double>(lds, A.lay.o_dense);
    T *xc = lds_v<T>(lds, A.lay.o_xc);
    // restriction: sixteen lanes per coarse row
    const int lanes = 16, lane = threadIdx.x & 15;
    for (int c = threadIdx.x / lanes; c < nc; c += kTailThreads / lanes) {
        double s = 0;
        for (int32_t q = mptr[c] + lane; q < mptr[c + 1]; q += lanes) s += (double)fres[mem[q]];
        s = lane_sum(s, lanes);
        if (lane == 0) rc[c] = s;
    }
    __syncthreads();
    for (int row = threadIdx.x / lanes; row < nc; row += kTailThreads / lanes) {
        double s = 0;
        for (int c = lane; c < nc; c += lanes) s += aug[(int64_t)row * 2 * nc + nc + c] * rc[c];
        s = lane_sum(s, lanes);
        if (lane == 0) xc[row] = (T)s;
    }
    __syncthreads();
    return xc;
}

// One visit of level first + D (the dense level when first + D == nlev); returns
// where the level's result lies in LDS.
template <typename T, int D>
__device__ __forceinline__ T *tail_visit(const TailArgs<T> &A, unsigned char *lds)
{
    const TailLayout &Y = A.lay;
    if constexpr (D > 0) {
        if (Y.first + D == Y.nlev) return tail_dense(A, Y.lv[D - 1], lds);
    }
    if constexpr (D < kTailDepth) {
        const TailLevelLds &L = Y.lv[D];
        const double lam = A.lam[Y.first + D];
        if constexpr (D == 0)
            tail_pre_global(A, L, lds, lam);
        else
            tail_pre_lds(A, Y.lv[D - 1], L, lds, lam);
        __syncthreads();
        T *d0 = lds_v<T>(lds, L.o_d0), *d1 = lds_v<T>(lds, L.o_d1);
        T *dc = d0, *dn = d1;
        T *xa = lds_v<T>(lds, L.o_x0), *xb = lds_v<T>(lds, L.o_x1);
        for (int i = 1; i < A.degree; ++i) {
            tail_cheb(A, L, lds, xa, dc, dn, lam, i);
            __syncthreads();
            T *t = dc;
            dc = dn;
            dn = t;
        }
        for (int c = 0; c < A.cycle; ++c) {
            tail_resid(L, lds, xa);
            __syncthreads();
            const T *e = tail_visit<T, D + 1>(A, lds);
            tail_post0(A, L, lds, xa, xb, e, lam);
            __syncthreads();
            dc = d0;
            dn = d1;
            for (int i = 1; i < A.degree; ++i) {
                tail_cheb(A, L, lds, xb, dc, dn, lam, i);
                __syncthreads();
                T *t = dc;
                dc = dn;
                dn = t;
            }
            if (c + 1 < A.cycle) {
                T *t = xa;
                xa = xb;
                xb = t;
            }
        }
        return xb;
    }
    return nullptr;   // not reached: the host limits the depth to kTailDepth smoothed levels
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_amg_tail(TailArgs<T> A)
{
    if (A.done && *A.done) return;
    extern __shared__ __align__(16) unsigned char lds[];
    // the image, 16-byte words, four per thread in flight
    const int nw = A.lay.img_bytes >> 4;
    const uint4 *src = reinterpret_cast<const uint4 *>(A.img);
    uint4 *dst = reinterpret_cast<uint4 *>(lds);
    for (int b0 = 0; b0 < nw; b0 += 8 * kTailThreads) {
        const int w = b0 + (int)threadIdx.x;
        // loads at clamped (in-bounds) indices, stores only where in range
        const uint4 v0 = src[min(w, nw - 1)], v1 = src[min(w + kTailThreads, nw - 1)],
                    v2 = src[min(w + 2 * kTailThreads, nw - 1)], v3 = src[min(w + 3 * kTailThreads, nw - 1)],
                    v4 = src[min(w + 4 * kTailThreads, nw - 1)], v5 = src[min(w + 5 * kTailThreads, nw - 1)],
                    v6 = src[min(w + 6 * kTailThreads, nw - 1)], v7 = src[min(w + 7 * kTailThreads, nw - 1)];
        if (w < nw) dst[w] = v0;
        if (w + kTailThreads < nw) dst[w + kTailThreads] = v1;
        if (w + 2 * kTailThreads < nw) dst[w + 2 * kTailThreads] = v2;
        if (w + 3 * kTailThreads < nw) dst[w + 3 * kTailThreads] = v3;
        if (w + 4 * kTailThreads < nw) dst[w + 4 * kTailThreads] = v4;
        if (w + 5 * kTailThreads < nw) dst[w + 5 * kTailThreads] = v5;
        if (w + 6 * kTailThreads < nw) dst[w + 6 * kTailThreads] = v6;
        if (w + 7 * kTailThreads < nw) dst[w + 7 * kTailThreads] = v7;
    }
    __syncthreads();
    const T *x = tail_visit<T, 0>(A, lds);
    const int n = A.lay.lv[0].n;
    T *out = A.basis ? A.out + (int64_t)blockIdx.x * n : A.out;
    for (int i = threadIdx.x; i < n; i += kTailThreads) out[i] = x[i];
}

// One visit of the one-workgroup levels through their tabulated operator, in
// two launches.  k_tail_restrict: rc = the finer residual restricted onto the n
// rows of level first (LPR lanes per row, each summing every LPR-th member in
// list order, then a fixed butterfly).  k_tail_apply: every workgroup reads rc
// into LDS and its 64 rows take out_i = sum_j op[j][i] rc_j, the four
// wavefronts summing every fourth column and adding their partial sums in order.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_tail_restrict(int n, const T *__restrict__ fres,
                                                       const int32_t *__restrict__ fmptr,
                                                       const int32_t *__restrict__ fmem, T *__restrict__ rc,
                                                       const int32_t *done)
{
    const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) / LPR);
    const int lane = threadIdx.x % LPR;
    if (i >= n) return;
    const int32_t beg = fmptr[i], end = fmptr[i + 1];
    if (done_with(done, end)) return;
    T s = 0;
    for (int32_t q = beg + lane; q < end; q += LPR) s += fres[fmem[q]];
    s = group_sum<T, LPR>(s);
    if (lane == 0) rc[i] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_tail_apply(int n, const T *__restrict__ rcg, const T *__restrict__ op,
                                                    T *__restrict__ out, const int32_t *done)
{
    if (done && *done) return;
    __shared__ T rc[kTailMaxRows];
    __shared__ T part[4][64];
    for (int i = threadIdx.x; i < n; i += 256) rc[i] = rcg[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    T acc = 0;
    if (i < n) {
#pragma unroll 8
        for (int j = wv; j < n; j += 4) acc += op[(int64_t)j * n + i] * rc[j];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && i < n) out[i] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

template <typename T>
lx_status amg_tail_prepare(int lds_bytes)
{
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_amg_tail<T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes) != hipSuccess)
        return fail(LX_EDEVICE, "cannot reserve %d bytes of LDS for the coarse AMG cycle", lds_bytes);
    return LX_OK;
}
template lx_status amg_tail_prepare<double>(int);
template lx_status amg_tail_prepare<float>(int);

// ================================================================== launchers

// Sliced-ELL passes come in two forms, 16-bit column offsets or 32-bit columns; one workgroup per slice.
#define LX_SELL_LAUNCH(LV, KERNEL, GRID, ...)                                                                   \
    do {                                                                                                      \
        if ((LV).sdel)                                                                                        \
            hipLaunchKernelGGL((KERNEL<T, true, kSellWaves>), GRID, dim3(64 * kSellWaves), 0, s, __VA_ARGS__);  \
        else                                                                                                  \
            hipLaunchKernelGGL((KERNEL<T, false, kSellWaves>), GRID, dim3(64 * kSellWaves), 0, s, __VA_ARGS__); \
    } while (0)

static unsigned rows_grid(int64_t n, int lpr) { return (unsigned)((n * lpr + 255) / 256); }
static unsigned flat_grid(int64_t n) { return (unsigned)((n + 255) / 256); }

// Lanes per block row of the velocity-block passes: 8 for the P1-P1 vertex
// pattern (about 15 blocks a row), 16 for denser patterns such as P2-P1's
// (about 28); LXNS_LPR (4, 8, 16 or 32) overrides.
static int block_lpr(const RowPattern &P)
{
    static const int env = [] {
        const char *e = getenv("LXNS_LPR");
        const int x = e ? atoi(e) : 0;
        return (x == 4 || x == 8 || x == 16 || x == 32) ? x : 0;
    }();
    static_assert(kMaxRowLanes >= 32, "Amg::partial is sized for kMaxRowLanes lanes per row");
    if (env) return env;
    return P.nblk >= 20 * P.nv ? 16 : 8;
}

#define LX_LPR_SWITCH(lpr, CALL) \
    switch (lpr) {               \
    case 4: {                    \
        constexpr int LP = 4;    \
        CALL;                    \
    } break;                     \
    case 8: {                    \
        constexpr int LP = 8;    \
        CALL;                    \
    } break;                     \
    case 32: {                   \
        constexpr int LP = 32;   \
        CALL;                    \
    } break;                     \
    default: {                   \
        constexpr int LP = 16;   \
        CALL;                    \
    } break;                     \
    }

template <typename T>
void launch_amg_setup(const SimpleView<T> &V, const T *Finv, const T *Dinv, Amg<T> &A, hipStream_t s)
{
    const RowPattern &P = V.Fp;
    const T *val = V.F;
    AmgLevel<T> &L0 = A.L[0];
    const dim3 gsf((unsigned)((V.np + kSfWaves - 1) / kSfWaves)), bsf(64 * kSfWaves);
    if (V.nu == V.np)
        hipLaunchKernelGGL((k_schur_form<T, 48, 384>), gsf, bsf, 0, s, V, Dinv, L0.rowptr, L0.col, L0.val, L0.soff);
    else
        hipLaunchKernelGGL((k_schur_form<T, 96, 640>), gsf, bsf, 0, s, V, Dinv, L0.rowptr, L0.col, L0.val, L0.soff);
    for (int l = 0; l < A.nlev; ++l) {
        AmgLevel<T> &L = A.L[l];
        unsigned g;
        if (L.soff) {
            g = flat_grid(L.n);
            hipLaunchKernelGGL((k_amg_rowinfo_sell<T>), dim3(g), dim3(256), 0, s, L, A.partial);
        } else {
            g = rows_grid(L.n, L.lpr);
            LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_rowinfo<T, LP>), dim3(g), dim3(256), 0, s, L.n, L.rowptr,
                                                    L.diag, L.val, L.dinv, A.partial));
        }
        hipLaunchKernelGGL(k_max_fin, dim3(1), dim3(256), 0, s, (int)g, A.partial, &A.lam[l]);
        AmgLevel<T> &C = A.L[l + 1];
        hipLaunchKernelGGL((k_amg_coarsen<T, 16>), dim3(rows_grid(C.nnz, 16)), dim3(256), 0, s, C.nnz, L.cptr, L.cidx,
                           L.val, C.val);
    }
    const AmgLevel<T> &D = A.L[A.nlev];
    hipLaunchKernelGGL(k_dense_init, dim3(flat_grid(2 * A.nc * A.nc)), dim3(256), 0, s, A.nc, A.dense);
    hipLaunchKernelGGL((k_dense_scatter<T>), dim3(flat_grid(D.nnz)), dim3(256), 0, s, D.nnz, A.nc, A.crow, D.col,
                       D.val, A.dense);
    if (A.nc <= kGjLdsMax)
        hipLaunchKernelGGL(k_dense_gj_lds, dim3(1), dim3(1024), 0, s, (int)A.nc, A.dense);
    else
        hipLaunchKernelGGL(k_dense_gj, dim3(1), dim3(1024), 0, s, (int)A.nc, A.dense);
    if (A.f_degree > 1) {
        // power iterations alternate fv -> fd1 -> fv; an even count ends in fv
        const int iters = A.f_warm ? A.f_pow_iters : A.f_pow_first;
        const int lpr = block_lpr(P);
        for (int it = 0; it < iters; ++it) {
            const bool even = (it % 2) == 0;
            const T *vin = (it == 0 && !A.f_warm) ? nullptr : (even ? A.fv : A.fd1);
            T *vout = even ? A.fd1 : A.fv;
            const int sin = even ? kNormA : kNormB, sout = even ? kNormB : kNormA;
            const double fac = (it == iters - 1) ? A.f_safety : 0.0;
            const unsigned g = rows_grid(P.nv, lpr);
            LX_LPR_SWITCH(lpr, hipLaunchKernelGGL((k_fpow<T, LP>), dim3(g), dim3(256), 0, s, P, val, Finv, vin, vout,
                                                  A.lam, sin, A.partial));
            hipLaunchKernelGGL(k_fpow_fin, dim3(1), dim3(256), 0, s, (int)g, A.partial, A.lam, sout, fac);
        }
        A.f_warm = true;
    }
    if (A.tail_op) {
        // the operator of the one-workgroup cycle: one workgroup per unit vector
        const AmgLevel<T> &F = A.L[A.tail.first - 1];
        TailArgs<T> t;
        t.lay = A.tail;
        t.img = A.tail_img;
        t.lam = A.lam;
        t.ratio = A.ratio;
        t.degree = A.degree;
        t.cycle = A.cycle_coarse;
        t.fres = F.res;
        t.fmptr = F.mptr;
        t.fmem = F.mem;
        t.out = A.tail_op;
        t.done = nullptr;
        t.basis = 1;
        hipLaunchKernelGGL((k_amg_tail<T>), dim3((unsigned)A.tail.lv[0].n), dim3(kTailThreads),
                           (size_t)A.tail.lds_bytes, s, t);
    }
}
template void launch_amg_setup<double>(const SimpleView<double> &, const double *, const double *, Amg<double> &,
                                       hipStream_t);
template void launch_amg_setup<float>(const SimpleView<float> &, const float *, const float *, Amg<float> &,
                                      hipStream_t);

template <typename T>
// prolong (optional): where the level's last pass also writes the finer level's
// corrected iterate fx0 + P x (returns true if it did).
static bool vcycle(Amg<T> &A, int l, const int32_t *done, hipStream_t s, T *prolong = nullptr,
                   const T *fx0 = nullptr)
{
    if (A.tail.first > 0 && l == A.tail.first) {
        const AmgLevel<T> &F = A.L[l - 1];
        TailArgs<T> t;
        t.lay = A.tail;
        t.img = A.tail_img;
        t.lam = A.lam;
        t.ratio = A.ratio;
        t.degree = A.degree;
        t.cycle = A.cycle_coarse;
        t.fres = F.res;
        t.fmptr = F.mptr;
        t.fmem = F.mem;
        t.out = A.L[l].x1;
        t.done = done;
        t.basis = 0;
        if (A.tail_op) {
            const int n = A.tail.lv[0].n;
            hipLaunchKernelGGL((k_tail_restrict<T, 16>), dim3((unsigned)((n * 16 + 255) / 256)), dim3(256), 0, s, n,
                               F.res, F.mptr, F.mem, A.tail_rc, done);
            hipLaunchKernelGGL((k_tail_apply<T>), dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, n, A.tail_rc,
                               A.tail_op, A.L[l].x1, done);
        } else {
            hipLaunchKernelGGL((k_amg_tail<T>), dim3(1), dim3(kTailThreads), (size_t)A.tail.lds_bytes, s, t);
        }
        return false;
    }
    if (l == A.nlev) {
        const bool fine = l == 0;
        const T *fres = fine ? A.L[0].r : A.L[l - 1].res;
        const int32_t *mptr = fine ? nullptr : A.L[l - 1].mptr, *mem = fine ? nullptr : A.L[l - 1].mem;
        hipLaunchKernelGGL((k_dense_solve<T>), dim3(1), dim3(256), 0, s, (int)A.nc, A.dense, fres, mptr, mem,
                           A.L[l].x1, done);
        return false;
    }
    AmgLevel<T> L = A.L[l];
    const double *lam = &A.lam[l];
    if (l > 0) {
        const AmgLevel<T> &F = A.L[l - 1];
        hipLaunchKernelGGL((k_amg_pre<T, 16>), dim3(rows_grid(L.n, 16)), dim3(256), 0, s, L, F.res, F.mptr, F.mem,
                           lam, A.ratio, done);
    }
    const dim3 gsell((unsigned)((L.n + 63) / 64));
    T *dc = L.d0, *dn = L.d1;
    for (int i = 1; i < A.degree; ++i) {
        if (L.soff)
            LX_SELL_LAUNCH(L, k_amg_cheb_sell, gsell, L, L.x0, dc, dn, lam, A.ratio, i, done);
        else
            LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_cheb<T, LP>), dim3(rows_grid(L.n, LP)), dim3(256), 0, s,
                                                    L, L.x0, dc, dn, lam, A.ratio, i, done));
        std::swap(dc, dn);
    }
    // gamma coarse corrections (1 on the finest level; cycle below it, 2 being a
    // W-cycle; cycle_coarse on the levels small enough for one workgroup's LDS,
    // where a correction costs barriers rather than launches and more of them
    // bring the coarse solve closer to exact), each followed by post-smoothing;
    // the iterate alternates between x0 and x1
    const int gamma = l == 0 ? 1 : l >= A.coarse_from ? A.cycle_coarse : A.cycle;
    bool prolonged = false;
    for (int c = 0; c < gamma; ++c) {
        if (L.soff)
            LX_SELL_LAUNCH(L, k_amg_resid_sell, gsell, L, L.x0, done);
        else
            LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_resid<T, LP>), dim3(rows_grid(L.n, LP)), dim3(256), 0, s,
                                                    L, L.x0, done));
        // a sliced-ELL level takes its corrected iterate from the coarser level's last pass, in d1
        // (free until the post-smoothing Chebyshev step writes it)
        const bool xp = vcycle(A, l + 1, done, s, L.soff ? L.d1 : nullptr, L.x0);
        if (L.soff && xp)
            LX_SELL_LAUNCH(L, k_amg_post0_sell_xp, gsell, L, L.d1, lam, A.ratio, done);
        else if (L.soff)
            LX_SELL_LAUNCH(L, k_amg_post0_sell, gsell, L, A.L[l + 1].x1, lam, A.ratio, done);
        else
            LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_post0<T, LP>), dim3(rows_grid(L.n, LP)), dim3(256), 0, s,
                                                    L, A.L[l + 1].x1, lam, A.ratio, done));
        dc = L.d0;
        dn = L.d1;
        for (int i = 1; i < A.degree; ++i) {
            const bool last = c + 1 == gamma && i + 1 == A.degree;
            if (L.soff)
                LX_SELL_LAUNCH(L, k_amg_cheb_sell, gsell, L, L.x1, dc, dn, lam, A.ratio, i, done);
            else if (last && prolong && fx0 && l > 0) {
                const AmgLevel<T> &F = A.L[l - 1];
                LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_cheb_prolong<T, LP>), dim3(rows_grid(L.n, LP)),
                                                        dim3(256), 0, s, L, L.x1, dc, dn, lam, A.ratio, i, done,
                                                        fx0, prolong, F.mptr, F.mem));
                prolonged = true;
            } else
                LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_cheb<T, LP>), dim3(rows_grid(L.n, LP)), dim3(256), 0,
                                                        s, L, L.x1, dc, dn, lam, A.ratio, i, done));
            std::swap(dc, dn);
        }
        if (c + 1 < gamma) std::swap(L.x0, L.x1);
    }
    // the level's result is read from x1
    A.L[l].x0 = L.x0;
    A.L[l].x1 = L.x1;
    return prolonged;
}

template <typename T>
void launch_simple_amg_apply(const SimpleView<T> &V, const T *Finv, const T *Dinv, Amg<T> &A, const T *r,
                             const double *scale_ptr, T *z, const int32_t *done, hipStream_t s, bool start_done)
{
    const RowPattern &P = V.Fp;
    const T *val = V.F;
    const int lpr = block_lpr(P);
    if (!start_done)
        hipLaunchKernelGGL((k_fz_start<T>), dim3(flat_grid(P.nv)), dim3(256), 0, s, P.nv, Finv, r, scale_ptr, z,
                           A.fr, A.fd0, &A.lam[kLamF], A.f_ratio, A.f_degree, done);
    T *dc = A.fd0, *dn = A.fd1;
    for (int i = 1; i < A.f_degree; ++i) {
        LX_LPR_SWITCH(lpr, hipLaunchKernelGGL((k_fcheb<T, LP>), dim3(rows_grid(P.nv, LP)), dim3(256), 0, s, P, val,
                                              Finv, z, A.fr, dc, dn, &A.lam[kLamF], A.f_ratio, i, done));
        std::swap(dc, dn);
    }
    LX_LPR_SWITCH(lpr, hipLaunchKernelGGL((k_zp_amg<T, LP>), dim3(rows_grid(V.np, LP)), dim3(256), 0, s, V, z,
                                          A.L[0], &A.lam[0], A.ratio, A.nlev > 0 ? 1 : 0, done));
    vcycle(A, 0, done, s);
    LX_LPR_SWITCH(lpr, hipLaunchKernelGGL((k_xu_amg<T, LP>), dim3(rows_grid(V.nu, LP)), dim3(256), 0, s, V, Dinv, z,
                                          A.L[0].x1, done));
}
template void launch_simple_amg_apply<double>(const SimpleView<double> &, const double *, const double *,
                                              Amg<double> &, const double *, const double *, double *,
                                              const int32_t *, hipStream_t, bool);
template void launch_simple_amg_apply<float>(const SimpleView<float> &, const float *, const float *, Amg<float> &,
                                             const float *, const double *, float *, const int32_t *, hipStream_t,
                                             bool);

}  // namespace lx
