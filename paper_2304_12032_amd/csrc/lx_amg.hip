// Device side of the SIMPLE block approximations (Sec. 2.4 names AMG and block
// Jacobi among the block approximations of its SIMPLE preconditioner):
//  * the Schur block S~ = C - B D^{-1} G is formed explicitly each step, and
//    approximated by one cycle of unsmoothed-aggregation multigrid with
//    Chebyshev smoothing on diag(A_l)^{-1} A_l and a dense inverse on the
//    coarsest level;
//  * the velocity block F is approximated by a Chebyshev iteration on
//    F~^{-1} F, F~ its nodal 3x3 diagonal blocks, whose upper bound comes from
//    a few power iterations warm-started from the previous step.
// Row kernels use LPR lanes per row and accumulate in FP64; every apply-phase
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
// of B's row i.  One wavefront per row i, lanes over the entries of the row;
// C_ik and G_jk are found by binary search (sorted columns).  The sum runs over
// B's row in order, so the result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(256) void k_schur_form(SimpleView<T> V, const T *__restrict__ Dinv,
                                                    const int32_t *__restrict__ srow,
                                                    const int32_t *__restrict__ scol, T *__restrict__ sval)
{
    const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= V.np) return;
    const int64_t nu = V.nu;
    const int32_t b0 = V.bptr[i], b1 = V.bptr[i + 1];
    for (int32_t e = srow[i] + lane; e < srow[i + 1]; e += 64) {
        const int32_t k = scol[e];
        const int32_t kc = find_col(V.ccol, V.cptr[i], V.cptr[i + 1], k);
        double acc = kc >= 0 ? (double)V.Cv[kc] : 0.0;
        for (int32_t k1 = b0; k1 < b1; ++k1) {
            const int32_t j = V.bcol[k1];
            const int32_t kg = find_col(V.gcol, V.gptr[j], V.gptr[j + 1], k);
            if (kg < 0) continue;
            acc -= (double)V.Bv[k1] * (double)Dinv[j] * (double)V.Gv[kg] +
                   (double)V.Bv[V.bs + k1] * (double)Dinv[nu + j] * (double)V.Gv[V.gs + kg] +
                   (double)V.Bv[2 * V.bs + k1] * (double)Dinv[2 * nu + j] * (double)V.Gv[2 * V.gs + kg];
        }
        sval[e] = (T)acc;
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
    double s = 0;
    if (row < n)
        for (int32_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += LPR) s += fabs((double)val[k]);
    s = group_sum<double, LPR>(s);
    double g = 0;
    if (row < n && lane == 0) {
        const int32_t dk = diag[row];
        const double a = dk >= 0 ? (double)val[dk] : 0.0;
        const double di = a != 0.0 ? 1.0 / a : 0.0;
        dinv[row] = (T)di;
        g = s * fabs(di);
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
// sum, in a fixed order, of the fine entries listed for it.
template <typename T>
__global__ void k_amg_coarsen(int64_t nnzc, const int32_t *__restrict__ cptr, const int32_t *__restrict__ cidx,
                              const T *__restrict__ fval, T *__restrict__ cval)
{
    const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= nnzc) return;
    double s = 0;
    for (int32_t q = cptr[c]; q < cptr[c + 1]; ++q) s += (double)fval[cidx[q]];
    cval[c] = (T)s;
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
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    const int64_t nb = P.nblk, nv = P.nv;
    using V = typename V4<T>::type;
    const double nin = v ? sqrt(lam[slot_in]) : sqrt(3.0 * (double)nv);
    double t0 = 0, t1 = 0, t2 = 0;
    if (row < nv)
        for (int32_t k = P.rowptr[row] + lane; k < P.rowptr[row + 1]; k += LPR) {
            const int32_t j = P.col[k];
            double x0, x1, x2;
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
            double a[9];
#pragma unroll
            for (int p = 0; p < 9; ++p) a[p] = (double)val[p * nb + k];
            t0 += a[0] * x0 + a[1] * x1 + a[2] * x2;
            t1 += a[3] * x0 + a[4] * x1 + a[5] * x2;
            t2 += a[6] * x0 + a[7] * x1 + a[8] * x2;
        }
    t0 = group_sum<double, LPR>(t0);
    t1 = group_sum<double, LPR>(t1);
    t2 = group_sum<double, LPR>(t2);
    double acc[1] = {0.0};
    if (row < nv && lane == 0) {
        double fi[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) fi[p] = (double)Finv[p * nv + row];
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
    const double sc = scale_ptr ? *scale_ptr : 1.0;
    using V = typename V4<T>::type;
    const V rv = reinterpret_cast<const V *>(r)[i];
    const double r0 = rv.v[0] * sc, r1 = rv.v[1] * sc, r2 = rv.v[2] * sc;
    double fi[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) fi[p] = (double)Finv[p * nv + i];
    double y0 = fi[0] * r0 + fi[1] * r1 + fi[2] * r2;
    double y1 = fi[3] * r0 + fi[4] * r1 + fi[5] * r2;
    double y2 = fi[6] * r0 + fi[7] * r1 + fi[8] * r2;
    V zv;
    if (degree > 1) {
        double theta, a, b;
        cheb_coef(*lamF, ratio, 0, theta, a, b);
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
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int64_t nb = P.nblk, nv = P.nv;
    using V = typename V4<T>::type;
    double t0 = 0, t1 = 0, t2 = 0;
    for (int32_t k = P.rowptr[row] + lane; k < P.rowptr[row + 1]; k += LPR) {
        const V xv = reinterpret_cast<const V *>(dcur)[P.col[k]];
        const double x0 = xv.v[0], x1 = xv.v[1], x2 = xv.v[2];
        double a[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) a[p] = (double)val[p * nb + k];
        t0 += a[0] * x0 + a[1] * x1 + a[2] * x2;
        t1 += a[3] * x0 + a[4] * x1 + a[5] * x2;
        t2 += a[6] * x0 + a[7] * x1 + a[8] * x2;
    }
    t0 = group_sum<double, LPR>(t0);
    t1 = group_sum<double, LPR>(t1);
    t2 = group_sum<double, LPR>(t2);
    if (lane != 0) return;
    double theta, a, b;
    cheb_coef(*lamF, ratio, step, theta, a, b);
    V f = reinterpret_cast<V *>(fr)[row];
    const double e0 = f.v[0] - t0, e1 = f.v[1] - t1, e2 = f.v[2] - t2;
    f.v[0] = (T)e0;
    f.v[1] = (T)e1;
    f.v[2] = (T)e2;
    reinterpret_cast<V *>(fr)[row] = f;
    double fi[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) fi[p] = (double)Finv[p * nv + row];
    const V dc = reinterpret_cast<const V *>(dcur)[row];
    V dn;
    dn.v[0] = (T)(a * dc.v[0] + b * (fi[0] * e0 + fi[1] * e1 + fi[2] * e2));
    dn.v[1] = (T)(a * dc.v[1] + b * (fi[3] * e0 + fi[4] * e1 + fi[5] * e2));
    dn.v[2] = (T)(a * dc.v[2] + b * (fi[6] * e0 + fi[7] * e1 + fi[8] * e2));
    dn.v[3] = T(0);
    reinterpret_cast<V *>(dnext)[row] = dn;
    V zv = reinterpret_cast<V *>(z)[row];
    zv.v[0] = (T)((double)zv.v[0] + dn.v[0]);
    zv.v[1] = (T)((double)zv.v[1] + dn.v[1]);
    zv.v[2] = (T)((double)zv.v[2] + dn.v[2]);
    reinterpret_cast<V *>(z)[row] = zv;
}

// t = z.p - sum_j B_ij z.u_j (z.p holds scale r.p): the right-hand side of the
// Schur solve, stored in L0.r; with smoothed levels also the Chebyshev start
// x0 = d0 = dinv t / theta, res = t.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_zp_amg(SimpleView<T> V, const T *__restrict__ z, AmgLevel<T> L,
                                                const double *lam, double ratio, int smooth, const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= V.np) return;
    using VT = typename V4<T>::type;
    double acc = 0;
    for (int32_t k = V.bptr[row] + lane; k < V.bptr[row + 1]; k += LPR) {
        const VT zj = reinterpret_cast<const VT *>(z)[V.bcol[k]];
        acc += (double)V.Bv[k] * zj.v[0] + (double)V.Bv[V.bs + k] * zj.v[1] + (double)V.Bv[2 * V.bs + k] * zj.v[2];
    }
    acc = group_sum<double, LPR>(acc);
    if (lane != 0) return;
    const double t = (double)z[4 * row + 3] - acc;
    L.r[row] = (T)t;
    if (smooth) {
        double theta, a, b;
        cheb_coef(*lam, ratio, 0, theta, a, b);
        const T x = (T)((double)L.dinv[row] * t / theta);
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
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= V.nu) return;
    const int64_t nu = V.nu;
    double a0 = 0, a1 = 0, a2 = 0;
    for (int32_t k = V.gptr[row] + lane; k < V.gptr[row + 1]; k += LPR) {
        const double pj = p[V.gcol[k]];
        a0 += (double)V.Gv[k] * pj;
        a1 += (double)V.Gv[V.gs + k] * pj;
        a2 += (double)V.Gv[2 * V.gs + k] * pj;
    }
    a0 = group_sum<double, LPR>(a0);
    a1 = group_sum<double, LPR>(a1);
    a2 = group_sum<double, LPR>(a2);
    if (lane != 0) return;
    using VT = typename V4<T>::type;
    VT zv = reinterpret_cast<VT *>(z)[row];
    zv.v[0] = (T)((double)zv.v[0] - (double)Dinv[row] * a0);
    zv.v[1] = (T)((double)zv.v[1] - (double)Dinv[nu + row] * a1);
    zv.v[2] = (T)((double)zv.v[2] - (double)Dinv[2 * nu + row] * a2);
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
    if (done && *done) return;
    const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (i >= L.n) return;
    double s = 0;
    for (int32_t q = mptr[i] + lane; q < mptr[i + 1]; q += LPR) s += (double)fres[mem[q]];
    s = group_sum<double, LPR>(s);
    if (lane != 0) return;
    double theta, a, b;
    cheb_coef(*lam, ratio, 0, theta, a, b);
    const T x = (T)((double)L.dinv[i] * s / theta);
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
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= L.n) return;
    double q = 0;
    for (int32_t k = L.rowptr[row] + lane; k < L.rowptr[row + 1]; k += LPR)
        q += (double)L.val[k] * (double)dcur[L.col[k]];
    q = group_sum<double, LPR>(q);
    if (lane != 0) return;
    double theta, a, b;
    cheb_coef(*lam, ratio, step, theta, a, b);
    const double r = (double)L.res[row] - q;
    L.res[row] = (T)r;
    const double dn = a * (double)dcur[row] + b * (double)L.dinv[row] * r;
    dnext[row] = (T)dn;
    x[row] = (T)((double)x[row] + dn);
}

// res = r - A x
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_resid(AmgLevel<T> L, const T *__restrict__ x, const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= L.n) return;
    double q = 0;
    for (int32_t k = L.rowptr[row] + lane; k < L.rowptr[row + 1]; k += LPR)
        q += (double)L.val[k] * (double)x[L.col[k]];
    q = group_sum<double, LPR>(q);
    if (lane == 0) L.res[row] = (T)((double)L.r[row] - q);
}

// Coarse correction and first post-smoothing step: y = x0 + P e,
// res = r - A y, d0 = dinv res / theta, x1 = y + d0.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_amg_post0(AmgLevel<T> L, const T *__restrict__ e, const double *lam,
                                                   double ratio, const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= L.n) return;
    double q = 0;
    for (int32_t k = L.rowptr[row] + lane; k < L.rowptr[row + 1]; k += LPR) {
        const int32_t j = L.col[k];
        q += (double)L.val[k] * ((double)L.x0[j] + (double)e[L.agg[j]]);
    }
    q = group_sum<double, LPR>(q);
    if (lane != 0) return;
    double theta, a, b;
    cheb_coef(*lam, ratio, 0, theta, a, b);
    const double r = (double)L.r[row] - q;
    const double d = (double)L.dinv[row] * r / theta;
    L.res[row] = (T)r;
    L.d0[row] = (T)d;
    L.x1[row] = (T)((double)L.x0[row] + (double)e[L.agg[row]] + d);
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

// ================================================================== launchers

static unsigned rows_grid(int64_t n, int lpr) { return (unsigned)((n * lpr + 255) / 256); }
static unsigned flat_grid(int64_t n) { return (unsigned)((n + 255) / 256); }

// Lanes per block row of the velocity-block passes (LXNS_LPR overrides, 4/8/16).
static int block_lpr()
{
    static const int v = [] {
        const char *e = getenv("LXNS_LPR");
        const int x = e ? atoi(e) : 8;
        return (x == 4 || x == 8 || x == 16) ? x : 8;
    }();
    return v;
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
    hipLaunchKernelGGL((k_schur_form<T>), dim3(rows_grid(V.np, 64)), dim3(256), 0, s, V, Dinv, L0.rowptr, L0.col,
                       L0.val);
    for (int l = 0; l < A.nlev; ++l) {
        AmgLevel<T> &L = A.L[l];
        const unsigned g = rows_grid(L.n, L.lpr);
        LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_rowinfo<T, LP>), dim3(g), dim3(256), 0, s, L.n, L.rowptr,
                                                L.diag, L.val, L.dinv, A.partial));
        hipLaunchKernelGGL(k_max_fin, dim3(1), dim3(256), 0, s, (int)g, A.partial, &A.lam[l]);
        AmgLevel<T> &C = A.L[l + 1];
        hipLaunchKernelGGL((k_amg_coarsen<T>), dim3(flat_grid(C.nnz)), dim3(256), 0, s, C.nnz, L.cptr, L.cidx, L.val,
                           C.val);
    }
    const AmgLevel<T> &D = A.L[A.nlev];
    hipLaunchKernelGGL(k_dense_init, dim3(flat_grid(2 * A.nc * A.nc)), dim3(256), 0, s, A.nc, A.dense);
    hipLaunchKernelGGL((k_dense_scatter<T>), dim3(flat_grid(D.nnz)), dim3(256), 0, s, D.nnz, A.nc, A.crow, D.col,
                       D.val, A.dense);
    hipLaunchKernelGGL(k_dense_gj, dim3(1), dim3(1024), 0, s, (int)A.nc, A.dense);
    if (A.f_degree > 1) {
        // power iterations alternate fv -> fd1 -> fv; an even count ends in fv
        const int iters = A.f_warm ? A.f_pow_iters : A.f_pow_first;
        const int lpr = block_lpr();
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
}
template void launch_amg_setup<double>(const SimpleView<double> &, const double *, const double *, Amg<double> &,
                                       hipStream_t);
template void launch_amg_setup<float>(const SimpleView<float> &, const float *, const float *, Amg<float> &,
                                      hipStream_t);

template <typename T>
static void vcycle(Amg<T> &A, int l, const int32_t *done, hipStream_t s)
{
    if (l == A.nlev) {
        const bool fine = l == 0;
        const T *fres = fine ? A.L[0].r : A.L[l - 1].res;
        const int32_t *mptr = fine ? nullptr : A.L[l - 1].mptr, *mem = fine ? nullptr : A.L[l - 1].mem;
        hipLaunchKernelGGL((k_dense_solve<T>), dim3(1), dim3(256), 0, s, (int)A.nc, A.dense, fres, mptr, mem,
                           A.L[l].x1, done);
        return;
    }
    AmgLevel<T> L = A.L[l];
    const double *lam = &A.lam[l];
    if (l > 0) {
        const AmgLevel<T> &F = A.L[l - 1];
        hipLaunchKernelGGL((k_amg_pre<T, 16>), dim3(rows_grid(L.n, 16)), dim3(256), 0, s, L, F.res, F.mptr, F.mem,
                           lam, A.ratio, done);
    }
    T *dc = L.d0, *dn = L.d1;
    for (int i = 1; i < A.degree; ++i) {
        LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_cheb<T, LP>), dim3(rows_grid(L.n, LP)), dim3(256), 0, s, L,
                                                L.x0, dc, dn, lam, A.ratio, i, done));
        std::swap(dc, dn);
    }
    // gamma coarse corrections (1: V-cycle, 2: W-cycle below the finest level),
    // each followed by post-smoothing; the iterate alternates between x0 and x1
    const int gamma = l > 0 ? A.cycle : 1;
    for (int c = 0; c < gamma; ++c) {
        LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_resid<T, LP>), dim3(rows_grid(L.n, LP)), dim3(256), 0, s, L,
                                                L.x0, done));
        vcycle(A, l + 1, done, s);
        LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_post0<T, LP>), dim3(rows_grid(L.n, LP)), dim3(256), 0, s, L,
                                                A.L[l + 1].x1, lam, A.ratio, done));
        dc = L.d0;
        dn = L.d1;
        for (int i = 1; i < A.degree; ++i) {
            LX_LPR_SWITCH(L.lpr, hipLaunchKernelGGL((k_amg_cheb<T, LP>), dim3(rows_grid(L.n, LP)), dim3(256), 0, s,
                                                    L, L.x1, dc, dn, lam, A.ratio, i, done));
            std::swap(dc, dn);
        }
        if (c + 1 < gamma) std::swap(L.x0, L.x1);
    }
    // the level's result is read from x1
    A.L[l].x0 = L.x0;
    A.L[l].x1 = L.x1;
}

template <typename T>
void launch_simple_amg_apply(const SimpleView<T> &V, const T *Finv, const T *Dinv, Amg<T> &A, const T *r,
                             const double *scale_ptr, T *z, const int32_t *done, hipStream_t s)
{
    const RowPattern &P = V.Fp;
    const T *val = V.F;
    const int lpr = block_lpr();
    hipLaunchKernelGGL((k_fz_start<T>), dim3(flat_grid(P.nv)), dim3(256), 0, s, P.nv, Finv, r, scale_ptr, z, A.fr,
                       A.fd0, &A.lam[kLamF], A.f_ratio, A.f_degree, done);
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
                                              const int32_t *, hipStream_t);
template void launch_simple_amg_apply<float>(const SimpleView<float> &, const float *, const float *, Amg<float> &,
                                             const float *, const double *, float *, const int32_t *, hipStream_t);

}  // namespace lx
