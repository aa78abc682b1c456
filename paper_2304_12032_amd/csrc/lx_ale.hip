// ALE mesh motion (paper Sec. 2.1.1 and the discrete mesh velocity of Sec. 2.3):
// harmonic extension of the boundary displacement on the reference mesh with
// a P1 Laplacian (stiffening alpha = 1), solved by Jacobi-preconditioned CG
// for the three components at once; then x^{n+1} = x^ + d^{n+1} and
// u_ALE = (alpha d^{n+1} - sum_l beta_l d^{n-l}) / dt at the vertices.
//
// Two ways to give the boundary data:
//  * d^ = law(t) D^ with a fixed shape D^: the extension operator is linear,
//    so the extension of D^ is computed once per shape and scaled by law(t)
//    every step (identical to solving the lifting problem with the scaled
//    data); setting a new shape triggers a new solve;
//  * nodal boundary displacements set for each step: the lifting problem is
//    solved every step, by CG started from the extrapolation of the
//    displacement history to t^{n+1} (the step's EXT weights).
#include <cmath>
#include <vector>

#include "lx_device.h"
#include "lx_sim.h"

namespace lx {

struct CgState {
    double rz[3], alpha[3], beta[3], rr[3], tol2[3];
    int32_t done, iters;
    uint32_t counter, pad;
};

// y = L x for [nv][3] vectors, scalar values per block slot
template <int LPR>
__device__ inline void lap_row(int64_t row, int lane, const int32_t *rowptr, const int32_t *col, const double *L,
                               const double *x, double &y0, double &y1, double &y2)
{
    y0 = y1 = y2 = 0;
    for (int32_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += LPR) {
        const double a = L[k];
        const double *xj = x + 3 * (int64_t)col[k];
        y0 += a * xj[0];
        y1 += a * xj[1];
        y2 += a * xj[2];
    }
    y0 = group_sum<double, LPR>(y0);
    y1 = group_sum<double, LPR>(y1);
    y2 = group_sum<double, LPR>(y2);
}

constexpr int kAleLPR = 16;

// rhs: boundary rows d_B; interior rows -sum_{j in B} Lfull_ij d_B(j).  d0: initial
// guess with boundary rows set.
__global__ __launch_bounds__(256) void k_ale_rhs(int64_t nv, const int32_t *rowptr, const int32_t *col,
                                                 const double *Lfull, const int32_t *mark, const double *shape,
                                                 double scale, double *rhs, double *d0)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / kAleLPR;
    const int lane = threadIdx.x % kAleLPR;
    if (row >= nv) return;
    double y[3] = {0, 0, 0};
    for (int32_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += kAleLPR) {
        const int64_t j = col[k];
        if (mark[j])
            for (int c = 0; c < 3; ++c) y[c] += Lfull[k] * scale * shape[3 * j + c];
    }
    for (int c = 0; c < 3; ++c) y[c] = group_sum<double, kAleLPR>(y[c]);
    if (lane == 0) {
        for (int c = 0; c < 3; ++c) {
            if (mark[row]) {
                rhs[3 * row + c] = scale * shape[3 * row + c];
                d0[3 * row + c] = scale * shape[3 * row + c];
            } else {
                rhs[3 * row + c] = -y[c];
            }
        }
    }
}

// r = rhs - L d; z = Dinv r; p = z; rz, rr, tolerance
__global__ __launch_bounds__(256) void k_cg_init(int64_t nv, const int32_t *rowptr, const int32_t *col,
                                                 const double *L, const double *dinv, const double *rhs,
                                                 const double *d, double *r, double *z, double *p, CgState *st,
                                                 double *partial, double rtol)
{
    __shared__ double lds[4 * 9];
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / kAleLPR;
    const int lane = threadIdx.x % kAleLPR;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (row < nv) {
        double y[3];
        lap_row<kAleLPR>(row, lane, rowptr, col, L, d, y[0], y[1], y[2]);
        if (lane == 0)
            for (int c = 0; c < 3; ++c) {
                double rc = rhs[3 * row + c] - y[c];
                double zc = dinv[row] * rc;
                r[3 * row + c] = rc;
                z[3 * row + c] = zc;
                p[3 * row + c] = zc;
                acc[c] = rc * zc;
                acc[3 + c] = rc * rc;
                acc[6 + c] = rhs[3 * row + c] * rhs[3 * row + c];
            }
    }
    block_sum<9>(acc, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < 9; ++j) partial[(int64_t)blockIdx.x * 9 + j] = acc[j];
    if (!arrive_last(&st->counter)) return;
    double tot[9];
    reduce_partials<9>(partial, gridDim.x, 9, tot, lds);
    if (threadIdx.x == 0) {
        bool done = true;
        for (int c = 0; c < 3; ++c) {
            st->rz[c] = tot[c];
            st->rr[c] = tot[3 + c];
            st->tol2[c] = rtol * rtol * tot[6 + c];
            if (st->rr[c] > st->tol2[c]) done = false;
        }
        st->done = done ? 1 : 0;
        st->iters = 0;
        st->counter = 0;
    }
}

// q = L p, alpha = rz / (p.q)
__global__ __launch_bounds__(256) void k_cg_ap(int64_t nv, const int32_t *rowptr, const int32_t *col,
                                               const double *L, const double *p, double *q, CgState *st,
                                               double *partial)
{
    if (st->done) return;
    __shared__ double lds[4 * 3];
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / kAleLPR;
    const int lane = threadIdx.x % kAleLPR;
    double acc[3] = {0, 0, 0};
    if (row < nv) {
        double y[3];
        lap_row<kAleLPR>(row, lane, rowptr, col, L, p, y[0], y[1], y[2]);
        if (lane == 0)
            for (int c = 0; c < 3; ++c) {
                q[3 * row + c] = y[c];
                acc[c] = p[3 * row + c] * y[c];
            }
    }
    block_sum<3>(acc, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < 3; ++j) partial[(int64_t)blockIdx.x * 3 + j] = acc[j];
    if (!arrive_last(&st->counter)) return;
    double tot[3];
    reduce_partials<3>(partial, gridDim.x, 3, tot, lds);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) st->alpha[c] = tot[c] > 0 ? st->rz[c] / tot[c] : 0.0;
        st->counter = 0;
    }
}

// d += alpha p; r -= alpha q; z = Dinv r; beta = rz_new / rz
__global__ __launch_bounds__(256) void k_cg_update(int64_t nv, const double *dinv, const double *p,
                                                   const double *q, double *d, double *r, double *z, CgState *st,
                                                   double *partial)
{
    if (st->done) return;
    __shared__ double lds[4 * 6];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const double a[3] = {st->alpha[0], st->alpha[1], st->alpha[2]};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < 3; ++c) {
            d[3 * i + c] += a[c] * p[3 * i + c];
            double rc = r[3 * i + c] - a[c] * q[3 * i + c];
            double zc = dinv[i] * rc;
            r[3 * i + c] = rc;
            z[3 * i + c] = zc;
            acc[c] += rc * zc;
            acc[3 + c] += rc * rc;
        }
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < 6; ++j) partial[(int64_t)blockIdx.x * 6 + j] = acc[j];
    if (!arrive_last(&st->counter)) return;
    double tot[6];
    reduce_partials<6>(partial, gridDim.x, 6, tot, lds);
    if (threadIdx.x == 0) {
        bool done = true;
        for (int c = 0; c < 3; ++c) {
            st->beta[c] = st->rz[c] > 0 ? tot[c] / st->rz[c] : 0.0;
            st->rz[c] = tot[c];
            st->rr[c] = tot[3 + c];
            if (st->rr[c] > st->tol2[c]) done = false;
        }
        st->done = done ? 1 : 0;
        st->iters += 1;
        st->counter = 0;
    }
}

__global__ void k_cg_dir(int64_t nv, const double *z, double *p, const CgState *st)
{
    if (st->done) return;
    const double b[3] = {st->beta[0], st->beta[1], st->beta[2]};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < 3; ++c) p[3 * i + c] = z[3 * i + c] + b[c] * p[3 * i + c];
}

// Initial guess of a per-step lifting solve: d = sum_l gamma_l d^{n-l}
__global__ void k_ale_guess(int64_t nv, const double *d0, const double *d1, const double *d2, StepCoef C,
                            double *ext)
{
    const double *D[3] = {d0, d1, d2};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nv; i += (int64_t)gridDim.x * blockDim.x) {
        double e = 0;
        for (int l = 0; l < C.nlev; ++l) e += C.gamma[l] * D[l][i];
        ext[i] = e;
    }
}

// x = x^ + d_new; uA = (alpha d_new - sum beta_l d^{n-l}) / dt; d_new = scale * ext
__global__ void k_ale_mesh(int64_t nv, const double *xh, const double *ext, double scale, const double *d0,
                           const double *d1, const double *d2, StepCoef C, double *dnew, double *x, double *uA)
{
    const double *D[3] = {d0, d1, d2};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nv; i += (int64_t)gridDim.x * blockDim.x) {
        double dn = scale * ext[i];
        double bdf = 0;
        for (int l = 0; l < C.nlev; ++l) bdf += C.beta[l] * D[l][i];
        dnew[i] = dn;
        x[i] = xh[i] + dn;
        uA[i] = (C.alpha * dn - bdf) / C.dt;
    }
}

// ------------------------------------------------------------------ host side

lx_status Sim::ale_setup()
{
    // P1 Laplacian on the reference mesh: int grad phi_a . grad phi_b
    std::vector<double> L(nblk, 0.0);
    for (int64_t e = 0; e < nt; ++e) {
        int32_t v[4];
        for (int a = 0; a < 4; ++a) v[a] = hs.tet_soa[a * nt + e];
        double J[3][3];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) J[i][k] = hs.xh[3 * v[k + 1] + i] - hs.xh[3 * v[0] + i];
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2],
               c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        double Ji[3][3] = {{c00 / det, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det,
                            (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det},
                           {c01 / det, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det,
                            (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det},
                           {c02 / det, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det,
                            (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det}};
        double gr[4][3];
        for (int j = 0; j < 3; ++j) {
            gr[1][j] = Ji[0][j];
            gr[2][j] = Ji[1][j];
            gr[3][j] = Ji[2][j];
            gr[0][j] = -(Ji[0][j] + Ji[1][j] + Ji[2][j]);
        }
        double vol = std::fabs(det) / 6.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                L[hs.eslot[(int64_t)(4 * a + b) * nt + e]] +=
                    vol * (gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2]);
    }
    std::vector<int32_t> mark(nv, 0);
    for (int32_t v : h_ale_nodes) mark[v] = 1;
    std::vector<double> Le(L), dinv(nv);
    for (int64_t i = 0; i < nv; ++i)
        for (int32_t k = hs.rowptr[i]; k < hs.rowptr[i + 1]; ++k) {
            const int32_t j = hs.col[k];
            if (mark[i]) Le[k] = (j == i) ? 1.0 : 0.0;
            else if (mark[j]) Le[k] = 0.0;
        }
    for (int64_t i = 0; i < nv; ++i) dinv[i] = 1.0 / Le[hs.diag[i]];
#define ALLOC(ptr, bytes)                                \
    do {                                                 \
        lx_status _s = dalloc((void **)&(ptr), (bytes)); \
        if (_s != LX_OK) return _s;                      \
    } while (0)
    ALLOC(d_lap, sizeof(double) * nblk);
    ALLOC(d_lapfull, sizeof(double) * nblk);
    ALLOC(d_lapdinv, sizeof(double) * nv);
    ALLOC(d_ale_mark, sizeof(int32_t) * nv);
    ALLOC(d_cg, sizeof(double) * 3 * nv * 6 + sizeof(CgState));
    ALLOC(d_dnew, sizeof(double) * 3 * nv);
    ALLOC(d_dbnd, sizeof(double) * 3 * nv);
    // reduction partials of the lifting CG (one row of 9 per workgroup of the row kernels)
    ALLOC(d_cg_partial, sizeof(double) * 9 * ((nv * kAleLPR + 255) / 256));
#undef ALLOC
    LX_HIP(hipMemcpyAsync(d_lap, Le.data(), sizeof(double) * nblk, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_lapfull, L.data(), sizeof(double) * nblk, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_lapdinv, dinv.data(), sizeof(double) * nv, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_ale_mark, mark.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemsetAsync(d_cg, 0, sizeof(double) * 3 * nv * 6 + sizeof(CgState), stream));
    LX_HIP(hipStreamSynchronize(stream));
    ale_ext_valid = false;
    return LX_OK;
}

// Harmonic extension into d_cg[ext] (CG to rtol 1e-13): of the shape D^ (data =
// nullptr), or of nodal boundary data starting from the guess already in ext.
lx_status Sim::ale_extend(const double *data)
{
    double *ext = d_cg, *rhs = d_cg + 3 * nv, *r = d_cg + 6 * nv, *z = d_cg + 9 * nv, *p = d_cg + 12 * nv,
           *q = d_cg + 15 * nv;
    CgState *cst = (CgState *)(d_cg + 18 * nv);
    const unsigned grow = (unsigned)((nv * kAleLPR + 255) / 256);
    const unsigned gvec = (unsigned)std::min<int64_t>((nv + 255) / 256, 1024);
    hipLaunchKernelGGL(k_ale_rhs, dim3(grow), dim3(256), 0, stream, nv, d_rowptr, d_col, d_lapfull, d_ale_mark,
                       data ? data : d_ale_shape, 1.0, rhs, ext);
    double *part = d_cg_partial;   // grow blocks * 9 doubles
    hipLaunchKernelGGL(k_cg_init, dim3(grow), dim3(256), 0, stream, nv, d_rowptr, d_col, d_lap, d_lapdinv, rhs, ext,
                       r, z, p, cst, part, 1e-13);
    CgState h;
    const int max_it = 50000;
    int it = 0;
    for (;;) {
        for (int k = 0; k < 25; ++k) {
            hipLaunchKernelGGL(k_cg_ap, dim3(grow), dim3(256), 0, stream, nv, d_rowptr, d_col, d_lap, p, q, cst, part);
            hipLaunchKernelGGL(k_cg_update, dim3(gvec), dim3(256), 0, stream, nv, d_lapdinv, p, q, ext, r, z, cst,
                               part);
            hipLaunchKernelGGL(k_cg_dir, dim3(gvec), dim3(256), 0, stream, nv, z, p, cst);
        }
        it += 25;
        LX_HIP(hipGetLastError());
        LX_HIP(hipMemcpyAsync(&h, cst, sizeof(CgState), hipMemcpyDeviceToHost, stream));
        LX_HIP(hipStreamSynchronize(stream));
        if (h.done) break;
        if (it >= max_it) return fail(LX_ENOCONV, "ALE lifting CG did not converge");
    }
    ale_iters = h.iters;
    ale_ext_valid = data == nullptr;
    return LX_OK;
}

lx_status Sim::ale_update(double t1, const StepCoef &C)
{
    double scale = 1.0;
    if (ale_nodal) {
        const unsigned g = (unsigned)std::min<int64_t>((3 * nv + 255) / 256, 4096);
        hipLaunchKernelGGL(k_ale_guess, dim3(g), dim3(256), 0, stream, nv, d_dhist[0],
                           prob.bdf_order > 1 ? d_dhist[1] : d_dhist[0], prob.bdf_order > 2 ? d_dhist[2] : d_dhist[0],
                           C, d_cg);
        lx_status s = ale_extend(d_dbnd);
        if (s != LX_OK) return s;
    } else {
        if (!ale_ext_valid) {
            lx_status s = ale_extend(nullptr);
            if (s != LX_OK) return s;
        }
        scale = law_value(prob.ale_law, t1);
    }
    const unsigned g = (unsigned)std::min<int64_t>((3 * nv + 255) / 256, 4096);
    hipLaunchKernelGGL(k_ale_mesh, dim3(g), dim3(256), 0, stream, nv, d_xh, d_cg, scale, d_dhist[0],
                       prob.bdf_order > 1 ? d_dhist[1] : d_dhist[0], prob.bdf_order > 2 ? d_dhist[2] : d_dhist[0],
                       C, d_dnew, d_x, d_uA);
    LX_HIP(hipGetLastError());
    return LX_OK;
}

void Sim::ale_commit()
{
    const int L = prob.bdf_order;
    double *oldest = d_dhist[L - 1];
    for (int l = L - 1; l > 0; --l) d_dhist[l] = d_dhist[l - 1];
    d_dhist[0] = d_dnew;
    d_dnew = oldest;
}

}  // namespace lx
