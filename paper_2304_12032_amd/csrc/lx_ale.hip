// ALE mesh motion (paper Sec. 2.1.1 and the discrete mesh velocity of Sec. 2.3):
// lifting of the boundary displacement on the reference mesh, eq. (lifting),
// with a P1 stiffness assembled once: the harmonic extension (a scalar
// Laplacian per block slot, the three components solved as three CGs side by
// side, Jacobi-preconditioned) or linear elasticity (3x3 blocks coupling the
// components, one CG, block-Jacobi-preconditioned), each weighted per element
// by the stiffening coefficient: 1, the Jacobian-based (J0/J)^chi, or the
// boundary-based max(d, beta)^-gamma with d the distance from the element's
// centroid to the moving boundary's faces (one pass over all faces per element
// on the device, at set-up).  Then x^{n+1} = x^ + d^{n+1} and
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

// The lifting operator on [nv][3] vectors: VEC = false, one scalar per block
// slot applied to each component (harmonic); VEC = true, 3x3 blocks stored as
// nine planes of length nblk, plane 3c+d (elasticity).
struct LiftOp {
    const int32_t *rowptr, *col;
    const double *K;
    int64_t nblk;
};

template <int LPR, bool VEC>
__device__ inline void lift_row(int64_t row, int lane, const LiftOp &A, const double *x, double y[3])
{
    y[0] = y[1] = y[2] = 0;
    for (int32_t k = A.rowptr[row] + lane; k < A.rowptr[row + 1]; k += LPR) {
        const double *xj = x + 3 * (int64_t)A.col[k];
        if (VEC) {
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) y[c] += A.K[(int64_t)(3 * c + d) * A.nblk + k] * xj[d];
        } else {
            const double a = A.K[k];
            for (int c = 0; c < 3; ++c) y[c] += a * xj[c];
        }
    }
    for (int c = 0; c < 3; ++c) y[c] = group_sum<double, LPR>(y[c]);
}

// z = P r at one vertex: P = 1 / diagonal (scalar) or the inverse 3x3 diagonal block
template <bool VEC>
__device__ inline void lift_prec(int64_t row, const double *dinv, const double r[3], double z[3])
{
    if (VEC) {
        const double *D = dinv + 9 * row;
        for (int c = 0; c < 3; ++c) z[c] = D[3 * c] * r[0] + D[3 * c + 1] * r[1] + D[3 * c + 2] * r[2];
    } else {
        for (int c = 0; c < 3; ++c) z[c] = dinv[row] * r[c];
    }
}

// One CG for the coupled system: the three per-component sums become one.
template <bool VEC, int K>
__device__ inline void lift_combine(double (&tot)[K], int first)
{
    if (VEC) {
        const double s = tot[first] + tot[first + 1] + tot[first + 2];
        tot[first] = tot[first + 1] = tot[first + 2] = s;
    }
}

// Lanes per row of the lifting products: a scalar (harmonic) row has one value per
// neighbour, so four lanes share a row and each walks about four neighbours with
// independent loads; a 3x3-block (elastic) row has nine, and takes sixteen lanes.
// The CG's row passes (k_cg_init, k_cg_ap) stride over the rows with at most
// kLiftBlocks workgroups, so that the one-workgroup kernels finishing their dot
// products add at most that many partial sums.
constexpr int kLiftBlocks = 2048;
template <bool VEC> constexpr int lift_lpr() { return VEC ? 16 : 4; }
template <bool VEC> unsigned lift_blocks(int64_t nv) { return (unsigned)((nv * lift_lpr<VEC>() + 255) / 256); }
template <bool VEC> unsigned lift_grid(int64_t nv) { return std::min<unsigned>(lift_blocks<VEC>(nv), kLiftBlocks); }

// rhs: boundary rows d_B; interior rows -sum_{j in B} Lfull_ij d_B(j).  d0 (may be
// null): initial guess whose boundary rows are set to d_B.
template <bool VEC>
__global__ __launch_bounds__(256) void k_ale_rhs(int64_t nv, LiftOp Afull, const int32_t *mark, const double *shape,
                                                 double scale, double *rhs, double *d0)
{
    constexpr int LPR = lift_lpr<VEC>();
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= nv) return;
    double y[3] = {0, 0, 0};
    for (int32_t k = Afull.rowptr[row] + lane; k < Afull.rowptr[row + 1]; k += LPR) {
        const int64_t j = Afull.col[k];
        if (mark[j]) {
            if (VEC) {
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d)
                        y[c] += Afull.K[(int64_t)(3 * c + d) * Afull.nblk + k] * scale * shape[3 * j + d];
            } else {
                for (int c = 0; c < 3; ++c) y[c] += Afull.K[k] * scale * shape[3 * j + c];
            }
        }
    }
    for (int c = 0; c < 3; ++c) y[c] = group_sum<double, LPR>(y[c]);
    if (lane == 0) {
        for (int c = 0; c < 3; ++c) {
            if (mark[row]) {
                rhs[3 * row + c] = scale * shape[3 * row + c];
                if (d0) d0[3 * row + c] = scale * shape[3 * row + c];
            } else {
                rhs[3 * row + c] = -y[c];
            }
        }
    }
}

// r = rhs - L d; z = Dinv r; p = z; rz, rr, tolerance
template <bool VEC>
__global__ __launch_bounds__(256) void k_cg_init(int64_t nv, LiftOp A, const double *dinv, const double *rhs,
                                                 const double *d, double *r, double *z, double *p, double *partial)
{
    constexpr int LPR = lift_lpr<VEC>(), RPB = 256 / LPR;
    __shared__ double lds[4 * 9];
    const int lane = threadIdx.x % LPR;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t row = xcd_block() * RPB + threadIdx.x / LPR; row < nv; row += (int64_t)gridDim.x * RPB) {
        double y[3];
        lift_row<LPR, VEC>(row, lane, A, d, y);
        if (lane == 0) {
            double rr[3], zz[3];
            for (int c = 0; c < 3; ++c) rr[c] = rhs[3 * row + c] - y[c];
            lift_prec<VEC>(row, dinv, rr, zz);
            for (int c = 0; c < 3; ++c) {
                r[3 * row + c] = rr[c];
                z[3 * row + c] = zz[c];
                p[3 * row + c] = zz[c];
                acc[c] += rr[c] * zz[c];
                acc[3 + c] += rr[c] * rr[c];
                acc[6 + c] += rhs[3 * row + c] * rhs[3 * row + c];
            }
        }
    }
    block_sum<9>(acc, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < 9; ++j) partial[(int64_t)blockIdx.x * 9 + j] = acc[j];
}

// One workgroup: the sums of k_cg_init's partials (fixed order) -> rz, rr, tolerance.
// Partials are finished by a kernel of their own rather than by the last block to
// arrive, which would cost every block a device-wide fence.
template <bool VEC>
__global__ __launch_bounds__(256) void k_cg_init_fin(int nb, CgState *st, const double *partial, double rtol)
{
    __shared__ double lds[4 * 9];
    double tot[9];
    reduce_partials<9>(partial, nb, 9, tot, lds);
    lift_combine<VEC>(tot, 0);
    lift_combine<VEC>(tot, 3);
    lift_combine<VEC>(tot, 6);
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

// q = K p, and partial sums of p.q for alpha = rz / (p.q)
template <bool VEC>
__global__ __launch_bounds__(256) void k_cg_ap(int64_t nv, LiftOp A, const double *p, double *q, CgState *st,
                                               double *partial)
{
    if (st->done) return;
    constexpr int LPR = lift_lpr<VEC>(), RPB = 256 / LPR;
    __shared__ double lds[4 * 3];
    const int lane = threadIdx.x % LPR;
    double acc[3] = {0, 0, 0};
    for (int64_t row = xcd_block() * RPB + threadIdx.x / LPR; row < nv; row += (int64_t)gridDim.x * RPB) {
        double y[3];
        lift_row<LPR, VEC>(row, lane, A, p, y);
        if (lane == 0)
            for (int c = 0; c < 3; ++c) {
                q[3 * row + c] = y[c];
                acc[c] += p[3 * row + c] * y[c];
            }
    }
    block_sum<3>(acc, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < 3; ++j) partial[(int64_t)blockIdx.x * 3 + j] = acc[j];
}

// One workgroup: alpha = rz / (p . q) from k_cg_ap's partials.
template <bool VEC>
__global__ __launch_bounds__(256) void k_cg_ap_fin(int nb, CgState *st, const double *partial)
{
    if (st->done) return;
    __shared__ double lds[4 * 3];
    double tot[3];
    reduce_partials<3>(partial, nb, 3, tot, lds);
    lift_combine<VEC>(tot, 0);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) st->alpha[c] = tot[c] > 0 ? st->rz[c] / tot[c] : 0.0;
        st->counter = 0;
    }
}

// d += alpha p; r -= alpha q; z = Dinv r; beta = rz_new / rz
template <bool VEC>
__global__ __launch_bounds__(256) void k_cg_update(int64_t nv, const double *dinv, const double *p,
                                                   const double *q, double *d, double *r, double *z, CgState *st,
                                                   double *partial)
{
    if (st->done) return;
    __shared__ double lds[4 * 6];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const double a[3] = {st->alpha[0], st->alpha[1], st->alpha[2]};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        double rr[3], zz[3];
        for (int c = 0; c < 3; ++c) {
            d[3 * i + c] += a[c] * p[3 * i + c];
            rr[c] = r[3 * i + c] - a[c] * q[3 * i + c];
        }
        lift_prec<VEC>(i, dinv, rr, zz);
        for (int c = 0; c < 3; ++c) {
            r[3 * i + c] = rr[c];
            z[3 * i + c] = zz[c];
            acc[c] += rr[c] * zz[c];
            acc[3 + c] += rr[c] * rr[c];
        }
    }
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < 6; ++j) partial[(int64_t)blockIdx.x * 6 + j] = acc[j];
}

// One workgroup: beta, rz, rr and the convergence test from k_cg_update's partials.
template <bool VEC>
__global__ __launch_bounds__(256) void k_cg_update_fin(int nb, CgState *st, const double *partial)
{
    if (st->done) return;
    __shared__ double lds[4 * 6];
    double tot[6];
    reduce_partials<6>(partial, nb, 6, tot, lds);
    lift_combine<VEC>(tot, 0);
    lift_combine<VEC>(tot, 3);
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

// p = z + beta p
__global__ void k_cg_dir(int64_t nv, const double *z, double *p, const CgState *st)
{
    if (st->done) return;
    const double b[3] = {st->beta[0], st->beta[1], st->beta[2]};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < 3; ++c) p[3 * i + c] = z[3 * i + c] + b[c] * p[3 * i + c];
}

// Distance from p to triangle (a, b, c): the closest point is found from the
// Voronoi regions of the triangle's vertices, edges and interior (the method of
// Ericson, Real-Time Collision Detection, Sec. 5.1.5).
__device__ inline double tri_dist(const double *p, const double *a, const double *b, const double *c)
{
    double ab[3], ac[3], ap[3], q[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ac[k] = c[k] - a[k];
        ap[k] = p[k] - a[k];
    }
    auto dot = [](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    auto at = [&](const double *o, double s, const double *u, double t, const double *v) {
        for (int k = 0; k < 3; ++k) q[k] = o[k] + s * u[k] + t * v[k];
    };
    const double d1 = dot(ab, ap), d2 = dot(ac, ap);
    double bp[3], cp[3];
    for (int k = 0; k < 3; ++k) {
        bp[k] = p[k] - b[k];
        cp[k] = p[k] - c[k];
    }
    const double d3 = dot(ab, bp), d4 = dot(ac, bp), d5 = dot(ab, cp), d6 = dot(ac, cp);
    const double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
    if (d1 <= 0.0 && d2 <= 0.0) {
        at(a, 0.0, ab, 0.0, ac);                                  // vertex a
    } else if (d3 >= 0.0 && d4 <= d3) {
        at(b, 0.0, ab, 0.0, ac);                                  // vertex b
    } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        at(a, d1 / (d1 - d3), ab, 0.0, ac);                       // edge ab
    } else if (d6 >= 0.0 && d5 <= d6) {
        at(c, 0.0, ab, 0.0, ac);                                  // vertex c
    } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        at(a, 0.0, ab, d2 / (d2 - d6), ac);                       // edge ac
    } else if (va <= 0.0 && d4 - d3 >= 0.0 && d5 - d6 >= 0.0) {
        double bc[3];
        for (int k = 0; k < 3; ++k) bc[k] = c[k] - b[k];
        at(b, (d4 - d3) / ((d4 - d3) + (d5 - d6)), bc, 0.0, ac);  // edge bc
    } else {
        const double den = 1.0 / (va + vb + vc);
        at(a, vb * den, ab, vc * den, ac);                        // interior
    }
    double d2s = 0.0;
    for (int k = 0; k < 3; ++k) d2s += (p[k] - q[k]) * (p[k] - q[k]);
    return sqrt(d2s);
}

// dist[e] = distance from centroid e to the nearest of nf faces (corner
// coordinates fx [nf][9]); the faces pass through LDS in tiles.
__global__ __launch_bounds__(256) void k_boundary_distance(int64_t nt, const double *__restrict__ cent, int64_t nf,
                                                           const double *__restrict__ fx, double *__restrict__ dist)
{
    __shared__ double tile[256 * 9];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double p[3] = {0, 0, 0};
    if (e < nt)
        for (int k = 0; k < 3; ++k) p[k] = cent[3 * e + k];
    double best = INFINITY;
    for (int64_t f0 = 0; f0 < nf; f0 += 256) {
        const int n = (int)min((int64_t)256, nf - f0);
        __syncthreads();
        for (int i = threadIdx.x; i < 9 * n; i += blockDim.x) tile[i] = fx[9 * f0 + i];
        __syncthreads();
        if (e < nt)
            for (int f = 0; f < n; ++f) best = fmin(best, tri_dist(p, tile + 9 * f, tile + 9 * f + 3, tile + 9 * f + 6));
    }
    if (e < nt) dist[e] = best;
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

// ---- projection onto earlier lifting solutions (LXNS_LIFT_PROJ=0 at creation
// turns it off)
//
// With nodal boundary data the lifting operator K stays the same from step to
// step and only the right-hand side changes, so the earlier solutions span a
// space where the new one nearly lies (exactly, for a motion that is a fixed
// shape times a time law).  Following the projection method for successive
// right-hand sides (Fischer, Comput. Methods Appl. Mech. Engrg. 163, 1998), the
// committed solutions are kept K-orthonormalised (Q, [kProjMax][3 nv]) and the
// CG starts from x0 = x_ext + Q Q^T (b - K x_ext): the extrapolated guess plus
// its best correction within span(Q) in the energy norm, never a worse start
// than x_ext.  All sums are per-workgroup partials finished in a fixed order.

// partial[b][i] = sum over the block's entries of Q_i . v, i < nq
__global__ __launch_bounds__(256) void k_proj_dots(int64_t n, const double *Q, int nq, const double *v,
                                                   double *partial)
{
    __shared__ double lds[4 * kProjMax];
    double acc[kProjMax];
#pragma unroll
    for (int i = 0; i < kProjMax; ++i) acc[i] = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double vj = v[j];
#pragma unroll
        for (int i = 0; i < kProjMax; ++i)
            if (i < nq) acc[i] += Q[i * n + j] * vj;
    }
    block_sum<kProjMax>(acc, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < kProjMax; ++i) partial[(int64_t)blockIdx.x * kProjMax + i] = acc[i];
}

// One workgroup: coef[i] = the sum of the partials of column i (fixed order).
__global__ __launch_bounds__(256) void k_proj_coef(int nb, int nq, const double *partial, double *coef)
{
    __shared__ double lds[4 * kProjMax];
    double tot[kProjMax];
    reduce_partials<kProjMax>(partial, nb, nq, tot, lds);
    if (threadIdx.x == 0)
        for (int i = 0; i < kProjMax; ++i) coef[i] = i < nq ? tot[i] : 0.0;
}

// x += sign sum_{i < nq} coef[i] Q_i
__global__ __launch_bounds__(256) void k_proj_add(int64_t n, const double *Q, int nq, const double *coef,
                                                  double sign, double *x)
{
    double c[kProjMax];
#pragma unroll
    for (int i = 0; i < kProjMax; ++i) c[i] = i < nq ? sign * coef[i] : 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        double a = 0;
#pragma unroll
        for (int i = 0; i < kProjMax; ++i)
            if (i < nq) a += c[i] * Q[i * n + j];
        x[j] += a;
    }
}

// y = K w and partial sums of w . y (the three components together)
template <bool VEC>
__global__ __launch_bounds__(256) void k_lift_apply_dot(int64_t nv, LiftOp A, const double *w, double *y,
                                                        double *partial)
{
    constexpr int LPR = lift_lpr<VEC>(), RPB = 256 / LPR;
    __shared__ double lds[4];
    const int lane = threadIdx.x % LPR;
    double acc[1] = {0};
    for (int64_t row = xcd_block() * RPB + threadIdx.x / LPR; row < nv; row += (int64_t)gridDim.x * RPB) {
        double yv[3];
        lift_row<LPR, VEC>(row, lane, A, w, yv);
        if (lane == 0)
            for (int c = 0; c < 3; ++c) {
                y[3 * row + c] = yv[c];
                acc[0] += w[3 * row + c] * yv[c];
            }
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

// One workgroup: the scale 1 / sqrt(w . K w) of the new basis vector, from
// k_lift_apply_dot's partials (nb1 of them), written to coef[0]; 0 when the
// energy of w is below 1e-16 of that of the solution d, d . b (column 0 of
// k_proj_dots's nb2 partials): w is then rounding noise of a solution already
// in the span, whose normalisation would break the basis' orthogonality.
__global__ __launch_bounds__(256) void k_proj_norm(int nb1, const double *partial1, int nb2, const double *partial2,
                                                   double *coef)
{
    __shared__ double lds[4 * kProjMax];
    double wkw[1], db[kProjMax];
    reduce_partials<1>(partial1, nb1, 1, wkw, lds);
    reduce_partials<kProjMax>(partial2, nb2, 1, db, lds);
    if (threadIdx.x == 0) coef[0] = wkw[0] > 1e-16 * db[0] && wkw[0] > 0 ? 1.0 / sqrt(wkw[0]) : 0.0;
}

__global__ void k_proj_scale(int64_t n, double *w, const double *coef)
{
    const double s = coef[0];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        w[j] *= s;
}

// ------------------------------------------------------------------ host side

lx_status Sim::ale_setup()
{
    // stiffening coefficient per element (reference mesh)
    std::vector<double> alpha(nt, 1.0);
    if (prob.stiffening == LX_STIFF_BOUNDARY) {
        lx_status s = ale_boundary_distance(alpha);
        if (s != LX_OK) return s;
        for (int64_t e = 0; e < nt; ++e) alpha[e] = std::pow(std::max(alpha[e], prob.stiff_p[0]), -prob.stiff_p[1]);
    }
    lift_vec = prob.lifting == LX_LIFT_ELASTIC;
    const int np = lift_vec ? 9 : 1;
    const double mu2 = prob.lift_E / (1.0 + prob.lift_nu);
    const double lam = prob.lift_E * prob.lift_nu / ((1.0 + prob.lift_nu) * (1.0 - 2.0 * prob.lift_nu));
    // P1 stiffness on the reference mesh: harmonic alpha int grad phi_a . grad phi_b, or the
    // elastic 3x3 blocks alpha vol (mu2 (delta_cd g_a.g_b + g_a[d] g_b[c]) / 2 + lam g_a[c] g_b[d])
    std::vector<double> L((size_t)np * nblk, 0.0);
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
        if (prob.stiffening == LX_STIFF_JACOBIAN) alpha[e] = std::pow(prob.stiff_p[0] / std::fabs(det), prob.stiff_p[1]);
        const double w = alpha[e] * std::fabs(det) / 6.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const int64_t slot = hs.eslot[(int64_t)(4 * a + b) * nt + e];
                const double gg = gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2];
                if (!lift_vec) {
                    L[slot] += w * gg;
                    continue;
                }
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d)
                        L[(size_t)(3 * c + d) * nblk + slot] +=
                            w * (mu2 * 0.5 * ((c == d ? gg : 0.0) + gr[a][d] * gr[b][c]) + lam * gr[a][c] * gr[b][d]);
            }
    }
    std::vector<int32_t> mark(nv, 0);
    for (int32_t v : h_ale_nodes) mark[v] = 1;
    // rows and columns of the boundary vertices eliminated (identity diagonal block): the
    // operator stays symmetric; the eliminated columns move to the right-hand side
    std::vector<double> Le(L), dinv((size_t)np * nv);
    for (int64_t i = 0; i < nv; ++i)
        for (int32_t k = hs.rowptr[i]; k < hs.rowptr[i + 1]; ++k) {
            const int32_t j = hs.col[k];
            for (int q = 0; q < np; ++q) {
                const bool diag_entry = j == i && (np == 1 || q % 4 == 0);
                if (mark[i]) Le[(size_t)q * nblk + k] = diag_entry ? 1.0 : 0.0;
                else if (mark[j]) Le[(size_t)q * nblk + k] = 0.0;
            }
        }
    for (int64_t i = 0; i < nv; ++i) {
        const int64_t k = hs.diag[i];
        if (!lift_vec) {
            dinv[i] = 1.0 / Le[k];
            continue;
        }
        double A[3][3], det3;
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) A[c][d] = Le[(size_t)(3 * c + d) * nblk + k];
        det3 = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        if (!(std::fabs(det3) > 0)) return fail(LX_EMESH, "singular lifting block at vertex %lld", (long long)i);
        double *D = &dinv[9 * i];
        D[0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det3;
        D[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det3;
        D[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det3;
        D[3] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det3;
        D[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det3;
        D[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det3;
        D[6] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det3;
        D[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det3;
        D[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det3;
    }
#define ALLOC(ptr, bytes)                                \
    do {                                                 \
        lx_status _s = dalloc((void **)&(ptr), (bytes)); \
        if (_s != LX_OK) return _s;                      \
    } while (0)
    ALLOC(d_lap, sizeof(double) * np * nblk);
    ALLOC(d_lapfull, sizeof(double) * np * nblk);
    ALLOC(d_lapdinv, sizeof(double) * np * nv);
    ALLOC(d_ale_mark, sizeof(int32_t) * nv);
    ALLOC(d_cg, sizeof(double) * 3 * nv * 6 + sizeof(CgState));
    ALLOC(d_dnew, sizeof(double) * 3 * nv);
    ALLOC(d_dbnd, sizeof(double) * 3 * nv);
    // reduction partials of the lifting CG (one row of 9 per workgroup of the row kernels)
    // (also the projection's: w . K w in the first kLiftBlocks, d . b from kProjMax * 1024 on)
    ALLOC(d_cg_partial, sizeof(double) * std::max(9 * std::max(kLiftBlocks, 1024), 2 * kProjMax * 1024));
    // projection basis (earlier lifting solutions, K-orthonormal) and its coefficients
    ALLOC(d_projQ, sizeof(double) * kProjMax * 3 * nv);
    ALLOC(d_proj_coef, sizeof(double) * 2 * kProjMax);
#undef ALLOC
    LX_HIP(hipMemcpyAsync(d_lap, Le.data(), sizeof(double) * Le.size(), hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_lapfull, L.data(), sizeof(double) * L.size(), hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_lapdinv, dinv.data(), sizeof(double) * dinv.size(), hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_ale_mark, mark.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemsetAsync(d_cg, 0, sizeof(double) * 3 * nv * 6 + sizeof(CgState), stream));
    LX_HIP(hipMemsetAsync(d_projQ, 0, sizeof(double) * kProjMax * 3 * nv, stream));
    LX_HIP(hipStreamSynchronize(stream));
    ale_ext_valid = false;
    proj_n = 0;
    return LX_OK;
}

// Distance from every element's centroid (reference mesh) to the nearest face of
// the moving boundary, into dist[nt]; device temporaries come from the caller's
// allocator (or hipMalloc) and are released before returning.
lx_status Sim::ale_boundary_distance(std::vector<double> &dist)
{
    const int64_t nf = (int64_t)h_ale_faces.size() / 3;
    if (nf == 0) return fail(LX_EINVAL, "boundary-based stiffening needs faces with the ALE tags");
    std::vector<double> cent(3 * nt), fx(9 * nf);
    for (int64_t e = 0; e < nt; ++e)
        for (int k = 0; k < 3; ++k) {
            double c = 0;
            for (int a = 0; a < 4; ++a) c += 0.25 * hs.xh[3 * hs.tet_soa[a * nt + e] + k];
            cent[3 * e + k] = c;
        }
    for (int64_t f = 0; f < nf; ++f)
        for (int l = 0; l < 3; ++l)
            for (int k = 0; k < 3; ++k) fx[9 * f + 3 * l + k] = hs.xh[3 * h_ale_faces[3 * f + l] + k];
    auto talloc = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (alloc_fn) p = alloc_fn(bytes, alloc_ctx);
        else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
        return p;
    };
    auto tfree = [&](void *p) {
        if (!p) return;
        if (free_fn) free_fn(p, alloc_ctx);
        else (void)hipFree(p);
    };
    double *dc = (double *)talloc(sizeof(double) * cent.size()), *df = (double *)talloc(sizeof(double) * fx.size()),
           *dd = (double *)talloc(sizeof(double) * nt);
    lx_status st = LX_OK;
    if (!dc || !df || !dd) {
        st = fail(LX_ENOMEM, "device memory for the boundary distances");
    } else if (hipMemcpyAsync(dc, cent.data(), sizeof(double) * cent.size(), hipMemcpyHostToDevice, stream) !=
                   hipSuccess ||
               hipMemcpyAsync(df, fx.data(), sizeof(double) * fx.size(), hipMemcpyHostToDevice, stream) != hipSuccess) {
        st = fail(LX_EDEVICE, "upload of the boundary-distance inputs failed");
    } else {
        hipLaunchKernelGGL(k_boundary_distance, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, stream, nt, dc, nf,
                           df, dd);
        dist.assign(nt, 0.0);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(dist.data(), dd, sizeof(double) * nt, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            st = fail(LX_EDEVICE, "boundary-distance kernel failed");
    }
    (void)hipStreamSynchronize(stream);
    tfree(dc);
    tfree(df);
    tfree(dd);
    return st;
}

// Lifting into d_cg[ext] (CG to rtol 1e-13): of the shape D^ (data = nullptr),
// or of nodal boundary data starting from the guess already in ext.  The
// iterations run in batches of kLiftBatch, with the host reading the state after
// each batch.
constexpr int kLiftBatch = 25;
template <bool VEC>
static void lift_iteration(int64_t nv, const LiftOp &A, const double *dinv, double *ext, double *r, double *z,
                           double *p, double *q, CgState *cst, double *part, unsigned gcg, unsigned gvec, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_ap<VEC>, dim3(gcg), dim3(256), 0, s, nv, A, p, q, cst, part);
    hipLaunchKernelGGL(k_cg_ap_fin<VEC>, dim3(1), dim3(256), 0, s, (int)gcg, cst, part);
    hipLaunchKernelGGL(k_cg_update<VEC>, dim3(gvec), dim3(256), 0, s, nv, dinv, p, q, ext, r, z, cst, part);
    hipLaunchKernelGGL(k_cg_update_fin<VEC>, dim3(1), dim3(256), 0, s, (int)gvec, cst, part);
    hipLaunchKernelGGL(k_cg_dir, dim3(gvec), dim3(256), 0, s, nv, z, p, cst);
}

lx_status Sim::ale_extend(const double *data)
{
    double *ext = d_cg, *rhs = d_cg + 3 * nv, *r = d_cg + 6 * nv, *z = d_cg + 9 * nv, *p = d_cg + 12 * nv,
           *q = d_cg + 15 * nv;
    CgState *cst = (CgState *)(d_cg + 18 * nv);
    const unsigned grow = lift_vec ? lift_blocks<true>(nv) : lift_blocks<false>(nv);   // k_ale_rhs
    const unsigned gcg = lift_vec ? lift_grid<true>(nv) : lift_grid<false>(nv);        // CG row passes
    const unsigned gvec = (unsigned)std::min<int64_t>((nv + 255) / 256, 1024);
    const LiftOp Afull{d_rowptr, d_col, d_lapfull, nblk}, A{d_rowptr, d_col, d_lap, nblk};
    double *part = d_cg_partial;   // gcg (or gvec) blocks * 9 doubles
    auto init = [&](bool finish) {
        if (lift_vec) {
            hipLaunchKernelGGL(k_cg_init<true>, dim3(gcg), dim3(256), 0, stream, nv, A, d_lapdinv, rhs, ext, r, z, p,
                               part);
            if (finish)
                hipLaunchKernelGGL(k_cg_init_fin<true>, dim3(1), dim3(256), 0, stream, (int)gcg, cst, part, 1e-13);
        } else {
            hipLaunchKernelGGL(k_cg_init<false>, dim3(gcg), dim3(256), 0, stream, nv, A, d_lapdinv, rhs, ext, r, z, p,
                               part);
            if (finish)
                hipLaunchKernelGGL(k_cg_init_fin<false>, dim3(1), dim3(256), 0, stream, (int)gcg, cst, part,
                                   1e-13);
        }
    };
    // With a projection basis the extrapolated guess keeps its own boundary rows: it
    // then lies in the span of the earlier solutions, and so does its error for a
    // motion those solutions span (setting the rows to d_B would take it out).
    const bool project = data && proj_n > 0 && lift_proj;
    if (lift_vec)
        hipLaunchKernelGGL(k_ale_rhs<true>, dim3(grow), dim3(256), 0, stream, nv, Afull, d_ale_mark,
                           data ? data : d_ale_shape, 1.0, rhs, project ? nullptr : ext);
    else
        hipLaunchKernelGGL(k_ale_rhs<false>, dim3(grow), dim3(256), 0, stream, nv, Afull, d_ale_mark,
                           data ? data : d_ale_shape, 1.0, rhs, project ? nullptr : ext);
    if (project) {
        // x0 = x_ext + Q Q^T (b - K x_ext)
        const unsigned gp = (unsigned)std::min<int64_t>((3 * nv + 255) / 256, 1024);
        init(false);
        hipLaunchKernelGGL(k_proj_dots, dim3(gp), dim3(256), 0, stream, 3 * nv, d_projQ, proj_n, r, part);
        hipLaunchKernelGGL(k_proj_coef, dim3(1), dim3(256), 0, stream, (int)gp, proj_n, part, d_proj_coef);
        hipLaunchKernelGGL(k_proj_add, dim3(gp), dim3(256), 0, stream, 3 * nv, d_projQ, proj_n, d_proj_coef, 1.0,
                           ext);
    }
    init(true);
    auto batch = [&](hipStream_t s) {
        for (int k = 0; k < kLiftBatch; ++k) {
            if (lift_vec)
                lift_iteration<true>(nv, A, d_lapdinv, ext, r, z, p, q, cst, part, gcg, gvec, s);
            else
                lift_iteration<false>(nv, A, d_lapdinv, ext, r, z, p, q, cst, part, gcg, gvec, s);
        }
    };
    CgState h;
    const int max_it = 50000;
    int it = 0;
    for (;;) {
        batch(stream);
        it += kLiftBatch;
        LX_HIP(hipGetLastError());
        LX_HIP(hipMemcpyAsync(&h, cst, sizeof(CgState), hipMemcpyDeviceToHost, stream));
        LX_HIP(hipStreamSynchronize(stream));
        if (h.done) break;
        if (it >= max_it) return fail(LX_ENOCONV, "ALE lifting CG did not converge");
    }
    ale_iters += h.iters;
    ale_ext_valid = data == nullptr;
    lift_solved = data != nullptr;
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

// Adds the step's lifting solution d (in d_cg, with its right-hand side b = K d)
// to the projection basis: w = d - Q Q^T b (K-orthogonal to Q, since Q^T K d =
// Q^T b), then w / sqrt(w . K w).  A full basis starts again from d alone.
void Sim::ale_add_solution()
{
    const double *d = d_cg, *b = d_cg + 3 * nv;
    double *tmp = d_cg + 15 * nv;   // the CG's product buffer, free after the solve
    if (proj_n == kProjMax) proj_n = 0;
    double *w = d_projQ + (int64_t)proj_n * 3 * nv;
    const unsigned gp = (unsigned)std::min<int64_t>((3 * nv + 255) / 256, 1024);
    double *part = d_cg_partial;
    (void)hipMemcpyAsync(w, d, sizeof(double) * 3 * nv, hipMemcpyDeviceToDevice, stream);
    if (proj_n > 0) {
        hipLaunchKernelGGL(k_proj_dots, dim3(gp), dim3(256), 0, stream, 3 * nv, d_projQ, proj_n, b, part);
        hipLaunchKernelGGL(k_proj_coef, dim3(1), dim3(256), 0, stream, (int)gp, proj_n, part, d_proj_coef);
        hipLaunchKernelGGL(k_proj_add, dim3(gp), dim3(256), 0, stream, 3 * nv, d_projQ, proj_n, d_proj_coef, -1.0,
                           w);
    }
    const LiftOp A{d_rowptr, d_col, d_lap, nblk};
    const unsigned gcg = lift_vec ? lift_grid<true>(nv) : lift_grid<false>(nv);
    double *part2 = part + kProjMax * 1024;   // d . b, after the kLiftBlocks partials of w . K w
    hipLaunchKernelGGL(k_proj_dots, dim3(gp), dim3(256), 0, stream, 3 * nv, d, 1, b, part2);
    if (lift_vec)
        hipLaunchKernelGGL(k_lift_apply_dot<true>, dim3(gcg), dim3(256), 0, stream, nv, A, w, tmp, part);
    else
        hipLaunchKernelGGL(k_lift_apply_dot<false>, dim3(gcg), dim3(256), 0, stream, nv, A, w, tmp, part);
    hipLaunchKernelGGL(k_proj_norm, dim3(1), dim3(256), 0, stream, (int)gcg, part, (int)gp, part2,
                       d_proj_coef + kProjMax);
    hipLaunchKernelGGL(k_proj_scale, dim3(gp), dim3(256), 0, stream, 3 * nv, w, d_proj_coef + kProjMax);
    ++proj_n;
}

void Sim::ale_commit()
{
    if (ale_nodal && lift_solved && lift_proj) ale_add_solution();
    const int L = prob.bdf_order;
    double *oldest = d_dhist[L - 1];
    for (int l = L - 1; l > 0; --l) d_dhist[l] = d_dhist[l - 1];
    d_dhist[0] = d_dnew;
    d_dnew = oldest;
}

}  // namespace lx
