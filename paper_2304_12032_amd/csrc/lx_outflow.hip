// Outflow boundary terms of P1-P1 problems and boundary integrals.
//
// Resistance condition (Sec. 2.2, resistance boundary conditions):
// sigma n = -(p0(t) + C_R int (u - u_ALE) . n) n.  Its flux functional is
// w . u with w_v = int phi_v n (area/3 n per face corner for flat P1 faces);
// the implicit coupling C_R w w^T is a rank-1 term applied beside the sparse
// matrix in every operator product, and -p0 w + C_R (w . u_ALE) w goes into
// the right-hand side.  Inertial backflow stabilisation (Sec. 2.2, Neumann
// conditions): beta rho/2 min(u_EXT . n, 0) u^{n+1} in the traction, i.e. the
// boundary mass term -beta rho/2 int min(u_EXT . n, 0) phi_b phi_a in every
// velocity component, by the edge-midpoint rule.  Rows of Dirichlet vertices
// get neither term.  Every sum runs in a fixed order: per-vertex and per-pair
// incidence lists in ascending face order, and one-workgroup tree reductions.
#include "lx_device.h"
#include "lx_outflow.h"

namespace lx {

namespace {

constexpr int kOfThreads = 256;

// Sum of v over the workgroup (fixed tree), valid in every thread.
__device__ double wg_sum(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int h = kOfThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    const double s = lds[0];
    __syncthreads();
    return s;
}

// Unit normal (oriented along dir; kept as listed where dir is zero or
// orthogonal) and area of triangle v on configuration x.
__device__ double face_normal(const double *x, const int32_t *v, double d0, double d1, double d2, double n[3])
{
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) {
        a[c] = x[3 * (int64_t)v[1] + c] - x[3 * (int64_t)v[0] + c];
        b[c] = x[3 * (int64_t)v[2] + c] - x[3 * (int64_t)v[0] + c];
    }
    n[0] = a[1] * b[2] - a[2] * b[1];
    n[1] = a[2] * b[0] - a[0] * b[2];
    n[2] = a[0] * b[1] - a[1] * b[0];
    const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double s = (n[0] * d0 + n[1] * d1 + n[2] * d2) < 0.0 ? -1.0 : 1.0;
    for (int c = 0; c < 3; ++c) n[c] = s * n[c] / len;
    return 0.5 * len;
}

// geom[f] = (n_x, n_y, n_z, area) of every face.
__global__ __launch_bounds__(256) void k_face_geom(int64_t nf, const int32_t *__restrict__ faces,
                                                   const double *__restrict__ x, double d0, double d1, double d2,
                                                   double *__restrict__ geom)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    double n[3];
    const double area = face_normal(x, faces + 3 * f, d0, d1, d2, n);
    geom[4 * f] = n[0];
    geom[4 * f + 1] = n[1];
    geom[4 * f + 2] = n[2];
    geom[4 * f + 3] = area;
}

// w_i = sum over the faces at boundary vertex i of area/3 n (incidence codes 3 f + l).
__global__ __launch_bounds__(256) void k_flux_weights(int64_t nbv, const int32_t *__restrict__ vptr,
                                                      const int32_t *__restrict__ vinc,
                                                      const double *__restrict__ geom, double *__restrict__ w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbv) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int32_t k = vptr[i]; k < vptr[i + 1]; ++k) {
        const int64_t f = vinc[k] / 3;
        const double a3 = geom[4 * f + 3] / 3.0;
        for (int c = 0; c < 3; ++c) s[c] += a3 * geom[4 * f + c];
    }
    for (int c = 0; c < 3; ++c) w[3 * i + c] = s[c];
}

// Backflow coefficient of every (row, column) vertex pair: the sum over its
// incidences (f << 4 | la << 2 | lb) of the face's midpoint terms in which
// both corners carry weight.
__global__ __launch_bounds__(256) void k_backflow_coef(int64_t npair, const int32_t *__restrict__ pptr,
                                                       const int32_t *__restrict__ pinc,
                                                       const int32_t *__restrict__ faces,
                                                       const double *__restrict__ geom, const double *__restrict__ h0,
                                                       const double *__restrict__ h1, const double *__restrict__ h2,
                                                       double g0, double g1, double g2, double coef,
                                                       double *__restrict__ pcoef)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npair) return;
    double s = 0.0;
    for (int32_t k = pptr[q]; k < pptr[q + 1]; ++k) {
        const int32_t code = pinc[k];
        const int64_t f = code >> 4;
        const int la = (code >> 2) & 3, lb = code & 3;
        const int32_t *v = faces + 3 * f;
        const double area = geom[4 * f + 3];
        double uE[3][3];
        for (int l = 0; l < 3; ++l)
            for (int c = 0; c < 3; ++c) {
                const int64_t o = 4 * (int64_t)v[l] + c;
                uE[l][c] = g0 * h0[o] + g1 * h1[o] + g2 * h2[o];
            }
        for (int m = 0; m < 3; ++m) {
            const int i = m, j = (m + 1) % 3;
            if (!((la == i || la == j) && (lb == i || lb == j))) continue;
            double un = 0.0;
            for (int c = 0; c < 3; ++c) un += 0.5 * (uE[i][c] + uE[j][c]) * geom[4 * f + c];
            const double neg = un < 0.0 ? un : 0.0;
            if (neg == 0.0) continue;
            s += -coef * (area / 3.0) * neg * 0.25;
        }
    }
    pcoef[q] = s;
}

// The pair coefficients into the diagonal planes F[c][c] of their blocks.
template <typename T>
__global__ __launch_bounds__(256) void k_backflow_add(int64_t npair, int64_t nblk, const int32_t *__restrict__ pblk,
                                                      const double *__restrict__ pcoef, T *__restrict__ val)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npair) return;
    const int64_t k = pblk[q];
    for (int c = 0; c < 3; ++c) val[(int64_t)(4 * c) * nblk + k] += (T)pcoef[q];
}

// r_a -= sum over a's pairs of coef x_b (velocity components), one row per thread.
__global__ __launch_bounds__(256) void k_backflow_apply(int64_t nrow, const int32_t *__restrict__ rptr,
                                                        const int32_t *__restrict__ rvert,
                                                        const int32_t *__restrict__ pcol,
                                                        const double *__restrict__ pcoef,
                                                        const double *__restrict__ x, double *__restrict__ r)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nrow) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int32_t k = rptr[q]; k < rptr[q + 1]; ++k) {
        const int64_t b = pcol[k];
        for (int c = 0; c < 3; ++c) s[c] += pcoef[k] * x[4 * b + c];
    }
    const int64_t a = rvert[q];
    for (int c = 0; c < 3; ++c) r[4 * a + c] -= s[c];
}

// y_i += sign C_R (w . x) w_i on the kept rows; one workgroup.
template <typename T>
__global__ __launch_bounds__(kOfThreads) void k_rank1(int64_t nbv, const int32_t *__restrict__ bv,
                                                      const double *__restrict__ w, const int32_t *__restrict__ keep,
                                                      double scale, const T *__restrict__ x, T *__restrict__ y,
                                                      const int32_t *__restrict__ done)
{
    __shared__ double lds[kOfThreads];
    if (done && *done) return;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nbv; i += kOfThreads)
        for (int c = 0; c < 3; ++c) s += w[3 * i + c] * (double)x[4 * (int64_t)bv[i] + c];
    const double a = scale * wg_sum(s, lds);
    for (int64_t i = threadIdx.x; i < nbv; i += kOfThreads)
        if (keep[i])
            for (int c = 0; c < 3; ++c) y[4 * (int64_t)bv[i] + c] += (T)(a * w[3 * i + c]);
}

// Right-hand side of a resistance condition: (-p0 + C_R (w . u_ALE)) w_i on the
// kept rows of out0 (and out1); uA [nv][3] or null.
__global__ __launch_bounds__(kOfThreads) void k_resist_rhs(int64_t nbv, const int32_t *__restrict__ bv,
                                                           const double *__restrict__ w,
                                                           const int32_t *__restrict__ keep, double cr, double p0,
                                                           const double *__restrict__ uA, double *out0, double *out1)
{
    __shared__ double lds[kOfThreads];
    double s = 0.0;
    if (uA)
        for (int64_t i = threadIdx.x; i < nbv; i += kOfThreads)
            for (int c = 0; c < 3; ++c) s += w[3 * i + c] * uA[3 * (int64_t)bv[i] + c];
    const double a = -p0 + cr * wg_sum(s, lds);
    for (int64_t i = threadIdx.x; i < nbv; i += kOfThreads)
        if (keep[i])
            for (int c = 0; c < 3; ++c) {
                const int64_t o = 4 * (int64_t)bv[i] + c;
                out0[o] += a * w[3 * i + c];
                if (out1) out1[o] += a * w[3 * i + c];
            }
}

// out = (int (u - u_ALE) . n, int p, area) over the faces; one workgroup.
__global__ __launch_bounds__(kOfThreads) void k_boundary_integrals(int64_t nf, const int32_t *__restrict__ faces,
                                                                   const double *__restrict__ x, double d0,
                                                                   double d1, double d2,
                                                                   const double *__restrict__ u,
                                                                   const double *__restrict__ uA,
                                                                   double *__restrict__ out)
{
    __shared__ double lds[kOfThreads];
    double q = 0.0, pi = 0.0, ar = 0.0;
    for (int64_t f = threadIdx.x; f < nf; f += kOfThreads) {
        const int32_t *v = faces + 3 * f;
        double n[3];
        const double area = face_normal(x, v, d0, d1, d2, n);
        for (int l = 0; l < 3; ++l) {
            double un = 0.0;
            for (int c = 0; c < 3; ++c)
                un += (u[4 * (int64_t)v[l] + c] - (uA ? uA[3 * (int64_t)v[l] + c] : 0.0)) * n[c];
            q += area / 3.0 * un;
            pi += area / 3.0 * u[4 * (int64_t)v[l] + 3];
        }
        ar += area;
    }
    q = wg_sum(q, lds);
    pi = wg_sum(pi, lds);
    ar = wg_sum(ar, lds);
    if (threadIdx.x == 0) {
        out[0] = q;
        out[1] = pi;
        out[2] = ar;
    }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_outflow_prepare(const OutflowDev &o, const double *x, const double *h0, const double *h1,
                            const double *h2, const double gamma[3], double rho, hipStream_t s)
{
    if (o.nf == 0) return;
    hipLaunchKernelGGL(k_face_geom, dim3(grid_of(o.nf)), dim3(256), 0, s, o.nf, o.faces, x, o.dir[0], o.dir[1],
                       o.dir[2], o.geom);
    if (o.cr > 0.0)
        hipLaunchKernelGGL(k_flux_weights, dim3(grid_of(o.nbv)), dim3(256), 0, s, o.nbv, o.vptr, o.vinc, o.geom, o.w);
    if (o.npair > 0)
        hipLaunchKernelGGL(k_backflow_coef, dim3(grid_of(o.npair)), dim3(256), 0, s, o.npair, o.pptr, o.pinc, o.faces,
                           o.geom, h0, h1, h2, gamma[0], gamma[1], gamma[2], 0.5 * o.beta * rho, o.pcoef);
}

template <typename T>
void launch_backflow_add(const OutflowDev &o, int64_t nblk, T *val, hipStream_t s)
{
    if (o.npair == 0) return;
    hipLaunchKernelGGL((k_backflow_add<T>), dim3(grid_of(o.npair)), dim3(256), 0, s, o.npair, nblk, o.pblk, o.pcoef,
                       val);
}

void launch_outflow_residual(const OutflowDev &o, double p0, const double *uA, const double *xs, double *r, double *b,
                             hipStream_t s)
{
    if (o.npair > 0)
        hipLaunchKernelGGL(k_backflow_apply, dim3(grid_of(o.nrow)), dim3(256), 0, s, o.nrow, o.rptr, o.rvert, o.pcol,
                           o.pcoef, xs, r);
    if (o.cr > 0.0) {
        hipLaunchKernelGGL(k_resist_rhs, dim3(1), dim3(kOfThreads), 0, s, o.nbv, o.bv, o.w, o.keep, o.cr, p0, uA, r,
                           b);
        hipLaunchKernelGGL((k_rank1<double>), dim3(1), dim3(kOfThreads), 0, s, o.nbv, o.bv, o.w, o.keep, -o.cr, xs, r,
                           (const int32_t *)nullptr);
    }
}

void launch_outflow_rhs(const OutflowDev &o, double p0, const double *uA, double *rhs, hipStream_t s)
{
    if (o.cr > 0.0)
        hipLaunchKernelGGL(k_resist_rhs, dim3(1), dim3(kOfThreads), 0, s, o.nbv, o.bv, o.w, o.keep, o.cr, p0, uA, rhs,
                           (double *)nullptr);
}

template <typename T>
void launch_rank1(const OutflowDev &o, const T *x, T *y, const int32_t *done, hipStream_t s)
{
    if (o.cr <= 0.0) return;
    hipLaunchKernelGGL((k_rank1<T>), dim3(1), dim3(kOfThreads), 0, s, o.nbv, o.bv, o.w, o.keep, o.cr, x, y, done);
}

void launch_boundary_integrals(int64_t nf, const int32_t *faces, const double *x, const double dir[3],
                               const double *u, const double *uA, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_boundary_integrals, dim3(1), dim3(kOfThreads), 0, s, nf, faces, x, dir[0], dir[1], dir[2],
                       u, uA, out);
}

template void launch_backflow_add<double>(const OutflowDev &, int64_t, double *, hipStream_t);
template void launch_backflow_add<float>(const OutflowDev &, int64_t, float *, hipStream_t);
template void launch_rank1<double>(const OutflowDev &, const double *, double *, const int32_t *, hipStream_t);
template void launch_rank1<float>(const OutflowDev &, const float *, float *, const int32_t *, hipStream_t);

}  // namespace lx
