// Fully implicit P1-P1 formulation (paper Sec. 2.3: u* = u^{n+1} - u_ALE in the
// advection and in tau_M, tau_C, and the implicit LES term) linearised by
// Newton's method (Sec. 2.4).
//
// The element residual R(u, p) is the same weak form as the semi-implicit
// element with u_EXT, p_EXT replaced by the unknowns:
//   R_ac = int (rho alpha/dt + sigma_R) u_c phi_a + rho (u* . grad u_c) phi_a
//              + mu grad u_c . grad phi_a [+ mu d_c u . grad phi_a] - p d_c phi_a - K_c phi_a
//              + tau_M r . T_ac + tau_C div u d_c phi_a,
//   R_a  = int div u phi_a + tau_M r . grad phi_a,
// with r = r_M(u, p) = rho (alpha u / dt + u* . grad u) + grad p + sigma_R u - K,
// K = f + rho u_BDF / dt + sigma_R u_ALE, and T_ac,j = rho ([c = j] u* . grad phi_a
// + u*_c d_j phi_a - tau_M r_c d_j phi_a) (SUPG, VMS, implicit LES; SUPG only for
// SUPG-PSPG).  Its consistent Jacobian comes from forward-mode differentiation:
// the residual is evaluated in dual numbers (value, derivative) once per local
// unknown, each pass giving one column.  One thread per element writes the
// 16 x 16 Jacobian and the residual; the slot pass sums them per block through
// the same incidence lists as the semi-implicit assembly, so the Newton system
// is built without atomics in a fixed order.
#include "lx_device.h"
#include "lx_newton.h"

namespace lx {

namespace {

struct Dual {
    double v, d;
};
__device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ inline Dual operator*(Dual a, double s) { return {s * a.v, s * a.d}; }
__device__ inline Dual operator+(Dual a, double s) { return {a.v + s, a.d}; }
__device__ inline Dual operator-(Dual a, double s) { return {a.v - s, a.d}; }
__device__ inline Dual inv(Dual a) { return {1.0 / a.v, -a.d / (a.v * a.v)}; }
__device__ inline Dual rsqrt_dual(Dual a)
{
    const double s = 1.0 / sqrt(a.v);
    return {s, -0.5 * a.d * s / a.v};
}

// Per element data that does not depend on the unknowns.
struct NElem {
    int32_t v[4];
    double dphi[4][3], G[3][3], GG, gg, vol;
    double uA[4][3];
    // per quadrature point: K (data side of the momentum residual), u_ALE, sigma_R, RIIS sum
    double Kq[4][3], uAq[4][3], sigR[4], riis2[4];
};

constexpr double kQa = 0.58541019662496845446, kQb = 0.13819660112501051518;

__device__ bool load_nelem(NElem &E, int64_t e, const NewtonArgs &A, const StepCoef &C)
{
    for (int a = 0; a < 4; ++a) E.v[a] = A.tet[(int64_t)a * A.nt + e];
    double J[3][3];
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) J[i][k] = A.x[3 * (int64_t)E.v[k + 1] + i] - A.x[3 * (int64_t)E.v[0] + i];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2],
                 c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (det == 0.0) return false;
    double Ji[3][3];
    Ji[0][0] = c00 / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = c01 / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = c02 / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    E.vol = fabs(det) / 6.0;
    for (int j = 0; j < 3; ++j) {
        E.dphi[1][j] = Ji[0][j];
        E.dphi[2][j] = Ji[1][j];
        E.dphi[3][j] = Ji[2][j];
        E.dphi[0][j] = -(Ji[0][j] + Ji[1][j] + Ji[2][j]);
    }
    E.GG = 0.0;
    E.gg = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double gi = Ji[0][i] + Ji[1][i] + Ji[2][i];
        E.gg += gi * gi;
        for (int j = 0; j < 3; ++j) {
            E.G[i][j] = Ji[0][i] * Ji[0][j] + Ji[1][i] * Ji[1][j] + Ji[2][i] * Ji[2][j];
            E.GG += E.G[i][j] * E.G[i][j];
        }
    }
    const double *H[3] = {A.h0, A.h1, A.h2};
    double K0[4][3], xh[4][3];
    for (int a = 0; a < 4; ++a) {
        const int64_t v = E.v[a];
        for (int c = 0; c < 3; ++c) {
            double ub = 0.0;
            for (int l = 0; l < C.nlev; ++l) ub += C.beta[l] * H[l][4 * v + c];
            K0[a][c] = (A.f ? A.f[3 * v + c] : 0.0) + C.rho * ub / C.dt;
            E.uA[a][c] = A.uA ? A.uA[3 * v + c] : 0.0;
            xh[a][c] = A.xh[3 * v + c];
        }
    }
    for (int q = 0; q < 4; ++q) {
        double lam[4], xq[3];
        for (int a = 0; a < 4; ++a) lam[a] = a == q ? kQa : kQb;
        for (int c = 0; c < 3; ++c) {
            xq[c] = 0.0;
            E.uAq[q][c] = 0.0;
            E.Kq[q][c] = 0.0;
            for (int a = 0; a < 4; ++a) {
                xq[c] += lam[a] * xh[a][c];
                E.uAq[q][c] += lam[a] * E.uA[a][c];
                E.Kq[q][c] += lam[a] * K0[a][c];
            }
        }
        double sigR = 0.0, riis2 = 0.0;
        for (int k = 0; k < C.n_valves; ++k) {
            const double *vp = C.valve[k];
            const double rel[3] = {xq[0] - vp[0], xq[1] - vp[1], xq[2] - vp[2]};
            const double z = rel[0] * vp[3] + rel[1] * vp[4] + rel[2] * vp[5];
            const double p0 = rel[0] - z * vp[3], p1 = rel[1] - z * vp[4], p2 = rel[2] - z * vp[5];
            const double rp = sqrt(p0 * p0 + p1 * p1 + p2 * p2);
            double dr = 0.0;
            if (rp < vp[6]) dr = vp[6] - rp;
            if (rp > vp[7]) dr = rp - vp[7];
            const double phi = sqrt(z * z + dr * dr), eps = vp[9];
            if (phi <= eps) {
                const double dl = (1.0 + cos(M_PI * phi / eps)) / (2.0 * eps), ratio = vp[8] / eps;
                sigR += ratio * dl;
                riis2 += ratio * ratio * dl * dl;
            }
        }
        E.sigR[q] = sigR;
        E.riis2[q] = riis2;
        for (int c = 0; c < 3; ++c) E.Kq[q][c] += sigR * E.uAq[q][c];
    }
    return true;
}

// R(u, p) in dual numbers.
__device__ void newton_residual(const NElem &E, const Dual u[4][3], const Dual p[4], const StepCoef &C, Dual R[16])
{
    for (int i = 0; i < 16; ++i) R[i] = {0.0, 0.0};
    const double rho = C.rho, mu = C.mu, adt = C.alpha / C.dt;
    Dual gU[3][3], gP[3], divu = {0.0, 0.0};
    for (int c = 0; c < 3; ++c) {
        gP[c] = {0.0, 0.0};
        for (int a = 0; a < 4; ++a) gP[c] = gP[c] + E.dphi[a][c] * p[a];
        for (int j = 0; j < 3; ++j) {
            gU[c][j] = {0.0, 0.0};
            for (int a = 0; a < 4; ++a) gU[c][j] = gU[c][j] + E.dphi[a][j] * u[a][c];
        }
    }
    divu = gU[0][0] + gU[1][1] + gU[2][2];
    for (int q = 0; q < 4; ++q) {
        double lam[4];
        for (int a = 0; a < 4; ++a) lam[a] = a == q ? kQa : kQb;
        const double w = 0.25 * E.vol, sigR = E.sigR[q];
        Dual uq[3], pq = {0.0, 0.0}, us[3];
        for (int a = 0; a < 4; ++a) pq = pq + lam[a] * p[a];
        for (int c = 0; c < 3; ++c) {
            uq[c] = {0.0, 0.0};
            for (int a = 0; a < 4; ++a) uq[c] = uq[c] + lam[a] * u[a][c];
            us[c] = uq[c] - E.uAq[q][c];
        }
        Dual tauM = {0.0, 0.0}, tauC = {0.0, 0.0};
        if (C.stab != LX_STAB_NONE) {
            Dual uGu = {0.0, 0.0};
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) uGu = uGu + E.G[i][j] * (us[i] * us[j]);
            const Dual s = rho * rho * uGu +
                           (C.sigma * C.sigma * rho * rho / (C.dt * C.dt) + C.C_r * mu * mu * E.GG + E.riis2[q]);
            tauM = rsqrt_dual(s);
            tauC = inv(tauM * E.gg);
        }
        Dual adv[3], r[3];
        for (int c = 0; c < 3; ++c) {
            adv[c] = us[0] * gU[c][0] + us[1] * gU[c][1] + us[2] * gU[c][2];
            r[c] = rho * (adt * uq[c] + adv[c]) + gP[c] + sigR * uq[c] - E.Kq[q][c];
        }
        Dual tr[3];
        for (int j = 0; j < 3; ++j) tr[j] = tauM * r[j];
        for (int a = 0; a < 4; ++a) {
            const Dual adv_phi = us[0] * E.dphi[a][0] + us[1] * E.dphi[a][1] + us[2] * E.dphi[a][2];
            Dual trdphi = tr[0] * E.dphi[a][0] + tr[1] * E.dphi[a][1] + tr[2] * E.dphi[a][2];
            for (int c = 0; c < 3; ++c) {
                Dual v = ((rho * adt + sigR) * lam[a]) * uq[c] + (rho * lam[a]) * adv[c];
                for (int j = 0; j < 3; ++j) v = v + (mu * E.dphi[a][j]) * gU[c][j];
                if (C.symgrad)
                    for (int d = 0; d < 3; ++d) v = v + (mu * E.dphi[a][d]) * gU[d][c];
                v = v - E.dphi[a][c] * pq - E.Kq[q][c] * lam[a];
                // tau_M r . T_ac: SUPG tr_c (u* . grad phi_a); VMS and implicit LES
                // (u*_c - tau_M r_c) (tr . grad phi_a)
                Dual st = tr[c] * adv_phi;
                if (C.stab == LX_STAB_VMS_LES) st = st + (us[c] - tr[c]) * trdphi;
                v = v + rho * st + (tauC * divu) * E.dphi[a][c];
                R[3 * a + c] = R[3 * a + c] + w * v;
            }
            R[12 + a] = R[12 + a] + w * (lam[a] * divu + trdphi);
        }
    }
}

// Jacobian column by column and the residual, into rec[e][272]: K[16][16] row-major, then R[16].
__global__ __launch_bounds__(64) void k_newton_p1(NewtonArgs A, StepCoef C)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.nt) return;
    NElem E;
    double *out = A.rec + e * kNewtonRec;
    if (!load_nelem(E, e, A, C)) {
        for (int i = 0; i < kNewtonRec; ++i) out[i] = 0.0;
        return;
    }
    double uv[4][3], pv[4];
    for (int a = 0; a < 4; ++a) {
        const double *s = A.xs + 4 * (int64_t)E.v[a];
        for (int c = 0; c < 3; ++c) uv[a][c] = s[c];
        pv[a] = s[3];
    }
    for (int j = 0; j < 16; ++j) {
        Dual u[4][3], p[4], R[16];
        for (int a = 0; a < 4; ++a) {
            for (int c = 0; c < 3; ++c) u[a][c] = {uv[a][c], 3 * a + c == j ? 1.0 : 0.0};
            p[a] = {pv[a], 12 + a == j ? 1.0 : 0.0};
        }
        newton_residual(E, u, p, C, R);
        for (int i = 0; i < 16; ++i) out[16 * i + j] = R[i].d;
        if (j == 0)
            for (int i = 0; i < 16; ++i) out[256 + i] = R[i].v;
    }
}

// Slot pass: block (i, j) sums the (a, b) blocks of its elements' Jacobians in list
// order; the diagonal slot of vertex i also gathers -R of its vertex rows.
__global__ __launch_bounds__(256) void k_gather_newton(NewtonArgs A)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.nblk) return;
    double acc[16], racc[4] = {0, 0, 0, 0};
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    int32_t vrow = -1;
    for (int32_t q = A.sinc_ptr[k]; q < A.sinc_ptr[k + 1]; ++q) {
        const int32_t code = A.sinc[q];
        const int64_t e = code >> 4;
        const int a = (code >> 2) & 3, b = code & 3;
        const double *K = A.rec + e * kNewtonRec;
        for (int c = 0; c < 3; ++c) {
            for (int d = 0; d < 3; ++d) acc[3 * c + d] += K[16 * (3 * a + c) + 3 * b + d];
            acc[9 + c] += K[16 * (3 * a + c) + 12 + b];
            acc[12 + c] += K[16 * (12 + a) + 3 * b + c];
        }
        acc[15] += K[16 * (12 + a) + 12 + b];
        if (a == b) {
            for (int c = 0; c < 3; ++c) racc[c] -= K[256 + 3 * a + c];
            racc[3] -= K[256 + 12 + a];
            vrow = A.tet[(int64_t)a * A.nt + e];
        }
    }
    for (int i = 0; i < 16; ++i) A.val[(int64_t)i * A.nblk + k] = acc[i];
    if (vrow >= 0)
        for (int c = 0; c < 4; ++c) A.rhs[4 * (int64_t)vrow + c] = racc[c];
}

// gd[k][c] = g[k][c] - xs[node k][c]: the Newton update's Dirichlet values
__global__ void k_dirichlet_delta(int64_t n_dir, const int32_t *node, const double *g, const double *xs, double *gd)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n_dir) return;
    gd[i] = g[i] - xs[4 * (int64_t)node[i / 3] + i % 3];
}

}  // namespace

void launch_newton_p1(const NewtonArgs &a, const StepCoef &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_newton_p1, dim3((unsigned)((a.nt + 63) / 64)), dim3(64), 0, s, a, c);
    hipLaunchKernelGGL(k_gather_newton, dim3((unsigned)((a.nblk + 255) / 256)), dim3(256), 0, s, a);
}

void launch_dirichlet_delta(int64_t n_dir, const int32_t *node, const double *g, const double *xs, double *gd,
                            hipStream_t s)
{
    if (n_dir == 0) return;
    hipLaunchKernelGGL(k_dirichlet_delta, dim3((unsigned)((3 * n_dir + 255) / 256)), dim3(256), 0, s, n_dir, node,
                       g, xs, gd);
}

}  // namespace lx
