/*
 * FP64 CPU oracle for one semi-implicit BDF step of the VMS-LES Navier-Stokes
 * system on tetrahedra (Africa et al., "lifex-cfd", arXiv 2304.12032).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the device library links, includes or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It is written to be checked against the paper by eye:
 * one loop over elements, one loop over quadrature points, and every matrix
 * entry written out from the weak form, with no factoring or fusion.
 *
 * Paper passages followed (section / equation names of the paper):
 *   - fully discrete weak form: Sec. 2.3, eq. (fullydiscrete_ns_ale_riis...)
 *   - diffusion forms: Sec. 2.3, eq. (diffusion-term)
 *   - SUPG-PSPG and VMS terms: Sec. 2.3, eqs. (stabilization_form_SUPG/VMS)
 *   - semi-implicit LES term: Sec. 2.3, eq. (stabilization_form_LES), 2nd case;
 *     the implicit formulation (its 1st case, u* = u^{n+1} - u_ALE) with
 *     Newton's method (Sec. 2.4), its Jacobian by the complex step
 *   - strong residuals r_M, r_C and tau_M, tau_C, G, g: Sec. 2.3
 *   - RIIS term and smoothed delta: Sec. 2.1.2, eq. (riis)
 *   - Neumann data: Sec. 2.2.3, eq. (bcs-neumann)
 *   - lifting problem (harmonic or linear elasticity, Jacobian- or
 *     boundary-based stiffening): Sec. 2.1.1, eq. (lifting)
 *   - inertial backflow stabilisation and resistance conditions: Sec. 2.2
 *     (Neumann and resistance boundary conditions); flow-rate and pressure
 *     integrals over boundary portions: Sec. 4
 *   - GMRES with the SIMPLE preconditioner: Sec. 2.4
 *
 * Readings where the paper is silent (kept identical on the device side and
 * listed in the design notes): local velocity index 3a+c, pressure 12+a;
 * vector-valued test functions phi_a e_c; the VMS term's component j is
 * sum_i u*_i d_j v_i; the LES term is -rho sum_ij atil_i b_j d_j v_i with atil
 * from (u_EXT, p_EXT); tau_M's first term uses the BDF order sigma; G and g
 * are built from the element map of the unit simplex with the element's
 * vertex order as given; the P1 quadrature is the symmetric 4-point degree-2
 * rule; the valve distance is measured at the quadrature point's reference
 * position; u_Sigma = 0.
 *
 * Threads: with OpenMP the element loop computes element matrices of a chunk
 * of elements in parallel and adds them into the global system serially in
 * element order; row loops (products, preconditioner set-up and apply) and
 * element-wise vector updates run in parallel; dot products sum fixed blocks
 * of 4096 entries in parallel and then the block sums in order.  Every result
 * is therefore bitwise the same for any number of threads.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_STAB_NONE 0
#define ORC_STAB_SUPG_PSPG 1
#define ORC_STAB_VMS_LES 2

typedef struct {
    double alpha;     /* BDF coefficient of u^{n+1} at this step                 */
    double sigma;     /* BDF order used at this step (first term of tau_M)       */
    double dt, rho, mu, C_r;
    int32_t stab;     /* ORC_STAB_*                                              */
    int32_t symgrad;  /* 0: gradient-gradient, 1: symmetric-gradient forms      */
    int32_t n_riis;
    int32_t pad;
    const double *riis; /* per valve 10 doubles: center[3], unit normal[3],
                           inner (orifice) radius, outer radius, R, eps         */
} orc_params;

/* ---------------------------------------------------------------- geometry */

/* Symmetric 4-point rule on the tetrahedron, degree 2: barycentric (a,b,b,b)
 * and permutations, a = (5+3 sqrt5)/20, b = (5-sqrt5)/20, each weight 1/4 of
 * the volume. */
void orc_quad_p1(double lam[4][4], double w[4])
{
    const double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0;
    const double b = (5.0 - sqrt(5.0)) / 20.0;
    for (int q = 0; q < 4; ++q) {
        for (int k = 0; k < 4; ++k) lam[q][k] = (k == q) ? a : b;
        w[q] = 0.25;
    }
}

/* J = [x1-x0, x2-x0, x3-x0] (columns) maps the unit simplex onto the element.
 * Returns det J, fills Jinv. */
static double jacobian(const double X[4][3], double Jinv[3][3])
{
    double J[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) J[i][k] = X[k + 1][i] - X[0][i];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Jinv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Jinv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Jinv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Jinv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Jinv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Jinv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Jinv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Jinv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Jinv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    return det;
}

/* Smoothed Dirac delta of half-width eps (Sec. 2.1.2). */
double orc_delta(double phi, double eps)
{
    if (fabs(phi) > eps) return 0.0;
    return (1.0 + cos(M_PI * phi / eps)) / (2.0 * eps);
}

/* Unsigned distance from point y to an annular disc (center c, unit normal n,
 * inner radius r0, outer radius r1).  A full disc has r0 = 0. */
double orc_valve_distance(const double *y, const double *v)
{
    double rel[3] = {y[0] - v[0], y[1] - v[1], y[2] - v[2]};
    double z = rel[0] * v[3] + rel[1] * v[4] + rel[2] * v[5];
    double p[3] = {rel[0] - z * v[3], rel[1] - z * v[4], rel[2] - z * v[5]};
    double rp = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    double dr = 0.0;
    if (rp < v[6]) dr = v[6] - rp;
    if (rp > v[7]) dr = rp - v[7];
    return sqrt(z * z + dr * dr);
}

/* tau_M and tau_C of Sec. 2.3 from the metric tensor G, metric vector g and
 * advection velocity u*, with the RIIS sum supplied as riis2 = sum R^2/eps^2 delta^2. */
void orc_tau(const orc_params *P, const double G[3][3], const double g[3], const double us[3],
             double riis2, double *tauM, double *tauC)
{
    double uGu = 0.0, GG = 0.0, gg = 0.0;
    for (int i = 0; i < 3; ++i) {
        gg += g[i] * g[i];
        for (int j = 0; j < 3; ++j) {
            uGu += us[i] * G[i][j] * us[j];
            GG += G[i][j] * G[i][j];
        }
    }
    double rho = P->rho, mu = P->mu;
    double s = P->sigma * P->sigma * rho * rho / (P->dt * P->dt) + rho * rho * uGu
             + P->C_r * mu * mu * GG + riis2;
    *tauM = 1.0 / sqrt(s);
    *tauC = 1.0 / ((*tauM) * gg);
}

/*
 * Element matrix Ke (16x16) and right-hand side Fe (16) of the P1-P1 element.
 * Inputs per local vertex a: current coordinates X, reference coordinates Xh,
 * extrapolated velocity uE and pressure pE, BDF velocity combination uB, ALE
 * velocity uA and forcing f (all P1 nodal values).  Returns det J.
 */
double orc_element_p1(const double X[4][3], const double Xh[4][3], const double uE[4][3],
                      const double uB[4][3], const double uA[4][3], const double pE[4],
                      const double f[4][3], const orc_params *P, double Ke[16][16], double Fe[16])
{
    double Jinv[3][3];
    double det = jacobian(X, Jinv);
    double vol = fabs(det) / 6.0;

    /* gradients of the barycentric basis: grad lambda_k = row k-1 of J^{-1} */
    double dphi[4][3];
    for (int j = 0; j < 3; ++j) {
        dphi[1][j] = Jinv[0][j];
        dphi[2][j] = Jinv[1][j];
        dphi[3][j] = Jinv[2][j];
        dphi[0][j] = -(Jinv[0][j] + Jinv[1][j] + Jinv[2][j]);
    }
    /* metric tensor G = J^{-T} J^{-1}, metric vector g = J^{-T} (1,1,1) */
    double G[3][3], g[3];
    for (int i = 0; i < 3; ++i) {
        g[i] = Jinv[0][i] + Jinv[1][i] + Jinv[2][i];
        for (int j = 0; j < 3; ++j)
            G[i][j] = Jinv[0][i] * Jinv[0][j] + Jinv[1][i] * Jinv[1][j] + Jinv[2][i] * Jinv[2][j];
    }

    memset(Ke, 0, sizeof(double) * 256);
    memset(Fe, 0, sizeof(double) * 16);

    double lam[4][4], wq[4];
    orc_quad_p1(lam, wq);
    const double rho = P->rho, mu = P->mu, dt = P->dt, alpha = P->alpha;

    for (int q = 0; q < 4; ++q) {
        const double *phi = lam[q];
        double w = wq[q] * vol;

        /* fields at the quadrature point */
        double uEq[3] = {0}, uBq[3] = {0}, uAq[3] = {0}, fq[3] = {0}, xh[3] = {0};
        double gradUE[3][3] = {{0}}, gradPE[3] = {0};
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) {
                uEq[c] += phi[a] * uE[a][c];
                uBq[c] += phi[a] * uB[a][c];
                uAq[c] += phi[a] * uA[a][c];
                fq[c] += phi[a] * f[a][c];
                xh[c] += phi[a] * Xh[a][c];
                gradPE[c] += pE[a] * dphi[a][c];
                for (int j = 0; j < 3; ++j) gradUE[c][j] += uE[a][c] * dphi[a][j];
            }

        /* RIIS: sigma_R = sum_k R_k/eps_k delta_k, riis2 = sum_k R_k^2/eps_k^2 delta_k^2 */
        double sigR = 0.0, riis2 = 0.0;
        for (int k = 0; k < P->n_riis; ++k) {
            const double *v = P->riis + 10 * k;
            double R = v[8], eps = v[9];
            double dl = orc_delta(orc_valve_distance(xh, v), eps);
            sigR += R / eps * dl;
            riis2 += (R * R) / (eps * eps) * dl * dl;
        }

        double us[3];
        for (int c = 0; c < 3; ++c) us[c] = uEq[c] - uAq[c];

        double tauM = 0.0, tauC = 0.0;
        if (P->stab != ORC_STAB_NONE) orc_tau(P, G, g, us, riis2, &tauM, &tauC);

        /* data collected on the right-hand side: K = f + rho u_BDF/dt + sigma_R u_ALE */
        double Kv[3];
        for (int c = 0; c < 3; ++c) Kv[c] = fq[c] + rho * uBq[c] / dt + sigR * uAq[c];

        /* strong momentum residual of the extrapolated state (mu Lap u = 0 for P1) */
        double at[3];
        for (int c = 0; c < 3; ++c) {
            double adv = 0.0;
            for (int j = 0; j < 3; ++j) adv += us[j] * gradUE[c][j];
            double rt = rho * (alpha * uEq[c] / dt + adv) + gradPE[c] + sigR * uEq[c] - Kv[c];
            at[c] = tauM * rt;
        }

        /* T[a][c][j]: the stabilisation test direction of test function phi_a e_c */
        double adv_phi[4], T[4][3][3], s[4];
        for (int a = 0; a < 4; ++a) {
            adv_phi[a] = us[0] * dphi[a][0] + us[1] * dphi[a][1] + us[2] * dphi[a][2];
        }
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c)
                for (int j = 0; j < 3; ++j) {
                    double t = (c == j) ? adv_phi[a] : 0.0;                       /* SUPG */
                    if (P->stab == ORC_STAB_VMS_LES) t += us[c] * dphi[a][j];     /* VMS  */
                    if (P->stab == ORC_STAB_VMS_LES) t -= at[c] * dphi[a][j];     /* LES  */
                    T[a][c][j] = rho * t;
                }
        /* s_b: momentum strong residual of the trial function phi_b e_d, per component */
        for (int b = 0; b < 4; ++b)
            s[b] = rho * (alpha / dt * phi[b] + adv_phi[b]) + sigR * phi[b];

        for (int a = 0; a < 4; ++a) {
            for (int c = 0; c < 3; ++c) {
                int ia = 3 * a + c;
                for (int b = 0; b < 4; ++b) {
                    double gg_ab = dphi[a][0] * dphi[b][0] + dphi[a][1] * dphi[b][1] + dphi[a][2] * dphi[b][2];
                    for (int d = 0; d < 3; ++d) {
                        int jb = 3 * b + d;
                        double v = 0.0;
                        if (c == d) {
                            v += (rho * alpha / dt + sigR) * phi[a] * phi[b];   /* time + RIIS */
                            v += rho * phi[a] * adv_phi[b];                     /* advection   */
                            v += mu * gg_ab;                                    /* diffusion   */
                        }
                        if (P->symgrad) v += mu * dphi[b][c] * dphi[a][d];
                        v += tauM * s[b] * T[a][c][d];                          /* SUPG/VMS/LES */
                        v += tauC * dphi[a][c] * dphi[b][d];                    /* grad-div    */
                        Ke[ia][jb] += w * v;
                    }
                    /* pressure trial psi_b = phi_b */
                    double v = -phi[b] * dphi[a][c];
                    v += tauM * (dphi[b][0] * T[a][c][0] + dphi[b][1] * T[a][c][1] + dphi[b][2] * T[a][c][2]);
                    Ke[ia][12 + b] += w * v;
                }
                double r = Kv[c] * phi[a];
                r += tauM * (Kv[0] * T[a][c][0] + Kv[1] * T[a][c][1] + Kv[2] * T[a][c][2]);
                Fe[ia] += w * r;
            }
            /* pressure test function q = psi_a */
            for (int b = 0; b < 4; ++b) {
                for (int d = 0; d < 3; ++d)
                    Ke[12 + a][3 * b + d] += w * (phi[a] * dphi[b][d] + tauM * s[b] * dphi[a][d]);
                double gg_ab = dphi[a][0] * dphi[b][0] + dphi[a][1] * dphi[b][1] + dphi[a][2] * dphi[b][2];
                Ke[12 + a][12 + b] += w * tauM * gg_ab;
            }
            Fe[12 + a] += w * tauM * (Kv[0] * dphi[a][0] + Kv[1] * dphi[a][1] + Kv[2] * dphi[a][2]);
        }
    }
    return det;
}

/* ----------------------------------------- fully implicit formulation */

/*
 * Element residual R(u, p) (16 entries, local index 3a+c, then 12+a) of the
 * fully implicit formulation (Sec. 2.3, eq. (fullydiscrete_ns_ale_riis...) with
 * u* = u^{n+1} - u_ALE and the implicit case of eq. (stabilization_form_LES)):
 * the same weak form as orc_element_p1 with every occurrence of u_EXT, p_EXT
 * replaced by the unknowns, so that the residual of the semi-implicit system
 * is Ke x - Fe.  Written in complex arithmetic and analytic in (u, p) (the
 * geometry, the valve distances and the data are real), so that the
 * complex-step derivative Im R(x + i h e_j) / h gives the Jacobian column j
 * to rounding (Squire and Trapp, SIAM Review 1998).
 */
typedef double complex orc_cplx;

static void residual_implicit(const double X[4][3], const double Xh[4][3], const orc_cplx u[4][3],
                              const orc_cplx p[4], const double uB[4][3], const double uA[4][3],
                              const double f[4][3], const orc_params *P, orc_cplx R[16])
{
    double Jinv[3][3];
    double det = jacobian(X, Jinv);
    double vol = fabs(det) / 6.0;
    double dphi[4][3];
    for (int j = 0; j < 3; ++j) {
        dphi[1][j] = Jinv[0][j];
        dphi[2][j] = Jinv[1][j];
        dphi[3][j] = Jinv[2][j];
        dphi[0][j] = -(Jinv[0][j] + Jinv[1][j] + Jinv[2][j]);
    }
    double G[3][3], g[3], GG = 0.0, gg = 0.0;
    for (int i = 0; i < 3; ++i) {
        g[i] = Jinv[0][i] + Jinv[1][i] + Jinv[2][i];
        gg += g[i] * g[i];
        for (int j = 0; j < 3; ++j) {
            G[i][j] = Jinv[0][i] * Jinv[0][j] + Jinv[1][i] * Jinv[1][j] + Jinv[2][i] * Jinv[2][j];
        }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) GG += G[i][j] * G[i][j];
    for (int i = 0; i < 16; ++i) R[i] = 0.0;
    double lam[4][4], wq[4];
    orc_quad_p1(lam, wq);
    const double rho = P->rho, mu = P->mu, dt = P->dt, alpha = P->alpha;
    for (int q = 0; q < 4; ++q) {
        const double *phi = lam[q];
        double w = wq[q] * vol;
        orc_cplx uq[3] = {0, 0, 0}, gradU[3][3] = {{0}}, pq = 0.0, gradP[3] = {0, 0, 0};
        double uBq[3] = {0}, uAq[3] = {0}, fq[3] = {0}, xh[3] = {0};
        for (int a = 0; a < 4; ++a) {
            pq += phi[a] * p[a];
            for (int c = 0; c < 3; ++c) {
                uq[c] += phi[a] * u[a][c];
                uBq[c] += phi[a] * uB[a][c];
                uAq[c] += phi[a] * uA[a][c];
                fq[c] += phi[a] * f[a][c];
                xh[c] += phi[a] * Xh[a][c];
                gradP[c] += p[a] * dphi[a][c];
                for (int j = 0; j < 3; ++j) gradU[c][j] += u[a][c] * dphi[a][j];
            }
        }
        double sigR = 0.0, riis2 = 0.0;
        for (int k = 0; k < P->n_riis; ++k) {
            const double *v = P->riis + 10 * k;
            double Rk = v[8], eps = v[9];
            double dl = orc_delta(orc_valve_distance(xh, v), eps);
            sigR += Rk / eps * dl;
            riis2 += (Rk * Rk) / (eps * eps) * dl * dl;
        }
        orc_cplx us[3];
        for (int c = 0; c < 3; ++c) us[c] = uq[c] - uAq[c];
        orc_cplx tauM = 0.0, tauC = 0.0;
        if (P->stab != ORC_STAB_NONE) {
            orc_cplx uGu = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) uGu += us[i] * G[i][j] * us[j];
            orc_cplx sM = P->sigma * P->sigma * rho * rho / (dt * dt) + rho * rho * uGu + P->C_r * mu * mu * GG + riis2;
            tauM = 1.0 / csqrt(sM);
            tauC = 1.0 / (tauM * gg);
        }
        double Kv[3];
        for (int c = 0; c < 3; ++c) Kv[c] = fq[c] + rho * uBq[c] / dt + sigR * uAq[c];
        /* strong momentum residual r_M(u, p) (mu Lap u = 0 for P1) and div u */
        orc_cplx r[3], adv[3], divu = gradU[0][0] + gradU[1][1] + gradU[2][2];
        for (int c = 0; c < 3; ++c) {
            adv[c] = us[0] * gradU[c][0] + us[1] * gradU[c][1] + us[2] * gradU[c][2];
            r[c] = rho * (alpha * uq[c] / dt + adv[c]) + gradP[c] + sigR * uq[c] - Kv[c];
        }
        for (int a = 0; a < 4; ++a) {
            orc_cplx adv_phi = us[0] * dphi[a][0] + us[1] * dphi[a][1] + us[2] * dphi[a][2];
            for (int c = 0; c < 3; ++c) {
                orc_cplx v = (rho * alpha / dt + sigR) * uq[c] * phi[a] + rho * adv[c] * phi[a];
                for (int j = 0; j < 3; ++j) v += mu * gradU[c][j] * dphi[a][j];
                if (P->symgrad)
                    for (int d = 0; d < 3; ++d) v += mu * gradU[d][c] * dphi[a][d];
                v += -pq * dphi[a][c] - Kv[c] * phi[a];
                /* SUPG (tau_M r_M, rho u* . grad v), VMS (tau_M r_M, rho u* . (grad v)^T) and
                 * implicit LES -(tau_M r_M (x) tau_M r_M, rho grad v), v = phi_a e_c */
                for (int j = 0; j < 3; ++j) {
                    orc_cplx t = (c == j) ? adv_phi : 0.0;
                    if (P->stab == ORC_STAB_VMS_LES) t += us[c] * dphi[a][j] - tauM * r[c] * dphi[a][j];
                    v += tauM * r[j] * rho * t;
                }
                v += tauC * divu * dphi[a][c];
                R[3 * a + c] += w * v;
            }
            orc_cplx vq = divu * phi[a];
            for (int j = 0; j < 3; ++j) vq += tauM * r[j] * dphi[a][j];
            R[12 + a] += w * vq;
        }
    }
}

/*
 * Newton element system of the implicit formulation at the state (u, p):
 * Re = R(u, p) and Ke = dR/d(u, p), column j by the complex step of size h
 * (1e-30 by default).  Returns det J.
 */
double orc_newton_element_p1(const double X[4][3], const double Xh[4][3], const double u[4][3], const double p[4],
                             const double uB[4][3], const double uA[4][3], const double f[4][3], const orc_params *P,
                             double h, double Ke[16][16], double Re[16])
{
    double Jinv[3][3];
    double det = jacobian(X, Jinv);
    if (!(h > 0.0)) h = 1e-30;
    orc_cplx uc[4][3], pc[4], R[16];
    for (int a = 0; a < 4; ++a) {
        pc[a] = p[a];
        for (int c = 0; c < 3; ++c) uc[a][c] = u[a][c];
    }
    residual_implicit(X, Xh, uc, pc, uB, uA, f, P, R);
    for (int i = 0; i < 16; ++i) Re[i] = creal(R[i]);
    for (int j = 0; j < 16; ++j) {
        if (j < 12) uc[j / 3][j % 3] += I * h;
        else pc[j - 12] += I * h;
        residual_implicit(X, Xh, uc, pc, uB, uA, f, P, R);
        for (int i = 0; i < 16; ++i) Ke[i][j] = cimag(R[i]) / h;
        if (j < 12) uc[j / 3][j % 3] = u[j / 3][j % 3];
        else pc[j - 12] = p[j - 12];
    }
    return det;
}

/* ------------------------------------------------------- global assembly */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Vertex adjacency (each vertex with itself and every vertex sharing a tet),
 * as CSR: vptr[nv+1], vadj[vptr[nv]] sorted.  Two passes: count, then fill.
 * Returns the adjacency size, or -1 on allocation failure; the caller passes
 * vadj = NULL first to get the size.
 */
int64_t orc_vertex_graph(int64_t nv, int64_t nt, int64_t nvpe, const int32_t *tets, int64_t *vptr,
                         int32_t *vadj)
{
    /* candidate lists with duplicates: each vertex gets nvpe entries per incident tet */
    int64_t *cnt = calloc((size_t)nv + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < nvpe; ++a) cnt[tets[e * nvpe + a] + 1] += nvpe;
    for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
    int32_t *cand = malloc(sizeof(int32_t) * (size_t)cnt[nv]);
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)nv);
    if (!cand || !fill) { free(cnt); free(cand); free(fill); return -1; }
    for (int64_t v = 0; v < nv; ++v) fill[v] = cnt[v];
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < nvpe; ++a) {
            int32_t va = tets[e * nvpe + a];
            for (int b = 0; b < nvpe; ++b) cand[fill[va]++] = tets[e * nvpe + b];
        }
    int64_t total = 0;
    if (vptr) vptr[0] = 0;
    for (int64_t v = 0; v < nv; ++v) {
        int32_t *lst = cand + cnt[v];
        int64_t n = cnt[v + 1] - cnt[v];
        qsort(lst, (size_t)n, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || lst[i] != lst[i - 1]) {
                if (vadj) vadj[total + u] = lst[i];
                ++u;
            }
        total += u;
        if (vptr) vptr[v + 1] = total;
    }
    free(cnt); free(cand); free(fill);
    return total;
}

/*
 * Scalar CSR pattern of the P1-P1 system, global numbering: velocity dof
 * (v, c) -> 3v + c, pressure dof v -> 3 nv + v.  Row r of vertex v holds the
 * columns {3w + d} for w in adj(v), d = 0..2, then {3 nv + w}.
 */
void orc_pattern_p1(int64_t nv, const int64_t *vptr, const int32_t *vadj, int64_t *rowptr,
                    int32_t *col)
{
    int64_t N = 4 * nv, pos = 0;
    rowptr[0] = 0;
    for (int64_t r = 0; r < N; ++r) {
        int64_t v = (r < 3 * nv) ? r / 3 : r - 3 * nv;
        for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k)
            for (int d = 0; d < 3; ++d) col[pos++] = (int32_t)(3 * vadj[k] + d);
        for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) col[pos++] = (int32_t)(3 * nv + vadj[k]);
        rowptr[r + 1] = pos;
    }
}

static int64_t find_col(const int64_t *rowptr, const int32_t *col, int64_t r, int32_t c)
{
    int64_t lo = rowptr[r], hi = rowptr[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] == c) return mid;
        if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * Assemble the P1-P1 system: for every element gather its nodal data, form
 * Ke, Fe with orc_element_p1 and add them into (val, rhs).  val and rhs must
 * be zeroed by the caller.  Field arrays are [nv][3] (velocity-like) or [nv].
 * Returns 0, or -(e+1) for the first element with |det J| <= 0.
 */
int64_t orc_assemble_p1(int64_t nv, int64_t nt, const double *x, const double *xh,
                        const int32_t *tets, const double *uE, const double *uB, const double *uA,
                        const double *pE, const double *f, const orc_params *P,
                        const int64_t *rowptr, const int32_t *col, double *val, double *rhs)
{
    enum { CHUNK = 8192 };
    double (*Kc)[16][16] = malloc(sizeof(double) * 256 * CHUNK);
    double (*Fc)[16] = malloc(sizeof(double) * 16 * CHUNK);
    double *detc = malloc(sizeof(double) * CHUNK);
    if (!Kc || !Fc || !detc) { free(Kc); free(Fc); free(detc); return -(nt + 1); }
    int64_t rc = 0;
    for (int64_t e0 = 0; e0 < nt && rc == 0; e0 += CHUNK) {
        const int64_t ne = (nt - e0 < CHUNK) ? nt - e0 : CHUNK;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < ne; ++i) {
            const int64_t e = e0 + i;
            double X[4][3], Xh[4][3], ue[4][3], ub[4][3], ua[4][3], pe[4], fe[4][3];
            for (int a = 0; a < 4; ++a) {
                const int32_t va = tets[4 * e + a];
                for (int c = 0; c < 3; ++c) {
                    X[a][c] = x[3 * va + c];
                    Xh[a][c] = xh[3 * va + c];
                    ue[a][c] = uE[3 * va + c];
                    ub[a][c] = uB[3 * va + c];
                    ua[a][c] = uA ? uA[3 * va + c] : 0.0;
                    fe[a][c] = f ? f[3 * va + c] : 0.0;
                }
                pe[a] = pE[va];
            }
            detc[i] = orc_element_p1(X, Xh, ue, ub, ua, pe, fe, P, Kc[i], Fc[i]);
        }
        for (int64_t i = 0; i < ne && rc == 0; ++i) {
            const int64_t e = e0 + i;
            if (!(fabs(detc[i]) > 0.0)) { rc = -(e + 1); break; }
            int64_t gdof[16];
            for (int a = 0; a < 4; ++a) {
                const int32_t va = tets[4 * e + a];
                for (int c = 0; c < 3; ++c) gdof[3 * a + c] = 3 * (int64_t)va + c;
                gdof[12 + a] = 3 * nv + va;
            }
            for (int r = 0; r < 16 && rc == 0; ++r) {
                rhs[gdof[r]] += Fc[i][r];
                for (int j = 0; j < 16; ++j) {
                    int64_t k = find_col(rowptr, col, gdof[r], (int32_t)gdof[j]);
                    if (k < 0) { rc = -(e + 1); break; }
                    val[k] += Kc[i][r][j];
                }
            }
        }
    }
    free(Kc); free(Fc); free(detc);
    return rc;
}

/*
 * Global Newton system of the implicit formulation at the state (u [nv][3],
 * p [nv]): val += dR/dx, rhs -= R (so that J dx = rhs is the Newton update),
 * element systems computed in parallel chunks and added in element order.
 * Returns 0, or -(e+1) for a degenerate element or a missing pattern entry.
 */
int64_t orc_assemble_p1_newton(int64_t nv, int64_t nt, const double *x, const double *xh, const int32_t *tets,
                               const double *u, const double *p, const double *uB, const double *uA, const double *f,
                               const orc_params *P, const int64_t *rowptr, const int32_t *col, double *val,
                               double *rhs)
{
    enum { CHUNK = 4096 };
    double (*Kc)[16][16] = malloc(sizeof(double) * 256 * CHUNK);
    double (*Fc)[16] = malloc(sizeof(double) * 16 * CHUNK);
    double *detc = malloc(sizeof(double) * CHUNK);
    if (!Kc || !Fc || !detc) { free(Kc); free(Fc); free(detc); return -(nt + 1); }
    int64_t rc = 0;
    for (int64_t e0 = 0; e0 < nt && rc == 0; e0 += CHUNK) {
        const int64_t ne = (nt - e0 < CHUNK) ? nt - e0 : CHUNK;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < ne; ++i) {
            const int64_t e = e0 + i;
            double X[4][3], Xh[4][3], ue[4][3], ub[4][3], ua[4][3], pe[4], fe[4][3];
            for (int a = 0; a < 4; ++a) {
                const int32_t va = tets[4 * e + a];
                for (int c = 0; c < 3; ++c) {
                    X[a][c] = x[3 * va + c];
                    Xh[a][c] = xh[3 * va + c];
                    ue[a][c] = u[3 * va + c];
                    ub[a][c] = uB[3 * va + c];
                    ua[a][c] = uA ? uA[3 * va + c] : 0.0;
                    fe[a][c] = f ? f[3 * va + c] : 0.0;
                }
                pe[a] = p[va];
            }
            detc[i] = orc_newton_element_p1(X, Xh, ue, pe, ub, ua, fe, P, 0.0, Kc[i], Fc[i]);
        }
        for (int64_t i = 0; i < ne && rc == 0; ++i) {
            const int64_t e = e0 + i;
            if (!(fabs(detc[i]) > 0.0)) { rc = -(e + 1); break; }
            int64_t gdof[16];
            for (int a = 0; a < 4; ++a) {
                const int32_t va = tets[4 * e + a];
                for (int c = 0; c < 3; ++c) gdof[3 * a + c] = 3 * (int64_t)va + c;
                gdof[12 + a] = 3 * nv + va;
            }
            for (int r = 0; r < 16 && rc == 0; ++r) {
                rhs[gdof[r]] -= Fc[i][r];
                for (int j = 0; j < 16; ++j) {
                    int64_t k = find_col(rowptr, col, gdof[r], (int32_t)gdof[j]);
                    if (k < 0) { rc = -(e + 1); break; }
                    val[k] += Kc[i][r][j];
                }
            }
        }
    }
    free(Kc); free(Fc); free(detc);
    return rc;
}

/*
 * Neumann term (h, v) on boundary triangles (Sec. 2.2.3): h is a nodal vector
 * traction [nv][3], interpolated linearly on each face and integrated with the
 * edge-midpoint rule (exact for the quadratic integrand).
 */
void orc_neumann_p1(int64_t nv, int64_t nf, const double *x, const int32_t *faces, const double *h,
                    double *rhs)
{
    (void)nv;
    for (int64_t e = 0; e < nf; ++e) {
        const int32_t *v = faces + 3 * e;
        double a[3], b[3];
        for (int c = 0; c < 3; ++c) {
            a[c] = x[3 * v[1] + c] - x[3 * v[0] + c];
            b[c] = x[3 * v[2] + c] - x[3 * v[0] + c];
        }
        double n[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        double area = 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        /* midpoint of edge (i,j): phi_i = phi_j = 1/2, weight area/3 */
        for (int m = 0; m < 3; ++m) {
            int i = m, j = (m + 1) % 3;
            for (int c = 0; c < 3; ++c) {
                double hq = 0.5 * (h[3 * v[i] + c] + h[3 * v[j] + c]);
                rhs[3 * (int64_t)v[i] + c] += area / 3.0 * hq * 0.5;
                rhs[3 * (int64_t)v[j] + c] += area / 3.0 * hq * 0.5;
            }
        }
    }
}

/* ------------------------------------------------ outflow boundary terms */

/* Outward unit normal and area of boundary triangle v[0..2] on configuration x:
 * the triangle's own normal, its sign chosen to agree with the condition's
 * outward direction dir (kept as given where dir is zero or orthogonal). */
static double face_normal(const double *x, const int32_t *v, const double *dir, double n[3])
{
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) {
        a[c] = x[3 * v[1] + c] - x[3 * v[0] + c];
        b[c] = x[3 * v[2] + c] - x[3 * v[0] + c];
    }
    n[0] = a[1] * b[2] - a[2] * b[1];
    n[1] = a[2] * b[0] - a[0] * b[2];
    n[2] = a[0] * b[1] - a[1] * b[0];
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double s = (n[0] * dir[0] + n[1] * dir[1] + n[2] * dir[2]) < 0.0 ? -1.0 : 1.0;
    for (int c = 0; c < 3; ++c) n[c] = s * n[c] / len;
    return 0.5 * len;
}

/* Resistance condition (Sec. 2.2, resistance boundary conditions): the flux
 * functional Q(u) = int_Gamma u . n is w . u with w[3v+c] = int_Gamma phi_v n_c,
 * which for P1 and flat faces is area/3 n_c per face corner.  w is added into. */
void orc_flux_weights(int64_t nf, const double *x, const int32_t *faces, const double *dir, double *w)
{
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t *v = faces + 3 * f;
        double n[3];
        double area = face_normal(x, v, dir, n);
        for (int l = 0; l < 3; ++l)
            for (int c = 0; c < 3; ++c) w[3 * (int64_t)v[l] + c] += area / 3.0 * n[c];
    }
}

/* Inertial backflow stabilisation (Sec. 2.2, Neumann conditions): the traction
 * gains beta rho/2 min(u . n, 0) u, taken semi-implicitly as
 * min(u_EXT . n, 0) u^{n+1}; on the left-hand side of the momentum equation
 * this is  - beta rho/2 int_Gamma min(u_EXT . n, 0) phi_b phi_a  in every
 * velocity component, integrated with the edge-midpoint rule (exact for
 * quadratics).  coef = beta rho / 2; rows of vertices with skip[v] != 0
 * (Dirichlet vertices) get nothing. */
void orc_backflow_p1(int64_t nf, const double *x, const int32_t *faces, const double *dir, const double *uE,
                     double coef, const char *skip, const int64_t *rowptr, const int32_t *col, double *val)
{
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t *v = faces + 3 * f;
        double n[3];
        double area = face_normal(x, v, dir, n);
        for (int m = 0; m < 3; ++m) {
            /* midpoint of the edge (v[m], v[m+1]): phi = 1/2 on its two ends, 0 on the third */
            int i = m, j = (m + 1) % 3;
            double un = 0.0;
            for (int c = 0; c < 3; ++c) un += 0.5 * (uE[3 * v[i] + c] + uE[3 * v[j] + c]) * n[c];
            double neg = un < 0.0 ? un : 0.0;
            if (neg == 0.0) continue;
            int ends[2] = {i, j};
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q) {
                    int64_t a = v[ends[p]], b = v[ends[q]];
                    if (skip[a]) continue;
                    double add = -coef * (area / 3.0) * neg * 0.25;
                    for (int c = 0; c < 3; ++c) {
                        int64_t r = 3 * a + c, cc = 3 * b + c;
                        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
                            if (col[k] == cc) {
                                val[k] += add;
                                break;
                            }
                    }
                }
        }
    }
}

/* Boundary integrals over faces (Sec. 4, flow rates and section pressures):
 * out[0] = int (u - u_ALE) . n (flux through the moving surface; uA may be
 * NULL), out[1] = int p, out[2] = area.  P1 data: area/3 times the corner sums. */
void orc_boundary_integrals(int64_t nf, const double *x, const int32_t *faces, const double *dir, const double *u,
                            const double *uA, const double *p, double *out)
{
    out[0] = out[1] = out[2] = 0.0;
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t *v = faces + 3 * f;
        double n[3];
        double area = face_normal(x, v, dir, n);
        for (int l = 0; l < 3; ++l) {
            double un = 0.0;
            for (int c = 0; c < 3; ++c) un += (u[3 * v[l] + c] - (uA ? uA[3 * v[l] + c] : 0.0)) * n[c];
            out[0] += area / 3.0 * un;
            out[1] += area / 3.0 * p[v[l]];
        }
        out[2] += area;
    }
}

/* Dirichlet rows: keep a_ii, zero the rest of the row, b_i = a_ii g_i. */
void orc_dirichlet_rows(int64_t nrows, const int64_t *rows, const double *g, const int64_t *rowptr,
                        const int32_t *col, double *val, double *rhs)
{
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t r = rows[k];
        double aii = 0.0;
        for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
            if (col[p] == r) aii = val[p];
            else val[p] = 0.0;
        }
        rhs[r] = aii * g[k];
    }
}

/* ------------------------------------------------------------- linear solve */

static void csr_mv(int64_t N, const int64_t *rowptr, const int32_t *col, const double *val,
                   const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; ++r) {
        double s = 0.0;
        for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) s += val[p] * x[col[p]];
        y[r] = s;
    }
}

/* Sum over fixed blocks of 4096 entries, then the block sums in order: the
   same rounding for any number of threads. */
static double dot(int64_t N, const double *a, const double *b)
{
    enum { BLK = 4096 };
    const int64_t nb = (N + BLK - 1) / BLK;
    double part[256];
    double s = 0.0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t n = (nb - b0 < 256) ? nb - b0 : 256;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            const int64_t lo = (b0 + k) * BLK, hi = (lo + BLK < N) ? lo + BLK : N;
            double t = 0.0;
            for (int64_t i = lo; i < hi; ++i) t += a[i] * b[i];
            part[k] = t;
        }
        for (int64_t k = 0; k < n; ++k) s += part[k];
    }
    return s;
}

typedef struct {
    int64_t nv;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
    double *Dinv;    /* [3nv] 1/F_ii                        */
    double *Finv;    /* [nv][9] inverse nodal 3x3 blocks    */
    double *Sinv;    /* [nv]  1/diag(C - B D^-1 G)          */
    double *tmp;     /* [4nv] work                          */
    int32_t degree;  /* Chebyshev degree for S~^{-1}; 0: diagonal only */
    double ratio;    /* lambda_max / lambda_min of the Chebyshev interval */
    double lam_max;  /* Gershgorin bound of diag(S~)^{-1} S~ */
    double *cw;      /* [6nv] Chebyshev work: r, d, y(3), t */
} simple_t;

static void inv3(const double A[9], double B[9])
{
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6])
               + A[2] * (A[3] * A[7] - A[4] * A[6]);
    B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

/* SIMPLE setup (Sec. 2.4, aSIMPLE with block-Jacobi blocks): D = diag(F),
 * F~ = nodal 3x3 diagonal blocks of F, S~ = diag(C - B D^-1 G). */
static int simple_setup(simple_t *S)
{
    int64_t nv = S->nv;
    const int64_t *rp = S->rowptr;
    const int32_t *col = S->col;
    const double *val = S->val;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        double blk[9];
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
                int64_t k = find_col(rp, col, 3 * v + c, (int32_t)(3 * v + d));
                blk[3 * c + d] = (k >= 0) ? val[k] : 0.0;
            }
        for (int c = 0; c < 3; ++c) S->Dinv[3 * v + c] = 1.0 / blk[4 * c];
        inv3(blk, S->Finv + 9 * v);
    }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        int64_t r = 3 * nv + v;
        double s = 0.0, cvv = 0.0;
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
            int32_t j = col[p];
            if (j == r) cvv = val[p];
            if (j < 3 * nv) {
                int64_t k = find_col(rp, col, j, (int32_t)r);
                double gji = (k >= 0) ? val[k] : 0.0;
                s += val[p] * S->Dinv[j] * gji;
            }
        }
        S->Sinv[v] = 1.0 / (cvv - s);
    }
    /* Gershgorin bound of diag(S~)^{-1} S~ with S~ = C - B D^{-1} G (not formed):
       row v: (sum |C_vw| + sum_(w,d) |B_v,(w,d)| sum_u |G_(w,d),u| / |D_(w,d)|) / |S~_vv| */
    S->lam_max = 0.0;
    if (S->degree > 0) {
        double *ag = S->cw;   /* [3nv] */
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < 3 * nv; ++r) {
            double a = 0.0;
            for (int64_t p = rp[r]; p < rp[r + 1]; ++p)
                if (col[p] >= 3 * nv) a += fabs(val[p]);
            ag[r] = a * fabs(S->Dinv[r]);
        }
        double lam = 0.0;
#pragma omp parallel for schedule(static) reduction(max : lam)
        for (int64_t v = 0; v < nv; ++v) {
            int64_t r = 3 * nv + v;
            double a = 0.0;
            for (int64_t p = rp[r]; p < rp[r + 1]; ++p)
                a += (col[p] >= 3 * nv) ? fabs(val[p]) : fabs(val[p]) * ag[col[p]];
            a *= fabs(S->Sinv[v]);
            if (a > lam) lam = a;
        }
        S->lam_max = lam;
    }
    return 0;
}

/* y = S~ d = C d - B D^{-1} G d for a pressure vector d (matrix-free). */
static void schur_mv(const simple_t *S, const double *d, double *gu, double *y)
{
    int64_t nv = S->nv;
    const int64_t *rp = S->rowptr;
    const int32_t *col = S->col;
    const double *val = S->val;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < 3 * nv; ++r) {
        double a = 0.0;
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p)
            if (col[p] >= 3 * nv) a += val[p] * d[col[p] - 3 * nv];
        gu[r] = S->Dinv[r] * a;
    }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        int64_t r = 3 * nv + v;
        double a = 0.0;
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p)
            a += (col[p] >= 3 * nv) ? val[p] * d[col[p] - 3 * nv] : -val[p] * gu[col[p]];
        y[v] = a;
    }
}

/* z ~= S~^{-1} t: Chebyshev iteration of the given degree on S~ z = t with
   diagonal scaling, started from z = 0, for eigenvalues of diag(S~)^{-1} S~ in
   [lam_max / ratio, lam_max] (Saad, Iterative Methods, Alg. 12.1). */
static void schur_cheb(const simple_t *S, const double *t, double *z)
{
    int64_t nv = S->nv;
    double *r = S->cw, *d = S->cw + nv, *gu = S->cw + 2 * nv, *q = S->cw + 5 * nv;
    double lmax = S->lam_max, lmin = lmax / S->ratio;
    double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    double sigma = theta / delta, rho = 1.0 / sigma;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        r[v] = t[v];
        d[v] = S->Sinv[v] * r[v] / theta;
        z[v] = d[v];
    }
    for (int i = 1; i < S->degree; ++i) {
        schur_mv(S, d, gu, q);
        double rho_new = 1.0 / (2.0 * sigma - rho);
#pragma omp parallel for schedule(static)
        for (int64_t v = 0; v < nv; ++v) {
            r[v] -= q[v];
            d[v] = rho_new * rho * d[v] + 2.0 * rho_new / delta * S->Sinv[v] * r[v];
            z[v] += d[v];
        }
        rho = rho_new;
    }
}

/* z = P^-1 r: z_u = F~^-1 r_u; z_p = S~^-1 (r_p - B z_u); x_u = z_u - D^-1 G z_p. */
static void simple_apply(const simple_t *S, const double *r, double *x)
{
    int64_t nv = S->nv;
    const int64_t *rp = S->rowptr;
    const int32_t *col = S->col;
    const double *val = S->val;
    double *zu = S->tmp;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int d = 0; d < 3; ++d) s += S->Finv[9 * v + 3 * c + d] * r[3 * v + d];
            zu[3 * v + c] = s;
        }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        int64_t row = 3 * nv + v;
        double s = r[row];
        for (int64_t p = rp[row]; p < rp[row + 1]; ++p)
            if (col[p] < 3 * nv) s -= val[p] * zu[col[p]];
        x[row] = s;
    }
    if (S->degree > 0) {
        double *t = S->cw + 6 * nv;
        memcpy(t, x + 3 * nv, sizeof(double) * nv);
        schur_cheb(S, t, x + 3 * nv);
    } else {
        for (int64_t v = 0; v < nv; ++v) x[3 * nv + v] *= S->Sinv[v];
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < 3 * nv; ++i) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (col[p] >= 3 * nv) s += val[p] * x[col[p]];
        x[i] = zu[i] - S->Dinv[i] * s;
    }
}

/*
 * Right-preconditioned restarted GMRES(m) with classical Gram-Schmidt applied
 * twice, Givens rotations on the Hessenberg matrix, and the SIMPLE
 * preconditioner (Sec. 2.4) whose Schur block S~ = C - B D^{-1} G is inverted
 * either by its diagonal (cheb_degree = 0) or by a Chebyshev polynomial of
 * the given degree in diag(S~)^{-1} S~.  Stops when ||b - A x|| <= rtol ||b||, checked with the true
 * residual at every restart.  x holds the initial guess on entry.  Returns the
 * number of iterations, or -1 if max_iters is reached first.  res_out gets
 * the final true relative residual.
 */
int64_t orc_gmres_simple(int64_t nv, const int64_t *rowptr, const int32_t *col, const double *val,
                         const double *b, double *x, int32_t m, double rtol, int64_t max_iters,
                         int32_t cheb_degree, double cheb_ratio, double *res_out)
{
    int64_t N = 4 * nv;
    simple_t S = {nv, rowptr, col, val, malloc(sizeof(double) * 3 * nv),
                  malloc(sizeof(double) * 9 * nv), malloc(sizeof(double) * nv),
                  malloc(sizeof(double) * N), cheb_degree, cheb_ratio, 0.0,
                  malloc(sizeof(double) * 7 * nv)};
    double *V = malloc(sizeof(double) * (size_t)N * (m + 1));
    double *w = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *gv = malloc(sizeof(double) * (m + 1)), *y = malloc(sizeof(double) * m);
    double *h1 = malloc(sizeof(double) * (m + 1));
    simple_setup(&S);

    double bnorm = sqrt(dot(N, b, b));
    if (bnorm == 0.0) bnorm = 1.0;
    int64_t it = 0;
    double rel = 0.0;
    for (;;) {
        csr_mv(N, rowptr, col, val, x, w);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) w[i] = b[i] - w[i];
        double beta = sqrt(dot(N, w, w));
        rel = beta / bnorm;
        if (rel <= rtol || it >= max_iters) break;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) V[i] = w[i] / beta;
        memset(gv, 0, sizeof(double) * (m + 1));
        gv[0] = beta;
        int k = 0;
        for (; k < m && it < max_iters; ++k, ++it) {
            double *vk = V + (size_t)k * N, *vn = V + (size_t)(k + 1) * N;
            simple_apply(&S, vk, z);
            csr_mv(N, rowptr, col, val, z, w);
            for (int j = 0; j <= k; ++j) H[j * m + k] = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int j = 0; j <= k; ++j) h1[j] = dot(N, V + (size_t)j * N, w);
                for (int j = 0; j <= k; ++j) {
                    const double *vj = V + (size_t)j * N;
#pragma omp parallel for schedule(static)
                    for (int64_t i = 0; i < N; ++i) w[i] -= h1[j] * vj[i];
                    H[j * m + k] += h1[j];
                }
            }
            double hn = sqrt(dot(N, w, w));
            H[(k + 1) * m + k] = hn;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) vn[i] = (hn > 0.0) ? w[i] / hn : 0.0;
            for (int j = 0; j < k; ++j) {
                double t = cs[j] * H[j * m + k] + sn[j] * H[(j + 1) * m + k];
                H[(j + 1) * m + k] = -sn[j] * H[j * m + k] + cs[j] * H[(j + 1) * m + k];
                H[j * m + k] = t;
            }
            double a = H[k * m + k], bb = H[(k + 1) * m + k];
            double r = hypot(a, bb);
            cs[k] = a / r;
            sn[k] = bb / r;
            H[k * m + k] = r;
            H[(k + 1) * m + k] = 0.0;
            gv[k + 1] = -sn[k] * gv[k];
            gv[k] = cs[k] * gv[k];
            if (fabs(gv[k + 1]) / bnorm <= rtol || hn == 0.0) { ++k; ++it; break; }
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = gv[i];
            for (int j = i + 1; j < k; ++j) s -= H[i * m + j] * y[j];
            y[i] = s / H[i * m + i];
        }
        memset(w, 0, sizeof(double) * N);
        for (int j = 0; j < k; ++j) {
            const double *vj = V + (size_t)j * N;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) w[i] += y[j] * vj[i];
        }
        simple_apply(&S, w, z);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) x[i] += z[i];
    }
    if (res_out) *res_out = rel;
    free(S.Dinv); free(S.Finv); free(S.Sinv); free(S.tmp); free(S.cw);
    free(V); free(w); free(z); free(H); free(cs); free(sn); free(gv); free(y); free(h1);
    return (rel <= rtol) ? it : -1;
}

/* ------------------------------------------------------------ P2-P1 element */

/* Local P2 nodes: vertices 0..3, then the midpoints of the edges
 * (0,1), (0,2), (0,3), (1,2), (1,3), (2,3) as nodes 4..9. */
static const int P2_EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

/* P2 basis values, gradients and (constant) Laplacians from the barycentric
 * coordinates lam and their gradients dl: phi_a = lam_a (2 lam_a - 1) at the
 * vertices, phi_ij = 4 lam_i lam_j at the edge midpoints. */
static void p2_basis(const double lam[4], const double dl[4][3], double phi[10], double dphi[10][3],
                     double lap[10])
{
    for (int a = 0; a < 4; ++a) {
        phi[a] = lam[a] * (2.0 * lam[a] - 1.0);
        for (int j = 0; j < 3; ++j) dphi[a][j] = (4.0 * lam[a] - 1.0) * dl[a][j];
        lap[a] = 4.0 * (dl[a][0] * dl[a][0] + dl[a][1] * dl[a][1] + dl[a][2] * dl[a][2]);
    }
    for (int e = 0; e < 6; ++e) {
        int i = P2_EDGE[e][0], k = P2_EDGE[e][1];
        phi[4 + e] = 4.0 * lam[i] * lam[k];
        for (int j = 0; j < 3; ++j) dphi[4 + e][j] = 4.0 * (lam[i] * dl[k][j] + lam[k] * dl[i][j]);
        lap[4 + e] = 8.0 * (dl[i][0] * dl[k][0] + dl[i][1] * dl[k][1] + dl[i][2] * dl[k][2]);
    }
}

/*
 * Element matrix Ke (34x34) and vector Fe (34) of the P2-P1 element.  Local
 * velocity index 3a+c (a = 0..9 P2 nodes), pressure 30+a (a = 0..3 vertices).
 * Nodal data: X, Xh (vertex coordinates, current and reference), uE, uB, uA, f
 * at the 10 P2 nodes, pE at the 4 vertices.  Quadrature: nq points with
 * barycentric coordinates qlam[nq][4] and weights qw summing to 1/6 (unit
 * simplex).  The same weak form as orc_element_p1, with -mu Lap terms in the
 * strong residuals (nonzero for P2).
 */
double orc_element_p2(const double X[4][3], const double Xh[4][3], const double uE[10][3],
                      const double uB[10][3], const double uA[10][3], const double pE[4],
                      const double f[10][3], const orc_params *P, int32_t nq, const double *qlam,
                      const double *qw, double Ke[34][34], double Fe[34])
{
    double Jinv[3][3];
    double det = jacobian(X, Jinv);
    double dl[4][3];
    for (int j = 0; j < 3; ++j) {
        dl[1][j] = Jinv[0][j];
        dl[2][j] = Jinv[1][j];
        dl[3][j] = Jinv[2][j];
        dl[0][j] = -(Jinv[0][j] + Jinv[1][j] + Jinv[2][j]);
    }
    double G[3][3], g[3];
    for (int i = 0; i < 3; ++i) {
        g[i] = Jinv[0][i] + Jinv[1][i] + Jinv[2][i];
        for (int j = 0; j < 3; ++j)
            G[i][j] = Jinv[0][i] * Jinv[0][j] + Jinv[1][i] * Jinv[1][j] + Jinv[2][i] * Jinv[2][j];
    }
    memset(Ke, 0, sizeof(double) * 34 * 34);
    memset(Fe, 0, sizeof(double) * 34);
    const double rho = P->rho, mu = P->mu, dt = P->dt, alpha = P->alpha;
    for (int q = 0; q < nq; ++q) {
        const double *lam = qlam + 4 * q;
        double w = qw[q] * fabs(det);
        double phi[10], dphi[10][3], lap[10];
        p2_basis(lam, dl, phi, dphi, lap);

        double uEq[3] = {0}, uBq[3] = {0}, uAq[3] = {0}, fq[3] = {0}, xh[3] = {0}, lapUE[3] = {0};
        double gradUE[3][3] = {{0}}, gradPE[3] = {0};
        for (int a = 0; a < 10; ++a)
            for (int c = 0; c < 3; ++c) {
                uEq[c] += phi[a] * uE[a][c];
                uBq[c] += phi[a] * uB[a][c];
                uAq[c] += phi[a] * uA[a][c];
                fq[c] += phi[a] * f[a][c];
                lapUE[c] += lap[a] * uE[a][c];
                for (int j = 0; j < 3; ++j) gradUE[c][j] += uE[a][c] * dphi[a][j];
            }
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) {
                xh[c] += lam[a] * Xh[a][c];
                gradPE[c] += pE[a] * dl[a][c];
            }
        double sigR = 0.0, riis2 = 0.0;
        for (int k = 0; k < P->n_riis; ++k) {
            const double *v = P->riis + 10 * k;
            double R = v[8], eps = v[9];
            double dlt = orc_delta(orc_valve_distance(xh, v), eps);
            sigR += R / eps * dlt;
            riis2 += (R * R) / (eps * eps) * dlt * dlt;
        }
        double us[3];
        for (int c = 0; c < 3; ++c) us[c] = uEq[c] - uAq[c];
        double tauM = 0.0, tauC = 0.0;
        if (P->stab != ORC_STAB_NONE) orc_tau(P, G, g, us, riis2, &tauM, &tauC);
        double Kv[3];
        for (int c = 0; c < 3; ++c) Kv[c] = fq[c] + rho * uBq[c] / dt + sigR * uAq[c];
        double at[3];
        for (int c = 0; c < 3; ++c) {
            double adv = 0.0;
            for (int j = 0; j < 3; ++j) adv += us[j] * gradUE[c][j];
            double rt = rho * (alpha * uEq[c] / dt + adv) + gradPE[c] - mu * lapUE[c] + sigR * uEq[c] - Kv[c];
            at[c] = tauM * rt;
        }
        double adv_phi[10], T[10][3][3], s[10];
        for (int a = 0; a < 10; ++a)
            adv_phi[a] = us[0] * dphi[a][0] + us[1] * dphi[a][1] + us[2] * dphi[a][2];
        for (int a = 0; a < 10; ++a)
            for (int c = 0; c < 3; ++c)
                for (int j = 0; j < 3; ++j) {
                    double t = (c == j) ? adv_phi[a] : 0.0;
                    if (P->stab == ORC_STAB_VMS_LES) t += us[c] * dphi[a][j];
                    if (P->stab == ORC_STAB_VMS_LES) t -= at[c] * dphi[a][j];
                    T[a][c][j] = rho * t;
                }
        for (int b = 0; b < 10; ++b)
            s[b] = rho * (alpha / dt * phi[b] + adv_phi[b]) - mu * lap[b] + sigR * phi[b];

        for (int a = 0; a < 10; ++a) {
            for (int c = 0; c < 3; ++c) {
                int ia = 3 * a + c;
                for (int b = 0; b < 10; ++b) {
                    double gg_ab = dphi[a][0] * dphi[b][0] + dphi[a][1] * dphi[b][1] + dphi[a][2] * dphi[b][2];
                    for (int d = 0; d < 3; ++d) {
                        double v = 0.0;
                        if (c == d) {
                            v += (rho * alpha / dt + sigR) * phi[a] * phi[b];
                            v += rho * phi[a] * adv_phi[b];
                            v += mu * gg_ab;
                        }
                        if (P->symgrad) v += mu * dphi[b][c] * dphi[a][d];
                        v += tauM * s[b] * T[a][c][d];
                        v += tauC * dphi[a][c] * dphi[b][d];
                        Ke[ia][3 * b + d] += w * v;
                    }
                }
                for (int b = 0; b < 4; ++b) {
                    double v = -lam[b] * dphi[a][c];
                    v += tauM * (dl[b][0] * T[a][c][0] + dl[b][1] * T[a][c][1] + dl[b][2] * T[a][c][2]);
                    Ke[ia][30 + b] += w * v;
                }
                double r = Kv[c] * phi[a];
                r += tauM * (Kv[0] * T[a][c][0] + Kv[1] * T[a][c][1] + Kv[2] * T[a][c][2]);
                Fe[ia] += w * r;
            }
        }
        for (int a = 0; a < 4; ++a) {
            for (int b = 0; b < 10; ++b)
                for (int d = 0; d < 3; ++d)
                    Ke[30 + a][3 * b + d] += w * (lam[a] * dphi[b][d] + tauM * s[b] * dl[a][d]);
            for (int b = 0; b < 4; ++b) {
                double gg_ab = dl[a][0] * dl[b][0] + dl[a][1] * dl[b][1] + dl[a][2] * dl[b][2];
                Ke[30 + a][30 + b] += w * tauM * gg_ab;
            }
            Fe[30 + a] += w * tauM * (Kv[0] * dl[a][0] + Kv[1] * dl[a][1] + Kv[2] * dl[a][2]);
        }
    }
    return det;
}

/* All P2-P1 element matrices of a mesh: nodes[e][10] are the global P2 node
 * ids (vertices then edges) of element e; fields are nodal arrays over the
 * P2 nodes (uE, uB, uA, f: [nu][3]) and the vertices (pE: [nv]); x and xh are
 * vertex coordinates.  Writes Ke_all[nt][34][34] and Fe_all[nt][34]. */
int64_t orc_elements_p2(int64_t nt, const double *x, const double *xh, const int32_t *tets,
                        const int32_t *nodes, const double *uE, const double *uB, const double *uA,
                        const double *pE, const double *f, const orc_params *P, int32_t nq,
                        const double *qlam, const double *qw, double *Ke_all, double *Fe_all)
{
    int64_t bad = nt;   /* first degenerate element, nt if none */
#pragma omp parallel for schedule(static) reduction(min : bad)
    for (int64_t e = 0; e < nt; ++e) {
        double X[4][3], Xh[4][3], ue[10][3], ub[10][3], ua[10][3], pe[4], fe[10][3];
        for (int a = 0; a < 4; ++a) {
            int32_t v = tets[4 * e + a];
            for (int c = 0; c < 3; ++c) {
                X[a][c] = x[3 * (int64_t)v + c];
                Xh[a][c] = xh[3 * (int64_t)v + c];
            }
            pe[a] = pE[v];
        }
        for (int a = 0; a < 10; ++a) {
            int64_t n = nodes[10 * e + a];
            for (int c = 0; c < 3; ++c) {
                ue[a][c] = uE[3 * n + c];
                ub[a][c] = uB[3 * n + c];
                ua[a][c] = uA ? uA[3 * n + c] : 0.0;
                fe[a][c] = f ? f[3 * n + c] : 0.0;
            }
        }
        double det = orc_element_p2(X, Xh, ue, ub, ua, pe, fe, P, nq, qlam, qw,
                                    (double(*)[34])(Ke_all + (size_t)e * 34 * 34), Fe_all + (size_t)e * 34);
        if (!(fabs(det) > 0.0) && e < bad) bad = e;
    }
    return bad < nt ? -(bad + 1) : 0;
}

/* ------------------------------------------------------------ mesh lifting */

/* Lifting problem of Sec. 2.1.1, eq. (lifting): -div(alpha sigma_L(d)) = 0 on the
 * reference mesh.  P1 element stiffness (12 x 12, index 3a+c) of
 *   harmonic (kind 0):  sigma_L = grad d
 *     K[3a+c][3b+d] = alpha vol delta_cd grad phi_a . grad phi_b
 *   linear elasticity (kind 1): sigma_L = E/(1+nu) sym grad d + E nu/((1+nu)(1-2nu)) div d I
 *     K[3a+c][3b+d] = alpha vol ( E/(1+nu) (delta_cd grad phi_a . grad phi_b
 *                                           + d_d phi_a d_c phi_b) / 2
 *                                 + E nu/((1+nu)(1-2nu)) d_c phi_a d_d phi_b )
 * (test function phi_a e_c, trial function phi_b e_d; the gradients are
 * constant on the element, so the one-point rule is exact).  Returns the volume. */
double orc_lifting_element(const double X[4][3], int32_t kind, double E, double nu, double alpha, double K[12][12])
{
    double M[4][4], Mi[4][4];
    /* barycentric gradients from the 4x4 system [1 x y z]: Mi rows 1..3 */
    for (int a = 0; a < 4; ++a) {
        M[a][0] = 1.0;
        for (int c = 0; c < 3; ++c) M[a][c + 1] = X[a][c];
    }
    /* Gauss-Jordan inverse with partial pivoting */
    double A[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) A[i][j] = j < 4 ? M[i][j] : (j - 4 == i ? 1.0 : 0.0);
    double det = 1.0;
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < 8; ++j) {
                double t = A[c][j];
                A[c][j] = A[piv][j];
                A[piv][j] = t;
            }
            det = -det;
        }
        det *= A[c][c];
        double inv = 1.0 / A[c][c];
        for (int j = 0; j < 8; ++j) A[c][j] *= inv;
        for (int r = 0; r < 4; ++r)
            if (r != c) {
                double f = A[r][c];
                for (int j = 0; j < 8; ++j) A[r][j] -= f * A[c][j];
            }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Mi[i][j] = A[i][j + 4];
    double g[4][3];   /* grad phi_a = column a of Mi, rows 1..3 */
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) g[a][c] = Mi[c + 1][a];
    double vol = fabs(det) / 6.0;
    double mu2 = E / (1.0 + nu), lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 4; ++b)
                for (int d = 0; d < 3; ++d) {
                    double gg = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
                    double v;
                    if (kind == 0)
                        v = (c == d) ? gg : 0.0;
                    else
                        v = mu2 * 0.5 * ((c == d ? gg : 0.0) + g[a][d] * g[b][c]) + lam * g[a][c] * g[b][d];
                    K[3 * a + c][3 * b + d] = alpha * vol * v;
                }
    return vol;
}

/* Every element's lifting stiffness on the reference coordinates xh, in COO
 * triplets (144 per element, element by element). */
void orc_lifting_matrix(int64_t nt, const double *xh, const int32_t *tets, int32_t kind, double E, double nu,
                        const double *alpha, int64_t *rows, int64_t *cols, double *vals)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nt; ++e) {
        double X[4][3], K[12][12];
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) X[a][c] = xh[3 * (int64_t)tets[4 * e + a] + c];
        orc_lifting_element(X, kind, E, nu, alpha[e], K);
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 12; ++j) {
                int64_t k = 144 * e + 12 * i + j;
                rows[k] = 3 * (int64_t)tets[4 * e + i / 3] + i % 3;
                cols[k] = 3 * (int64_t)tets[4 * e + j / 3] + j % 3;
                vals[k] = K[i][j];
            }
    }
}

/* Distance from point p to triangle (a, b, c): if the projection of p on the
 * triangle's plane lies inside the triangle, the distance to the plane;
 * otherwise the smallest distance to its three edges (as segments). */
static double seg_dist2(const double *p, const double *a, const double *b)
{
    double ab[3], ap[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ap[k] = p[k] - a[k];
    }
    double t = (ap[0] * ab[0] + ap[1] * ab[1] + ap[2] * ab[2]) / (ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double q = ap[k] - t * ab[k];
        d2 += q * q;
    }
    return d2;
}

double orc_point_triangle_distance(const double *p, const double *a, const double *b, const double *c)
{
    double u[3], v[3], w[3];
    for (int k = 0; k < 3; ++k) {
        u[k] = b[k] - a[k];
        v[k] = c[k] - a[k];
        w[k] = p[k] - a[k];
    }
    /* barycentric coordinates of the projection: solve [u.u u.v; u.v v.v] (s, t) = (w.u, w.v) */
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2], vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    double wu = w[0] * u[0] + w[1] * u[1] + w[2] * u[2], wv = w[0] * v[0] + w[1] * v[1] + w[2] * v[2];
    double den = uu * vv - uv * uv;
    double s = (vv * wu - uv * wv) / den, t = (uu * wv - uv * wu) / den;
    if (s >= 0.0 && t >= 0.0 && s + t <= 1.0) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double q = w[k] - s * u[k] - t * v[k];
            d2 += q * q;
        }
        return sqrt(d2);
    }
    double d2 = seg_dist2(p, a, b), e2 = seg_dist2(p, b, c), f2 = seg_dist2(p, c, a);
    if (e2 < d2) d2 = e2;
    if (f2 < d2) d2 = f2;
    return sqrt(d2);
}

/* Boundary-based stiffening (Sec. 2.1.1): distance from each element's
 * centroid (reference coordinates) to the nearest of the nf boundary faces. */
void orc_boundary_distance(int64_t nt, const double *xh, const int32_t *tets, int64_t nf, const int32_t *faces,
                           double *dist)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nt; ++e) {
        double p[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) p[c] += 0.25 * xh[3 * (int64_t)tets[4 * e + a] + c];
        double best = INFINITY;
        for (int64_t f = 0; f < nf; ++f) {
            double d = orc_point_triangle_distance(p, xh + 3 * (int64_t)faces[3 * f], xh + 3 * (int64_t)faces[3 * f + 1],
                                                   xh + 3 * (int64_t)faces[3 * f + 2]);
            if (d < best) best = d;
        }
        dist[e] = best;
    }
}

/* Threads used by the parallel loops (OpenMP builds); returns the count in effect. */
int32_t orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
