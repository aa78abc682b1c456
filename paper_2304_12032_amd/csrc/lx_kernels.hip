// HIP kernels for gfx950: P1-P1 VMS-LES element assembly and matrix-free FP64
// residual, boundary rows, SIMPLE block preconditioner, block-CSR SpMV and the
// GMRES orthogonalisation / Hessenberg kernels.
//
// The element integrals follow the fully discrete weak form of the paper
// (Sec. 2.3): BDF time term, semi-implicit advection with u* = u_EXT - u_ALE,
// gradient-gradient (optionally symmetric-gradient) diffusion, the RIIS
// resistive term with its smoothed delta (Sec. 2.1.2), SUPG-PSPG + grad-div,
// the VMS cross term and the semi-implicit LES term, with tau_M, tau_C built
// from the metric tensor G = J^{-T} J^{-1} and vector g = J^{-T} 1.
//
// Unlike a per-entry evaluation, the P1 assembly accumulates a handful of
// per-element moments over the quadrature points (X_ab, Y_bc, Z_a, W_c, S_b,
// sum tau_M, sum tau_C and three right-hand-side moments): for P1 every basis
// gradient is constant on the element, so each stabilised entry factors into
// a gradient product times a quadrature sum.  One thread per element writes
// these moments as a small record; a second pass, one thread per block of the
// pattern, expands and sums the records of the elements sharing that block in
// a fixed order, so the matrix is built without atomics and deterministically.
#include <hip/hip_ext.h>

#include <cstdlib>

#include "lx_device.h"
#include "lx_kernels.h"

namespace lx {

// symmetric 4-point degree-2 rule: barycentric (qa, qb, qb, qb) and permutations
#define LX_QA 0.58541019662496845446
#define LX_QB 0.13819660112501051518

// ------------------------------------------------------------------ element data

template <typename T>
struct Elem {
    int32_t v[4];
    T dphi[4][3];
    T G[3][3], g[3], GG, gg;
    T vol;
    T uE[4][3];   // u_EXT at the vertices
    T K0[4][3];   // f + rho u_BDF / dt at the vertices
    T uA[4][3];   // u_ALE at the vertices
    T gU[3][3];   // grad u_EXT (constant), gU[c][j] = d_j u_c
    T gP[3];      // grad p_EXT (constant)
    T xh[4][3];   // reference coordinates (valve distance)
};

template <typename T>
__device__ inline bool load_elem(Elem<T> &E, int64_t e, int64_t nt, const int32_t *tet, const double *x,
                                 const double *xh, const double *h0, const double *h1, const double *h2,
                                 const double *uA, const double *f, const StepCoef &C)
{
#pragma unroll
    for (int a = 0; a < 4; ++a) E.v[a] = tet[a * nt + e];
    // edge vectors and J^{-1} in FP64 (an FP32 inverse of a flat element loses
    // digits in every gradient), then rounded to T
    double X0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) X0[i] = x[3 * (int64_t)E.v[0] + i];
    double J[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) J[i][k] = x[3 * (int64_t)E.v[k + 1] + i] - X0[i];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    double Ji[3][3];
    Ji[0][0] = c00 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][0] = c01 * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][0] = c02 * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    E.vol = (T)(fabs(det) / 6.0);
    // J^{-1} rounded to T; the gradients, G and g are formed from it in T so that
    // sum_a grad phi_a = 0 holds in T arithmetic as well
    T Jt[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Jt[i][j] = (T)Ji[i][j];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        E.dphi[1][j] = Jt[0][j];
        E.dphi[2][j] = Jt[1][j];
        E.dphi[3][j] = Jt[2][j];
        E.dphi[0][j] = -(Jt[0][j] + Jt[1][j] + Jt[2][j]);
    }
    E.GG = 0;
    E.gg = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        E.g[i] = Jt[0][i] + Jt[1][i] + Jt[2][i];
        E.gg += E.g[i] * E.g[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            E.G[i][j] = Jt[0][i] * Jt[0][j] + Jt[1][i] * Jt[1][j] + Jt[2][i] * Jt[2][j];
            E.GG += E.G[i][j] * E.G[i][j];
        }
    }
    const double *H[3] = {h0, h1, h2};
    const double rdt = C.rho / C.dt;
#pragma unroll
    for (int j = 0; j < 3; ++j) E.gP[j] = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int64_t v = E.v[a];
        double ue[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, pe = 0;
        for (int l = 0; l < C.nlev; ++l) {
            const double *h = H[l] + 4 * v;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ue[c] += C.gamma[l] * h[c];
                ub[c] += C.beta[l] * h[c];
            }
            pe += C.gamma[l] * h[3];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            E.uE[a][c] = (T)ue[c];
            E.K0[a][c] = (T)((f ? f[3 * v + c] : 0.0) + rdt * ub[c]);
            E.uA[a][c] = uA ? (T)uA[3 * v + c] : T(0);
            E.xh[a][c] = (T)xh[3 * v + c];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) E.gP[j] += (T)pe * E.dphi[a][j];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            E.gU[c][j] = E.uE[0][c] * E.dphi[0][j] + E.uE[1][c] * E.dphi[1][j] + E.uE[2][c] * E.dphi[2][j] +
                         E.uE[3][c] * E.dphi[3][j];
    return det != 0.0;
}

// Quadrature-point quantities shared by assembly and residual.
template <typename T>
struct QP {
    T lam[4];
    T uEq[3], uAq[3], Kv[3], us[3], dv[3];
    T Aq, sigR, tauM, tauC;
    T adv[4];
    T s[4];
};

template <typename T>
__device__ inline void eval_qp(const Elem<T> &E, int q, const StepCoef &C, QP<T> &Q)
{
    const T qa = (T)LX_QA, qb = (T)LX_QB, dq = qa - qb;
#pragma unroll
    for (int a = 0; a < 4; ++a) Q.lam[a] = (a == q) ? qa : qb;
    T xq[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Q.uEq[c] = qb * (E.uE[0][c] + E.uE[1][c] + E.uE[2][c] + E.uE[3][c]) + dq * E.uE[q][c];
        Q.uAq[c] = qb * (E.uA[0][c] + E.uA[1][c] + E.uA[2][c] + E.uA[3][c]) + dq * E.uA[q][c];
        T k0 = qb * (E.K0[0][c] + E.K0[1][c] + E.K0[2][c] + E.K0[3][c]) + dq * E.K0[q][c];
        Q.Kv[c] = k0;
        xq[c] = qb * (E.xh[0][c] + E.xh[1][c] + E.xh[2][c] + E.xh[3][c]) + dq * E.xh[q][c];
    }
    // RIIS: sigma_R = sum R/eps delta(phi), riis2 = sum R^2/eps^2 delta^2
    T sigR = 0, riis2 = 0;
    for (int k = 0; k < C.n_valves; ++k) {
        const double *vp = C.valve[k];
        T rel[3] = {xq[0] - (T)vp[0], xq[1] - (T)vp[1], xq[2] - (T)vp[2]};
        T z = rel[0] * (T)vp[3] + rel[1] * (T)vp[4] + rel[2] * (T)vp[5];
        T p0 = rel[0] - z * (T)vp[3], p1 = rel[1] - z * (T)vp[4], p2 = rel[2] - z * (T)vp[5];
        T rp = lx_sqrt(p0 * p0 + p1 * p1 + p2 * p2);
        T dr = 0;
        if (rp < (T)vp[6]) dr = (T)vp[6] - rp;
        if (rp > (T)vp[7]) dr = rp - (T)vp[7];
        T phi = lx_sqrt(z * z + dr * dr);
        T eps = (T)vp[9];
        if (phi <= eps) {
            T dl = (T(1) + lx_cos((T)M_PI * phi / eps)) / (T(2) * eps);
            T ratio = (T)vp[8] / eps;
            sigR += ratio * dl;
            riis2 += ratio * ratio * dl * dl;
        }
    }
    Q.sigR = sigR;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Q.us[c] = Q.uEq[c] - Q.uAq[c];
        Q.Kv[c] += sigR * Q.uAq[c];
    }
    const T rho = (T)C.rho, adt = (T)(C.alpha / C.dt);
    Q.Aq = rho * adt + sigR;
    Q.tauM = 0;
    Q.tauC = 0;
    if (C.stab != LX_STAB_NONE) {
        T uGu = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) uGu += Q.us[i] * E.G[i][j] * Q.us[j];
        T tsum = (T)(C.sigma * C.sigma * C.rho * C.rho / (C.dt * C.dt)) + rho * rho * uGu +
                 (T)(C.C_r * C.mu * C.mu) * E.GG + riis2;
        Q.tauM = T(1) / lx_sqrt(tsum);
        Q.tauC = T(1) / (Q.tauM * E.gg);
    }
    // dv = rho (u* - tau_M r_M(u_EXT, p_EXT)) used by the VMS and LES parts
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T adv = Q.us[0] * E.gU[c][0] + Q.us[1] * E.gU[c][1] + Q.us[2] * E.gU[c][2];
        T rt = rho * (adt * Q.uEq[c] + adv) + E.gP[c] + sigR * Q.uEq[c] - Q.Kv[c];
        Q.dv[c] = (C.stab == LX_STAB_VMS_LES) ? rho * (Q.us[c] - Q.tauM * rt) : T(0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        Q.adv[a] = Q.us[0] * E.dphi[a][0] + Q.us[1] * E.dphi[a][1] + Q.us[2] * E.dphi[a][2];
        Q.s[a] = Q.Aq * Q.lam[a] + rho * Q.adv[a];
    }
}

// ------------------------------------------------------------------ assembly

// Record layout: groups of four values, so that the slot gather reads each with
// one vector load (offsets into the kRStride values of an element):
//   D_v = (grad phi_v, Z_v), E_v = (Y_v, S_v), X_v = (X_v0 .. X_v3) with
//   X_ab = X_ab + mu|K| grad phi_a . grad phi_b, G1 = (W, sum w tau_C),
//   G2 = (sum w tau_M, mu|K|, |K|/4, 0).  The right-hand side (u_x, u_y, u_z, p) of
//   each vertex ([4][4] per element) follows all nt records, so that the records the
//   gather revisits for the element's other vertex rows are as small as they can be
//   and more of them stay in a die's L2 meanwhile.
enum : int {
    kRD = 0,        // D_v [4][4]
    kRE = 16,       // E_v [4][4]
    kRX = 32,       // X_v [4][4]
    kRG1 = 48,      // W[3], sum w tau_C
    kRG2 = 52,      // sum w tau_M, mu|K|, |K|/4, 0
    kRStride = 56   // values per record; the right-hand side block starts at nt kRStride
};
static_assert(kRStride + 16 <= kRec, "element record too small");

// Element pass of the assembly: one thread per element evaluates the quadrature
// moments and writes the element's record.
template <typename T, bool RHS>
__global__ __launch_bounds__(256) void k_element_p1(AsmArgs<T> A, StepCoef C)
{
    const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
    if (e >= A.nt) return;
    Elem<T> E;
    load_elem<T>(E, e, A.nt, A.tet, A.x, A.xh, A.h0, A.h1, A.h2, A.uA, A.f, C);
    const T rho = (T)C.rho;
    const T w = E.vol * T(0.25);
    T X[4][4], Y[4][3], Z[4], W[3], S[4], TC = 0, TM = 0;
    T KP[4][3], KW[3][3], KT[3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        Z[a] = 0;
        S[a] = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) X[a][b] = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Y[a][c] = 0;
            KP[a][c] = 0;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        W[c] = 0;
        KT[c] = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j) KW[c][j] = 0;
    }

#pragma unroll
    for (int q = 0; q < 4; ++q) {
        QP<T> Q;
        eval_qp<T>(E, q, C, Q);
        const T wt = w * Q.tauM;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                X[a][b] += w * (Q.Aq * Q.lam[a] * Q.lam[b] + rho * Q.lam[a] * Q.adv[b]) +
                           wt * rho * Q.s[b] * Q.adv[a];
            Z[a] += wt * rho * Q.adv[a];
            S[a] += wt * Q.s[a];
#pragma unroll
            for (int c = 0; c < 3; ++c) Y[a][c] += wt * Q.s[a] * Q.dv[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) W[c] += wt * Q.dv[c];
        TC += w * Q.tauC;
        TM += wt;
        if (RHS) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) KP[a][c] += w * Q.Kv[c] * (Q.lam[a] + Q.tauM * rho * Q.adv[a]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                KT[c] += wt * Q.Kv[c];
#pragma unroll
                for (int j = 0; j < 3; ++j) KW[c][j] += wt * Q.dv[c] * Q.Kv[j];
            }
        }
    }
    const T mv = (T)C.mu * E.vol;
    T *R = A.rec + (int64_t)e * kRStride;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            R[kRD + 4 * a + d] = E.dphi[a][d];
            R[kRE + 4 * a + d] = Y[a][d];
        }
        R[kRD + 4 * a + 3] = Z[a];
        R[kRE + 4 * a + 3] = S[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T gab = E.dphi[a][0] * E.dphi[b][0] + E.dphi[a][1] * E.dphi[b][1] + E.dphi[a][2] * E.dphi[b][2];
            R[kRX + 4 * a + b] = X[a][b] + mv * gab;
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) R[kRG1 + c] = W[c];
    R[kRG1 + 3] = TC;
    R[kRG2] = TM;
    R[kRG2 + 1] = mv;
    R[kRG2 + 2] = E.vol * T(0.25);   // integral of one basis function
    R[kRG2 + 3] = T(0);
    if (RHS) {
        T *Rr = A.rec + (int64_t)A.nt * kRStride + 16 * e;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Rr[4 * a + c] = KP[a][c] + KW[c][0] * E.dphi[a][0] + KW[c][1] * E.dphi[a][1] +
                                KW[c][2] * E.dphi[a][2];
            Rr[4 * a + 3] = KT[0] * E.dphi[a][0] + KT[1] * E.dphi[a][1] + KT[2] * E.dphi[a][2];
        }
    }
}

// What one (block, element) pair reads from the element's record.
template <typename T, bool RHS>
struct SlotIn {
    typename V4<T>::type Da, Db, Eb, G1, G2, Rh;
    T Xab;
    int64_t e;
    int a, b;
};

template <typename T, bool RHS>
__device__ __forceinline__ void slot_load(const T *__restrict__ rec, const T *__restrict__ rhs, int32_t code,
                                          SlotIn<T, RHS> &s)
{
    using V = typename V4<T>::type;
    s.e = code >> 4;
    s.a = (code >> 2) & 3;
    s.b = code & 3;
    const V *R = reinterpret_cast<const V *>(rec + s.e * kRStride);
    s.Da = R[kRD / 4 + s.a];
    s.Db = R[kRD / 4 + s.b];
    s.Eb = R[kRE / 4 + s.b];
    s.Xab = rec[s.e * kRStride + kRX + 4 * s.a + s.b];
    s.G1 = R[kRG1 / 4];
    s.G2 = R[kRG2 / 4];
    if (RHS && s.a == s.b) s.Rh = reinterpret_cast<const V *>(rhs + 16 * s.e)[s.a];
}

template <typename T, bool RHS>
__device__ __forceinline__ void slot_add(const SlotIn<T, RHS> &s, int symgrad, T acc[16], T racc[4])
{
    const T da[3] = {s.Da.v[0], s.Da.v[1], s.Da.v[2]}, db[3] = {s.Db.v[0], s.Db.v[1], s.Db.v[2]};
    const T Yb[3] = {s.Eb.v[0], s.Eb.v[1], s.Eb.v[2]}, W[3] = {s.G1.v[0], s.G1.v[1], s.G1.v[2]};
    const T Xab = s.Xab, Za = s.Da.v[3], Sb = s.Eb.v[3];
    const T TC = s.G1.v[3], TM = s.G2.v[0], w1 = s.G2.v[2];
    const T mv = symgrad ? s.G2.v[1] : T(0);
    const T gab = da[0] * db[0] + da[1] * db[1] + da[2] * db[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            T F = da[d] * Yb[c] + TC * da[c] * db[d] + mv * db[c] * da[d];
            if (c == d) F += Xab;
            acc[3 * c + d] += F;
        }
        acc[9 + c] += -w1 * da[c] + db[c] * Za + gab * W[c];
        acc[12 + c] += w1 * db[c] + da[c] * Sb;
    }
    acc[15] += TM * gab;
    if (RHS && s.a == s.b)
#pragma unroll
        for (int c = 0; c < 4; ++c) racc[c] += s.Rh.v[c];
}

// Slot pass: every block (i, j) of the pattern sums, in the fixed order of its
// incidence list, the 4x4 block (a, b) of each element containing the edge
// (i, j), expanded from the element's record:
//   F_cd = dphi_a,d Y_b,c + tau_C dphi_a,c dphi_b,d + [c = d] X_ab (+ mu|K| dphi_b,c dphi_a,d)
//   G_c  = -|K|/4 dphi_a,c + dphi_b,c Z_a + (dphi_a . dphi_b) W_c
//   B_c  =  |K|/4 dphi_b,c + dphi_a,c S_b
//   C    = (sum tau_M w) (dphi_a . dphi_b)
// Sums run in T (the assembly precision) and each plane entry is written once (no atomics).  With
// RHS, the diagonal slot of vertex i also gathers the vertex's right-hand side.
// The list is walked two elements at a time with the next two codes loaded ahead, so that a
// lane keeps two records' loads and the following codes in flight instead of one
// code-then-record round trip per element; the sum order is the list order all the same.
template <typename T, bool RHS>
__global__ __launch_bounds__(256) void k_gather_p1(AsmArgs<T> A, int symgrad)
{
    const int64_t k = xcd_block() * blockDim.x + threadIdx.x;
    if (k >= A.nblk) return;
    T acc[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) acc[p] = 0;
    T racc[4] = {0, 0, 0, 0};
    int64_t ediag = -1;
    int adiag = 0;
    const T *rhs = A.rec + (int64_t)A.nt * kRStride;
    const int32_t q1 = A.sinc_ptr[k + 1];
    int32_t q = A.sinc_ptr[k];
    int32_t c0 = q < q1 ? A.sinc[q] : 0, c1 = q + 1 < q1 ? A.sinc[q + 1] : 0;
    for (; q + 1 < q1; q += 2) {
        // the next two codes, unconditionally (clamped to the list's last entry, whose value is
        // then unused), so that no branch joins the loads and their wait moves to the next trip
        const int32_t n0 = A.sinc[min(q + 2, q1 - 1)], n1 = A.sinc[min(q + 3, q1 - 1)];
        SlotIn<T, RHS> s0, s1;
        slot_load<T, RHS>(A.rec, rhs, c0, s0);
        slot_load<T, RHS>(A.rec, rhs, c1, s1);
        __builtin_amdgcn_sched_barrier(0);   // both records' loads issue before any arithmetic
        slot_add<T, RHS>(s0, symgrad, acc, racc);
        slot_add<T, RHS>(s1, symgrad, acc, racc);
        if (RHS && s1.a == s1.b) {
            ediag = s1.e;
            adiag = s1.a;
        }
        c0 = n0;
        c1 = n1;
    }
    if (q < q1) {
        SlotIn<T, RHS> s0;
        slot_load<T, RHS>(A.rec, rhs, c0, s0);
        slot_add<T, RHS>(s0, symgrad, acc, racc);
        if (RHS && s0.a == s0.b) {
            ediag = s0.e;
            adiag = s0.a;
        }
    }
    // the planes are read by later kernels only: streaming stores leave the L2 to the records
#pragma unroll
    for (int p = 0; p < 16; ++p) __builtin_nontemporal_store(acc[p], A.val + (int64_t)p * A.nblk + k);
    if (RHS && ediag >= 0) {
        T *r = A.rhs + 4 * A.tet[(int64_t)adiag * A.nt + ediag];
#pragma unroll
        for (int c = 0; c < 4; ++c) r[c] = (T)racc[c];
    }
}

template <typename T>
void launch_assemble_p1(const AsmArgs<T> &a, const StepCoef &c, hipStream_t s)
{
    const dim3 ge((unsigned)((a.nt + 255) / 256)), gs((unsigned)((a.nblk + 255) / 256));
    if (a.rhs) {
        hipLaunchKernelGGL((k_element_p1<T, true>), ge, dim3(256), 0, s, a, c);
        hipLaunchKernelGGL((k_gather_p1<T, true>), gs, dim3(256), 0, s, a, c.symgrad);
    } else {
        hipLaunchKernelGGL((k_element_p1<T, false>), ge, dim3(256), 0, s, a, c);
        hipLaunchKernelGGL((k_gather_p1<T, false>), gs, dim3(256), 0, s, a, c.symgrad);
    }
}
template void launch_assemble_p1<double>(const AsmArgs<double> &, const StepCoef &, hipStream_t);
template void launch_assemble_p1<float>(const AsmArgs<float> &, const StepCoef &, hipStream_t);

// ------------------------------------------------------------------ FP64 residual

// r = b - A xs on every row except Dirichlet velocity rows, evaluated element
// by element at the quadrature points from the strong residual of the iterate
// (no matrix is formed).  FULL: also b and the FP64 diagonal of the Dirichlet
// velocity rows (a separate instance, so the plain residual keeps fewer
// registers live).  The element pass writes each element's vertex
// contributions to a record; k_residual_gather sums them per vertex in the
// fixed order of the vertex's incidence list.
template <bool FULL>
__global__ __launch_bounds__(256) void k_residual_p1(ResArgs A, StepCoef C)
{
    const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
    if (e >= A.nt) return;
    Elem<double> E;
    load_elem<double>(E, e, A.nt, A.tet, A.x, A.xh, A.h0, A.h1, A.h2, A.uA, A.f, C);
    const double rho = C.rho, mu = C.mu;
    const double w = E.vol * 0.25;
    double xu[4][3], xp[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double *p = A.xs + 4 * (int64_t)E.v[a];
#pragma unroll
        for (int c = 0; c < 3; ++c) xu[a][c] = p[c];
        xp[a] = p[3];
    }
    double gX[3][3], gXP[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            gX[c][j] = xu[0][c] * E.dphi[0][j] + xu[1][c] * E.dphi[1][j] + xu[2][c] * E.dphi[2][j] +
                       xu[3][c] * E.dphi[3][j];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) gXP[j] += xp[a] * E.dphi[a][j];
    const double divX = gX[0][0] + gX[1][1] + gX[2][2];
    int32_t dir[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) dir[a] = A.dir_index[E.v[a]];

    double ru[4][3], rp[4], bu[4][3], bp[4], dg[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        rp[a] = bp[a] = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) ru[a][c] = bu[a][c] = dg[a][c] = 0;
    }
    const double qa = LX_QA, qb = LX_QB, dq = qa - qb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        QP<double> Q;
        eval_qp<double>(E, q, C, Q);
        double xuq[3], xpq;
#pragma unroll
        for (int c = 0; c < 3; ++c) xuq[c] = qb * (xu[0][c] + xu[1][c] + xu[2][c] + xu[3][c]) + dq * xu[q][c];
        xpq = qb * (xp[0] + xp[1] + xp[2] + xp[3]) + dq * xp[q];
        double rM[3], advX[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            advX[c] = Q.us[0] * gX[c][0] + Q.us[1] * gX[c][1] + Q.us[2] * gX[c][2];
            rM[c] = Q.Aq * xuq[c] + rho * advX[c] + gXP[c] - Q.Kv[c];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double la = Q.lam[a], ad = Q.adv[a];
            const double rMd = rM[0] * E.dphi[a][0] + rM[1] * E.dphi[a][1] + rM[2] * E.dphi[a][2];
            const double Kd = Q.Kv[0] * E.dphi[a][0] + Q.Kv[1] * E.dphi[a][1] + Q.Kv[2] * E.dphi[a][2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double gal = Q.Kv[c] * la - Q.Aq * xuq[c] * la - rho * advX[c] * la -
                             mu * (gX[c][0] * E.dphi[a][0] + gX[c][1] * E.dphi[a][1] + gX[c][2] * E.dphi[a][2]) +
                             xpq * E.dphi[a][c];
                if (C.symgrad)
                    gal -= mu * (gX[0][c] * E.dphi[a][0] + gX[1][c] * E.dphi[a][1] + gX[2][c] * E.dphi[a][2]);
                double st = -Q.tauM * (rho * ad * rM[c] + Q.dv[c] * rMd) - Q.tauC * divX * E.dphi[a][c];
                ru[a][c] += w * (gal + st);
                if (FULL) bu[a][c] += w * (Q.Kv[c] * la + Q.tauM * (rho * ad * Q.Kv[c] + Q.dv[c] * Kd));
                if (FULL && dir[a] >= 0) {
                    const double dca = E.dphi[a][c];
                    dg[a][c] += w * (Q.Aq * la * la + rho * la * ad +
                                     Q.tauM * Q.s[a] * (rho * ad + Q.dv[c] * dca) + Q.tauC * dca * dca);
                }
            }
            rp[a] += w * (-la * divX - Q.tauM * rMd);
            if (FULL) bp[a] += w * Q.tauM * Kd;
        }
    }
    const double mv = mu * E.vol;
    const int64_t n4 = 4 * A.nt;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const bool free_u = dir[a] < 0;
        double *R = A.rec + 4 * (int64_t)A.vpos[(int64_t)a * A.nt + e];
#pragma unroll
        for (int c = 0; c < 3; ++c) R[c] = free_u ? ru[a][c] : 0.0;
        R[3] = rp[a];
        if (FULL) {
#pragma unroll
            for (int c = 0; c < 3; ++c) R[4 * n4 + c] = free_u ? bu[a][c] : 0.0;
            R[4 * n4 + 3] = bp[a];
        }
        if (FULL && !free_u) {   // read back for Dirichlet vertices only
            const double gaa = E.dphi[a][0] * E.dphi[a][0] + E.dphi[a][1] * E.dphi[a][1] + E.dphi[a][2] * E.dphi[a][2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double d = dg[a][c] + mv * gaa;
                if (C.symgrad) d += mv * E.dphi[a][c] * E.dphi[a][c];
                R[8 * n4 + c] = d;
            }
        }
    }
}

// Vertex pass of the residual: sums the contributions of the elements around
// each vertex, which lie one after the other in vertex-incidence order (the
// order of the vertex's diagonal-block incidence list), and writes r, b and the
// Dirichlet diagonal once.
__global__ __launch_bounds__(256) void k_residual_gather(ResArgs A)
{
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= A.nv) return;
    const int64_t n4 = 4 * A.nt;
    const int32_t di = A.dir_index[i];
    const bool want_dg = A.dg && di >= 0;
    double r[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0}, d[3] = {0, 0, 0};
    for (int32_t q = A.vinc_ptr[i]; q < A.vinc_ptr[i + 1]; ++q) {
        const double *R = A.rec + 4 * (int64_t)q;
        using V = typename V4<double>::type;
        const V rv = *reinterpret_cast<const V *>(R);
#pragma unroll
        for (int c = 0; c < 4; ++c) r[c] += rv.v[c];
        if (A.b) {
            const V bv = *reinterpret_cast<const V *>(R + 4 * n4);
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] += bv.v[c];
        }
        if (want_dg)
#pragma unroll
            for (int c = 0; c < 3; ++c) d[c] += R[8 * n4 + c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) A.r[4 * i + c] = r[c];
    if (A.b)
#pragma unroll
        for (int c = 0; c < 4; ++c) A.b[4 * i + c] = b[c];
    if (want_dg)
#pragma unroll
        for (int c = 0; c < 3; ++c) A.dg[3 * (int64_t)di + c] = d[c];
}

void launch_residual_p1(const ResArgs &a, const StepCoef &c, hipStream_t s)
{
    const dim3 g((unsigned)((a.nt + 255) / 256));
    if (a.b)
        hipLaunchKernelGGL(k_residual_p1<true>, g, dim3(256), 0, s, a, c);
    else
        hipLaunchKernelGGL(k_residual_p1<false>, g, dim3(256), 0, s, a, c);
    hipLaunchKernelGGL(k_residual_gather, dim3((unsigned)((a.nv + 255) / 256)), dim3(256), 0, s, a);
}

// ------------------------------------------------------------------ boundary data

__global__ void k_dirichlet_values(int64_t n_dir, const int32_t *dir_node, const int32_t *dir_bc, BCSet S,
                                   const double *x, const double *uA, const double *gnodal, double *g)
{
    const int64_t k = xcd_block() * blockDim.x + threadIdx.x;
    if (k >= n_dir) return;
    const int64_t v = dir_node[k];
    const BCVal &B = S.bc[dir_bc[k]];
    double out[3] = {0, 0, 0};
    if (B.type == LX_BC_NOSLIP) {
        if (uA)
            for (int c = 0; c < 3; ++c) out[c] = uA[3 * v + c];
    } else if (B.profile == LX_PROFILE_NODAL) {
        for (int c = 0; c < 3; ++c) out[c] = gnodal[3 * k + c];
    } else if (B.profile == LX_PROFILE_PARABOLIC) {
        double r2 = 0;
        for (int c = 0; c < 3; ++c) {
            double d = x[3 * v + c] - B.center[c];
            r2 += d * d;
        }
        const double R = B.radius;
        const double s = -2.0 * (R * R - r2) / (M_PI * R * R * R * R);
        for (int c = 0; c < 3; ++c) out[c] = B.scale * s * B.normal[c];
    } else {  // uniform
        for (int c = 0; c < 3; ++c) out[c] = -B.scale * B.normal[c];
    }
    for (int c = 0; c < 3; ++c) g[3 * k + c] = out[c];
}

void launch_dirichlet_values(int64_t n_dir, const int32_t *dir_node, const int32_t *dir_bc, const BCSet &bcs,
                             const double *x, const double *uA, const double *gnodal, double *g,
                             hipStream_t s)
{
    if (n_dir == 0) return;
    hipLaunchKernelGGL(k_dirichlet_values, dim3((unsigned)((n_dir + 255) / 256)), dim3(256), 0, s, n_dir,
                       dir_node, dir_bc, bcs, x, uA, gnodal, g);
}

// Dirichlet velocity rows: keep the diagonal entry a_ii of each component,
// zero the rest of the row (F and G parts), b_i = a_ii g_i.
template <typename T>
__global__ void k_dirichlet_rows(int64_t n_dir, const int32_t *dir_node, const double *g, RowPattern P, T *val,
                                 T *rhs)
{
    const int64_t k = xcd_block() * blockDim.x + threadIdx.x;
    if (k >= n_dir) return;
    const int64_t i = dir_node[k];
    const int64_t dk = P.diag[i];
    const int64_t nb = P.nblk;
    for (int64_t s = P.rowptr[i]; s < P.rowptr[i + 1]; ++s) {
        for (int c = 0; c < 3; ++c) {
            for (int d = 0; d < 3; ++d)
                if (s != dk || c != d) val[(3 * c + d) * nb + s] = T(0);
            val[(9 + c) * nb + s] = T(0);
        }
    }
    if (rhs)
        for (int c = 0; c < 3; ++c) rhs[4 * i + c] = (T)((double)val[(4 * c) * nb + dk] * g[3 * k + c]);
}

template <typename T>
void launch_dirichlet_rows(int64_t n_dir, const int32_t *dir_node, const double *g, const RowPattern &P, T *val,
                           T *rhs, hipStream_t s)
{
    if (n_dir == 0) return;
    hipLaunchKernelGGL((k_dirichlet_rows<T>), dim3((unsigned)((n_dir + 127) / 128)), dim3(128), 0, s, n_dir,
                       dir_node, g, P, val, rhs);
}
template void launch_dirichlet_rows<double>(int64_t, const int32_t *, const double *, const RowPattern &,
                                            double *, double *, hipStream_t);
template void launch_dirichlet_rows<float>(int64_t, const int32_t *, const double *, const RowPattern &,
                                           float *, float *, hipStream_t);

__global__ void k_dirichlet_residual(int64_t n_dir, const int32_t *dir_node, const double *g, const double *dg,
                                     const double *xs, double *r, double *b)
{
    const int64_t k = xcd_block() * blockDim.x + threadIdx.x;
    if (k >= n_dir) return;
    const int64_t i = dir_node[k];
    for (int c = 0; c < 3; ++c) {
        r[4 * i + c] = dg[3 * k + c] * (g[3 * k + c] - xs[4 * i + c]);
        if (b) b[4 * i + c] = dg[3 * k + c] * g[3 * k + c];
    }
}

void launch_dirichlet_residual(int64_t n_dir, const int32_t *dir_node, const double *g, const double *dg,
                               const double *xs, double *r, double *b, hipStream_t s)
{
    if (n_dir == 0) return;
    hipLaunchKernelGGL(k_dirichlet_residual, dim3((unsigned)((n_dir + 255) / 256)), dim3(256), 0, s, n_dir,
                       dir_node, g, dg, xs, r, b);
}

// Neumann term (h, v) on boundary triangles with a nodal (or constant) traction
// vector, linear on each face, integrated by the edge-midpoint rule.
__global__ void k_neumann(int64_t nf, const int32_t *faces, const double *x, const double *hn, double h0,
                          double h1, double h2, double *o0, double *o1, float *o32)
{
    const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
    if (e >= nf) return;
    int64_t v[3] = {faces[3 * e], faces[3 * e + 1], faces[3 * e + 2]};
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) {
        a[c] = x[3 * v[1] + c] - x[3 * v[0] + c];
        b[c] = x[3 * v[2] + c] - x[3 * v[0] + c];
    }
    double n0 = a[1] * b[2] - a[2] * b[1], n1 = a[2] * b[0] - a[0] * b[2], n2 = a[0] * b[1] - a[1] * b[0];
    double area = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    double h[3][3];
    for (int i = 0; i < 3; ++i) {
        h[i][0] = hn ? hn[3 * v[i]] : h0;
        h[i][1] = hn ? hn[3 * v[i] + 1] : h1;
        h[i][2] = hn ? hn[3 * v[i] + 2] : h2;
    }
    // int h_c phi_i = area/12 (2 h_i + h_j + h_k)
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) {
            double val = area / 12.0 * (2.0 * h[i][c] + h[(i + 1) % 3][c] + h[(i + 2) % 3][c]);
            if (o0) atomic_add(&o0[4 * v[i] + c], val);
            if (o1) atomic_add(&o1[4 * v[i] + c], val);
            if (o32) atomic_add(&o32[4 * v[i] + c], (float)val);
        }
}

void launch_neumann(int64_t nf, const int32_t *faces, const double *x, const double *hnodal, const double hc[3],
                    double *out0, double *out1, float *out32, hipStream_t s)
{
    if (nf == 0) return;
    hipLaunchKernelGGL(k_neumann, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, nf, faces, x, hnodal,
                       hc[0], hc[1], hc[2], out0, out1, out32);
}

// ------------------------------------------------------------------ SIMPLE

// D = diag(F); F~^{-1}: inverse of the nodal 3x3 diagonal block of F;
// with Sinv, also S~ = diag(C - B D^{-1} G), reading G_ji through the transposed
// slot (LPR lanes per row, partial sums combined by a fixed butterfly).
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_simple_setup(RowPattern P, const T *val, T *Finv, T *Dinv, T *Sinv)
{
    const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (i >= P.nv) return;
    const int64_t nb = P.nblk, nv = P.nv, dk = P.diag[i];
    if (Sinv) {
        T s = 0;
        for (int64_t k = P.rowptr[i] + lane; k < P.rowptr[i + 1]; k += LPR) {
            const int64_t j = P.col[k], ts = P.tslot[k], dj = P.diag[j];
            for (int d = 0; d < 3; ++d)
                s += val[(12 + d) * nb + k] * val[(9 + d) * nb + ts] / val[(4 * d) * nb + dj];
        }
        s = group_sum<T, LPR>(s);
        if (lane == 0) Sinv[i] = T(1) / (val[15 * nb + dk] - s);
    }
    if (lane != 0) return;
    T A[9];
    for (int p = 0; p < 9; ++p) A[p] = val[p * nb + dk];
    T c0 = A[4] * A[8] - A[5] * A[7], c1 = A[5] * A[6] - A[3] * A[8], c2 = A[3] * A[7] - A[4] * A[6];
    T id = T(1) / (A[0] * c0 + A[1] * c1 + A[2] * c2);
    T B[9] = {c0 * id, (A[2] * A[7] - A[1] * A[8]) * id, (A[1] * A[5] - A[2] * A[4]) * id,
              c1 * id, (A[0] * A[8] - A[2] * A[6]) * id, (A[2] * A[3] - A[0] * A[5]) * id,
              c2 * id, (A[1] * A[6] - A[0] * A[7]) * id, (A[0] * A[4] - A[1] * A[3]) * id};
    for (int p = 0; p < 9; ++p) Finv[p * nv + i] = (T)B[p];
    for (int c = 0; c < 3; ++c) Dinv[c * nv + i] = T(1) / A[4 * c];
}

// Sinv may be null (the AMG Schur block does not use diag(S~)).
template <typename T>
void launch_simple_setup(const RowPattern &P, const T *val, T *Finv, T *Dinv, T *Sinv, hipStream_t s)
{
    hipLaunchKernelGGL((k_simple_setup<T, 16>), dim3((unsigned)((P.nv * 16 + 255) / 256)), dim3(256), 0, s, P, val,
                       Finv, Dinv, Sinv);
}
template void launch_simple_setup<double>(const RowPattern &, const double *, double *, double *, double *,
                                          hipStream_t);
template void launch_simple_setup<float>(const RowPattern &, const float *, float *, float *, float *,
                                         hipStream_t);

constexpr int kLPR = 16;

// ---- Gershgorin bound of diag(S~)^{-1} S~

// ag[c][i] = |1/D_(i,c)| sum_j |G_ij[c]|
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_schur_ag(RowPattern P, const T *val, const T *Dinv, T *ag)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int64_t nb = P.nblk, nv = P.nv;
    T a0 = 0, a1 = 0, a2 = 0;
    for (int32_t k = P.rowptr[row] + lane; k < P.rowptr[row + 1]; k += LPR) {
        a0 += fabs(val[9 * nb + k]);
        a1 += fabs(val[10 * nb + k]);
        a2 += fabs(val[11 * nb + k]);
    }
    a0 = group_sum<T, LPR>(a0);
    a1 = group_sum<T, LPR>(a1);
    a2 = group_sum<T, LPR>(a2);
    if (lane == 0) {
        ag[row] = a0 * fabs(Dinv[row]);
        ag[nv + row] = a1 * fabs(Dinv[nv + row]);
        ag[2 * nv + row] = a2 * fabs(Dinv[2 * nv + row]);
    }
}

// gers[i] = |1/S~_ii| (sum_j |C_ij| + sum_j sum_d |B_ij[d]| ag[d][j])
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_schur_gers(RowPattern P, const T *val, const T *Sinv, const T *ag, T *gers)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int64_t nb = P.nblk, nv = P.nv;
    T a = 0;
    for (int32_t k = P.rowptr[row] + lane; k < P.rowptr[row + 1]; k += LPR) {
        const int64_t j = P.col[k];
        a += fabs(val[15 * nb + k]) + fabs(val[12 * nb + k]) * ag[j] + fabs(val[13 * nb + k]) * ag[nv + j] +
             fabs(val[14 * nb + k]) * ag[2 * nv + j];
    }
    a = group_sum<T, LPR>(a);
    if (lane == 0) gers[row] = a * fabs(Sinv[row]);
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_max(int64_t n, const T *x, GmState *st, double *partial)
{
    __shared__ double lds[4];
    double m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, (double)x[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
    if (!arrive_last(&st->counter)) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = 0;
        for (unsigned b = 0; b < gridDim.x; ++b) mm = fmax(mm, partial[b]);
        st->lam_max = mm;
        st->counter = 0;
    }
}

template <typename T>
void launch_schur_bound(const RowPattern &P, const T *val, const T *Dinv, const T *Sinv, T *work, GmState *st,
                        double *partial, int nb, hipStream_t s)
{
    const unsigned g = (unsigned)((P.nv * kLPR + 255) / 256);
    hipLaunchKernelGGL((k_schur_ag<T, kLPR>), dim3(g), dim3(256), 0, s, P, val, Dinv, work);
    hipLaunchKernelGGL((k_schur_gers<T, kLPR>), dim3(g), dim3(256), 0, s, P, val, Sinv, work, work + 3 * P.nv);
    hipLaunchKernelGGL((k_max<T>), dim3(nb), dim3(kRedThreads), 0, s, P.nv, work + 3 * P.nv, st, partial);
}
template void launch_schur_bound<double>(const RowPattern &, const double *, const double *, const double *,
                                         double *, GmState *, double *, int, hipStream_t);
template void launch_schur_bound<float>(const RowPattern &, const float *, const float *, const float *, float *,
                                        GmState *, double *, int, hipStream_t);

// ---- SIMPLE apply

// z.u = F~^{-1} (scale r.u)   (node-local); z.p = scale r.p for the next pass
template <typename T>
__global__ void k_simple_zu(int64_t nv, const T *Finv, const T *r, const double *scale_ptr, T *z,
                            const int32_t *done)
{
    if (done && *done) return;
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const T sc = scale_ptr ? (T)(*scale_ptr) : T(1);
    using V = typename V4<T>::type;
    V rv = reinterpret_cast<const V *>(r)[i];
    T r0 = rv.v[0] * sc, r1 = rv.v[1] * sc, r2 = rv.v[2] * sc;
    V zv;
    zv.v[0] = Finv[0 * nv + i] * r0 + Finv[1 * nv + i] * r1 + Finv[2 * nv + i] * r2;
    zv.v[1] = Finv[3 * nv + i] * r0 + Finv[4 * nv + i] * r1 + Finv[5 * nv + i] * r2;
    zv.v[2] = Finv[6 * nv + i] * r0 + Finv[7 * nv + i] * r1 + Finv[8 * nv + i] * r2;
    zv.v[3] = rv.v[3] * sc;
    reinterpret_cast<V *>(z)[i] = zv;
}

// t = z.p - sum_j B_ij z.u_j (z.p holds scale*r.p on entry); degree 0: z.p = S~^{-1}_diag t;
// degree > 0: Chebyshev step 0 (rc = t, cur.w = d0 = Sinv t / theta, z.p = d0).
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_simple_zp(RowPattern P, const T *val, const T *Sinv, T *z, int degree,
                                                   double ratio, T *rc, T *cur, const GmState *st,
                                                   const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int64_t nb = P.nblk;
    const int32_t beg = P.rowptr[row], end = P.rowptr[row + 1];
    using V = typename V4<T>::type;
    T acc = 0;
    for (int32_t k = beg + lane; k < end; k += LPR) {
        const V zj = reinterpret_cast<const V *>(z)[P.col[k]];
        acc += val[12 * nb + k] * zj.v[0] + val[13 * nb + k] * zj.v[1] + val[14 * nb + k] * zj.v[2];
    }
    acc = group_sum<T, LPR>(acc);
    if (lane == 0) {
        const T t = (T)(z[4 * row + 3] - acc);
        if (degree == 0) {
            z[4 * row + 3] = Sinv[row] * t;
        } else {
            double theta, a, b;
            cheb_coef(st->lam_max, ratio, 0, theta, a, b);
            const T d = Sinv[row] * t / (T)theta;
            rc[row] = t;
            cur[4 * row + 3] = d;
            z[4 * row + 3] = d;
        }
    }
}

// Chebyshev pass A: cur.xyz = D^{-1} (G d), d = cur.w   (velocity side of S~ d)
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_cheb_gd(RowPattern P, const T *val, const T *Dinv, T *cur,
                                                 const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int64_t nb = P.nblk, nv = P.nv;
    T a0 = 0, a1 = 0, a2 = 0;
    for (int32_t k = P.rowptr[row] + lane; k < P.rowptr[row + 1]; k += LPR) {
        const T dj = cur[4 * (int64_t)P.col[k] + 3];
        a0 += val[9 * nb + k] * dj;
        a1 += val[10 * nb + k] * dj;
        a2 += val[11 * nb + k] * dj;
    }
    a0 = group_sum<T, LPR>(a0);
    a1 = group_sum<T, LPR>(a1);
    a2 = group_sum<T, LPR>(a2);
    if (lane == 0) {
        cur[4 * row + 0] = (T)(Dinv[row] * a0);
        cur[4 * row + 1] = (T)(Dinv[nv + row] * a1);
        cur[4 * row + 2] = (T)(Dinv[2 * nv + row] * a2);
    }
}

// Chebyshev pass B (step i >= 1): q = C d - B y = S~ d with (y, d) = cur (one
// 4-vector gather per block); rc -= q; next.w = a d + b Sinv rc; z.p += next.w
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_cheb_step(RowPattern P, const T *val, const T *Sinv, const T *cur,
                                                   T *rc, T *next, T *z, int i, double ratio, const GmState *st,
                                                   const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int64_t nb = P.nblk;
    using V = typename V4<T>::type;
    T q = 0;
    for (int32_t k = P.rowptr[row] + lane; k < P.rowptr[row + 1]; k += LPR) {
        const V c = reinterpret_cast<const V *>(cur)[P.col[k]];
        q += val[15 * nb + k] * c.v[3] -
             (val[12 * nb + k] * c.v[0] + val[13 * nb + k] * c.v[1] + val[14 * nb + k] * c.v[2]);
    }
    q = group_sum<T, LPR>(q);
    if (lane == 0) {
        double theta, a, b;
        cheb_coef(st->lam_max, ratio, i, theta, a, b);
        const T r = rc[row] - q;
        rc[row] = r;
        const T dnew = (T)a * cur[4 * row + 3] + (T)b * Sinv[row] * r;
        next[4 * row + 3] = (T)dnew;
        z[4 * row + 3] = (T)(z[4 * row + 3] + dnew);
    }
}

// z.u -= D^{-1} sum_j G_ij z.p_j
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_simple_xu(RowPattern P, const T *val, const T *Dinv, T *z,
                                                   const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int64_t nb = P.nblk, nv = P.nv;
    const int32_t beg = P.rowptr[row], end = P.rowptr[row + 1];
    T a0 = 0, a1 = 0, a2 = 0;
    for (int32_t k = beg + lane; k < end; k += LPR) {
        const T zp = z[4 * (int64_t)P.col[k] + 3];
        a0 += val[9 * nb + k] * zp;
        a1 += val[10 * nb + k] * zp;
        a2 += val[11 * nb + k] * zp;
    }
    a0 = group_sum<T, LPR>(a0);
    a1 = group_sum<T, LPR>(a1);
    a2 = group_sum<T, LPR>(a2);
    if (lane == 0) {
        z[4 * row + 0] = (T)(z[4 * row + 0] - Dinv[row] * a0);
        z[4 * row + 1] = (T)(z[4 * row + 1] - Dinv[nv + row] * a1);
        z[4 * row + 2] = (T)(z[4 * row + 2] - Dinv[2 * nv + row] * a2);
    }
}

// Lanes per block row of the sparse row passes (4, 8 or 16; LXNS_LPR overrides).
static int lanes_per_row()
{
    static const int v = [] {
        const char *e = getenv("LXNS_LPR");
        const int x = e ? atoi(e) : 8;
        return (x == 4 || x == 8 || x == 16) ? x : 8;
    }();
    return v;
}

template <typename T, int LPR>
static void simple_apply_lpr(const RowPattern &P, const Simple<T> &S, const T *r, const double *scale_ptr, T *z,
                             const int32_t *done, hipStream_t s)
{
    const int64_t nv = P.nv;
    hipLaunchKernelGGL((k_simple_zu<T>), dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, nv, S.Finv, r,
                       scale_ptr, z, done);
    const unsigned g = (unsigned)((nv * LPR + 255) / 256);
    T *rc = S.work, *ca = S.work + nv, *cb = S.work + 5 * nv;   // rc [nv]; two [nv][4] (y, d) buffers
    hipLaunchKernelGGL((k_simple_zp<T, LPR>), dim3(g), dim3(256), 0, s, P, S.val, S.Sinv, z, S.degree, S.ratio, rc,
                       ca, S.st, done);
    for (int i = 1; i < S.degree; ++i) {
        hipLaunchKernelGGL((k_cheb_gd<T, LPR>), dim3(g), dim3(256), 0, s, P, S.val, S.Dinv, ca, done);
        hipLaunchKernelGGL((k_cheb_step<T, LPR>), dim3(g), dim3(256), 0, s, P, S.val, S.Sinv, ca, rc, cb, z, i,
                           S.ratio, S.st, done);
        std::swap(ca, cb);
    }
    hipLaunchKernelGGL((k_simple_xu<T, LPR>), dim3(g), dim3(256), 0, s, P, S.val, S.Dinv, z, done);
}

template <typename T>
void launch_simple_apply(const RowPattern &P, const Simple<T> &S, const T *r, const double *scale_ptr, T *z,
                         const int32_t *done, hipStream_t s)
{
    switch (lanes_per_row()) {
    case 4: simple_apply_lpr<T, 4>(P, S, r, scale_ptr, z, done, s); break;
    case 16: simple_apply_lpr<T, 16>(P, S, r, scale_ptr, z, done, s); break;
    default: simple_apply_lpr<T, 8>(P, S, r, scale_ptr, z, done, s); break;
    }
}
template void launch_simple_apply<double>(const RowPattern &, const Simple<double> &, const double *,
                                          const double *, double *, const int32_t *, hipStream_t);
template void launch_simple_apply<float>(const RowPattern &, const Simple<float> &, const float *, const double *,
                                         float *, const int32_t *, hipStream_t);

// ------------------------------------------------------------------ SpMV

// y = A x over the block-CSR planes: LPR lanes per block row, each lane one
// 4x4 block per iteration (16 unit-stride plane loads + one gathered 4-vector),
// then a cross-lane reduction of the 4 row sums.  NT: the planes exceed the
// last-level cache (ld_mat).
template <typename T, int LPR, bool NT>
__global__ __launch_bounds__(256) void k_spmv(RowPattern P, const T *__restrict__ val, const T *__restrict__ x,
                                              T *__restrict__ y, const int32_t *done)
{
    const int64_t row = (xcd_block() * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= P.nv) return;
    const int64_t nb = P.nblk;
    const int32_t beg = P.rowptr[row], end = P.rowptr[row + 1];
    if (done_with(done, end)) return;
    using V = typename V4<T>::type;
    // sums in the working precision T (FP32 inner solves accumulate in FP32)
    T y0 = 0, y1 = 0, y2 = 0, y3 = 0;
    for (int32_t k = beg + lane; k < end; k += LPR) {
        const V xv = reinterpret_cast<const V *>(x)[P.col[k]];
        const T x0 = xv.v[0], x1 = xv.v[1], x2 = xv.v[2], x3 = xv.v[3];
        T a[16];
#pragma unroll
        for (int p = 0; p < 16; ++p) a[p] = ld_mat<NT>(&val[p * nb + k]);
        y0 += a[0] * x0 + a[1] * x1 + a[2] * x2 + a[9] * x3;
        y1 += a[3] * x0 + a[4] * x1 + a[5] * x2 + a[10] * x3;
        y2 += a[6] * x0 + a[7] * x1 + a[8] * x2 + a[11] * x3;
        y3 += a[12] * x0 + a[13] * x1 + a[14] * x2 + a[15] * x3;
    }
    y0 = group_sum<T, LPR>(y0);
    y1 = group_sum<T, LPR>(y1);
    y2 = group_sum<T, LPR>(y2);
    y3 = group_sum<T, LPR>(y3);
    if (lane == 0) {
        V out;
        out.v[0] = (T)y0;
        out.v[1] = (T)y1;
        out.v[2] = (T)y2;
        out.v[3] = (T)y3;
        reinterpret_cast<V *>(y)[row] = out;
    }
}

bool streamed(int64_t bytes)
{
    static const bool on = [] {
        const char *e = getenv("LXNS_STREAM_LOADS");
        return !(e && *e == '0');
    }();
    return on && bytes > kLastLevelCacheBytes;
}

// Lanes per block row of the SpMV (4, 8 or 16; LXNS_LPR_SPMV overrides).
static int lanes_per_row_spmv()
{
    static const int v = [] {
        const char *e = getenv("LXNS_LPR_SPMV");
        const int x = e ? atoi(e) : 16;
        return (x == 4 || x == 8 || x == 16) ? x : 16;
    }();
    return v;
}

// ev0/ev1 (optional): events stamped by the dispatch itself around the kernel
template <typename T>
void launch_spmv(const RowPattern &P, const T *val, const T *x, T *y, const int32_t *done, hipStream_t s,
                 hipEvent_t ev0, hipEvent_t ev1)
{
    const int lpr = lanes_per_row_spmv();
    const unsigned g = (unsigned)((P.nv * lpr + 255) / 256);
    auto go = [&](auto nt) {
        constexpr bool NT = decltype(nt)::value;
        if (lpr == 4)
            hipExtLaunchKernelGGL((k_spmv<T, 4, NT>), dim3(g), dim3(256), 0, s, ev0, ev1, 0, P, val, x, y, done);
        else if (lpr == 8)
            hipExtLaunchKernelGGL((k_spmv<T, 8, NT>), dim3(g), dim3(256), 0, s, ev0, ev1, 0, P, val, x, y, done);
        else
            hipExtLaunchKernelGGL((k_spmv<T, 16, NT>), dim3(g), dim3(256), 0, s, ev0, ev1, 0, P, val, x, y, done);
    };
    if (streamed(16 * P.nblk * (int64_t)sizeof(T)))
        go(std::true_type{});
    else
        go(std::false_type{});
}
template void launch_spmv<double>(const RowPattern &, const double *, const double *, double *, const int32_t *,
                                  hipStream_t, hipEvent_t, hipEvent_t);
template void launch_spmv<float>(const RowPattern &, const float *, const float *, float *, const int32_t *,
                                 hipStream_t, hipEvent_t, hipEvent_t);

// ------------------------------------------------------------------ reductions


// Reductions run in two kernels: the data-parallel pass writes one partial sum
// per block (or per chunk and vector), and a one-block kernel adds them in a
// fixed order.  Kernel boundaries order the two, so no block waits for or
// fences against another (a device-scope fence per block is expensive on a
// multi-die GPU), and every result is independent of scheduling.

// Blocks of the elementwise passes: about four elements per thread.
static unsigned vec_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 1023) / 1024, 4096)); }

int64_t gm_partial_size(int64_t n)
{
    const int64_t nbx = (n + kDotChunk - 1) / kDotChunk;
    return std::max<int64_t>((kMaxRestart + 1) * nbx, vec_blocks(n)) + 64;
}

// Sum of the block's per-thread values, valid in thread 0 (blockDim 256).
__device__ inline double block_total(double v, double *lds)
{
    double a[1] = {v};
    block_sum<1>(a, lds);
    return a[0];
}

// r = b - Ax (or b), V0 = r; partial[block] = sum r^2.
template <typename T>
__global__ __launch_bounds__(256) void k_gm_start(int64_t n, const T *b, const T *Ax, T *V0, double *partial)
{
    __shared__ double lds[4];
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double r = Ax ? to_d(b[i]) - to_d(Ax[i]) : to_d(b[i]);
        const T rt = (T)r;
        V0[i] = rt;
        acc += to_d(rt) * to_d(rt);
    }
    const double t = block_total(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Fixed-order sum of partial[0..nb) in one block of 256 threads (valid in thread 0).
__device__ inline double sum_partials(const double *partial, int nb, double *lds)
{
    double s = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[b];
    return block_total(s, lds);
}

// beta = ||r||: starts a cycle (g = beta e_1, V_0 scale 1/beta) or stops it.
__global__ __launch_bounds__(256) void k_gm_start_fin(int nb, const double *partial, GmState *st)
{
    __shared__ double lds[4];
    const double tot = sum_partials(partial, nb, lds);
    if (threadIdx.x == 0) {
        const double beta = sqrt(tot);
        st->resid = beta;
        st->g[0] = beta;
        for (int j = 1; j <= kMaxRestart; ++j) st->g[j] = 0;
        st->s[0] = beta > 0 ? 1.0 / beta : 0.0;
        st->kused = 0;
        st->reorth = 0;
        st->n_reorth = 0;
        st->converged = (beta <= st->tol_abs) ? 1 : 0;
        st->breakdown = (beta != beta) ? 1 : 0;
        st->done = (st->converged || st->breakdown) ? 1 : 0;
    }
}

template <typename T>
void launch_gm_start(int64_t n, const T *b, const T *Ax, T *V0, GmState *st, double *partial, hipStream_t s)
{
    const unsigned nb = vec_blocks(n);
    hipLaunchKernelGGL((k_gm_start<T>), dim3(nb), dim3(256), 0, s, n, b, Ax, V0, partial);
    hipLaunchKernelGGL(k_gm_start_fin, dim3(1), dim3(256), 0, s, (int)nb, partial, st);
}
template void launch_gm_start<double>(int64_t, const double *, const double *, double *, GmState *, double *,
                                      hipStream_t);
template void launch_gm_start<float>(int64_t, const float *, const float *, float *, GmState *, double *,
                                     hipStream_t);

// partial[j * gridDim.x + bx] = <Vhat_j, w> over chunk bx, j = blockIdx.y; the
// row j = nv (if the grid has it) is <w, w>.  second: the second Gram-Schmidt
// pass, skipped unless the first one asked for it.
template <typename T>
__global__ __launch_bounds__(256) void k_gm_dot(int64_t n, const T *V, int64_t ldv, const T *w, double *partial,
                                                const GmState *st, int nv, int second)
{
    if (st->done || (second && !st->reorth)) return;
    __shared__ double lds[4];
    const T *v = (int)blockIdx.y < nv ? V + (int64_t)blockIdx.y * ldv : w;
    const int64_t i0 = (int64_t)blockIdx.x * kDotChunk;
    const int64_t i1 = i0 + kDotChunk < n ? i0 + kDotChunk : n;
    double acc = 0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc += to_d(v[i]) * to_d(w[i]);
    const double t = block_total(acc, lds);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// The rest of one Gram-Schmidt pass, in every block: dot_j = sum_b partial[j][b]
// (fixed order, one wavefront per j, the same in every block), h_j = s_j dot_j
// with V_j = s_j Vhat_j, and the block's share of Vhat_{k+1} = w - sum_j h_j V_j
// (the second pass, second = 1, takes w = Vhat_{k+1} in place).  Block 0 also
// keeps the books: the first pass writes H[j][k] = h_j and asks for the second
// one when the projection removed more than the share reorth_frac of ||w||^2
// (row k + 1 of the partials holds <w, w>; the library sets 0.9, i.e.
// ||w - V h|| < ||w|| / sqrt(10), a stricter form of the
// Daniel-Gragg-Kaufman-Stewart test, whose 1/sqrt(2) asks for it at nearly
// every step of these solves); the second pass adds its h_j to H[j][k].  The
// pass that ends the step takes ||Vhat_{k+1}||^2 = <w, w> - sum_j h_j^2 (the
// basis is orthonormal to working precision; the test above keeps the
// difference at least a tenth of <w, w>), and applies the Givens update of
// column k and the convergence test; with fz, it also starts the velocity
// block's Chebyshev iteration on V_{k+1} = s_{k+1} Vhat_{k+1} (every block knows
// ||Vhat_{k+1}|| from the same sums).  One thread per node (4-vector).  A block
// that starts after block 0 has ended the cycle returns at once: Vhat_{k+1} is
// then never read.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_gm_axpy_fin(int64_t n, int k, int nbx, T *V, int64_t ldv, const T *w,
                                                     GmState *st, const double *partial, int second, FzStart<T> fz)
{
    if (st->done || (second && !st->reorth)) return;
    __shared__ double red[K + 1];
    __shared__ double coef[K];
    __shared__ double col[K + 1];
    __shared__ double gcs[K], gsn[K];
    __shared__ double fin[2];   // ||Vhat_{k+1}|| if this pass ends the step; 1 if the step needs another pass
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int j = wid; j <= k + 1; j += 4) {
        double s = 0;
        for (int b = lane; b < nbx; b += 64) s += partial[(int64_t)j * nbx + b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) red[j] = s;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        const int j = threadIdx.x;
        const double sj = j <= k ? st->s[j] : 0.0;
        const double h = j <= k ? red[j] * sj : 0.0;
        coef[j] = h * sj;
        red[j] = j <= k ? h : red[j];   // rows 0..k now hold h_j; row k + 1 keeps <w, w>
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double p = 0;
        for (int j = 0; j <= k; ++j) p += red[j] * red[j];
        const double ww = red[k + 1];
        const double d = ww - p;
        fin[0] = d > 0 ? sqrt(d) : 0.0;
        fin[1] = (second || p <= st->reorth_frac * ww) ? 0.0 : 1.0;   // also taken on a non-finite value
    }
    __syncthreads();
    const double hn = fin[0];
    const bool again = fin[1] != 0.0;
    using VT = typename V4<T>::type;
    T *Vn = V + (int64_t)(k + 1) * ldv;
    const bool start = fz.z && !again;
    const double sc = hn > 0 ? 1.0 / hn : 0.0;   // s_{k+1}, as block 0 stores it
    double theta = 1.0, ca, cb;
    if (start && fz.degree > 1) cheb_coef(*fz.lamF, fz.ratio, 0, theta, ca, cb);
    const int64_t nv = n >> 2;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const VT wv = reinterpret_cast<const VT *>(w)[v];
        double a[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = to_d(wv.v[c]);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j <= k) {
                const VT x = reinterpret_cast<const VT *>(V + j * ldv)[v];
#pragma unroll
                for (int c = 0; c < 4; ++c) a[c] -= coef[j] * to_d(x.v[c]);
            }
        VT o;
#pragma unroll
        for (int c = 0; c < 4; ++c) o.v[c] = (T)a[c];
        reinterpret_cast<VT *>(Vn)[v] = o;
        if (start) {
            const double r0 = to_d(o.v[0]) * sc, r1 = to_d(o.v[1]) * sc, r2 = to_d(o.v[2]) * sc;
            double fi[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) fi[q] = to_d(fz.Finv[q * nv + v]);
            double y0 = fi[0] * r0 + fi[1] * r1 + fi[2] * r2;
            double y1 = fi[3] * r0 + fi[4] * r1 + fi[5] * r2;
            double y2 = fi[6] * r0 + fi[7] * r1 + fi[8] * r2;
            VT zv;
            if (fz.degree > 1) {
                y0 /= theta;
                y1 /= theta;
                y2 /= theta;
                VT f, d;
                f.v[0] = (T)r0;
                f.v[1] = (T)r1;
                f.v[2] = (T)r2;
                f.v[3] = T(0);
                reinterpret_cast<VT *>(fz.fr)[v] = f;
                d.v[0] = (T)y0;
                d.v[1] = (T)y1;
                d.v[2] = (T)y2;
                d.v[3] = T(0);
                reinterpret_cast<VT *>(fz.fd)[v] = d;
                zv.v[0] = d.v[0];
                zv.v[1] = d.v[1];
                zv.v[2] = d.v[2];
            } else {
                zv.v[0] = (T)y0;
                zv.v[1] = (T)y1;
                zv.v[2] = (T)y2;
            }
            zv.v[3] = (T)(to_d(o.v[3]) * sc);
            reinterpret_cast<VT *>(fz.z)[v] = zv;
        }
    }
    if (blockIdx.x != 0) return;
    // ---- block 0: Hessenberg column k, second-pass decision, Givens update
    const int M = kMaxRestart;
    double *H = st->H;
    if (threadIdx.x <= (unsigned)k) {
        const int j = threadIdx.x;
        const double hj = second ? H[j * M + k] + red[j] : red[j];
        H[j * M + k] = hj;
        col[j] = hj;
        if (j < k) {
            gcs[j] = st->cs[j];
            gsn[j] = st->sn[j];
        }
    }
    if (threadIdx.x == 0 && !second) {
        st->reorth = again ? 1 : 0;
        st->n_reorth += again ? 1 : 0;
    }
    __syncthreads();
    if (again || threadIdx.x != 0) return;
    for (int j = 0; j < k; ++j) {
        const double t = gcs[j] * col[j] + gsn[j] * col[j + 1];
        col[j + 1] = -gsn[j] * col[j] + gcs[j] * col[j + 1];
        col[j] = t;
    }
    const double a = col[k];
    const double r = hypot(a, hn);
    const double c = (r > 0) ? a / r : 1.0, sn = (r > 0) ? hn / r : 0.0;
    for (int j = 0; j < k; ++j) H[j * M + k] = col[j];
    H[k * M + k] = r;
    H[(k + 1) * M + k] = 0.0;
    st->cs[k] = c;
    st->sn[k] = sn;
    const double gk = st->g[k];
    st->g[k + 1] = -sn * gk;
    st->g[k] = c * gk;
    st->s[k + 1] = sc;
    const double res = fabs(sn * gk);
    st->resid = res;
    st->kused = k + 1;
    const bool bad = !(res == res) || !(r > 0);
    st->breakdown = bad ? 1 : 0;
    st->converged = (!bad && res <= st->tol_abs) ? 1 : 0;
    // a zero new direction means the Krylov space is invariant: the solution is exact
    if (!bad && hn == 0.0) st->converged = 1;
    st->done = (st->converged || bad) ? 1 : 0;
}

#define LX_GM_K_DISPATCH(KERNEL, T, grid, ...)                                                                \
    do {                                                                                                       \
        if (k + 1 <= 8)                                                                                        \
            hipLaunchKernelGGL((KERNEL<T, 8>), grid, dim3(256), 0, s, __VA_ARGS__);                           \
        else if (k + 1 <= 16)                                                                                  \
            hipLaunchKernelGGL((KERNEL<T, 16>), grid, dim3(256), 0, s, __VA_ARGS__);                          \
        else if (k + 1 <= 32)                                                                                  \
            hipLaunchKernelGGL((KERNEL<T, 32>), grid, dim3(256), 0, s, __VA_ARGS__);                          \
        else                                                                                                   \
            hipLaunchKernelGGL((KERNEL<T, 64>), grid, dim3(256), 0, s, __VA_ARGS__);                          \
    } while (0)

// One Arnoldi step's classical Gram-Schmidt of w against Vhat_0..Vhat_k, with a
// second pass when the first one cancelled much of w (selective
// reorthogonalisation; the device decides, the second-pass kernels return at
// once otherwise), then Vhat_{k+1} and the Givens update.
template <typename T>
void launch_gm_orth(int64_t n, int k, T *V, int64_t ldv, T *w, GmState *st, double *partial, hipStream_t s,
                    const FzStart<T> *fz)
{
    const int nbx = (int)((n + kDotChunk - 1) / kDotChunk);
    const unsigned nbv = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n / 4 + 255) / 256, 4096));
    const dim3 gd(nbx, k + 2), gv(nbv);
    T *vn = V + (int64_t)(k + 1) * ldv;
    const FzStart<T> f = fz ? *fz : FzStart<T>();
    hipLaunchKernelGGL((k_gm_dot<T>), gd, dim3(256), 0, s, n, V, ldv, w, partial, st, k + 1, 0);
    LX_GM_K_DISPATCH(k_gm_axpy_fin, T, gv, n, k, nbx, V, ldv, w, st, partial, 0, f);
    hipLaunchKernelGGL((k_gm_dot<T>), gd, dim3(256), 0, s, n, V, ldv, vn, partial, st, k + 1, 1);
    LX_GM_K_DISPATCH(k_gm_axpy_fin, T, gv, n, k, nbx, V, ldv, vn, st, partial, 1, f);
}
template void launch_gm_orth<double>(int64_t, int, double *, int64_t, double *, GmState *, double *, hipStream_t,
                                     const FzStart<double> *);
template void launch_gm_orth<float>(int64_t, int, float *, int64_t, float *, GmState *, double *, hipStream_t,
                                    const FzStart<float> *);

// y = H^{-1} g over the kused columns: back substitution by one wavefront, the
// triangle staged in LDS; lane j keeps g_j minus the terms of the y found so
// far and holds y_j once its turn has come.
__global__ __launch_bounds__(64) void k_gm_solve_y(GmState *st)
{
    __shared__ double Hs[kMaxRestart][kMaxRestart + 1];
    const int M = kMaxRestart, k = st->kused, lane = threadIdx.x;
    for (int idx = lane; idx < k * k; idx += 64) {
        const int i = idx / k, j = idx - i * k;
        Hs[i][j] = st->H[i * M + j];
    }
    double gl = lane < k ? st->g[lane] : 0.0;
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        const double yi = __shfl(gl, i) / Hs[i][i];
        if (lane < i) gl -= Hs[lane][i] * yi;
        if (lane == i) gl = yi;
    }
    if (lane < k) st->y[lane] = gl;
}

void launch_gm_solve_y(GmState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_solve_y, dim3(1), dim3(64), 0, s, st);
}

// x += sum_j y_j Z_j over the kused preconditioned directions (flexible GMRES update)
template <typename T>
__global__ void k_gm_update(int64_t n, const T *Z, int64_t ldz, const GmState *st, T *x)
{
    const int k = st->kused;
    __shared__ double y[kMaxRestart];
    if (threadIdx.x < kMaxRestart) y[threadIdx.x] = (threadIdx.x < (unsigned)k) ? st->y[threadIdx.x] : 0.0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = to_d(x[i]);
        for (int j = 0; j < k; ++j) s += y[j] * to_d(Z[j * ldz + i]);
        x[i] = (T)s;
    }
}

template <typename T>
void launch_gm_update(int64_t n, const T *Z, int64_t ldz, const GmState *st, T *x, hipStream_t s)
{
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL((k_gm_update<T>), dim3(g), dim3(256), 0, s, n, Z, ldz, st, x);
}
template void launch_gm_update<double>(int64_t, const double *, int64_t, const GmState *, double *, hipStream_t);
template void launch_gm_update<float>(int64_t, const float *, int64_t, const GmState *, float *, hipStream_t);

template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(int64_t n, const T *x, double *partial)
{
    __shared__ double lds[4];
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += to_d(x[i]) * to_d(x[i]);
    const double t = block_total(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_norm_fin(int nb, const double *partial, GmState *st, double rtol, int slot)
{
    __shared__ double lds[4];
    const double tot = sum_partials(partial, nb, lds);
    if (threadIdx.x == 0) {
        st->norms[slot] = sqrt(tot);
        if (rtol > 0) st->tol_abs = rtol * st->norms[slot];
    }
}

template <typename T>
void launch_norm(int64_t n, const T *x, GmState *st, double rtol, double *partial, int slot, hipStream_t s)
{
    const unsigned nb = vec_blocks(n);
    hipLaunchKernelGGL((k_sumsq<T>), dim3(nb), dim3(256), 0, s, n, x, partial);
    hipLaunchKernelGGL(k_norm_fin, dim3(1), dim3(256), 0, s, (int)nb, partial, st, rtol, slot);
}
template void launch_norm<double>(int64_t, const double *, GmState *, double, double *, int, hipStream_t);
template void launch_norm<float>(int64_t, const float *, GmState *, double, double *, int, hipStream_t);

// ------------------------------------------------------------------ vector utilities

template <typename T>
__global__ void k_fill(int64_t n, T *x, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}
template <typename T>
void launch_fill(int64_t n, T *x, T v, hipStream_t s)
{
    if (n <= 0) return;
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((k_fill<T>), dim3(g), dim3(256), 0, s, n, x, v);
}
template void launch_fill<double>(int64_t, double *, double, hipStream_t);
template void launch_fill<float>(int64_t, float *, float, hipStream_t);
template void launch_fill<int32_t>(int64_t, int32_t *, int32_t, hipStream_t);

template <typename TD, typename TS>
__global__ void k_axpy(int64_t n, TD *y, const TS *x, const double *scale_ptr, double scale)
{
    const double a = scale_ptr ? scale * (*scale_ptr) : scale;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (TD)((double)y[i] + a * (double)x[i]);
}
template <typename TD, typename TS>
void launch_axpy(int64_t n, TD *y, const TS *x, const double *scale_ptr, double scale, hipStream_t s)
{
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((k_axpy<TD, TS>), dim3(g), dim3(256), 0, s, n, y, x, scale_ptr, scale);
}
template void launch_axpy<double, double>(int64_t, double *, const double *, const double *, double, hipStream_t);
template void launch_axpy<float, float>(int64_t, float *, const float *, const double *, double, hipStream_t);
template void launch_axpy<double, float>(int64_t, double *, const float *, const double *, double, hipStream_t);

// x = g0 h0 + g1 h1 + g2 h2 (h1, h2 may be null when their weight is 0)
__global__ void k_extrapolate(int64_t n, double *x, const double *h0, const double *h1, const double *h2,
                              const double *h3, double g0, double g1, double g2, double g3)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = g0 * h0[i];
        if (h1) v += g1 * h1[i];
        if (h2) v += g2 * h2[i];
        if (h3) v += g3 * h3[i];
        x[i] = v;
    }
}

void launch_extrapolate(int64_t n, double *x, const double *h0, const double *h1, const double *h2, double g0,
                        double g1, double g2, hipStream_t s, const double *h3, double g3)
{
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_extrapolate, dim3(g), dim3(256), 0, s, n, x, h0, h1, h2, h3, g0, g1, g2, g3);
}

template <typename TD, typename TS>
__global__ void k_scale_copy(int64_t n, TD *dst, const TS *src, double a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (TD)((double)src[i] * a);
}
template <typename TD, typename TS>
void launch_scale_copy(int64_t n, TD *dst, const TS *src, double factor, hipStream_t s)
{
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((k_scale_copy<TD, TS>), dim3(g), dim3(256), 0, s, n, dst, src, factor);
}
template void launch_scale_copy<float, double>(int64_t, float *, const double *, double, hipStream_t);
template void launch_scale_copy<double, double>(int64_t, double *, const double *, double, hipStream_t);
template void launch_scale_copy<double, float>(int64_t, double *, const float *, double, hipStream_t);

__global__ void k_set_dirichlet_x(int64_t n_dir, const int32_t *dir_node, const double *g, double *xs)
{
    const int64_t k = xcd_block() * blockDim.x + threadIdx.x;
    if (k >= n_dir) return;
    const int64_t i = dir_node[k];
    for (int c = 0; c < 3; ++c) xs[4 * i + c] = g[3 * k + c];
}
void launch_set_dirichlet_x(int64_t n_dir, const int32_t *dir_node, const double *g, double *xs, hipStream_t s)
{
    if (n_dir == 0) return;
    hipLaunchKernelGGL(k_set_dirichlet_x, dim3((unsigned)((n_dir + 255) / 256)), dim3(256), 0, s, n_dir, dir_node,
                       g, xs);
}


// How well each initial guess would have predicted the solution x just
// computed from the history h_0..h_3 (newest first): sums of squares of
// x - (g0 h0 + g1 h1 + g2 h2) (the BDF extrapolation), x - (3h0 - 3h1 + h2)
// (quadratic, nk >= 2) and x - (4h0 - 6h1 + 4h2 - h3) (cubic, nk >= 3).
// Per-block partials, then one wave sums them in a fixed order into out[0..2].
constexpr int kGuessErrBlocks = 256;
__global__ __launch_bounds__(256) void k_guess_err(int64_t n, int nk, const double *x, const double *h0,
                                                   const double *h1, const double *h2, const double *h3, double g0,
                                                   double g1, double g2, double *partial)
{
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = x[i], a = h0[i], b = h1[i], c = h2[i];
        const double d0 = v - (g0 * a + g1 * b + g2 * c);
        e0 += d0 * d0;
        if (nk >= 2) {
            const double d1 = v - (3.0 * (a - b) + c);
            e1 += d1 * d1;
        }
        if (nk >= 3) {
            const double d2 = v - (4.0 * (a + c) - 6.0 * b - h3[i]);
            e2 += d2 * d2;
        }
    }
    __shared__ double red[3][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        e0 += __shfl_down(e0, o, 64);
        e1 += __shfl_down(e1, o, 64);
        e2 += __shfl_down(e2, o, 64);
    }
    if (lane == 0) {
        red[0][wv] = e0;
        red[1][wv] = e1;
        red[2][wv] = e2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int q = threadIdx.x;
        partial[blockIdx.x * 3 + q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
    }
}

__global__ void k_guess_err_sum(int nblk, const double *partial, double *out)
{
    for (int q = 0; q < 3; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64) v += partial[b * 3 + q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (threadIdx.x == 0) out[q] = v;
    }
}

void launch_guess_err(int64_t n, int nk, const double *x, const double *const *h, const double *gamma,
                      double *partial, double *out, hipStream_t s)
{
    const int nblk = (int)std::min<int64_t>((n + 255) / 256, kGuessErrBlocks);
    hipLaunchKernelGGL(k_guess_err, dim3(nblk), dim3(256), 0, s, n, nk, x, h[0], h[1], h[2], h[3], gamma[0],
                       gamma[1], gamma[2], partial);
    hipLaunchKernelGGL(k_guess_err_sum, dim3(1), dim3(64), 0, s, nblk, partial, out);
}

}  // namespace lx
