// P2-P1 kernels: element matrices with the degree-5 rule, fixed-order slot
// gathers into the split block-CSR parts, Dirichlet rows, the quadratic
// boundary traction, SIMPLE diagonal blocks and the split SpMV.
//
// The element integrals are those of the P1 path (fully discrete weak form of
// Sec. 2.3 with SUPG-PSPG + grad-div, VMS cross term and semi-implicit LES),
// evaluated per quadrature point since the P2 gradients vary on the element;
// the strong residuals include -mu Lap u with the constant Hessians of the P2
// basis.  One wavefront per element: its lanes first evaluate the quadrature
// points (one lane each), then accumulate the 34 x 34 matrix and the
// right-hand side in parallel over entry groups, and write the element record
// that the slot gathers read.
#include <hip/hip_ext.h>

#include "lx_device.h"
#include "lx_p2.h"

namespace lx {

// local edge k joins local vertices kE[k][0], kE[k][1]
__constant__ int kE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

struct P2Lds {
    double dl[4][3];      // grad lambda_a (constant)
    double G[3][3], g[3], GG, gg, vol6;
    double xh[4][3];
    double uE[10][3], uB[10][3], f[10][3], pE[4], lap[10];
    double gP[3];
    // quadrature-point data
    double w[kP2Q], M[kP2Q], tM[kP2Q], tC[kP2Q];
    double phi[kP2Q][10], dphi[kP2Q][10][3], adv[kP2Q][10], s[kP2Q][10], T[kP2Q][10][9], K[kP2Q][3];
    double lam[kP2Q][4];
};

__global__ __launch_bounds__(64) void k_element_p2(P2AsmArgs A, StepCoef C, int symgrad)
{
    __shared__ P2Lds S;
    const int64_t e = blockIdx.x;
    const int lane = threadIdx.x;
    if (e >= A.nt) return;
    const int64_t nt = A.nt;
    // geometry (every lane, identical)
    int32_t v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] = A.tet[a * nt + e];
    double J[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) J[i][k] = A.x[3 * (int64_t)v[k + 1] + i] - A.x[3 * (int64_t)v[0] + i];
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
    if (lane == 0) {
        for (int j = 0; j < 3; ++j) {
            S.dl[1][j] = Ji[0][j];
            S.dl[2][j] = Ji[1][j];
            S.dl[3][j] = Ji[2][j];
            S.dl[0][j] = -(Ji[0][j] + Ji[1][j] + Ji[2][j]);
        }
        S.GG = 0;
        S.gg = 0;
        for (int i = 0; i < 3; ++i) {
            S.g[i] = Ji[0][i] + Ji[1][i] + Ji[2][i];
            S.gg += S.g[i] * S.g[i];
            for (int j = 0; j < 3; ++j) {
                S.G[i][j] = Ji[0][i] * Ji[0][j] + Ji[1][i] * Ji[1][j] + Ji[2][i] * Ji[2][j];
                S.GG += S.G[i][j] * S.G[i][j];
            }
        }
        S.vol6 = fabs(det);
    }
    // nodal data: lane a < 10 loads node a
    const double *H[3] = {A.h0, A.h1, A.h2};
    const double rdt = C.rho / C.dt;
    if (lane < 10) {
        const int64_t nd = A.nodes[(int64_t)lane * nt + e];
        double ue[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, pe = 0;
        for (int l = 0; l < C.nlev; ++l) {
            const double *h = H[l] + 4 * nd;
            for (int c = 0; c < 3; ++c) {
                ue[c] += C.gamma[l] * h[c];
                ub[c] += C.beta[l] * h[c];
            }
            pe += C.gamma[l] * h[3];
        }
        for (int c = 0; c < 3; ++c) {
            S.uE[lane][c] = ue[c];
            S.uB[lane][c] = ub[c];
            S.f[lane][c] = A.f ? A.f[3 * nd + c] : 0.0;
        }
        if (lane < 4) {
            S.pE[lane] = pe;
            for (int c = 0; c < 3; ++c) S.xh[lane][c] = A.xh[3 * nd + c];
        }
    }
    __syncthreads();
    if (lane < 10) {
        // constant Laplacians of the P2 basis
        double lp;
        if (lane < 4) {
            lp = 4.0 * (S.dl[lane][0] * S.dl[lane][0] + S.dl[lane][1] * S.dl[lane][1] + S.dl[lane][2] * S.dl[lane][2]);
        } else {
            const int i = kE[lane - 4][0], j = kE[lane - 4][1];
            lp = 8.0 * (S.dl[i][0] * S.dl[j][0] + S.dl[i][1] * S.dl[j][1] + S.dl[i][2] * S.dl[j][2]);
        }
        S.lap[lane] = lp;
    }
    if (lane == 10)
        for (int c = 0; c < 3; ++c)
            S.gP[c] = S.pE[0] * S.dl[0][c] + S.pE[1] * S.dl[1][c] + S.pE[2] * S.dl[2][c] + S.pE[3] * S.dl[3][c];
    __syncthreads();

    // ---- one lane per quadrature point
    const double rho = C.rho, mu = C.mu, adt = C.alpha / C.dt;
    if (lane < kP2Q) {
        const int q = lane;
        double L[4];
        for (int a = 0; a < 4; ++a) L[a] = A.rules->lam[q][a];
        const double w = A.rules->w[q] * S.vol6;
        double phi[10], dphi[10][3];
        for (int a = 0; a < 4; ++a) {
            phi[a] = L[a] * (2.0 * L[a] - 1.0);
            for (int j = 0; j < 3; ++j) dphi[a][j] = (4.0 * L[a] - 1.0) * S.dl[a][j];
        }
        for (int k = 0; k < 6; ++k) {
            const int i = kE[k][0], j2 = kE[k][1];
            phi[4 + k] = 4.0 * L[i] * L[j2];
            for (int j = 0; j < 3; ++j) dphi[4 + k][j] = 4.0 * (L[i] * S.dl[j2][j] + L[j2] * S.dl[i][j]);
        }
        double uq[3] = {0, 0, 0}, ubq[3] = {0, 0, 0}, fq[3] = {0, 0, 0}, lapU[3] = {0, 0, 0};
        double gU[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int a = 0; a < 10; ++a)
            for (int c = 0; c < 3; ++c) {
                uq[c] += phi[a] * S.uE[a][c];
                ubq[c] += phi[a] * S.uB[a][c];
                fq[c] += phi[a] * S.f[a][c];
                lapU[c] += S.lap[a] * S.uE[a][c];
                for (int j = 0; j < 3; ++j) gU[c][j] += S.uE[a][c] * dphi[a][j];
            }
        double xq[3];
        for (int c = 0; c < 3; ++c) xq[c] = L[0] * S.xh[0][c] + L[1] * S.xh[1][c] + L[2] * S.xh[2][c] + L[3] * S.xh[3][c];
        // RIIS: smoothed delta of the distance to each annular disc
        double sigR = 0, riis2 = 0;
        for (int k = 0; k < C.n_valves; ++k) {
            const double *vp = C.valve[k];
            const double rel[3] = {xq[0] - vp[0], xq[1] - vp[1], xq[2] - vp[2]};
            const double z = rel[0] * vp[3] + rel[1] * vp[4] + rel[2] * vp[5];
            const double p0 = rel[0] - z * vp[3], p1 = rel[1] - z * vp[4], p2 = rel[2] - z * vp[5];
            const double rp = sqrt(p0 * p0 + p1 * p1 + p2 * p2);
            double dr = 0;
            if (rp < vp[6]) dr = vp[6] - rp;
            if (rp > vp[7]) dr = rp - vp[7];
            const double phid = sqrt(z * z + dr * dr), eps = vp[9];
            if (phid <= eps) {
                const double dlt = (1.0 + cos(M_PI * phid / eps)) / (2.0 * eps);
                const double ratio = vp[8] / eps;
                sigR += ratio * dlt;
                riis2 += ratio * ratio * dlt * dlt;
            }
        }
        double tauM = 0, tauC = 0;
        if (C.stab != LX_STAB_NONE) {
            double uGu = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) uGu += uq[i] * S.G[i][j] * uq[j];
            const double tsum = C.sigma * C.sigma * rho * rho / (C.dt * C.dt) + rho * rho * uGu +
                                C.C_r * mu * mu * S.GG + riis2;
            tauM = 1.0 / sqrt(tsum);
            tauC = 1.0 / (tauM * S.gg);
        }
        double Kv[3], at[3];
        for (int c = 0; c < 3; ++c) Kv[c] = fq[c] + rdt * ubq[c];
        for (int c = 0; c < 3; ++c) {
            const double ad = uq[0] * gU[c][0] + uq[1] * gU[c][1] + uq[2] * gU[c][2];
            const double rt = rho * (adt * uq[c] + ad) + S.gP[c] - mu * lapU[c] + sigR * uq[c] - Kv[c];
            at[c] = tauM * rt;
        }
        S.w[q] = w;
        S.M[q] = rho * adt + sigR;
        S.tM[q] = tauM;
        S.tC[q] = tauC;
        for (int a = 0; a < 4; ++a) S.lam[q][a] = L[a];
        for (int c = 0; c < 3; ++c) S.K[q][c] = Kv[c];
        const bool vms = C.stab == LX_STAB_VMS_LES;
        for (int a = 0; a < 10; ++a) {
            const double ad = uq[0] * dphi[a][0] + uq[1] * dphi[a][1] + uq[2] * dphi[a][2];
            S.phi[q][a] = phi[a];
            for (int j = 0; j < 3; ++j) S.dphi[q][a][j] = dphi[a][j];
            S.adv[q][a] = ad;
            S.s[q][a] = rho * (adt * phi[a] + ad) - mu * S.lap[a] + sigR * phi[a];
            for (int c = 0; c < 3; ++c)
                for (int j = 0; j < 3; ++j) {
                    double t = (c == j) ? ad : 0.0;
                    if (vms) t += (uq[c] - at[c]) * dphi[a][j];
                    S.T[q][a][3 * c + j] = rho * t;
                }
        }
    }
    __syncthreads();

    // ---- entry groups over the lanes
    double *R = A.rec + e * (int64_t)kP2Rec;
    for (int it = lane; it < 210; it += 64) {
        if (it < 100) {
            // F block of velocity nodes (a, b): rows 3a + c, columns 3b + d
            const int a = it / 10, b = it % 10;
            double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int q = 0; q < kP2Q; ++q) {
                const double w = S.w[q];
                const double *da = S.dphi[q][a], *db = S.dphi[q][b];
                const double gab = da[0] * db[0] + da[1] * db[1] + da[2] * db[2];
                const double diag = S.M[q] * S.phi[q][a] * S.phi[q][b] + rho * S.phi[q][a] * S.adv[q][b] + mu * gab;
                const double ts = S.tM[q] * S.s[q][b], tc = S.tC[q];
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d) {
                        double v = ts * S.T[q][a][3 * c + d] + tc * da[c] * db[d];
                        if (c == d) v += diag;
                        if (symgrad) v += mu * db[c] * da[d];
                        acc[3 * c + d] += w * v;
                    }
            }
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) R[(3 * a + c) * 34 + 3 * b + d] = acc[3 * c + d];
        } else if (it < 140) {
            // G: velocity node a, pressure vertex b
            const int a = (it - 100) / 4, b = (it - 100) % 4;
            double acc[3] = {0, 0, 0};
            for (int q = 0; q < kP2Q; ++q) {
                const double w = S.w[q], tm = S.tM[q];
                for (int c = 0; c < 3; ++c) {
                    const double *Tc = &S.T[q][a][3 * c];
                    acc[c] += w * (-S.lam[q][b] * S.dphi[q][a][c] +
                                   tm * (S.dl[b][0] * Tc[0] + S.dl[b][1] * Tc[1] + S.dl[b][2] * Tc[2]));
                }
            }
            for (int c = 0; c < 3; ++c) R[(3 * a + c) * 34 + 30 + b] = acc[c];
        } else if (it < 180) {
            // B: pressure vertex a, velocity node b
            const int a = (it - 140) / 10, b = (it - 140) % 10;
            double acc[3] = {0, 0, 0};
            for (int q = 0; q < kP2Q; ++q) {
                const double w = S.w[q], ts = S.tM[q] * S.s[q][b];
                for (int d = 0; d < 3; ++d) acc[d] += w * (S.lam[q][a] * S.dphi[q][b][d] + ts * S.dl[a][d]);
            }
            for (int d = 0; d < 3; ++d) R[(30 + a) * 34 + 3 * b + d] = acc[d];
        } else if (it < 196) {
            // C: pressure vertices (a, b)
            const int a = (it - 180) / 4, b = (it - 180) % 4;
            const double gab = S.dl[a][0] * S.dl[b][0] + S.dl[a][1] * S.dl[b][1] + S.dl[a][2] * S.dl[b][2];
            double acc = 0;
            for (int q = 0; q < kP2Q; ++q) acc += S.w[q] * S.tM[q] * gab;
            R[(30 + a) * 34 + 30 + b] = acc;
        } else if (it < 206) {
            // right-hand side of velocity node a
            const int a = it - 196;
            double acc[3] = {0, 0, 0};
            for (int q = 0; q < kP2Q; ++q) {
                const double w = S.w[q], tm = S.tM[q];
                const double *K = S.K[q];
                for (int c = 0; c < 3; ++c) {
                    const double *Tc = &S.T[q][a][3 * c];
                    acc[c] += w * (K[c] * S.phi[q][a] + tm * (K[0] * Tc[0] + K[1] * Tc[1] + K[2] * Tc[2]));
                }
            }
            for (int c = 0; c < 3; ++c) R[1156 + 3 * a + c] = acc[c];
        } else {
            // right-hand side of pressure vertex a
            const int a = it - 206;
            double acc = 0;
            for (int q = 0; q < kP2Q; ++q) {
                const double *K = S.K[q];
                acc += S.w[q] * S.tM[q] * (K[0] * S.dl[a][0] + K[1] * S.dl[a][1] + K[2] * S.dl[a][2]);
            }
            R[1156 + 30 + a] = acc;
        }
    }
}

// ---- slot gathers (one thread per slot, records summed in list order)

__global__ __launch_bounds__(256) void k_gather_p2f(P2AsmArgs A, P2Sys<double> S, double *rhs)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S.nf) return;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, r[3] = {0, 0, 0};
    bool diag = false;
    int64_t node = -1;
    for (int32_t q = A.finc_ptr[k]; q < A.finc_ptr[k + 1]; ++q) {
        const int32_t code = A.finc[q];
        const int64_t e = code >> 7;
        const int ab = code & 127, a = ab / 10, b = ab % 10;
        const double *R = A.rec + e * (int64_t)kP2Rec;
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) acc[3 * c + d] += R[(3 * a + c) * 34 + 3 * b + d];
        if (a == b) {
            for (int c = 0; c < 3; ++c) r[c] += R[1156 + 3 * a + c];
            diag = true;
            node = A.nodes[(int64_t)a * A.nt + e];
        }
    }
    for (int p = 0; p < 9; ++p) S.F[(int64_t)p * S.nf + k] = acc[p];
    if (rhs && diag)
        for (int c = 0; c < 3; ++c) rhs[4 * node + c] = r[c];
}

__global__ __launch_bounds__(256) void k_gather_p2g(P2AsmArgs A, P2Sys<double> S)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S.ng) return;
    double acc[3] = {0, 0, 0};
    for (int32_t q = A.ginc_ptr[k]; q < A.ginc_ptr[k + 1]; ++q) {
        const int32_t code = A.ginc[q];
        const int64_t e = code >> 7;
        const int ab = code & 127, a = ab / 10, b = ab % 10;
        const double *R = A.rec + e * (int64_t)kP2Rec;
        for (int c = 0; c < 3; ++c) acc[c] += R[(3 * a + c) * 34 + 30 + b];
    }
    for (int c = 0; c < 3; ++c) S.G[(int64_t)c * S.ng + k] = acc[c];
}

__global__ __launch_bounds__(256) void k_gather_p2b(P2AsmArgs A, P2Sys<double> S)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S.nb) return;
    double acc[3] = {0, 0, 0};
    for (int32_t q = A.binc_ptr[k]; q < A.binc_ptr[k + 1]; ++q) {
        const int32_t code = A.binc[q];
        const int64_t e = code >> 7;
        const int ab = code & 127, a = ab / 10, b = ab % 10;
        const double *R = A.rec + e * (int64_t)kP2Rec;
        for (int d = 0; d < 3; ++d) acc[d] += R[(30 + a) * 34 + 3 * b + d];
    }
    for (int d = 0; d < 3; ++d) S.B[(int64_t)d * S.nb + k] = acc[d];
}

// C on the vertex pattern (incidence codes 16 e + 4 a + b of the P1 path)
__global__ __launch_bounds__(256) void k_gather_p2c(P2AsmArgs A, P2Sys<double> S, double *rhs)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S.nc) return;
    double acc = 0, r = 0;
    int64_t vert = -1;
    for (int32_t q = A.cinc_ptr[k]; q < A.cinc_ptr[k + 1]; ++q) {
        const int32_t code = A.cinc[q];
        const int64_t e = code >> 4;
        const int a = (code >> 2) & 3, b = code & 3;
        const double *R = A.rec + e * (int64_t)kP2Rec;
        acc += R[(30 + a) * 34 + 30 + b];
        if (a == b) {
            r += R[1156 + 30 + a];
            vert = A.tet[(int64_t)a * A.nt + e];
        }
    }
    S.C[k] = acc;
    if (rhs && vert >= 0) rhs[4 * vert + 3] = r;
}

void launch_assemble_p2(const P2AsmArgs &a, const StepCoef &c, const P2Sys<double> &S, double *rhs, hipStream_t s)
{
    hipLaunchKernelGGL(k_element_p2, dim3((unsigned)a.nt), dim3(64), 0, s, a, c, c.symgrad);
    hipLaunchKernelGGL(k_gather_p2f, dim3((unsigned)((S.nf + 255) / 256)), dim3(256), 0, s, a, S, rhs);
    hipLaunchKernelGGL(k_gather_p2g, dim3((unsigned)((S.ng + 255) / 256)), dim3(256), 0, s, a, S);
    hipLaunchKernelGGL(k_gather_p2b, dim3((unsigned)((S.nb + 255) / 256)), dim3(256), 0, s, a, S);
    hipLaunchKernelGGL(k_gather_p2c, dim3((unsigned)((S.nc + 255) / 256)), dim3(256), 0, s, a, S, rhs);
}

// ---- Dirichlet rows

template <typename T>
__global__ void k_dirichlet_rows_p2(int64_t n_dir, const int32_t *dir_node, const double *g, P2Sys<T> S,
                                    const int32_t *fdiag, T *rhs)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_dir) return;
    const int64_t i = dir_node[k];
    const int32_t dk = fdiag[i];
    for (int32_t s = S.fptr[i]; s < S.fptr[i + 1]; ++s)
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d)
                if (!(s == dk && c == d)) S.F[(int64_t)(3 * c + d) * S.nf + s] = T(0);
    for (int32_t s = S.gptr[i]; s < S.gptr[i + 1]; ++s)
        for (int c = 0; c < 3; ++c) S.G[(int64_t)c * S.ng + s] = T(0);
    if (rhs)
        for (int c = 0; c < 3; ++c) rhs[4 * i + c] = (T)((double)S.F[(int64_t)(4 * c) * S.nf + dk] * g[3 * k + c]);
}

template <typename T>
void launch_dirichlet_rows_p2(int64_t n_dir, const int32_t *dir_node, const double *g, const P2Sys<T> &S,
                              const int32_t *fdiag, T *rhs, hipStream_t s)
{
    if (n_dir == 0) return;
    hipLaunchKernelGGL((k_dirichlet_rows_p2<T>), dim3((unsigned)((n_dir + 255) / 256)), dim3(256), 0, s, n_dir,
                       dir_node, g, S, fdiag, rhs);
}
template void launch_dirichlet_rows_p2<double>(int64_t, const int32_t *, const double *, const P2Sys<double> &,
                                               const int32_t *, double *, hipStream_t);

// ---- Neumann traction on quadratic boundary triangles

__global__ void k_neumann_p2(int64_t nf, const int32_t *faces6, const double *xn, const double *hn, double h0,
                             double h1, double h2, const P2Rules *R, double *out)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int64_t nd[6];
    for (int a = 0; a < 6; ++a) nd[a] = faces6[6 * f + a];
    double u[3], v[3];
    for (int c = 0; c < 3; ++c) {
        u[c] = xn[3 * nd[1] + c] - xn[3 * nd[0] + c];
        v[c] = xn[3 * nd[2] + c] - xn[3 * nd[0] + c];
    }
    const double n0 = u[1] * v[2] - u[2] * v[1], n1 = u[2] * v[0] - u[0] * v[2], n2 = u[0] * v[1] - u[1] * v[0];
    const double jac = sqrt(n0 * n0 + n1 * n1 + n2 * n2);   // 2 * area
    double hv[6][3];
    for (int a = 0; a < 6; ++a) {
        hv[a][0] = hn ? hn[3 * nd[a]] : h0;
        hv[a][1] = hn ? hn[3 * nd[a] + 1] : h1;
        hv[a][2] = hn ? hn[3 * nd[a] + 2] : h2;
    }
    double acc[6][3] = {{0}};
    for (int q = 0; q < kP2FQ; ++q) {
        const double L0 = R->flam[q][0], L1 = R->flam[q][1], L2 = R->flam[q][2];
        const double ph[6] = {L0 * (2 * L0 - 1), L1 * (2 * L1 - 1), L2 * (2 * L2 - 1), 4 * L0 * L1, 4 * L1 * L2,
                              4 * L2 * L0};
        double hq[3] = {0, 0, 0};
        for (int a = 0; a < 6; ++a)
            for (int c = 0; c < 3; ++c) hq[c] += ph[a] * hv[a][c];
        const double w = R->fw[q] * jac;
        for (int a = 0; a < 6; ++a)
            for (int c = 0; c < 3; ++c) acc[a][c] += w * hq[c] * ph[a];
    }
    for (int a = 0; a < 6; ++a)
        for (int c = 0; c < 3; ++c) atomic_add(&out[4 * nd[a] + c], acc[a][c]);
}

void launch_neumann_p2(int64_t nf, const int32_t *faces6, const double *xnode, const double *hn,
                       const double hconst[3], const P2Rules *rules, double *out, hipStream_t s)
{
    if (nf == 0) return;
    hipLaunchKernelGGL(k_neumann_p2, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, nf, faces6, xnode, hn,
                       hconst[0], hconst[1], hconst[2], rules, out);
}

// ---- SIMPLE diagonal blocks

template <typename T>
__global__ void k_simple_setup_p2(P2Sys<T> S, const int32_t *fdiag, T *Finv, T *Dinv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.nu) return;
    const int32_t dk = fdiag[i];
    T A[9];
    for (int p = 0; p < 9; ++p) A[p] = S.F[(int64_t)p * S.nf + dk];
    const T c0 = A[4] * A[8] - A[5] * A[7], c1 = A[5] * A[6] - A[3] * A[8], c2 = A[3] * A[7] - A[4] * A[6];
    const T id = T(1) / (A[0] * c0 + A[1] * c1 + A[2] * c2);
    const T Bm[9] = {c0 * id, (A[2] * A[7] - A[1] * A[8]) * id, (A[1] * A[5] - A[2] * A[4]) * id,
                          c1 * id, (A[0] * A[8] - A[2] * A[6]) * id, (A[2] * A[3] - A[0] * A[5]) * id,
                          c2 * id, (A[1] * A[6] - A[0] * A[7]) * id, (A[0] * A[4] - A[1] * A[3]) * id};
    for (int p = 0; p < 9; ++p) Finv[(int64_t)p * S.nu + i] = (T)Bm[p];
    for (int c = 0; c < 3; ++c) Dinv[(int64_t)c * S.nu + i] = (T)(T(1) / A[4 * c]);
}

template <typename T>
void launch_simple_setup_p2(const P2Sys<T> &S, const int32_t *fdiag, T *Finv, T *Dinv, hipStream_t s)
{
    hipLaunchKernelGGL((k_simple_setup_p2<T>), dim3((unsigned)((S.nu + 127) / 128)), dim3(128), 0, s, S, fdiag,
                       Finv, Dinv);
}
template void launch_simple_setup_p2<double>(const P2Sys<double> &, const int32_t *, double *, double *,
                                             hipStream_t);
template void launch_simple_setup_p2<float>(const P2Sys<float> &, const int32_t *, float *, float *, hipStream_t);

// ---- split SpMV: velocity rows (F, G), then pressure rows (B, C)

template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_spmv_p2u(P2Sys<T> S, const T *__restrict__ x, T *__restrict__ y,
                                                  const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= S.nu) return;
    using V = typename V4<T>::type;
    T y0 = 0, y1 = 0, y2 = 0;
    for (int32_t k = S.fptr[row] + lane; k < S.fptr[row + 1]; k += LPR) {
        const V xv = reinterpret_cast<const V *>(x)[S.fcol[k]];
        T a[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) a[p] = S.F[(int64_t)p * S.nf + k];
        y0 += a[0] * xv.v[0] + a[1] * xv.v[1] + a[2] * xv.v[2];
        y1 += a[3] * xv.v[0] + a[4] * xv.v[1] + a[5] * xv.v[2];
        y2 += a[6] * xv.v[0] + a[7] * xv.v[1] + a[8] * xv.v[2];
    }
    for (int32_t k = S.gptr[row] + lane; k < S.gptr[row + 1]; k += LPR) {
        const T xp = x[4 * (int64_t)S.gcol[k] + 3];
        y0 += S.G[k] * xp;
        y1 += S.G[S.ng + k] * xp;
        y2 += S.G[2 * S.ng + k] * xp;
    }
    y0 = group_sum<T, LPR>(y0);
    y1 = group_sum<T, LPR>(y1);
    y2 = group_sum<T, LPR>(y2);
    if (lane == 0) {
        y[4 * row] = (T)y0;
        y[4 * row + 1] = (T)y1;
        y[4 * row + 2] = (T)y2;
        if (row >= S.nv) y[4 * row + 3] = T(0);
    }
}

template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_spmv_p2p(P2Sys<T> S, const T *__restrict__ x, T *__restrict__ y,
                                                  const int32_t *done)
{
    if (done && *done) return;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= S.nv) return;
    using V = typename V4<T>::type;
    T acc = 0;
    for (int32_t k = S.bptr[row] + lane; k < S.bptr[row + 1]; k += LPR) {
        const V xv = reinterpret_cast<const V *>(x)[S.bcol[k]];
        acc += S.B[k] * xv.v[0] + S.B[S.nb + k] * xv.v[1] + S.B[2 * S.nb + k] * xv.v[2];
    }
    for (int32_t k = S.cptr[row] + lane; k < S.cptr[row + 1]; k += LPR)
        acc += S.C[k] * x[4 * (int64_t)S.ccol[k] + 3];
    acc = group_sum<T, LPR>(acc);
    if (lane == 0) y[4 * row + 3] = (T)acc;
}

template <typename T>
void launch_spmv_p2(const P2Sys<T> &S, const T *x, T *y, const int32_t *done, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1)
{
    const unsigned gu = (unsigned)((S.nu * 16 + 255) / 256), gp = (unsigned)((S.nv * 16 + 255) / 256);
    if (ev0) (void)hipEventRecord(ev0, s);
    hipLaunchKernelGGL((k_spmv_p2u<T, 16>), dim3(gu), dim3(256), 0, s, S, x, y, done);
    hipLaunchKernelGGL((k_spmv_p2p<T, 16>), dim3(gp), dim3(256), 0, s, S, x, y, done);
    if (ev1) (void)hipEventRecord(ev1, s);
}
template void launch_spmv_p2<double>(const P2Sys<double> &, const double *, double *, const int32_t *, hipStream_t,
                                     hipEvent_t, hipEvent_t);
template void launch_spmv_p2<float>(const P2Sys<float> &, const float *, float *, const int32_t *, hipStream_t,
                                    hipEvent_t, hipEvent_t);

void launch_round_p2(const P2Sys<double> &S64, const P2Sys<float> &S32, hipStream_t s)
{
    launch_scale_copy<float, double>(9 * S64.nf, S32.F, S64.F, 1.0, s);
    launch_scale_copy<float, double>(3 * S64.ng, S32.G, S64.G, 1.0, s);
    launch_scale_copy<float, double>(3 * S64.nb, S32.B, S64.B, 1.0, s);
    launch_scale_copy<float, double>(S64.nc, S32.C, S64.C, 1.0, s);
}

}  // namespace lx
