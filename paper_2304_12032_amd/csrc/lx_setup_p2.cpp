// Host set-up of the P2-P1 (Taylor-Hood) system: edge enumeration and P2 node
// numbering (vertices first, then edge midpoints ordered by their vertex pair),
// the split patterns of the F (node-node, 3x3 blocks), G (node-vertex), B
// (vertex-node) blocks -- C uses the vertex pattern of the P1 path -- and the
// slot -> (element, local entry) incidence lists of the assembly gathers.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <utility>

#include "lx_p2.h"

namespace lx {

// Local P2 nodes: the four vertices, then the midpoints of the edges in this order.
static const int kEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

int32_t p2_edge_node(const P2Setup &p2, int64_t nv, int32_t a, int32_t b)
{
    if (a > b) std::swap(a, b);
    const uint64_t key = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
    auto it = std::lower_bound(p2.edge_key.begin(), p2.edge_key.end(), key);
    if (it == p2.edge_key.end() || *it != key) return -1;
    return (int32_t)(nv + (it - p2.edge_key.begin()));
}

// CSR pattern and incidence lists from (row, col, code) entries generated in
// increasing code order: rows are bucketed, each bucket stably sorted by column,
// so every slot lists its codes in increasing order.
template <class Gen>
static void build_split(int64_t nrows, Gen gen, std::vector<int32_t> &rowptr, std::vector<int32_t> &col,
                        std::vector<int32_t> &iptr, std::vector<int32_t> &inc)
{
    std::vector<int64_t> cnt(nrows + 1, 0);
    gen([&](int32_t r, int32_t, int32_t) { ++cnt[r + 1]; });
    for (int64_t i = 0; i < nrows; ++i) cnt[i + 1] += cnt[i];
    std::vector<std::pair<int32_t, int32_t>> ent(cnt[nrows]);   // (col, code)
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        gen([&](int32_t r, int32_t c, int32_t code) { ent[fill[r]++] = {c, code}; });
    }
    rowptr.assign(nrows + 1, 0);
    col.clear();
    iptr.assign(1, 0);
    inc.clear();
    inc.reserve(ent.size());
    for (int64_t i = 0; i < nrows; ++i) {
        auto b = ent.begin() + cnt[i], e = ent.begin() + cnt[i + 1];
        std::stable_sort(b, e, [](const std::pair<int32_t, int32_t> &x, const std::pair<int32_t, int32_t> &y) {
            return x.first < y.first;
        });
        for (auto it = b; it != e; ++it) {
            if (it == b || it->first != (it - 1)->first) {
                col.push_back(it->first);
                iptr.push_back(iptr.back());
            }
            inc.push_back(it->second);
            ++iptr.back();
        }
        rowptr[i + 1] = (int32_t)col.size();
    }
}

lx_status build_setup_p2(const HostSetup &hs, P2Setup &p2)
{
    const int64_t nv = hs.nv, nt = hs.nt;
    if (nt >= ((int64_t)1 << 31) / 128) return fail(LX_EINVAL, "P2-P1: too many tets for 32-bit incidence codes");
    const int32_t *T = hs.tet_soa.data();   // [4][nt]
    // edges of all elements, unique, ordered by (lower, higher) vertex id
    std::vector<uint64_t> keys((size_t)6 * nt);
    for (int64_t e = 0; e < nt; ++e)
        for (int k = 0; k < 6; ++k) {
            int32_t a = T[kEdge[k][0] * nt + e], b = T[kEdge[k][1] * nt + e];
            if (a > b) std::swap(a, b);
            keys[6 * e + k] = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
        }
    std::vector<uint64_t> uk(keys);
    std::sort(uk.begin(), uk.end());
    uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
    p2.edge_key = uk;
    p2.ne = (int64_t)uk.size();
    p2.nu = nv + p2.ne;
    if (p2.nu >= ((int64_t)1 << 31)) return fail(LX_EINVAL, "P2-P1: too many nodes");
    p2.nodes.assign((size_t)10 * nt, 0);
    for (int64_t e = 0; e < nt; ++e) {
        for (int a = 0; a < 4; ++a) p2.nodes[a * nt + e] = T[a * nt + e];
        for (int k = 0; k < 6; ++k) {
            auto it = std::lower_bound(uk.begin(), uk.end(), keys[6 * e + k]);
            p2.nodes[(4 + k) * nt + e] = (int32_t)(nv + (it - uk.begin()));
        }
    }
    p2.xnode.assign(3 * p2.nu, 0.0);
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) p2.xnode[3 * i + c] = hs.xh[3 * i + c];
    for (int64_t k = 0; k < p2.ne; ++k) {
        const int64_t a = (int64_t)(uk[k] >> 32), b = (int64_t)(uk[k] & 0xffffffffu);
        for (int c = 0; c < 3; ++c) p2.xnode[3 * (nv + k) + c] = 0.5 * (hs.xh[3 * a + c] + hs.xh[3 * b + c]);
    }
    const int32_t *N = p2.nodes.data();
    // F: node rows x node columns, local (a, b) in 0..9
    build_split(p2.nu,
                [&](auto emit) {
                    for (int64_t e = 0; e < nt; ++e)
                        for (int a = 0; a < 10; ++a)
                            for (int b = 0; b < 10; ++b)
                                emit(N[a * nt + e], N[b * nt + e], (int32_t)(128 * e + 10 * a + b));
                },
                p2.fptr, p2.fcol, p2.finc_ptr, p2.finc);
    // G: node rows x vertex columns, local a in 0..9, b in 0..3
    build_split(p2.nu,
                [&](auto emit) {
                    for (int64_t e = 0; e < nt; ++e)
                        for (int a = 0; a < 10; ++a)
                            for (int b = 0; b < 4; ++b)
                                emit(N[a * nt + e], T[b * nt + e], (int32_t)(128 * e + 10 * a + b));
                },
                p2.gptr, p2.gcol, p2.ginc_ptr, p2.ginc);
    // B: vertex rows x node columns, local a in 0..3, b in 0..9
    build_split(nv,
                [&](auto emit) {
                    for (int64_t e = 0; e < nt; ++e)
                        for (int a = 0; a < 4; ++a)
                            for (int b = 0; b < 10; ++b)
                                emit(T[a * nt + e], N[b * nt + e], (int32_t)(128 * e + 10 * a + b));
                },
                p2.bptr, p2.bcol, p2.binc_ptr, p2.binc);
    if ((int64_t)p2.fcol.size() * 9 >= INT32_MAX || (int64_t)p2.finc.size() >= INT32_MAX)
        return fail(LX_EINVAL, "P2-P1: velocity pattern too large for 32-bit offsets");
    p2.fdiag.assign(p2.nu, -1);
    for (int64_t i = 0; i < p2.nu; ++i)
        for (int32_t k = p2.fptr[i]; k < p2.fptr[i + 1]; ++k)
            if (p2.fcol[k] == i) p2.fdiag[i] = k;
    return LX_OK;
}

}  // namespace lx

namespace lx {

// n-point Gauss-Jacobi rule on [0, 1] for the weight (1 - u)^alpha by the
// Golub-Welsch construction: the nodes are the eigenvalues of the symmetric
// tridiagonal Jacobi matrix of the recurrence of the Jacobi polynomials
// P^(alpha, 0) on [-1, 1], the weights mu0 times the squared first eigenvector
// components; the eigenproblem is solved by cyclic Jacobi rotations.
static void gauss_jacobi01(int n, double alpha, double *x, double *w)
{
    const double be = 0.0;
    double J[8][8] = {{0}};
    for (int k = 0; k < n; ++k) {
        const double s = 2.0 * k + alpha + be;
        J[k][k] = (k == 0) ? (be - alpha) / (alpha + be + 2.0) : (be * be - alpha * alpha) / (s * (s + 2.0));
        if (k + 1 < n) {
            const double m = k + 1.0, t = 2.0 * m + alpha + be;
            const double b2 = 4.0 * m * (m + alpha) * (m + be) * (m + alpha + be) / (t * t * (t + 1.0) * (t - 1.0));
            J[k][k + 1] = J[k + 1][k] = std::sqrt(b2);
        }
    }
    double V[8][8] = {{0}};
    for (int k = 0; k < n; ++k) V[k][k] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += J[p][q] * J[p][q];
        if (off < 1e-30) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (std::fabs(J[p][q]) < 1e-300) continue;
                const double th = 0.5 * (J[q][q] - J[p][p]) / J[p][q];
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {   // J <- J R
                    const double a = J[k][p], b = J[k][q];
                    J[k][p] = c * a - sn * b;
                    J[k][q] = sn * a + c * b;
                }
                for (int k = 0; k < n; ++k) {   // J <- R^T J
                    const double a = J[p][k], b = J[q][k];
                    J[p][k] = c * a - sn * b;
                    J[q][k] = sn * a + c * b;
                }
                for (int k = 0; k < n; ++k) {   // V <- V R
                    const double a = V[k][p], b = V[k][q];
                    V[k][p] = c * a - sn * b;
                    V[k][q] = sn * a + c * b;
                }
            }
    }
    // mu0 = int_{-1}^{1} (1-x)^alpha dx = 2^(alpha+1) / (alpha + 1)
    const double mu0 = std::pow(2.0, alpha + 1.0) / (alpha + 1.0);
    for (int k = 0; k < n; ++k) {
        x[k] = 0.5 * (1.0 + J[k][k]);                                   // map to [0, 1]
        w[k] = mu0 * V[0][k] * V[0][k] / std::pow(2.0, alpha + 1.0);    // weight (1-u)^alpha on [0, 1]
    }
}

void p2_rules(P2Rules &R)
{
    double u1[3], w1[3], u2[3], w2[3], u3[3], w3[3];
    gauss_jacobi01(3, 2.0, u1, w1);
    gauss_jacobi01(3, 1.0, u2, w2);
    gauss_jacobi01(3, 0.0, u3, w3);
    // Duffy collapse of the cube onto the simplex: x1 = u1, x2 = u2 (1 - u1),
    // x3 = u3 (1 - u1)(1 - u2); the Jacobian factors are the Jacobi weights
    int q = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k, ++q) {
                const double x1 = u1[i], x2 = u2[j] * (1.0 - u1[i]), x3 = u3[k] * (1.0 - u1[i]) * (1.0 - u2[j]);
                R.lam[q][0] = 1.0 - x1 - x2 - x3;
                R.lam[q][1] = x1;
                R.lam[q][2] = x2;
                R.lam[q][3] = x3;
                R.w[q] = w1[i] * w2[j] * w3[k];
            }
    double v1[3], z1[3], v2[3], z2[3];
    gauss_jacobi01(3, 1.0, v1, z1);
    gauss_jacobi01(3, 0.0, v2, z2);
    q = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j, ++q) {
            const double x1 = v1[i], x2 = v2[j] * (1.0 - v1[i]);
            R.flam[q][0] = 1.0 - x1 - x2;
            R.flam[q][1] = x1;
            R.flam[q][2] = x2;
            R.fw[q] = z1[i] * z2[j];
        }
}

}  // namespace lx
