// Host-side setup: mesh validation, reverse Cuthill-McKee vertex renumbering,
// element reordering, the block-CSR pattern shared by the F/G/B/C blocks of the
// P1-P1 system (one 4x4 block per vertex pair sharing a tetrahedron), the
// element -> block-slot map and the transposed-slot map.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "lx_common.h"

namespace lx {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

lx_status fail(lx_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

static double tet_det(const double *X, const int32_t *v)
{
    double J[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) J[i][k] = X[3 * v[k + 1] + i] - X[3 * v[0] + i];
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Vertex adjacency (including self) as CSR, sorted, from the element list.
static void vertex_graph(int64_t nv, int64_t nt, const int32_t *tets, std::vector<int32_t> &ptr,
                         std::vector<int32_t> &adj)
{
    std::vector<int32_t> cnt(nv + 1, 0);
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a) cnt[tets[4 * e + a] + 1]++;
    for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
    std::vector<int32_t> v2e(cnt[nv]);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a) v2e[fill[tets[4 * e + a]]++] = (int32_t)e;
    ptr.assign(nv + 1, 0);
    adj.clear();
    adj.reserve((size_t)nv * 16);
    std::vector<int32_t> buf;
    for (int64_t v = 0; v < nv; ++v) {
        buf.clear();
        for (int32_t k = cnt[v]; k < cnt[v + 1]; ++k) {
            const int32_t *t = tets + 4 * (int64_t)v2e[k];
            for (int a = 0; a < 4; ++a) buf.push_back(t[a]);
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
        adj.insert(adj.end(), buf.begin(), buf.end());
        ptr[v + 1] = (int32_t)adj.size();
    }
}

// Reverse Cuthill-McKee: BFS from a pseudo-peripheral vertex of each connected
// component, visiting neighbours by increasing degree, then reversed.
static std::vector<int32_t> rcm_order(int64_t nv, const std::vector<int32_t> &ptr,
                                      const std::vector<int32_t> &adj)
{
    std::vector<int32_t> order;
    order.reserve(nv);
    std::vector<char> seen(nv, 0);
    std::vector<int32_t> deg(nv);
    for (int64_t v = 0; v < nv; ++v) deg[v] = ptr[v + 1] - ptr[v];
    std::vector<int32_t> level(nv, -1);
    auto bfs_far = [&](int32_t s) {
        // returns the last vertex of a BFS from s (a far vertex)
        std::vector<int32_t> q{s};
        std::vector<int32_t> touched{s};
        level[s] = 0;
        size_t h = 0;
        int32_t last = s;
        while (h < q.size()) {
            int32_t v = q[h++];
            last = v;
            for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k) {
                int32_t w = adj[k];
                if (level[w] < 0) {
                    level[w] = level[v] + 1;
                    q.push_back(w);
                    touched.push_back(w);
                }
            }
        }
        for (int32_t v : touched) level[v] = -1;
        return last;
    };
    std::vector<int32_t> nb;
    for (int64_t s0 = 0; s0 < nv; ++s0) {
        if (seen[s0]) continue;
        int32_t s = bfs_far(bfs_far((int32_t)s0));
        size_t head = order.size();
        order.push_back(s);
        seen[s] = 1;
        while (head < order.size()) {
            int32_t v = order[head++];
            nb.clear();
            for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k)
                if (!seen[adj[k]]) {
                    seen[adj[k]] = 1;
                    nb.push_back(adj[k]);
                }
            std::stable_sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

lx_status build_setup(const lx_mesh *m, HostSetup &hs)
{
    if (!m || !m->coords || !m->tets || m->n_vertices <= 0 || m->n_tets <= 0)
        return fail(LX_EINVAL, "mesh: empty or NULL arrays");
    if (m->n_vertices >= (int64_t)1 << 31 || m->n_tets >= (int64_t)1 << 31)
        return fail(LX_EINVAL, "mesh: more than 2^31 vertices or tets");
    const int64_t nv = m->n_vertices, nt = m->n_tets;
    hs.nv = nv;
    hs.nt = nt;
    for (int64_t k = 0; k < 4 * nt; ++k)
        if (m->tets[k] < 0 || m->tets[k] >= nv)
            return fail(LX_EMESH, "mesh: tet %lld references vertex %d out of range", (long long)(k / 4),
                        m->tets[k]);
    // degenerate-element check: |det J| <= 1e-14 h^3 with h the longest edge
    for (int64_t e = 0; e < nt; ++e) {
        const int32_t *v = m->tets + 4 * e;
        double h2 = 0;
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) {
                double d2 = 0;
                for (int c = 0; c < 3; ++c) {
                    double d = m->coords[3 * v[a] + c] - m->coords[3 * v[b] + c];
                    d2 += d * d;
                }
                h2 = std::max(h2, d2);
            }
        double h = std::sqrt(h2);
        if (!(std::fabs(tet_det(m->coords, v)) > 1e-14 * h * h * h))
            return fail(LX_EMESH, "mesh: tet %lld is degenerate", (long long)e);
    }
    // renumber vertices
    std::vector<int32_t> ptr, adj;
    vertex_graph(nv, nt, m->tets, ptr, adj);
    hs.perm_v = rcm_order(nv, ptr, adj);
    hs.iperm_v.assign(nv, 0);
    for (int64_t i = 0; i < nv; ++i) hs.iperm_v[hs.perm_v[i]] = (int32_t)i;
    hs.xh.resize(3 * nv);
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) hs.xh[3 * i + c] = m->coords[3 * (int64_t)hs.perm_v[i] + c];
    // renumbered connectivity (local order kept), elements sorted by smallest new vertex id
    std::vector<int32_t> tnew(4 * nt);
    std::vector<int64_t> key(nt);
    for (int64_t e = 0; e < nt; ++e) {
        int32_t mn = INT32_MAX;
        for (int a = 0; a < 4; ++a) {
            tnew[4 * e + a] = hs.iperm_v[m->tets[4 * e + a]];
            mn = std::min(mn, tnew[4 * e + a]);
        }
        key[e] = mn;
    }
    hs.perm_e.resize(nt);
    std::iota(hs.perm_e.begin(), hs.perm_e.end(), 0);
    std::stable_sort(hs.perm_e.begin(), hs.perm_e.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    std::vector<int32_t> tsorted(4 * nt);
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a) tsorted[4 * e + a] = tnew[4 * hs.perm_e[e] + a];
    hs.tet_soa.resize(4 * nt);
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a) hs.tet_soa[a * nt + e] = tsorted[4 * e + a];
    // pattern in the new numbering
    vertex_graph(nv, nt, tsorted.data(), ptr, adj);
    if ((int64_t)adj.size() >= ((int64_t)1 << 31) / 16)
        return fail(LX_EINVAL, "mesh: block count too large for 32-bit slots");
    hs.rowptr = ptr;
    hs.col = adj;
    const int64_t nblk = (int64_t)adj.size();
    hs.diag.assign(nv, -1);
    for (int64_t v = 0; v < nv; ++v)
        for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k)
            if (adj[k] == v) hs.diag[v] = k;
    auto find = [&](int32_t r, int32_t c) -> int32_t {
        auto b = adj.begin() + ptr[r], en = adj.begin() + ptr[r + 1];
        auto it = std::lower_bound(b, en, c);
        return (it != en && *it == c) ? (int32_t)(it - adj.begin()) : -1;
    };
    hs.tslot.resize(nblk);
    for (int64_t v = 0; v < nv; ++v)
        for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k) hs.tslot[k] = find(adj[k], (int32_t)v);
    hs.eslot.resize(16 * nt);
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                hs.eslot[(int64_t)(4 * a + b) * nt + e] = find(tsorted[4 * e + a], tsorted[4 * e + b]);
    // slot -> (element, local block) incidence, ordered by element then local block
    if (16 * nt >= INT32_MAX) return fail(LX_ENOMEM, "mesh too large for 32-bit incidence codes");
    hs.sinc_ptr.assign(nblk + 1, 0);
    for (int64_t q = 0; q < 16 * nt; ++q) ++hs.sinc_ptr[hs.eslot[q] + 1];
    for (int64_t k = 0; k < nblk; ++k) hs.sinc_ptr[k + 1] += hs.sinc_ptr[k];
    hs.sinc.assign(16 * nt, 0);
    {
        std::vector<int32_t> fill(hs.sinc_ptr.begin(), hs.sinc_ptr.end() - 1);
        for (int64_t e = 0; e < nt; ++e)
            for (int ab = 0; ab < 16; ++ab) {
                const int32_t k = hs.eslot[(int64_t)ab * nt + e];
                hs.sinc[fill[k]++] = (int32_t)(16 * e + ab);
            }
    }
    // vertex incidence for the residual pass: the diagonal slots' lists one after
    // the other, and where each (element, local vertex) lands in them
    hs.vinc_ptr.assign(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v)
        hs.vinc_ptr[v + 1] = hs.vinc_ptr[v] + (hs.sinc_ptr[hs.diag[v] + 1] - hs.sinc_ptr[hs.diag[v]]);
    hs.vpos.assign(4 * nt, -1);
    for (int64_t v = 0; v < nv; ++v) {
        const int32_t k = hs.diag[v];
        for (int32_t q = hs.sinc_ptr[k]; q < hs.sinc_ptr[k + 1]; ++q) {
            const int32_t code = hs.sinc[q];
            hs.vpos[(int64_t)((code >> 2) & 3) * nt + (code >> 4)] = hs.vinc_ptr[v] + (q - hs.sinc_ptr[k]);
        }
    }
    if (hs.vinc_ptr[nv] != 4 * nt || std::find(hs.vpos.begin(), hs.vpos.end(), -1) != hs.vpos.end())
        return fail(LX_EMESH, "inconsistent vertex incidence");
    return LX_OK;
}

}  // namespace lx

extern "C" const char *lx_last_error(void) { return lx::g_err; }
