// Host set-up of the Schur-block multigrid hierarchy: the pattern of
// S~ = C - B D^{-1} G, greedy aggregation and the fixed index lists that turn
// each step's fine values into coarse ones.
#include <algorithm>
#include <numeric>
#include <utility>

#include "lx_amg.h"

namespace lx {

// Greedy aggregation on a graph (CSR, self loops allowed): first every row whose
// neighbours are all free becomes a root and takes its neighbourhood; then each
// remaining row joins the aggregate that most of its neighbours belong to
// (lowest aggregate id on ties).  Rows are visited in index order.
static int64_t aggregate(int64_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                         std::vector<int32_t> &agg)
{
    agg.assign(n, -1);
    int64_t na = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        bool free_nb = true;
        for (int32_t k = rp[i]; k < rp[i + 1] && free_nb; ++k)
            if (ci[k] != i && agg[ci[k]] >= 0) free_nb = false;
        if (!free_nb) continue;
        agg[i] = (int32_t)na;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) agg[ci[k]] = (int32_t)na;
        ++na;
    }
    std::vector<std::pair<int32_t, int32_t>> cnt;
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        cnt.clear();
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t a = agg[ci[k]];
            if (a < 0) continue;
            auto it = std::find_if(cnt.begin(), cnt.end(), [&](const std::pair<int32_t, int32_t> &p) {
                return p.first == a;
            });
            if (it == cnt.end())
                cnt.push_back({a, 1});
            else
                ++it->second;
        }
        if (cnt.empty()) {
            agg[i] = (int32_t)na++;
            continue;
        }
        int32_t best = cnt[0].first, bc = cnt[0].second;
        for (auto &p : cnt)
            if (p.second > bc || (p.second == bc && p.first < best)) {
                best = p.first;
                bc = p.second;
            }
        agg[i] = best;
    }
    // rows that joined an aggregate in the second pass were not yet neighbours of
    // a root when that root was made; nothing else to fix
    return na;
}

// Coarse pattern of P^T A P for piecewise-constant P and the contribution lists.
static void coarsen(AmgLevelHost &f, AmgLevelHost &c, int64_t nc)
{
    const int64_t n = f.n;
    f.mptr.assign(nc + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++f.mptr[f.agg[i] + 1];
    for (int64_t a = 0; a < nc; ++a) f.mptr[a + 1] += f.mptr[a];
    f.mem.assign(n, 0);
    {
        std::vector<int32_t> fill(f.mptr.begin(), f.mptr.end() - 1);
        for (int64_t i = 0; i < n; ++i) f.mem[fill[f.agg[i]]++] = (int32_t)i;
    }
    c.n = nc;
    c.rowptr.assign(nc + 1, 0);
    c.col.clear();
    f.cptr.assign(1, 0);
    f.cidx.clear();
    f.cidx.reserve(f.col.size());
    std::vector<std::pair<int32_t, int32_t>> ent;   // (coarse column, fine entry)
    for (int64_t a = 0; a < nc; ++a) {
        ent.clear();
        for (int32_t q = f.mptr[a]; q < f.mptr[a + 1]; ++q) {
            const int32_t i = f.mem[q];
            for (int32_t k = f.rowptr[i]; k < f.rowptr[i + 1]; ++k) ent.push_back({f.agg[f.col[k]], k});
        }
        std::sort(ent.begin(), ent.end());
        for (size_t q = 0; q < ent.size(); ++q) {
            if (q == 0 || ent[q].first != ent[q - 1].first) {
                c.col.push_back(ent[q].first);
                f.cptr.push_back(f.cptr.back());
            }
            f.cidx.push_back(ent[q].second);
            ++f.cptr.back();
        }
        c.rowptr[a + 1] = (int32_t)c.col.size();
    }
    c.diag.assign(nc, -1);
    for (int64_t a = 0; a < nc; ++a)
        for (int32_t k = c.rowptr[a]; k < c.rowptr[a + 1]; ++k)
            if (c.col[k] == a) c.diag[a] = k;
}

lx_status amg_build_host(const HostSetup &hs, AmgHost &H)
{
    const int64_t nv = hs.nv;
    const std::vector<int32_t> &rp = hs.rowptr, &ci = hs.col;
    H.lev.clear();
    H.lev.emplace_back();
    AmgLevelHost &L0 = H.lev[0];
    L0.n = nv;
    // S~ = C - B D^{-1} G: entry (i, k) for k in the neighbourhood of a neighbour of i
    L0.rowptr.assign(nv + 1, 0);
    std::vector<int32_t> row;
    std::vector<char> mark(nv, 0);
    for (int pass = 0; pass < 2; ++pass) {
        int64_t nnz = 0;
        for (int64_t i = 0; i < nv; ++i) {
            row.clear();
            for (int32_t k1 = rp[i]; k1 < rp[i + 1]; ++k1) {
                const int32_t j = ci[k1];
                for (int32_t k2 = rp[j]; k2 < rp[j + 1]; ++k2) {
                    const int32_t k = ci[k2];
                    if (!mark[k]) {
                        mark[k] = 1;
                        row.push_back(k);
                    }
                }
            }
            for (int32_t k : row) mark[k] = 0;
            if (pass == 0) {
                nnz += (int64_t)row.size();
                L0.rowptr[i + 1] = (int32_t)row.size();
            } else {
                std::sort(row.begin(), row.end());
                std::copy(row.begin(), row.end(), L0.col.begin() + L0.rowptr[i]);
            }
        }
        if (pass == 0) {
            if (nnz >= INT32_MAX) return fail(LX_ENOMEM, "Schur pattern too large for 32-bit offsets");
            for (int64_t i = 0; i < nv; ++i) L0.rowptr[i + 1] += L0.rowptr[i];
            L0.col.assign(nnz, 0);
        }
    }
    L0.diag.assign(nv, -1);
    for (int64_t i = 0; i < nv; ++i)
        for (int32_t k = L0.rowptr[i]; k < L0.rowptr[i + 1]; ++k)
            if (L0.col[k] == i) L0.diag[i] = k;

    while (H.lev.back().n > kAmgDenseMax) {
        if ((int)H.lev.size() > kAmgMaxLevels)
            return fail(LX_EINVAL, "AMG: more than %d levels needed", kAmgMaxLevels);
        AmgLevelHost &f = H.lev.back();
        // level 0 aggregates over the vertex graph, coarser levels over their own pattern
        const bool fine = H.lev.size() == 1;
        const int64_t nc = aggregate(f.n, fine ? rp : f.rowptr, fine ? ci : f.col, f.agg);
        if (nc * 10 > f.n * 9)
            return fail(LX_EINVAL, "AMG: aggregation stalled at %lld rows", (long long)f.n);
        AmgLevelHost c;
        coarsen(f, c, nc);
        H.lev.push_back(std::move(c));
    }
    return LX_OK;
}

}  // namespace lx

namespace lx {

static int32_t align16(int64_t x) { return (int32_t)((x + 15) & ~int64_t(15)); }

TailLayout amg_tail_layout(int nlev, const int64_t *n, const int64_t *nnz, int vbytes, int64_t max_lds)
{
    for (int first = 1; first < nlev; ++first) {
        if (nlev - first > kTailDepth) continue;
        bool small = true;
        for (int m = first; m < nlev; ++m) small = small && n[m] <= kTailMaxRows;
        if (!small) continue;
        // with the member lists in the image, and space to stage the finer residual
        // in member order; with the lists only; with neither
        for (int variant = 0; variant < 3; ++variant) {
            const bool lists = variant < 2, stage = variant == 0;
            TailLayout T;
            T.first = first;
            T.nlev = nlev;
            T.nc = (int)n[nlev];
            int64_t o = 0;
            T.o_dense = 0;
            o = align16(o + 8 * 2 * n[nlev] * n[nlev]);
            if (lists) {
                T.o_fmptr = (int32_t)o;
                o = align16(o + 4 * (n[first] + 1));
                T.o_fmem = (int32_t)o;
                o = align16(o + 4 * n[first - 1]);
            }
            for (int m = first; m < nlev; ++m) {
                TailLevelLds &L = T.lv[m - first];
                L.n = (int32_t)n[m];
                L.nnz = (int32_t)nnz[m];
                L.nn = (int32_t)n[m + 1];
                L.lanes = 1;
                while (L.lanes < 16 && (int64_t)L.n * L.lanes * 2 <= kTailThreads) L.lanes *= 2;
                L.o_val = (int32_t)o;
                o = align16(o + (int64_t)vbytes * L.nnz);
                L.o_dinv = (int32_t)o;
                o = align16(o + (int64_t)vbytes * L.n);
                L.o_rowptr = (int32_t)o;
                o = align16(o + 4 * ((int64_t)L.n + 1));
                L.o_col = (int32_t)o;
                o = align16(o + 4 * (int64_t)L.nnz);
                L.o_agg = (int32_t)o;
                o = align16(o + 4 * (int64_t)L.n);
                L.o_mptr = (int32_t)o;
                o = align16(o + 4 * ((int64_t)L.nn + 1));
                L.o_mem = (int32_t)o;
                o = align16(o + 4 * (int64_t)L.n);
            }
            T.img_bytes = (int32_t)o;
            for (int m = first; m < nlev; ++m) {
                TailLevelLds &L = T.lv[m - first];
                int32_t *vo[6] = {&L.o_r, &L.o_res, &L.o_x0, &L.o_x1, &L.o_d0, &L.o_d1};
                for (int v = 0; v < 6; ++v) {
                    *vo[v] = (int32_t)o;
                    o = align16(o + (int64_t)vbytes * L.n);
                }
            }
            T.o_rc = (int32_t)o;
            o = align16(o + 8 * n[nlev]);
            T.o_xc = (int32_t)o;
            o = align16(o + (int64_t)vbytes * n[nlev]);
            if (stage) {
                T.o_fstage = (int32_t)o;
                o = align16(o + (int64_t)vbytes * n[first - 1]);
            }
            T.lds_bytes = (int32_t)o;
            if (o <= max_lds) return T;
        }
    }
    return TailLayout();
}

}  // namespace lx
