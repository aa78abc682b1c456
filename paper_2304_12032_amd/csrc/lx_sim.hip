// The simulation object behind the C ABI: device state, one time step (FP64,
// or FP32 with FP64 iterative refinement) and the GMRES driver.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <memory>

#include "lx_kernels.h"
#include "lx_sim.h"

namespace lx {

// ------------------------------------------------------------------ helpers

double law_value(const lx_time_law &L, double t)
{
    const double *p = L.p;
    switch (L.kind) {
    case LX_LAW_CONSTANT:
        return p[0];
    case LX_LAW_PULSATILE:
        return p[0] + (p[1] - p[0]) * 0.5 * (1.0 - std::cos(2.0 * M_PI * t / p[2]));
    case LX_LAW_RAMP:
        if (t < p[2]) return p[0];
        if (t < p[2] + p[3]) return p[0] + 0.5 * (p[1] - p[0]) * (1.0 - std::cos(M_PI * (t - p[2]) / p[3]));
        return p[1];
    case LX_LAW_RAMP2: {
        double tau = p[6] > 0 ? std::fmod(t, p[6]) : t;
        if (tau < p[2]) return p[0];
        if (tau < p[2] + p[3]) return p[0] + 0.5 * (p[1] - p[0]) * (1.0 - std::cos(M_PI * (tau - p[2]) / p[3]));
        if (tau < p[4]) return p[1];
        if (tau < p[4] + p[5]) return p[1] + 0.5 * (p[0] - p[1]) * (1.0 - std::cos(M_PI * (tau - p[4]) / p[5]));
        return p[0];
    }
    case LX_LAW_LINEAR:
        return p[0] + p[1] * t;
    case LX_LAW_SINE:
        return p[0] * std::sin(p[1] * t + p[2]);
    }
    return 0.0;
}

static const double kAlpha[4] = {0, 1.0, 1.5, 11.0 / 6.0};
static const double kBeta[4][3] = {{0, 0, 0}, {1.0, 0, 0}, {2.0, -0.5, 0}, {3.0, -1.5, 1.0 / 3.0}};
static const double kGamma[4][3] = {{0, 0, 0}, {1.0, 0, 0}, {2.0, -1.0, 0}, {3.0, -3.0, 1.0}};

lx_status Sim::dalloc(void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) return LX_OK;
    if (alloc_fn) {
        *p = alloc_fn(bytes, alloc_ctx);
        if (!*p) return fail(LX_ENOMEM, "caller allocator returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) return fail(LX_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    allocs.push_back(*p);
    device_bytes += (int64_t)bytes;
    return LX_OK;
}

Sim::~Sim()
{
    if (device >= 0) (void)hipSetDevice(device);
    if (stream) (void)hipStreamSynchronize(stream);
    for (void *p : allocs) {
        if (free_fn) free_fn(p, alloc_ctx);
        else (void)hipFree(p);
    }
    if (h_st) (void)hipHostFree(h_st);
    if (h_chk) (void)hipHostFree(h_chk);
    if (h_gerr) (void)hipHostFree(h_gerr);
    if (h_norms0) (void)hipHostFree(h_norms0);
    for (auto &ev : ev_chk)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &ev : ev_pool) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    if (ev_step0) (void)hipEventDestroy(ev_step0);
    if (ev_step1) (void)hipEventDestroy(ev_step1);
    if (ev_asm1) (void)hipEventDestroy(ev_asm1);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (stream_aux) (void)hipStreamDestroy(stream_aux);
    for (auto &g : gx_step)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : g_step)
        if (g) (void)hipGraphDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// ------------------------------------------------------------------ creation

lx_status Sim::create(const lx_device *dev, const lx_mesh *mesh, const lx_problem *pr, const lx_solver *sv)
{
    if (!pr || !sv) return fail(LX_EINVAL, "problem/solver NULL");
    if (pr->fe != LX_P1P1 && pr->fe != LX_P2P1) return fail(LX_EINVAL, "fe must be LX_P1P1 or LX_P2P1");
    if (pr->fe == LX_P2P1 && pr->ale) return fail(LX_EINVAL, "ALE is built for the P1-P1 pair only");
    if (pr->fe == LX_P2P1 && sv->precond != LX_PC_AMG)
        return fail(LX_EINVAL, "the P2-P1 pair uses the AMG preconditioner (LX_PC_AMG)");
    if (pr->bdf_order < 1 || pr->bdf_order > 3) return fail(LX_EINVAL, "bdf_order must be 1..3");
    if (!(pr->dt > 0) || !(pr->rho > 0) || !(pr->mu >= 0)) return fail(LX_EINVAL, "dt, rho must be > 0, mu >= 0");
    if (pr->semi_implicit != 0 && pr->semi_implicit != 1) return fail(LX_EINVAL, "semi_implicit must be 0 or 1");
    if (pr->semi_implicit == 0) {
        if (pr->fe != LX_P1P1) return fail(LX_EINVAL, "the implicit formulation is built for the P1-P1 pair");
        if (sv->max_ir < 1) return fail(LX_EINVAL, "implicit formulation: max_ir (Newton updates) must be >= 1");
    }
    if (pr->n_riis < 0 || pr->n_riis > kMaxValves) return fail(LX_EINVAL, "at most %d RIIS surfaces", kMaxValves);
    if (pr->n_bc < 0 || pr->n_bc > kMaxBC) return fail(LX_EINVAL, "at most %d boundary conditions", kMaxBC);
    if (sv->restart < 1 || sv->restart > kMaxRestart) return fail(LX_EINVAL, "restart must be 1..%d", kMaxRestart);
    if (sv->precision != LX_FP64 && sv->precision != LX_FP32_IR) return fail(LX_EINVAL, "bad precision");
    if (pr->stab < 0 || pr->stab > 2) return fail(LX_EINVAL, "bad stabilisation");
    if (sv->precond != LX_PC_AMG && sv->precond != LX_PC_CHEB_SCHUR) return fail(LX_EINVAL, "bad precond");
    if (sv->precond == LX_PC_CHEB_SCHUR) {
        if (sv->schur_degree < 0 || sv->schur_degree > 32) return fail(LX_EINVAL, "schur_degree must be 0..32");
        if (sv->schur_degree > 0 && !(sv->schur_ratio > 1.0)) return fail(LX_EINVAL, "schur_ratio must be > 1");
    } else {
        if (sv->f_degree < 0 || sv->f_degree > 16) return fail(LX_EINVAL, "f_degree must be 0..16");
        if (sv->amg_degree < 0 || sv->amg_degree > 8) return fail(LX_EINVAL, "amg_degree must be 0..8");
        if (sv->amg_cycle < 0 || sv->amg_cycle > 3) return fail(LX_EINVAL, "amg_cycle must be 0..3");
        if (sv->amg_coarse_cycle < 0 || sv->amg_coarse_cycle > 6)
            return fail(LX_EINVAL, "amg_coarse_cycle must be 0..6");
        if (sv->f_ratio != 0.0 && !(sv->f_ratio > 1.0)) return fail(LX_EINVAL, "f_ratio must be 0 or > 1");
        if (sv->amg_ratio != 0.0 && !(sv->amg_ratio > 1.0)) return fail(LX_EINVAL, "amg_ratio must be 0 or > 1");
    }

    prob = *pr;
    solver = *sv;
    if (solver.precond == LX_PC_AMG) {
        // the Jacobi-scaled P2 velocity block (mass-dominated) has a wider spectrum
        // than the P1 one, so its Chebyshev iteration gets more steps and a wider interval
        const bool q2 = pr->fe == LX_P2P1;
        if (solver.f_degree == 0) solver.f_degree = q2 ? 12 : 3;
        if (solver.amg_degree == 0) solver.amg_degree = 2;
        if (solver.f_ratio == 0.0) solver.f_ratio = q2 ? 300.0 : 5.0;
        if (solver.amg_ratio == 0.0) solver.amg_ratio = 30.0;
        if (solver.amg_cycle == 0) solver.amg_cycle = 2;
        if (solver.amg_coarse_cycle == 0) solver.amg_coarse_cycle = 3;
    }
    for (int i = 0; i < pr->n_bc; ++i) {
        BCDesc b;
        b.spec = pr->bc[i];
        if (b.spec.n_tags > 0 && !b.spec.tags) return fail(LX_EINVAL, "bc %d: tags NULL", i);
        b.tags.assign(b.spec.tags, b.spec.tags + b.spec.n_tags);
        b.spec.tags = nullptr;
        if (b.spec.type < 0 || b.spec.type > 3) return fail(LX_EINVAL, "bc %d: bad type", i);
        if (b.spec.resistance < 0 || b.spec.backflow < 0)
            return fail(LX_EINVAL, "bc %d: negative resistance or backflow coefficient", i);
        if (b.spec.backflow > 0 && b.spec.type != LX_BC_NEUMANN && b.spec.type != LX_BC_RESISTANCE)
            return fail(LX_EINVAL, "bc %d: backflow stabilisation applies to Neumann and resistance conditions", i);
        if (pr->fe == LX_P2P1 && (b.spec.type == LX_BC_RESISTANCE || b.spec.backflow > 0))
            return fail(LX_EINVAL, "bc %d: resistance and backflow terms are built for P1-P1", i);
        bcs.push_back(b);
    }
    prob.bc = nullptr;
    valves.assign(pr->riis, pr->riis + pr->n_riis);
    prob.riis = nullptr;
    if (pr->ale) {
        ale_tags.assign(pr->ale_tags, pr->ale_tags + pr->n_ale_tags);
        if (pr->lifting != LX_LIFT_HARMONIC && pr->lifting != LX_LIFT_ELASTIC)
            return fail(LX_EINVAL, "lifting must be LX_LIFT_HARMONIC or LX_LIFT_ELASTIC");
        if (pr->lifting == LX_LIFT_ELASTIC && !(pr->lift_E > 0 && pr->lift_nu >= 0 && pr->lift_nu < 0.5))
            return fail(LX_EINVAL, "elastic lifting needs lift_E > 0 and 0 <= lift_nu < 1/2");
        if (pr->stiffening < LX_STIFF_NONE || pr->stiffening > LX_STIFF_BOUNDARY)
            return fail(LX_EINVAL, "stiffening must be LX_STIFF_NONE, _JACOBIAN or _BOUNDARY");
        if (pr->stiffening != LX_STIFF_NONE && !(pr->stiff_p[0] > 0 && pr->stiff_p[1] > 0))
            return fail(LX_EINVAL, "stiffening parameters must be positive");
    }
    prob.ale_tags = nullptr;
    if (prob.C_r <= 0) prob.C_r = (prob.fe == LX_P2P1) ? 60.0 : 30.0;

    lx_status st = build_setup(mesh, hs);
    if (st != LX_OK) return st;
    nv = hs.nv;
    nt = hs.nt;
    nblk = (int64_t)hs.col.size();
    p2 = prob.fe == LX_P2P1;
    if (p2) {
        st = build_setup_p2(hs, p2h);
        if (st != LX_OK) return st;
        nu = p2h.nu;
    } else {
        nu = nv;
    }
    N = 4 * nu;

    // boundary sets in the new numbering: face vertices (P2-P1: then the face's
    // edge nodes (0,1) (1,2) (2,0))
    std::vector<int32_t> owner(nu, -1);
    bool edge_missing = false;
    auto face_vertices = [&](const std::vector<int32_t> &tags, std::vector<int32_t> &out_faces) {
        out_faces.clear();
        for (int64_t f = 0; f < mesh->n_bfaces; ++f) {
            int32_t tg = mesh->bface_tag[f];
            if (std::find(tags.begin(), tags.end(), tg) == tags.end()) continue;
            int32_t w[3];
            for (int k = 0; k < 3; ++k) {
                int32_t v = mesh->bfaces[3 * f + k];
                if (v < 0 || v >= nv) return false;
                w[k] = hs.iperm_v[v];
                out_faces.push_back(w[k]);
            }
            if (p2)
                for (int k = 0; k < 3; ++k) {
                    const int32_t m = p2_edge_node(p2h, nv, w[k], w[(k + 1) % 3]);
                    if (m < 0) edge_missing = true;
                    out_faces.push_back(m < 0 ? 0 : m);
                }
        }
        return true;
    };
    std::vector<int32_t> fv;
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < (int)bcs.size(); ++i) {
            int ty = bcs[i].spec.type;
            if ((pass == 0 && ty != LX_BC_NOSLIP) || (pass == 1 && ty != LX_BC_DIRICHLET)) continue;
            if (!face_vertices(bcs[i].tags, fv)) return fail(LX_EMESH, "boundary face vertex out of range");
            for (int32_t v : fv)
                if (owner[v] < 0) owner[v] = i;
        }
    h_dir_index.assign(nu, -1);
    for (int64_t v = 0; v < nu; ++v)
        if (owner[v] >= 0) {
            h_dir_index[v] = (int32_t)h_dir_node.size();
            h_dir_node.push_back((int32_t)v);
            h_dir_bc.push_back(owner[v]);
        }
    n_dir = (int64_t)h_dir_node.size();
    h_gnodal.assign(3 * std::max<int64_t>(n_dir, 1), 0.0);
    // faces of the Neumann conditions (P1-P1: of every condition, for the boundary integrals)
    for (int i = 0; i < (int)bcs.size(); ++i) {
        if (bcs[i].spec.type != LX_BC_NEUMANN && p2) continue;
        if (!face_vertices(bcs[i].tags, fv)) return fail(LX_EMESH, "boundary face vertex out of range");
        bcs[i].nf = (int64_t)fv.size() / (p2 ? 6 : 3);
        bcs[i].h_faces = fv;
    }
    if (edge_missing) return fail(LX_EMESH, "a boundary face is not a face of any tetrahedron");
    if (prob.ale) {
        if (!face_vertices(ale_tags, fv)) return fail(LX_EMESH, "boundary face vertex out of range");
        h_ale_faces = fv;
        std::vector<char> mark(nv, 0);
        for (int32_t v : fv) mark[v] = 1;
        for (int64_t v = 0; v < nv; ++v)
            if (mark[v]) h_ale_nodes.push_back((int32_t)v);
    }

    if (solver.precond == LX_PC_AMG) {
        lx_status sa = amg_build_host(hs, amgh);
        if (sa != LX_OK) return sa;
    }

    // ---- device side: everything above is host-only validation and setup
    device = dev ? dev->device : 0;
    if (dev && (!dev->alloc) != (!dev->free)) return fail(LX_EINVAL, "lx_device: set both alloc and free, or neither");
    if (dev && dev->alloc) {
        alloc_fn = dev->alloc;
        free_fn = dev->free;
        alloc_ctx = dev->ctx;
    }
    LX_HIP(hipSetDevice(device));
    st = noalloc_init(device);
    if (st != LX_OK) return st;
    if (dev && dev->hip_stream) {
        stream = (hipStream_t)dev->hip_stream;
        own_stream = false;
    } else {
        LX_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        own_stream = true;
    }

#define ALLOC(ptr, bytes)                                      \
    do {                                                       \
        lx_status _s = dalloc((void **)&(ptr), (bytes));       \
        if (_s != LX_OK) return _s;                            \
    } while (0)
    ALLOC(d_xh, sizeof(double) * 3 * nv);
    ALLOC(d_x, sizeof(double) * 3 * nv);
    ALLOC(d_tet, sizeof(int32_t) * 4 * nt);
    ALLOC(d_sinc_ptr, sizeof(int32_t) * (nblk + 1));
    ALLOC(d_sinc, sizeof(int32_t) * 16 * nt);
    if (!p2) {
        ALLOC(d_vinc_ptr, sizeof(int32_t) * (nv + 1));
        ALLOC(d_vpos, sizeof(int32_t) * 4 * nt);
    }
    if (p2) {
        const P2Setup &q = p2h;
        ALLOC(d_nodes, sizeof(int32_t) * 10 * nt);
        ALLOC(d_fptr, sizeof(int32_t) * (nu + 1));
        ALLOC(d_fcol, sizeof(int32_t) * q.fcol.size());
        ALLOC(d_fdiag, sizeof(int32_t) * nu);
        ALLOC(d_gptr, sizeof(int32_t) * (nu + 1));
        ALLOC(d_gcol, sizeof(int32_t) * q.gcol.size());
        ALLOC(d_bptr, sizeof(int32_t) * (nv + 1));
        ALLOC(d_bcol, sizeof(int32_t) * q.bcol.size());
        ALLOC(d_finc_ptr, sizeof(int32_t) * q.finc_ptr.size());
        ALLOC(d_finc, sizeof(int32_t) * q.finc.size());
        ALLOC(d_ginc_ptr, sizeof(int32_t) * q.ginc_ptr.size());
        ALLOC(d_ginc, sizeof(int32_t) * q.ginc.size());
        ALLOC(d_binc_ptr, sizeof(int32_t) * q.binc_ptr.size());
        ALLOC(d_binc, sizeof(int32_t) * q.binc.size());
        ALLOC(d_xnode, sizeof(double) * 3 * nu);
        ALLOC(d_rules, sizeof(P2Rules));
        ALLOC(d_rec2, sizeof(double) * (int64_t)kP2Rec * nt);
        s64.nv = s32.nv = nv;
        s64.nu = s32.nu = nu;
        s64.nt = s32.nt = nt;
        s64.nf = s32.nf = (int64_t)q.fcol.size();
        s64.ng = s32.ng = (int64_t)q.gcol.size();
        s64.nb = s32.nb = (int64_t)q.bcol.size();
        s64.nc = s32.nc = nblk;
    }
    ALLOC(d_rowptr, sizeof(int32_t) * (nv + 1));
    ALLOC(d_col, sizeof(int32_t) * nblk);
    ALLOC(d_diag, sizeof(int32_t) * nv);
    ALLOC(d_tslot, sizeof(int32_t) * nblk);
    ALLOC(d_dir_index, sizeof(int32_t) * nu);
    ALLOC(d_perm, sizeof(int32_t) * nv);
    if (n_dir > 0) {
        ALLOC(d_dir_node, sizeof(int32_t) * n_dir);
        ALLOC(d_dir_bc, sizeof(int32_t) * n_dir);
        ALLOC(d_g, sizeof(double) * 3 * n_dir);
        ALLOC(d_gnodal, sizeof(double) * 3 * n_dir);
        ALLOC(d_dg, sizeof(double) * 3 * n_dir);
    }
    const int L = prob.bdf_order;
    // more levels than BDF2 needs: the initial guess extrapolates up to four solutions
    for (int l = 0; l < std::max(L, 4); ++l) ALLOC(d_hist[l], sizeof(double) * N);
    ALLOC(d_xs, sizeof(double) * N);
    if (prob.forcing) ALLOC(d_f, sizeof(double) * 3 * nu);
    if (prob.ale) {
        ALLOC(d_uA, sizeof(double) * 3 * nv);
        for (int l = 0; l < L; ++l) ALLOC(d_dhist[l], sizeof(double) * 3 * nv);
        ALLOC(d_ale_shape, sizeof(double) * 3 * nv);
        lx_status s2 = ale_setup();
        if (s2 != LX_OK) return s2;
    }
    for (auto &b : bcs)
        if ((b.spec.type == LX_BC_NEUMANN || !p2) && b.nf > 0) {
            ALLOC(b.d_faces, sizeof(int32_t) * b.h_faces.size());
            if (b.spec.profile.kind == LX_PROFILE_NODAL) ALLOC(b.d_hnodal, sizeof(double) * 3 * nu);
        }
    const int m = solver.restart;
    nb_red = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (N + 2047) / 2048));
    ALLOC(d_st, sizeof(GmState));
    ALLOC(d_partial, sizeof(double) * std::max<int64_t>((int64_t)nb_red * 64, gm_partial_size(N)));
    LX_HIP(hipHostMalloc((void **)&h_st, sizeof(GmState), hipHostMallocDefault));
    LX_HIP(hipHostMalloc((void **)&h_chk, 2 * sizeof(GmState), hipHostMallocDefault));
    LX_HIP(hipHostMalloc((void **)&h_gerr, 4 * sizeof(double), hipHostMallocDefault));
    ALLOC(d_gerr, sizeof(double) * (kGuessErrPartial + 4));
    for (auto &ev : ev_chk) LX_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    {
        const char *ge = getenv("LXNS_GRAPH");
        use_graphs = !(ge && *ge == '0');
        const char *lp = getenv("LXNS_LIFT_PROJ");
        lift_proj = !(lp && *lp == '0');
        if (use_graphs) {
            LX_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
            g_step.assign(6 * kMaxRestart, nullptr);
            gx_step.assign(6 * kMaxRestart, nullptr);
        }
    }
    if (p2) {
        // FP64 split system in both precisions (the refinement residual uses it)
        ALLOC(s64.F, sizeof(double) * 9 * s64.nf);
        ALLOC(s64.G, sizeof(double) * 3 * s64.ng);
        ALLOC(s64.B, sizeof(double) * 3 * s64.nb);
        ALLOC(s64.C, sizeof(double) * s64.nc);
        s64.fptr = s32.fptr = d_fptr;
        s64.fcol = s32.fcol = d_fcol;
        s64.gptr = s32.gptr = d_gptr;
        s64.gcol = s32.gcol = d_gcol;
        s64.bptr = s32.bptr = d_bptr;
        s64.bcol = s32.bcol = d_bcol;
        s64.cptr = s32.cptr = d_rowptr;
        s64.ccol = s32.ccol = d_col;
        ALLOC(d_rhs64, sizeof(double) * N);
        if (solver.precision != LX_FP64) {
            ALLOC(s32.F, sizeof(float) * 9 * s32.nf);
            ALLOC(s32.G, sizeof(float) * 3 * s32.ng);
            ALLOC(s32.B, sizeof(float) * 3 * s32.nb);
            ALLOC(s32.C, sizeof(float) * s32.nc);
        }
    } else if (solver.precision == LX_FP64 || solver.asm_fp64) {
        ALLOC(d_rec64, sizeof(double) * kRec * nt);
    } else {
        ALLOC(d_rec32, sizeof(float) * kRec * nt);
    }
    if (!prob.semi_implicit) {
        ALLOC(d_nrec, sizeof(double) * kNewtonRec * nt);
        ALLOC(d_dx, sizeof(double) * N);
        ALLOC(d_gdelta, sizeof(double) * 3 * std::max<int64_t>(n_dir, 1));
        if (solver.precision != LX_FP64) {
            // FP32 updates: the Newton system is still formed in FP64, then rounded
            ALLOC(d_val64, sizeof(double) * kPlanes * nblk);
            ALLOC(d_rhs64, sizeof(double) * N);
        }
    }
    if (solver.precision == LX_FP64) {
        if (!p2) ALLOC(d_val64, sizeof(double) * kPlanes * nblk);
        if (!d_rhs64) ALLOC(d_rhs64, sizeof(double) * N);
        ALLOC(d_Finv64, sizeof(double) * 9 * nu);
        ALLOC(d_Dinv64, sizeof(double) * 3 * nu);
        ALLOC(d_Sinv64, sizeof(double) * nv);
        ALLOC(d_V64, sizeof(double) * N * (m + 1));
        ALLOC(d_Z64, sizeof(double) * N * m);
        ALLOC(d_sw64, sizeof(double) * 9 * nv);
        ALLOC(d_w64, sizeof(double) * N);
    } else {
        if (!p2) ALLOC(d_val32, sizeof(float) * kPlanes * nblk);
        ALLOC(d_Finv32, sizeof(float) * 9 * nu);
        ALLOC(d_Dinv32, sizeof(float) * 3 * nu);
        ALLOC(d_Sinv32, sizeof(float) * nv);
        ALLOC(d_V32, sizeof(float) * N * (m + 1));
        if (solver.asm_fp64 && !p2 && !d_val64) ALLOC(d_val64, sizeof(double) * kPlanes * nblk);
        ALLOC(d_Z32, sizeof(float) * N * m);
        ALLOC(d_sw32, sizeof(float) * 9 * nv);
        ALLOC(d_w32, sizeof(float) * N);
        ALLOC(d_x32, sizeof(float) * N);
        ALLOC(d_r32, sizeof(float) * N);
        ALLOC(d_r64, sizeof(double) * N);
        ALLOC(d_b64, sizeof(double) * N);
        if (!p2) ALLOC(d_rrec, sizeof(double) * kRRec * nt);
    }
#undef ALLOC
    if (solver.precond == LX_PC_AMG) {
        lx_status sa = solver.precision == LX_FP64 ? setup_amg<double>(amg64) : setup_amg<float>(amg32);
        if (sa != LX_OK) return sa;
        amgh = AmgHost();
    }
    // ---- uploads
    LX_HIP(hipMemcpyAsync(d_xh, hs.xh.data(), sizeof(double) * 3 * nv, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_x, hs.xh.data(), sizeof(double) * 3 * nv, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_tet, hs.tet_soa.data(), sizeof(int32_t) * 4 * nt, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_sinc_ptr, hs.sinc_ptr.data(), sizeof(int32_t) * (nblk + 1), hipMemcpyHostToDevice,
                          stream));
    LX_HIP(hipMemcpyAsync(d_sinc, hs.sinc.data(), sizeof(int32_t) * 16 * nt, hipMemcpyHostToDevice, stream));
    if (!p2) {
        LX_HIP(hipMemcpyAsync(d_vinc_ptr, hs.vinc_ptr.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice,
                              stream));
        LX_HIP(hipMemcpyAsync(d_vpos, hs.vpos.data(), sizeof(int32_t) * 4 * nt, hipMemcpyHostToDevice, stream));
    }
    LX_HIP(hipMemcpyAsync(d_rowptr, hs.rowptr.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_col, hs.col.data(), sizeof(int32_t) * nblk, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_diag, hs.diag.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_tslot, hs.tslot.data(), sizeof(int32_t) * nblk, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_dir_index, h_dir_index.data(), sizeof(int32_t) * nu, hipMemcpyHostToDevice, stream));
    LX_HIP(hipMemcpyAsync(d_perm, hs.perm_v.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice, stream));
    if (p2) {
        const P2Setup &q = p2h;
        auto up = [&](int32_t *d, const std::vector<int32_t> &h) {
            return hipMemcpyAsync(d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, stream);
        };
        LX_HIP(up(d_nodes, q.nodes));
        LX_HIP(up(d_fptr, q.fptr));
        LX_HIP(up(d_fcol, q.fcol));
        LX_HIP(up(d_fdiag, q.fdiag));
        LX_HIP(up(d_gptr, q.gptr));
        LX_HIP(up(d_gcol, q.gcol));
        LX_HIP(up(d_bptr, q.bptr));
        LX_HIP(up(d_bcol, q.bcol));
        LX_HIP(up(d_finc_ptr, q.finc_ptr));
        LX_HIP(up(d_finc, q.finc));
        LX_HIP(up(d_ginc_ptr, q.ginc_ptr));
        LX_HIP(up(d_ginc, q.ginc));
        LX_HIP(up(d_binc_ptr, q.binc_ptr));
        LX_HIP(up(d_binc, q.binc));
        LX_HIP(hipMemcpyAsync(d_xnode, q.xnode.data(), sizeof(double) * 3 * nu, hipMemcpyHostToDevice, stream));
        P2Rules rules;
        p2_rules(rules);
        LX_HIP(hipMemcpyAsync(d_rules, &rules, sizeof(P2Rules), hipMemcpyHostToDevice, stream));
        LX_HIP(hipStreamSynchronize(stream));   // rules is a stack object
    }
    if (n_dir > 0) {
        LX_HIP(hipMemcpyAsync(d_dir_node, h_dir_node.data(), sizeof(int32_t) * n_dir, hipMemcpyHostToDevice, stream));
        LX_HIP(hipMemcpyAsync(d_dir_bc, h_dir_bc.data(), sizeof(int32_t) * n_dir, hipMemcpyHostToDevice, stream));
        launch_fill<double>(3 * n_dir, d_gnodal, 0.0, stream);
    }
    for (auto &b : bcs)
        if (b.d_faces)
            LX_HIP(hipMemcpyAsync(b.d_faces, b.h_faces.data(), sizeof(int32_t) * b.h_faces.size(),
                                  hipMemcpyHostToDevice, stream));
    if (!p2) {
        lx_status so = outflow_setup();
        if (so != LX_OK) return so;
    }
    for (int l = 0; l < std::max(L, 4); ++l) launch_fill<double>(N, d_hist[l], 0.0, stream);
    launch_fill<double>(N, d_xs, 0.0, stream);
    if (d_f) launch_fill<double>(3 * nu, d_f, 0.0, stream);
    if (prob.ale) {
        launch_fill<double>(3 * nv, d_uA, 0.0, stream);
        for (int l = 0; l < L; ++l) launch_fill<double>(3 * nv, d_dhist[l], 0.0, stream);
        launch_fill<double>(3 * nv, d_dnew, 0.0, stream);
        launch_fill<double>(3 * nv, d_ale_shape, 0.0, stream);
    }
    for (auto &b : bcs)
        if (b.d_hnodal) launch_fill<double>(3 * nu, b.d_hnodal, 0.0, stream);
    LX_HIP(hipMemsetAsync(d_st, 0, sizeof(GmState), stream));
    {
        const char *e = getenv("LXNS_REORTH_FRAC");
        const double frac = e ? atof(e) : 0.9;   // second Gram-Schmidt pass below ||w|| / sqrt(10)
        LX_HIP(hipMemcpyAsync(&d_st->reorth_frac, &frac, sizeof(double), hipMemcpyHostToDevice, stream));
        LX_HIP(hipStreamSynchronize(stream));
    }
    LX_HIP(hipEventCreate(&ev_step0));
    LX_HIP(hipEventCreate(&ev_step1));
    LX_HIP(hipEventCreate(&ev_asm1));
    {
        static const bool overlap = [] {
            const char *e = getenv("LXNS_OVERLAP");
            return !(e && strcmp(e, "0") == 0);
        }();
        // (the implicit formulation forms its systems in the Newton loop: nothing to overlap)
        if (overlap && prob.semi_implicit && !p2 && solver.precision != LX_FP64 && !solver.asm_fp64 &&
            nt >= (1 << 19)) {
            LX_HIP(hipStreamCreateWithFlags(&stream_aux, hipStreamNonBlocking));
            LX_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
            LX_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
            const lx_status as = dalloc((void **)&d_partial_aux, sizeof(double) * gm_partial_size(N));
            if (as != LX_OK) return as;
            LX_HIP(hipHostMalloc((void **)&h_norms0, 2 * sizeof(double), hipHostMallocDefault));
        }
    }
    LX_HIP(hipStreamSynchronize(stream));
    LX_HIP(hipGetLastError());
    t = prob.t0;
    nlev = 0;
    return LX_OK;
}

RowPattern Sim::pattern() const
{
    RowPattern P;
    P.nv = nv;
    P.nblk = nblk;
    P.rowptr = d_rowptr;
    P.col = d_col;
    P.diag = d_diag;
    P.tslot = d_tslot;
    return P;
}

// Device arrays of the Schur-block hierarchy (patterns uploaded once; values
// are refreshed every step by launch_amg_setup).
template <typename T>
lx_status Sim::setup_amg(Amg<T> &A)
{
    const int nl = (int)amgh.lev.size();
    A.nlev = nl - 1;
    A.degree = solver.amg_degree;
    A.ratio = solver.amg_ratio;
    A.f_degree = solver.f_degree;
    A.f_ratio = solver.f_ratio;
    A.f_warm = false;
    A.cycle = solver.amg_cycle;
    A.cycle_coarse = solver.amg_coarse_cycle;
    const char *env = getenv("LXNS_AMG_LPR");
    const int lpr_env = env ? atoi(env) : 0;
    // the power iterations on F run with block_lpr lanes per row (up to kMaxRowLanes) and
    // write one partial sum per workgroup into A.partial
    int64_t maxgrid = (nu * kMaxRowLanes + 255) / 256;
    auto up = [&](int32_t *&d, const std::vector<int32_t> &h) -> lx_status {
        lx_status s = dalloc((void **)&d, sizeof(int32_t) * std::max<size_t>(h.size(), 1));
        if (s != LX_OK) return s;
        if (!h.empty()) LX_HIP(hipMemcpyAsync(d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, stream));
        return LX_OK;
    };
    auto vec = [&](T *&d, int64_t n) { return dalloc((void **)&d, sizeof(T) * std::max<int64_t>(n, 1)); };
#define CK(x)                          \
    do {                               \
        lx_status _s = (x);            \
        if (_s != LX_OK) return _s;    \
    } while (0)
    // one-workgroup coarse cycle: the suffix of the hierarchy that fits one
    // workgroup's LDS (LXNS_AMG_TAIL=0 keeps every level on its own launches)
    {
        int64_t ln[kAmgMaxLevels + 1], lnnz[kAmgMaxLevels + 1];
        for (int l = 0; l < nl; ++l) {
            ln[l] = amgh.lev[l].n;
            lnnz[l] = (int64_t)amgh.lev[l].col.size();
        }
        int max_lds = 0;
        LX_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
        const char *te = getenv("LXNS_AMG_TAIL");
        const bool use_tail = !(te && *te == '0');
        // the levels that fit take cycle_coarse coarse corrections, whichever kernels cycle them
        const TailLayout fit = amg_tail_layout(A.nlev, ln, lnnz, (int)sizeof(T), max_lds);
        A.coarse_from = fit.first > 0 ? fit.first : A.nlev + 1;
        A.tail = use_tail ? fit : TailLayout();
        // a device that refuses the LDS reservation runs every level on its own launches
        if (A.tail.first > 0 && amg_tail_prepare<T>(A.tail.lds_bytes) != LX_OK) A.tail = TailLayout();
        if (A.tail.first > 0) {
            CK(dalloc((void **)&A.tail_img, (size_t)A.tail.img_bytes));
            LX_HIP(hipMemsetAsync(A.tail_img, 0, (size_t)A.tail.img_bytes, stream));
            // the tabulated operator of that cycle (LXNS_TAIL_OP=0: cycle at every visit)
            const char *to = getenv("LXNS_TAIL_OP");
            if (!(to && *to == '0')) {
                const int64_t n = A.tail.lv[0].n;
                CK(dalloc((void **)&A.tail_op, sizeof(T) * (size_t)(n * n)));
                CK(dalloc((void **)&A.tail_rc, sizeof(T) * (size_t)n));
            }
        }
    }
    auto in_img = [&](int l) { return A.tail.first > 0 && l >= A.tail.first && l < A.nlev; };
    // the finest smoothed level in sliced-ELL order (LXNS_AMG_SELL=0: plain CSR)
    const char *se = getenv("LXNS_AMG_SELL");
    const bool sell0 = A.nlev > 0 && !(se && *se == '0');
    std::vector<int32_t> soff0;
    auto img_up = [&](int32_t *&d, int32_t off, const std::vector<int32_t> &h) -> lx_status {
        d = reinterpret_cast<int32_t *>(A.tail_img + off);
        if (!h.empty()) LX_HIP(hipMemcpyAsync(d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, stream));
        return LX_OK;
    };
    for (int l = 0; l < nl; ++l) {
        const AmgLevelHost &H = amgh.lev[l];
        AmgLevel<T> &L = A.L[l];
        L.n = H.n;
        L.nnz = (int64_t)H.col.size();
        const double avg = (double)L.nnz / (double)std::max<int64_t>(L.n, 1);
        L.lpr = avg >= 12 ? 16 : avg >= 6 ? 8 : 4;
        if (lpr_env == 4 || lpr_env == 8 || lpr_env == 16 || lpr_env == 32) L.lpr = lpr_env;
        maxgrid = std::max<int64_t>(maxgrid, (L.n * L.lpr + 255) / 256);
        const bool img = in_img(l);
        const TailLevelLds *Y = img ? &A.tail.lv[l - A.tail.first] : nullptr;
        if (img) {
            CK(img_up(L.rowptr, Y->o_rowptr, H.rowptr));
            CK(img_up(L.col, Y->o_col, H.col));
            L.val = reinterpret_cast<T *>(A.tail_img + Y->o_val);
        } else {
            CK(up(L.rowptr, H.rowptr));
            CK(up(L.col, H.col));
            if (l == 0 && sell0) {
                // the finest level in sliced-ELL order (padding: zero values, own column)
                const int64_t n = H.n, ns = (n + 63) / 64;
                soff0.assign(ns + 1, 0);
                std::vector<int32_t> swid(ns, 0);
                for (int64_t s = 0; s < ns; ++s) {
                    int32_t w = 0;
                    for (int64_t i = 64 * s; i < std::min<int64_t>(n, 64 * s + 64); ++i)
                        w = std::max(w, H.rowptr[i + 1] - H.rowptr[i]);
                    swid[s] = w;
                    soff0[s + 1] = soff0[s] + 64 * w;
                }
                L.nsell = soff0[ns];
                std::vector<int32_t> scol(L.nsell);
                bool d16 = true;
                for (int64_t i = 0; i < n; ++i) {
                    const int64_t base = soff0[i >> 6] + (i & 63);
                    const int32_t len = H.rowptr[i + 1] - H.rowptr[i];
                    for (int32_t j = 0; j < swid[i >> 6]; ++j) {
                        const int32_t c = j < len ? H.col[H.rowptr[i] + j] : (int32_t)i;
                        scol[base + 64 * (int64_t)j] = c;
                        d16 = d16 && c - i >= -32768 && c - i <= 32767;
                    }
                }
                // lanes of the last slice past row n - 1 hold padding and are never read
                CK(up(L.soff, soff0));
                CK(up(L.swid, swid));
                if (d16) {
                    // every column within 32767 of its row: 16-bit offsets
                    std::vector<int16_t> sdel(L.nsell, 0);
                    for (int64_t i = 0; i < n; ++i) {
                        const int64_t base = soff0[i >> 6] + (i & 63);
                        for (int32_t j = 0; j < swid[i >> 6]; ++j)
                            sdel[base + 64 * (int64_t)j] = (int16_t)(scol[base + 64 * (int64_t)j] - i);
                    }
                    CK(dalloc((void **)&L.sdel, sizeof(int16_t) * sdel.size()));
                    LX_HIP(hipMemcpyAsync(L.sdel, sdel.data(), sizeof(int16_t) * sdel.size(), hipMemcpyHostToDevice,
                                          stream));
                } else {
                    CK(up(L.scol, scol));
                }
                LX_HIP(hipStreamSynchronize(stream));   // swid, scol and sdel are local vectors
                CK(vec(L.val, L.nsell));
                LX_HIP(hipMemsetAsync(L.val, 0, sizeof(T) * L.nsell, stream));
            } else {
                CK(vec(L.val, L.nnz));
            }
        }
        CK(up(L.diag, H.diag));
        CK(vec(L.x1, L.n));
        if (l < A.nlev) {
            if (img) {
                CK(img_up(L.agg, Y->o_agg, H.agg));
                CK(img_up(L.mptr, Y->o_mptr, H.mptr));
                CK(img_up(L.mem, Y->o_mem, H.mem));
                L.dinv = reinterpret_cast<T *>(A.tail_img + Y->o_dinv);
            } else {
                CK(up(L.agg, H.agg));
                CK(up(L.mptr, H.mptr));
                CK(up(L.mem, H.mem));
                CK(vec(L.dinv, L.n));
            }
            CK(up(L.cptr, H.cptr));
            if (l == 0 && sell0) {
                // coarse entries sum the finest level's entries at their sliced-ELL positions
                std::vector<int32_t> row_of(H.col.size());
                for (int64_t i = 0; i < H.n; ++i)
                    for (int32_t k = H.rowptr[i]; k < H.rowptr[i + 1]; ++k) row_of[k] = (int32_t)i;
                std::vector<int32_t> cidx(H.cidx.size());
                for (size_t q = 0; q < H.cidx.size(); ++q)
                    cidx[q] = (int32_t)sell_pos(soff0, H.rowptr, row_of[H.cidx[q]], H.cidx[q]);
                CK(up(L.cidx, cidx));
            } else {
                CK(up(L.cidx, H.cidx));
            }
            CK(vec(L.x0, L.n));
            CK(vec(L.res, L.n));
            CK(vec(L.d0, L.n));
            CK(vec(L.d1, L.n));
        }
        if (l < A.nlev || l == 0) CK(vec(L.r, L.n));
    }
    const AmgLevelHost &Hc = amgh.lev.back();
    A.nc = Hc.n;
    std::vector<int32_t> crow(Hc.col.size());
    for (int64_t i = 0; i < Hc.n; ++i)
        for (int32_t k = Hc.rowptr[i]; k < Hc.rowptr[i + 1]; ++k) crow[k] = (int32_t)i;
    CK(up(A.crow, crow));
    if (A.tail.first > 0) {
        A.dense = reinterpret_cast<double *>(A.tail_img + A.tail.o_dense);
        if (A.tail.o_fmem >= 0) {
            const AmgLevelHost &Hf = amgh.lev[A.tail.first - 1];
            int32_t *dm = nullptr;
            CK(img_up(dm, A.tail.o_fmptr, Hf.mptr));
            CK(img_up(dm, A.tail.o_fmem, Hf.mem));
        }
    } else {
        CK(dalloc((void **)&A.dense, sizeof(double) * 2 * A.nc * std::max<int64_t>(A.nc, 1)));
    }
    CK(dalloc((void **)&A.lam, sizeof(double) * kLamSlots));
    CK(dalloc((void **)&A.partial, sizeof(double) * (maxgrid + 64)));
    CK(dalloc((void **)&A.counter, sizeof(uint32_t) * 4));
    CK(vec(A.fr, 4 * nu));
    CK(vec(A.fd0, 4 * nu));
    CK(vec(A.fd1, 4 * nu));
    CK(vec(A.fv, 4 * nu));
#undef CK
    if (const char *v = getenv("LXNS_VERBOSE"))
        if (*v && *v != '0') {
            if (A.tail.first > 0)
                fprintf(stderr, "[lxns] AMG one-workgroup cycle from level %d: %d image bytes, %d LDS bytes\n",
                        A.tail.first, A.tail.img_bytes, A.tail.lds_bytes);
            for (int l = 0; l < nl; ++l)
                fprintf(stderr, "[lxns] AMG level %d%s: %lld rows, %lld entries, lanes/row %d%s\n", l,
                        l == A.nlev ? " (dense)" : "", (long long)A.L[l].n, (long long)A.L[l].nnz, A.L[l].lpr,
                        A.tail.first > 0 && l >= A.tail.first ? " (one-workgroup cycle)" : "");
        }
    LX_HIP(hipMemsetAsync(A.lam, 0, sizeof(double) * kLamSlots, stream));
    LX_HIP(hipMemsetAsync(A.counter, 0, sizeof(uint32_t) * 4, stream));
    launch_fill<T>(4 * nu, A.fr, T(0), stream);
    launch_fill<T>(4 * nu, A.fd0, T(0), stream);
    launch_fill<T>(4 * nu, A.fd1, T(0), stream);
    launch_fill<T>(4 * nu, A.fv, T(0), stream);
    return LX_OK;
}

// ------------------------------------------------------------------ timing

// A pair of events for one timed launch.  record = true: bracket the launch with
// hipEventRecord (timer_end closes it); record = false: the caller hands the pair
// to hipExtLaunchKernelGGL, which stamps the kernel's own start and end.
std::pair<hipEvent_t, hipEvent_t> *Sim::timer_begin(int kind, int iter, bool record)
{
    if (solver.collect_timing <= 0) return nullptr;
    if (kind == 0 && (spmv_seq++ % solver.collect_timing) != 0) return nullptr;
    if (ev_used >= ev_pool.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return nullptr;
        if (hipEventCreate(&b) != hipSuccess) return nullptr;
        ev_pool.push_back({a, b});
        ev_tag.push_back({0, 0});
    }
    auto *p = &ev_pool[ev_used];
    ev_tag[ev_used] = {kind, iter};
    ++ev_used;
    if (record) (void)hipEventRecord(p->first, stream);
    return p;
}

void Sim::timer_end(std::pair<hipEvent_t, hipEvent_t> *p)
{
    if (p) (void)hipEventRecord(p->second, stream);
}

// Accumulate recorded kernel times; in-cycle SpMVs with iteration index >= kused
// were skipped by the device-side exit and are not counted.
void Sim::timer_flush(int kused, lx_step_stats &acc)
{
    for (size_t i = 0; i < ev_used; ++i) {
        const int kind = ev_tag[i].first, it = ev_tag[i].second;
        // products of a cycle's steps from kused on exited on the done flag; their events are
        // not queried (a cycle that a check stopped is flushed before they need have run)
        if (kind == 0 && it >= 0 && it >= kused) continue;
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev_pool[i].first, ev_pool[i].second) != hipSuccess) continue;
        if (kind == 0) {
            acc.spmv_ms += ms;
            acc.spmv_calls += 1;
        } else if (kind == 1) {
            acc.asm_ms += ms;
            acc.asm_calls += 1;
        } else if (kind == 2) {
            acc.resid_ms += ms;
            acc.resid_calls += 1;
        }
    }
    ev_used = 0;
}

// ------------------------------------------------------------------ GMRES

template <typename T>
struct Ops;
template <>
struct Ops<double> {
    static double *val(Sim *s) { return s->d_val64; }
    static double *Finv(Sim *s) { return s->d_Finv64; }
    static double *Dinv(Sim *s) { return s->d_Dinv64; }
    static double *Sinv(Sim *s) { return s->d_Sinv64; }
    static double *V(Sim *s) { return s->d_V64; }
    static double *w(Sim *s) { return s->d_w64; }
    static double *sw(Sim *s) { return s->d_sw64; }
    static double *Z(Sim *s) { return s->d_Z64; }
    static Amg<double> &amg(Sim *s) { return s->amg64; }
    static P2Sys<double> &sys(Sim *s) { return s->s64; }
};
template <>
struct Ops<float> {
    static float *val(Sim *s) { return s->d_val32; }
    static float *Finv(Sim *s) { return s->d_Finv32; }
    static float *Dinv(Sim *s) { return s->d_Dinv32; }
    static float *Sinv(Sim *s) { return s->d_Sinv32; }
    static float *V(Sim *s) { return s->d_V32; }
    static float *w(Sim *s) { return s->d_w32; }
    static float *sw(Sim *s) { return s->d_sw32; }
    static float *Z(Sim *s) { return s->d_Z32; }
    static Amg<float> &amg(Sim *s) { return s->amg32; }
    static P2Sys<float> &sys(Sim *s) { return s->s32; }
};

// The preconditioner's view of the system in precision T.
template <typename T>
SimpleView<T> Sim::view()
{
    if (!p2) return simple_view_p1<T>(pattern(), Ops<T>::val(this));
    const P2Sys<T> &S = Ops<T>::sys(this);
    SimpleView<T> V;
    V.nu = nu;
    V.np = nv;
    V.Fp.nv = nu;
    V.Fp.nblk = S.nf;
    V.Fp.rowptr = S.fptr;
    V.Fp.col = S.fcol;
    V.Fp.diag = d_fdiag;
    V.Fp.tslot = nullptr;
    V.Fp.remap = 0;   // vertex rows (many more entries) come first
    V.F = S.F;
    V.gptr = S.gptr;
    V.gcol = S.gcol;
    V.Gv = S.G;
    V.gs = S.ng;
    V.bptr = S.bptr;
    V.bcol = S.bcol;
    V.Bv = S.B;
    V.bs = S.nb;
    V.cptr = S.cptr;
    V.ccol = S.ccol;
    V.Cv = S.C;
    return V;
}

// y = A x in precision T (tm: events that time the launch, or null)
template <typename T>
void Sim::spmv(const T *x, T *y, const int32_t *done, std::pair<hipEvent_t, hipEvent_t> *tm, hipStream_t s)
{
    if (!s) s = stream;
    if (p2)
        launch_spmv_p2<T>(Ops<T>::sys(this), x, y, done, s, tm ? tm->first : nullptr, tm ? tm->second : nullptr);
    else
        launch_spmv<T>(pattern(), Ops<T>::val(this), x, y, done, s, tm ? tm->first : nullptr,
                       tm ? tm->second : nullptr);
    for (const OutflowDev &o : outflow) launch_rank1<T>(o, x, y, done, s);
}

// the scalar part of the GMRES state (everything from tol_abs on), which the host reads
static const size_t kStOff = offsetof(GmState, tol_abs);

lx_status Sim::read_state()
{
    LX_HIP(hipMemcpyAsync((char *)h_st + kStOff, (char *)d_st + kStOff, sizeof(GmState) - kStOff,
                          hipMemcpyDeviceToHost, stream));
    LX_HIP(hipStreamSynchronize(stream));
    return LX_OK;
}

static bool verbose()
{
    static const bool v = [] {
        const char *e = getenv("LXNS_VERBOSE");
        return e && *e && *e != '0';
    }();
    return v;
}

// Flexible (right-preconditioned) restarted GMRES(m) with CGS2 orthogonalisation:
// the preconditioned directions Z_j = M^{-1} v_j are kept and x += Z y at the end
// of a cycle, so the update uses exactly the vectors of the Arnoldi process.
// b and x
// are device vectors of length N; x holds the initial guess (x_zero: it is 0).
// An inner solve (of iterative refinement) stops as soon as the Givens
// residual estimate meets rtol inside a cycle; the outer FP64 residual judges
// the correction, so the true residual is not re-verified in low precision.
template <typename T>
lx_status Sim::gmres(const T *b, T *x, bool x_zero, double rtol, int max_iters, GmResult &res,
                     lx_step_stats &tstats, bool inner, int kind)
{
    const RowPattern P = pattern();
    const T *val = Ops<T>::val(this);
    T *V = Ops<T>::V(this), *w = Ops<T>::w(this), *Z = Ops<T>::Z(this);
    const Simple<T> SP{val, Ops<T>::Finv(this), Ops<T>::Dinv(this), Ops<T>::Sinv(this), solver.schur_degree,
                       solver.schur_ratio, Ops<T>::sw(this), d_st};
    const int m = solver.restart;
    const int64_t ld = N;
    launch_norm<T>(N, b, d_st, rtol, d_partial, 0, stream);
    if (x_zero) launch_fill<T>(N, x, T(0), stream);
    int it = 0;
    res = GmResult();
    for (int cycle = 0;; ++cycle) {
        if (x_zero && cycle == 0) {
            launch_gm_start<T>(N, b, nullptr, V, d_st, d_partial, stream);
        } else {
            auto *tm = timer_begin(0, -1, false);
            spmv<T>(x, w, nullptr, tm);
            launch_gm_start<T>(N, b, w, V, d_st, d_partial, stream);
        }
        const int kmax = std::min(m, max_iters - it);
        // The host learns of convergence from the done flag, copied to pinned
        // memory behind an event after chosen Arnoldi steps and read one step
        // later, while the next step is already queued: the device never waits
        // for the host, and a converged cycle leaves one step of early-exit
        // launches behind.  Steps are checked from two before the column count
        // of the same cycle in the last solve of this kind, every step if that
        // is unknown, and every eighth step in any case.
        const int kp = (kind >= 0 && kind < 8 && cycle < 8) ? k_hint[kind][cycle] : 0;
        int pending = -1, snap = -1;
        for (int k = 0; k < kmax; ++k) {
            T *zk = Z + k * ld;
            const bool amg = solver.precond == LX_PC_AMG;
            // Arnoldi step k: z_k = M^{-1} v_k, w = A z_k, Gram-Schmidt (from the second
            // step on, the pass that formed v_k already started the velocity block on it)
            // The Arnoldi step in two parts around the product: the preconditioner
            // apply, and the Gram-Schmidt pass (with the next step's head start)
            auto pre = [&](hipStream_t s) {
                if (amg)
                    launch_simple_amg_apply<T>(view<T>(), SP.Finv, SP.Dinv, Ops<T>::amg(this), V + k * ld,
                                               &d_st->s[k], zk, &d_st->done, s, k > 0);
                else
                    launch_simple_apply<T>(P, SP, V + k * ld, &d_st->s[k], zk, &d_st->done, s);
            };
            auto post = [&](hipStream_t s) {
                FzStart<T> fz;
                if (amg) fz = amg_fz_start(Ops<T>::amg(this), SP.Finv, Z + (k + 1) * ld);
                launch_gm_orth<T>(N, k, V, ld, w, d_st, d_partial, s, amg && k + 1 < kmax ? &fz : nullptr);
            };
            auto replay = [&](int slot, auto &&part) {
                if (!gx_step[slot]) {
                    LX_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
                    part(cap_stream);
                    LX_HIP(hipStreamEndCapture(cap_stream, &g_step[slot]));
                    LX_HIP(hipGraphInstantiate(&gx_step[slot], g_step[slot], nullptr, nullptr, 0));
                }
                LX_HIP(hipGraphLaunch(gx_step[slot], stream));
                return LX_OK;
            };
            if (use_graphs) {
                const int key = 2 * k + (k + 1 < kmax ? 0 : 1);
                // a timed step replays its two parts as graphs of their own around
                // the product, launched directly so that its events stamp the kernel
                auto *tm = timer_begin(0, k, false);
                if (tm) {
                    if (lx_status e = replay(2 * kMaxRestart + k, pre); e != LX_OK) return e;
                    spmv<T>(zk, w, &d_st->done, tm, stream);
                    if (lx_status e = replay(4 * kMaxRestart + key, post); e != LX_OK) return e;
                } else {
                    auto whole = [&](hipStream_t s) {
                        pre(s);
                        spmv<T>(zk, w, &d_st->done, nullptr, s);
                        post(s);
                    };
                    if (lx_status e = replay(key, whole); e != LX_OK) return e;
                }
            } else {
                pre(stream);
                spmv<T>(zk, w, &d_st->done, timer_begin(0, k, false), stream);
                post(stream);
            }
            if (pending >= 0) {
                LX_HIP(hipEventSynchronize(ev_chk[pending & 1]));
                const bool stop = h_chk[pending & 1].done != 0;
                if (stop) {
                    snap = pending;
                    break;
                }
                pending = -1;
            }
            const bool check = kp > 0 ? (k + 2 >= kp || (k + 1) % 8 == 0) : true;
            if (check && k + 1 < kmax) {
                LX_HIP(hipMemcpyAsync((char *)&h_chk[k & 1] + kStOff, (char *)d_st + kStOff, sizeof(GmState) - kStOff,
                                      hipMemcpyDeviceToHost, stream));
                LX_HIP(hipEventRecord(ev_chk[k & 1], stream));
                pending = k;
            }
        }
        LX_HIP(hipGetLastError());
        // A cycle stopped by a check already holds the state as that step left it: the step
        // queued after it exits on the done flag and writes nothing, so the host takes that
        // copy and queues the cycle's update without waiting for the device (the stamps of
        // that step's product, if any, are not read: its column is at or past kused).
        if (snap >= 0) {
            memcpy((char *)h_st + kStOff, (char *)&h_chk[snap & 1] + kStOff, sizeof(GmState) - kStOff);
        } else {
            lx_status s = read_state();
            if (s != LX_OK) return s;
        }
        lx_status s = LX_OK;
        timer_flush(h_st->kused, tstats);
        if (kind >= 0 && kind < 8 && cycle < 8) k_hint[kind][cycle] = h_st->kused;
        res.bnorm = h_st->norms[0];
        if (h_st->kused == 0) {
            // the cycle start found the true residual below tolerance (or broke down)
            res.resid = h_st->resid;
            res.converged = h_st->converged != 0;
            res.iters = it;
            return LX_OK;
        }
        ++res.restarts;
        it += h_st->kused;
        if (verbose())
            fprintf(stderr, "[lxns] gmres<%s> cycle %d: k=%d est=%.3e tol=%.3e bnorm=%.3e second passes %d\n",
                    sizeof(T) == 4 ? "f32" : "f64", cycle, h_st->kused, h_st->resid, h_st->tol_abs, h_st->norms[0],
                    h_st->n_reorth);
        launch_gm_solve_y(d_st, stream);
        launch_gm_update<T>(N, Z, ld, d_st, x, stream);
        if (inner && h_st->converged) {
            res.iters = it;
            res.resid = h_st->resid;
            res.converged = true;
            return LX_OK;
        }
        if (inner && it >= max_iters) {
            res.iters = it;
            res.resid = h_st->resid;
            res.converged = false;
            return LX_OK;
        }
        if (h_st->breakdown) {
            res.iters = it;
            res.resid = h_st->resid;
            return fail(LX_ENOCONV, "GMRES breakdown (non-finite value) after %d iterations", it);
        }
        if (it >= max_iters && !h_st->converged) {
            // final true residual
            spmv<T>(x, w, nullptr, nullptr);
            launch_gm_start<T>(N, b, w, V, d_st, d_partial, stream);
            s = read_state();
            if (s != LX_OK) return s;
            res.iters = it;
            res.resid = h_st->resid;
            res.converged = h_st->converged != 0;
            return LX_OK;
        }
        x_zero = false;
    }
}
template lx_status Sim::gmres<double>(const double *, double *, bool, double, int, GmResult &, lx_step_stats &,
                                      bool, int);
template lx_status Sim::gmres<float>(const float *, float *, bool, double, int, GmResult &, lx_step_stats &,
                                     bool, int);

// ------------------------------------------------------------------ step

void Sim::coefficients(double t1, StepCoef &C, BCSet &B) const
{
    memset(&C, 0, sizeof(C));
    const int order = std::max(1, std::min(prob.bdf_order, std::max(nlev, 1)));
    C.alpha = kAlpha[order];
    C.sigma = order;
    C.dt = prob.dt;
    C.rho = prob.rho;
    C.mu = prob.mu;
    C.C_r = prob.C_r;
    for (int l = 0; l < 3; ++l) {
        C.beta[l] = kBeta[order][l];
        C.gamma[l] = kGamma[order][l];
    }
    C.nlev = order;
    C.stab = prob.stab;
    C.symgrad = prob.diffusion == LX_DIFF_SYMGRAD;
    C.n_valves = (int)valves.size();
    for (int k = 0; k < C.n_valves; ++k) {
        const lx_riis &v = valves[k];
        double nn = std::sqrt(v.normal[0] * v.normal[0] + v.normal[1] * v.normal[1] + v.normal[2] * v.normal[2]);
        for (int c = 0; c < 3; ++c) {
            C.valve[k][c] = v.center[c];
            C.valve[k][3 + c] = v.normal[c] / nn;
        }
        C.valve[k][6] = law_value(v.orifice_radius, t1);
        C.valve[k][7] = v.outer_radius;
        C.valve[k][8] = v.R;
        C.valve[k][9] = v.eps;
    }
    memset(&B, 0, sizeof(B));
    B.n = (int)bcs.size();
    B.ale = prob.ale;
    for (int i = 0; i < B.n; ++i) {
        const lx_boundary &s = bcs[i].spec;
        B.bc[i].type = s.type;
        B.bc[i].profile = s.profile.kind;
        B.bc[i].scale = s.theta * law_value(s.law, t1);
        for (int c = 0; c < 3; ++c) {
            B.bc[i].center[c] = s.profile.center[c];
            B.bc[i].normal[c] = s.profile.normal[c];
        }
        B.bc[i].radius = s.profile.radius;
    }
}

// Coefficients, mesh motion and boundary values of the coming step.
lx_status Sim::prepare(double t1, StepCoef &C)
{
    BCSet B;
    coefficients(t1, C, B);
    if (prob.ale) {
        lx_status s = ale_update(t1, C);
        if (s != LX_OK) return s;
    }
    for (const OutflowDev &o : outflow)
        launch_outflow_prepare(o, d_x, hist(0), hist(1), hist(2), C.gamma, prob.rho, stream);
    if (n_dir > 0) {
        if (dirty_gnodal) {
            LX_HIP(hipMemcpyAsync(d_gnodal, h_gnodal.data(), sizeof(double) * 3 * n_dir, hipMemcpyHostToDevice,
                                  stream));
            dirty_gnodal = false;
        }
        launch_dirichlet_values(n_dir, d_dir_node, d_dir_bc, B, p2 ? d_xnode : d_x, d_uA, d_gnodal, d_g, stream);
    }
    return LX_OK;
}

// Everything that builds the system of the coming step (no solve).
lx_status Sim::build_system(double t1, StepCoef &C, lx_step_stats &tstats)
{
    (void)tstats;
    lx_status ps = prepare(t1, C);
    if (ps != LX_OK) return ps;
    return assemble_system(t1, C);
}

// The system at t1 after prepare(): assembly, Dirichlet rows, preconditioner set-up.
// fork_residual (P1-P1 FP32 with the second stream): once the FP32 matrix is
// assembled, the FP64 residual of the guess d_xs starts on the second stream and
// runs beside the preconditioner set-up; ev_join marks its end.
lx_status Sim::assemble_system(double t1, StepCoef &C, bool fork_residual)
{
    if (p2) return build_system_p2(t1, C);
    const RowPattern P = pattern();
    if (solver.precision == LX_FP64) {
        launch_fill<double>(N, d_rhs64, 0.0, stream);
        AsmArgs<double> A{nt, nblk, d_tet, d_sinc_ptr, d_sinc, d_rec64, d_x, d_xh, hist(0), hist(1), hist(2), d_uA,
                          d_f, d_val64, d_rhs64};
        auto *tm = timer_begin(1, 0);
        launch_assemble_p1<double>(A, C, stream);
        timer_end(tm);
        add_neumann(t1, d_rhs64, nullptr);
        for (const OutflowDev &o : outflow) {
            launch_backflow_add<double>(o, nblk, d_val64, stream);
            launch_outflow_rhs(o, outflow_p0(o, t1), prob.ale ? d_uA : nullptr, d_rhs64, stream);
        }
        launch_dirichlet_rows<double>(n_dir, d_dir_node, d_g, P, d_val64, d_rhs64, stream);
        launch_simple_setup<double>(P, d_val64, d_Finv64, d_Dinv64, solver.precond == LX_PC_AMG ? nullptr : d_Sinv64,
                                  stream);
        if (solver.precond == LX_PC_AMG)
            launch_amg_setup<double>(view<double>(), d_Finv64, d_Dinv64, amg64, stream);
        else if (solver.schur_degree > 0)
            launch_schur_bound<double>(P, d_val64, d_Dinv64, d_Sinv64, d_sw64, d_st, d_partial, nb_red, stream);
    } else {
        if (solver.asm_fp64) {
            AsmArgs<double> A{nt, nblk, d_tet, d_sinc_ptr, d_sinc, d_rec64, d_x, d_xh, hist(0), hist(1), hist(2),
                              d_uA, d_f, d_val64, nullptr};
            auto *tm = timer_begin(1, 0);
            launch_assemble_p1<double>(A, C, stream);
            timer_end(tm);
            launch_scale_copy<float, double>(kPlanes * nblk, d_val32, d_val64, 1.0, stream);
        } else {
            AsmArgs<float> A{nt, nblk, d_tet, d_sinc_ptr, d_sinc, d_rec32, d_x, d_xh, hist(0), hist(1), hist(2),
                             d_uA, d_f, d_val32, nullptr};
            auto *tm = timer_begin(1, 0);
            launch_assemble_p1<float>(A, C, stream);
            timer_end(tm);
        }
        for (const OutflowDev &o : outflow) launch_backflow_add<float>(o, nblk, d_val32, stream);
        launch_dirichlet_rows<float>(n_dir, d_dir_node, d_g, P, d_val32, (float *)nullptr, stream);
        if (fork_residual) {
            // the residual reads the element data and the history, not the FP32
            // system; it shares no buffer that either side writes
            LX_HIP(hipEventRecord(ev_fork, stream));
            LX_HIP(hipStreamWaitEvent(stream_aux, ev_fork, 0));
            std::swap(stream, stream_aux);
            const lx_status rs = residual64(C, d_xs, true, t1);
            std::swap(stream, stream_aux);
            if (rs != LX_OK) return rs;
            // ||b|| and ||r|| behind it on the same stream (norm slots 1 and 2; the set-up on
            // the first stream writes other fields of the state) and their copy to the host
            launch_norm<double>(N, d_b64, d_st, 0.0, d_partial_aux, 1, stream_aux);
            launch_norm<double>(N, d_r64, d_st, 0.0, d_partial_aux, 2, stream_aux);
            LX_HIP(hipMemcpyAsync(h_norms0, &d_st->norms[1], 2 * sizeof(double), hipMemcpyDeviceToHost, stream_aux));
            LX_HIP(hipEventRecord(ev_join, stream_aux));
        }
        launch_simple_setup<float>(P, d_val32, d_Finv32, d_Dinv32, solver.precond == LX_PC_AMG ? nullptr : d_Sinv32,
                                  stream);
        if (solver.precond == LX_PC_AMG)
            launch_amg_setup<float>(view<float>(), d_Finv32, d_Dinv32, amg32, stream);
        else if (solver.schur_degree > 0)
            launch_schur_bound<float>(P, d_val32, d_Dinv32, d_Sinv32, d_sw32, d_st, d_partial, nb_red, stream);
    }
    LX_HIP(hipGetLastError());
    return LX_OK;
}

// P2-P1: element records + slot gathers (FP64), Neumann traction, Dirichlet
// rows, then the SIMPLE blocks and the AMG hierarchy in the solve precision.
lx_status Sim::build_system_p2(double t1, StepCoef &C)
{
    launch_fill<double>(N, d_rhs64, 0.0, stream);
    P2AsmArgs A{nt, nv, nu, d_tet, d_nodes, d_x, d_xh, hist(0), hist(1), hist(2), d_f, d_rules, d_rec2,
                d_finc_ptr, d_finc, d_ginc_ptr, d_ginc, d_binc_ptr, d_binc, d_sinc_ptr, d_sinc, d_fdiag, d_diag};
    auto *tm = timer_begin(1, 0);
    launch_assemble_p2(A, C, s64, d_rhs64, stream);
    timer_end(tm);
    add_neumann(t1, d_rhs64, nullptr);
    launch_dirichlet_rows_p2<double>(n_dir, d_dir_node, d_g, s64, d_fdiag, d_rhs64, stream);
    if (solver.precision == LX_FP64) {
        launch_simple_setup_p2<double>(s64, d_fdiag, d_Finv64, d_Dinv64, stream);
        launch_amg_setup<double>(view<double>(), d_Finv64, d_Dinv64, amg64, stream);
    } else {
        launch_round_p2(s64, s32, stream);
        launch_simple_setup_p2<float>(s32, d_fdiag, d_Finv32, d_Dinv32, stream);
        launch_amg_setup<float>(view<float>(), d_Finv32, d_Dinv32, amg32, stream);
    }
    LX_HIP(hipGetLastError());
    return LX_OK;
}

// Host lists of the outflow conditions (resistance, backflow): boundary vertices
// with their face incidences, and the backflow vertex pairs with their blocks.
lx_status Sim::outflow_setup()
{
    lx_status a = dalloc((void **)&d_bint, sizeof(double) * 4);
    if (a != LX_OK) return a;
    std::vector<std::vector<int32_t>> keep_alive;
    auto up32 = [&](int32_t **dst, std::vector<int32_t> v) -> lx_status {
        if (v.empty()) v.push_back(0);
        lx_status r = dalloc((void **)dst, sizeof(int32_t) * v.size());
        if (r != LX_OK) return r;
        keep_alive.push_back(std::move(v));
        const auto &h = keep_alive.back();
        LX_HIP(hipMemcpyAsync(*dst, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, stream));
        return LX_OK;
    };
    for (int i = 0; i < (int)bcs.size(); ++i) {
        const BCDesc &B = bcs[i];
        const bool res = B.spec.type == LX_BC_RESISTANCE && B.spec.resistance > 0;
        const bool back = B.spec.backflow > 0;
        if ((!res && !back) || B.nf == 0) continue;
        OutflowDev o;
        o.bc = i;
        for (int c = 0; c < 3; ++c) o.dir[c] = B.spec.profile.normal[c];
        o.cr = res ? B.spec.resistance : 0.0;
        o.beta = back ? B.spec.backflow : 0.0;
        o.nf = B.nf;
        o.faces = B.d_faces;
        const std::vector<int32_t> &F = B.h_faces;
        // boundary vertices and their face corners (codes 3 f + l, ascending f)
        std::vector<int32_t> bv(F.begin(), F.end());
        std::sort(bv.begin(), bv.end());
        bv.erase(std::unique(bv.begin(), bv.end()), bv.end());
        o.nbv = (int64_t)bv.size();
        auto slot = [&](int32_t v) { return (int64_t)(std::lower_bound(bv.begin(), bv.end(), v) - bv.begin()); };
        std::vector<int32_t> vptr(o.nbv + 1, 0), vinc(3 * o.nf), keep(o.nbv);
        for (int64_t k = 0; k < 3 * o.nf; ++k) vptr[slot(F[k]) + 1]++;
        for (int64_t j = 0; j < o.nbv; ++j) vptr[j + 1] += vptr[j];
        {
            std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
            for (int64_t k = 0; k < 3 * o.nf; ++k) vinc[fill[slot(F[k])]++] = (int32_t)k;
        }
        for (int64_t j = 0; j < o.nbv; ++j) keep[j] = h_dir_index[bv[j]] < 0 ? 1 : 0;
        // backflow pairs (a, b), a kept: incidences in ascending face order
        std::vector<std::pair<std::pair<int32_t, int32_t>, int32_t>> inc;   // ((a, b), code)
        if (back)
            for (int64_t f = 0; f < o.nf; ++f)
                for (int la = 0; la < 3; ++la)
                    for (int lb = 0; lb < 3; ++lb) {
                        const int32_t va = F[3 * f + la], vb = F[3 * f + lb];
                        if (h_dir_index[va] >= 0) continue;
                        inc.push_back({{va, vb}, (int32_t)((f << 4) | (la << 2) | lb)});
                    }
        std::stable_sort(inc.begin(), inc.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
        std::vector<int32_t> pblk, pcol, pptr{0}, pinc, rptr{0}, rvert;
        for (size_t k = 0; k < inc.size(); ++k) {
            const bool new_pair = k == 0 || inc[k].first != inc[k - 1].first;
            if (new_pair) {
                const int32_t va = inc[k].first.first, vb = inc[k].first.second;
                int32_t blk = -1;
                for (int32_t q = hs.rowptr[va]; q < hs.rowptr[va + 1]; ++q)
                    if (hs.col[q] == vb) blk = q;
                if (blk < 0) return fail(LX_EMESH, "bc %d: boundary face edge missing from the matrix pattern", i);
                if (k > 0) pptr.push_back((int32_t)k);
                if (rvert.empty() || rvert.back() != va) {
                    if (!rvert.empty()) rptr.push_back((int32_t)pblk.size());
                    rvert.push_back(va);
                }
                pblk.push_back(blk);
                pcol.push_back(vb);
            }
            pinc.push_back(inc[k].second);
        }
        pptr.push_back((int32_t)inc.size());
        rptr.push_back((int32_t)pblk.size());
        o.npair = (int64_t)pblk.size();
        o.nrow = (int64_t)rvert.size();
        if (o.npair == 0) {
            pptr.assign(1, 0);
            rptr.assign(1, 0);
        }
        lx_status r;
        if ((r = up32(&o.bv, bv)) != LX_OK || (r = up32(&o.vptr, vptr)) != LX_OK ||
            (r = up32(&o.vinc, vinc)) != LX_OK || (r = up32(&o.keep, keep)) != LX_OK ||
            (r = up32(&o.pblk, pblk)) != LX_OK || (r = up32(&o.pcol, pcol)) != LX_OK ||
            (r = up32(&o.pptr, pptr)) != LX_OK || (r = up32(&o.pinc, pinc)) != LX_OK ||
            (r = up32(&o.rptr, rptr)) != LX_OK || (r = up32(&o.rvert, rvert)) != LX_OK)
            return r;
        if ((r = dalloc((void **)&o.geom, sizeof(double) * 4 * o.nf)) != LX_OK ||
            (r = dalloc((void **)&o.w, sizeof(double) * 3 * o.nbv)) != LX_OK ||
            (r = dalloc((void **)&o.pcoef, sizeof(double) * std::max<int64_t>(o.npair, 1))) != LX_OK)
            return r;
        launch_fill<double>(3 * o.nbv, o.w, 0.0, stream);
        launch_fill<double>(std::max<int64_t>(o.npair, 1), o.pcoef, 0.0, stream);
        outflow.push_back(o);
    }
    LX_HIP(hipStreamSynchronize(stream));   // the host lists are local
    return LX_OK;
}

double Sim::outflow_p0(const OutflowDev &o, double t1) const
{
    const lx_boundary &b = bcs[o.bc].spec;
    return b.type == LX_BC_RESISTANCE ? b.theta * law_value(b.law, t1) : 0.0;
}

void Sim::add_neumann(double t1, double *out0, double *out1)
{
    for (auto &b : bcs) {
        if (b.spec.type != LX_BC_NEUMANN || b.nf == 0) continue;
        double hc[3] = {0, 0, 0};
        const double *hn = nullptr;
        if (b.spec.profile.kind == LX_PROFILE_NODAL) {
            if (!b.nodal_set) continue;
            hn = b.d_hnodal;
        } else {
            // sigma n = -theta h(t) n
            double h = b.spec.theta * law_value(b.spec.law, t1);
            if (h == 0.0) continue;
            for (int c = 0; c < 3; ++c) hc[c] = -h * b.spec.profile.normal[c];
        }
        if (p2) {
            launch_neumann_p2(b.nf, b.d_faces, d_xnode, hn, hc, d_rules, out0, stream);
            if (out1) launch_neumann_p2(b.nf, b.d_faces, d_xnode, hn, hc, d_rules, out1, stream);
        } else {
            launch_neumann(b.nf, b.d_faces, d_x, hn, hc, out0, out1, nullptr, stream);
        }
    }
}

// FP64 matrix-free residual r = b - A xs (first: also b and the Dirichlet diagonal).
lx_status Sim::residual64(const StepCoef &C, const double *xs, bool first, double t1)
{
    if (p2) {
        // b is the assembled FP64 right-hand side; r = b - A64 xs by the FP64 SpMV
        if (first) LX_HIP(hipMemcpyAsync(d_b64, d_rhs64, sizeof(double) * N, hipMemcpyDeviceToDevice, stream));
        auto *tm = timer_begin(2, 0);
        launch_spmv_p2<double>(s64, xs, d_r64, nullptr, stream);
        timer_end(tm);
        launch_scale_copy<double, double>(N, d_r64, d_r64, -1.0, stream);
        launch_axpy<double, double>(N, d_r64, d_b64, nullptr, 1.0, stream);
        LX_HIP(hipGetLastError());
        return LX_OK;
    }
    return residual64_into(C, xs, first, t1, d_rrec, d_r64, d_b64, true);
}

// P1-P1 FP64 matrix-free residual into given buffers: element contributions in
// rec [kRRec nt], r = b - A xs [nv][4] and (first) b [nv][4]; every entry of the
// three is written before it is read.  timed: stamp the pass (collect_timing).
lx_status Sim::residual64_into(const StepCoef &C, const double *xs, bool first, double t1, double *rec, double *r,
                               double *b, bool timed)
{
    // the vertex pass writes every row of r (and of b); Dirichlet diagonals are summed into dg
    if (first && n_dir > 0) launch_fill<double>(3 * n_dir, d_dg, 0.0, stream);
    ResArgs R{nt, nv, d_tet, d_vinc_ptr, d_vpos, rec, d_x, d_xh, hist(0), hist(1), hist(2), d_uA, d_f,
              xs, d_dir_index, r, first ? b : nullptr, first ? d_dg : nullptr};
    auto *tm = timed ? timer_begin(2, 0) : nullptr;
    launch_residual_p1(R, C, stream);
    timer_end(tm);
    add_neumann(t1, r, first ? b : nullptr);
    for (const OutflowDev &o : outflow)
        launch_outflow_residual(o, outflow_p0(o, t1), prob.ale ? d_uA : nullptr, xs, r, first ? b : nullptr, stream);
    launch_dirichlet_residual(n_dir, d_dir_node, d_g, d_dg, xs, r, first ? b : nullptr, stream);
    LX_HIP(hipGetLastError());
    return LX_OK;
}

// Newton's method for the implicit formulation, from the guess in d_xs: at each
// iterate the Jacobian and -R are assembled (Neumann data, Dirichlet rows set to
// the update g - x), the SIMPLE/AMG preconditioner is built on the Jacobian and
// GMRES solves the update (to rtol, or to a tenth of the Newton target near the
// end).  Stops when ||R|| <= ir_rtol ||R_0|| or the last update is below
// ir_rtol ||x||.
// The Newton system at the iterate d_xs: Jacobian in d_val64, -R in d_rhs64 (after prepare()).
void Sim::newton_system(double t1, const StepCoef &C)
{
    const RowPattern P = pattern();
    NewtonArgs A{nt, nblk, d_tet, d_sinc_ptr, d_sinc, d_x, d_xh, d_xs, hist(0), hist(1), hist(2),
                 prob.ale ? d_uA : nullptr, d_f, d_nrec, d_val64, d_rhs64};
    launch_fill<double>(N, d_rhs64, 0.0, stream);
    auto *tm = timer_begin(1, 0);
    launch_newton_p1(A, C, stream);
    timer_end(tm);
    add_neumann(t1, d_rhs64, nullptr);
    // outflow terms are linear in the new state (the backflow coefficient is taken at
    // u_EXT): the backflow block joins the Jacobian, -R gains the resistance data minus
    // (backflow + C_R w w^T) xs; the rank-1 part of the Jacobian is applied in the product
    for (const OutflowDev &o : outflow) {
        launch_backflow_add<double>(o, nblk, d_val64, stream);
        launch_outflow_residual(o, outflow_p0(o, t1), prob.ale ? d_uA : nullptr, d_xs, d_rhs64, nullptr, stream);
    }
    launch_dirichlet_delta(n_dir, d_dir_node, d_g, d_xs, d_gdelta, stream);
    launch_dirichlet_rows<double>(n_dir, d_dir_node, d_gdelta, P, d_val64, d_rhs64, stream);
}

lx_status Sim::newton(double t1, const StepCoef &C, lx_step_stats &S)
{
    const RowPattern P = pattern();
    double r0 = 0.0, rn = 0.0;
    bool conv = false;
    int it = 0, total = 0;
    for (;; ++it) {
        newton_system(t1, C);
        launch_norm<double>(N, d_rhs64, d_st, 0.0, d_partial, 1, stream);
        if (it > 0) {
            // the last update: FP64 in d_dx, or FP32 in d_x32
            if (solver.precision == LX_FP64)
                launch_norm<double>(N, d_dx, d_st, 0.0, d_partial, 2, stream);
            else
                launch_norm<float>(N, d_x32, d_st, 0.0, d_partial, 2, stream);
            launch_norm<double>(N, d_xs, d_st, 0.0, d_partial, 3, stream);
        }
        lx_status st = read_state();
        if (st != LX_OK) return st;
        rn = h_st->norms[1];
        if (it == 0) r0 = rn;
        if (verbose())
            fprintf(stderr, "[lxns] Newton %d: ||R|| %.3e (%.3e of the start)\n", it, rn, r0 > 0 ? rn / r0 : 0.0);
        if (!(rn == rn)) break;
        if (rn <= solver.ir_rtol * r0 || rn == 0.0 || (it > 0 && h_st->norms[2] <= solver.ir_rtol * h_st->norms[3])) {
            conv = true;
            break;
        }
        if (it >= solver.max_ir || total >= solver.max_iters) break;
        // each update to rtol, but no tighter than the Newton test needs: a residual already near
        // ir_rtol ||R_0|| is solved only to a tenth of that level (inexact Newton), so that the
        // linear tolerance never falls below what the Jacobian's conditioning allows
        const double lin = std::min(0.5, std::max(solver.rtol, 0.1 * solver.ir_rtol * r0 / rn));
        GmResult gr;
        if (solver.precision == LX_FP64) {
            launch_simple_setup<double>(P, d_val64, d_Finv64, d_Dinv64,
                                        solver.precond == LX_PC_AMG ? nullptr : d_Sinv64, stream);
            if (solver.precond == LX_PC_AMG)
                launch_amg_setup<double>(view<double>(), d_Finv64, d_Dinv64, amg64, stream);
            else if (solver.schur_degree > 0)
                launch_schur_bound<double>(P, d_val64, d_Dinv64, d_Sinv64, d_sw64, d_st, d_partial, nb_red, stream);
            st = gmres<double>(d_rhs64, d_dx, true, lin, solver.max_iters - total, gr, S);
            if (st != LX_OK) return st;
            launch_axpy<double, double>(N, d_xs, d_dx, nullptr, 1.0, stream);
        } else {
            // FP32 update: the FP64 Jacobian and -R rounded, the preconditioner and GMRES in
            // FP32 (to no tighter than inner_rtol, what FP32 sums resolve), the update added
            // to the FP64 iterate; the FP64 residual of the next iterate decides, as in
            // iterative refinement
            launch_scale_copy<float, double>(kPlanes * nblk, d_val32, d_val64, 1.0, stream);
            launch_scale_copy<float, double>(N, d_r32, d_rhs64, 1.0, stream);
            launch_simple_setup<float>(P, d_val32, d_Finv32, d_Dinv32,
                                       solver.precond == LX_PC_AMG ? nullptr : d_Sinv32, stream);
            if (solver.precond == LX_PC_AMG)
                launch_amg_setup<float>(view<float>(), d_Finv32, d_Dinv32, amg32, stream);
            else if (solver.schur_degree > 0)
                launch_schur_bound<float>(P, d_val32, d_Dinv32, d_Sinv32, d_sw32, d_st, d_partial, nb_red, stream);
            st = gmres<float>(d_r32, d_x32, true, std::max(lin, solver.inner_rtol), solver.max_iters - total, gr, S,
                              true, std::min(it + 1, 7));
            if (st != LX_OK) return st;
            launch_axpy<double, float>(N, d_xs, d_x32, nullptr, 1.0, stream);
        }
        total += gr.iters;
        S.restarts += gr.restarts;
    }
    S.gmres_iters = total;
    S.newton_iters = it;
    S.rel_residual = r0 > 0 ? rn / r0 : rn;
    S.converged = conv;
    return LX_OK;
}

lx_status Sim::step(lx_step_stats *out)
{
    LX_HIP(hipSetDevice(device));
    lx_step_stats S;
    memset(&S, 0, sizeof(S));
    const double t1 = t + prob.dt;
    const int L = prob.bdf_order;
    ale_iters = 0;
    lift_solved = false;
    LX_HIP(hipEventRecord(ev_step0, stream));
    StepCoef C;
    const bool overlap = stream_aux != nullptr;
    // the implicit formulation assembles its Newton systems inside the Newton loop
    lx_status st = (overlap || !prob.semi_implicit) ? prepare(t1, C) : build_system(t1, C, S);
    if (st != LX_OK) return st;
    if (!overlap) LX_HIP(hipEventRecord(ev_asm1, stream));
    // initial guess, with the new Dirichlet values: the polynomial through the
    // last four (three) solutions evaluated at t^{n+1}, or the extrapolation
    // with the step's BDF weights (u_EXT, p_EXT); x_order picks the one that
    // best predicted the previous step's solution (measured after each step),
    // limited by the levels that exist.  The guess sets only where GMRES
    // starts; it stops on ||b - A x|| <= rtol ||b|| whatever the start.
    // LXNS_X0_ORDER=2|3 caps the order, LXNS_X0=prev starts from the previous
    // solution.
    static const bool extrap = [] {
        const char *e = getenv("LXNS_X0");
        return !(e && strcmp(e, "prev") == 0);
    }();
    static const int xorder = [] {
        const char *e = getenv("LXNS_X0_ORDER");
        const int k = e ? atoi(e) : 4;
        return k >= 2 && k <= 4 ? k : 4;
    }();
    const int K = std::min(std::min(x_order, xorder), nhist);
    if (extrap && K == 4)
        // the cubic through the last four solutions at t^{n+1} (constant step)
        launch_extrapolate(N, d_xs, d_hist[0], d_hist[1], d_hist[2], 4.0, -6.0, 4.0, stream, d_hist[3], -1.0);
    else if (extrap && K == 3)
        // the quadratic through the last three solutions at t^{n+1} (constant step)
        launch_extrapolate(N, d_xs, d_hist[0], d_hist[1], d_hist[2], 3.0, -3.0, 1.0, stream);
    else if (extrap)
        launch_extrapolate(N, d_xs, d_hist[0], C.gamma[1] != 0 ? d_hist[1] : nullptr,
                           C.gamma[2] != 0 ? d_hist[2] : nullptr, C.gamma[0], C.gamma[1], C.gamma[2], stream);
    else
        LX_HIP(hipMemcpyAsync(d_xs, d_hist[0], sizeof(double) * N, hipMemcpyDeviceToDevice, stream));
    launch_set_dirichlet_x(n_dir, d_dir_node, d_g, d_xs, stream);
    if (overlap) {
        // The FP64 residual of the guess (matrix-free, from the element data and the
        // history) does not read the FP32 system: it runs on the second stream while
        // the preconditioner is set up.
        st = assemble_system(t1, C, true);
        if (st != LX_OK) return st;
        LX_HIP(hipEventRecord(ev_asm1, stream));
        LX_HIP(hipStreamWaitEvent(stream, ev_join, 0));
    }
    // scoring of the guess orders against the solution (read after the final sync); the
    // refinement loop scores each iterate it checks before reading its residual, so that the
    // last check's host round trip covers the scoring too
    const int nk = extrap ? std::min(nhist, 4) - 1 : 0;
    bool scored = false;
    auto score_guess = [&]() -> lx_status {
        if (nk < 2) return LX_OK;
        const double *h[4] = {d_hist[0], d_hist[1], d_hist[2], d_hist[3]};
        launch_guess_err(N, nk, d_xs, h, C.gamma, d_gerr, d_gerr + kGuessErrPartial, stream);
        LX_HIP(hipMemcpyAsync(h_gerr, d_gerr + kGuessErrPartial, 3 * sizeof(double), hipMemcpyDeviceToHost, stream));
        scored = true;
        return LX_OK;
    };
    GmResult gr;
    if (!prob.semi_implicit) {
        st = newton(t1, C, S);
        if (st != LX_OK) return st;
    } else if (solver.precision == LX_FP64) {
        st = gmres<double>(d_rhs64, d_xs, false, solver.rtol, solver.max_iters, gr, S);
        if (st != LX_OK) return st;
        S.gmres_iters = gr.iters;
        S.restarts = gr.restarts;
        S.rel_residual = gr.bnorm > 0 ? gr.resid / gr.bnorm : gr.resid;
        S.converged = gr.converged;
    } else {
        // FP32 matrix and inner GMRES inside FP64 iterative refinement
        double n0[2];
        if (overlap) {
            // formed on the second stream: wait for that stream only, while the set-up runs on
            LX_HIP(hipEventSynchronize(ev_join));
            n0[0] = h_norms0[0];
            n0[1] = h_norms0[1];
        } else {
            st = residual64(C, d_xs, true, t1);
            if (st != LX_OK) return st;
            launch_norm<double>(N, d_b64, d_st, 0.0, d_partial, 1, stream);
            launch_norm<double>(N, d_r64, d_st, 0.0, d_partial, 2, stream);
            st = read_state();
            if (st != LX_OK) return st;
            n0[0] = h_st->norms[1];
            n0[1] = h_st->norms[2];
        }
        const double bnorm = n0[0] > 0 ? n0[0] : 1.0;
        double rnorm = n0[1];
        int total = 0, ir = 0;
        bool conv = rnorm <= solver.ir_rtol * bnorm;
        while (!conv && ir < solver.max_ir && total < solver.max_iters) {
            // aim the inner tolerance at finishing in one more refinement step, but not below inner_rtol
            double want = 0.3 * solver.ir_rtol * bnorm / rnorm;
            double rin = std::max(solver.inner_rtol, std::min(want, 0.5));
            launch_scale_copy<float, double>(N, d_r32, d_r64, 1.0 / rnorm, stream);
            GmResult g32;
            st = gmres<float>(d_r32, d_x32, true, rin, solver.max_iters - total, g32, S, true, std::min(ir + 1, 7));
            if (st != LX_OK) return st;
            total += g32.iters;
            S.restarts += g32.restarts;
            launch_axpy<double, float>(N, d_xs, d_x32, nullptr, rnorm, stream);
            ++ir;
            st = residual64(C, d_xs, false, t1);
            if (st != LX_OK) return st;
            launch_norm<double>(N, d_r64, d_st, 0.0, d_partial, 2, stream);
            st = score_guess();
            if (st != LX_OK) return st;
            st = read_state();
            if (st != LX_OK) return st;
            if (verbose())
                fprintf(stderr, "[lxns] IR %d: inner rtol %.2e, %d iterations, FP64 rel. residual %.3e -> %.3e\n", ir,
                        rin, g32.iters, rnorm / bnorm, h_st->norms[2] / bnorm);
            rnorm = h_st->norms[2];
            conv = rnorm <= solver.ir_rtol * bnorm;
            if (!(rnorm == rnorm)) break;
            if (g32.iters == 0 && !g32.converged) break;
        }
        S.gmres_iters = total;
        S.ir_iters = ir;
        S.rel_residual = rnorm / bnorm;
        S.converged = conv;
        timer_flush(0, S);
    }
    if (!scored) {
        st = score_guess();
        if (st != LX_OK) return st;
    }
    LX_HIP(hipEventRecord(ev_step1, stream));
    LX_HIP(hipEventSynchronize(ev_step1));
    float ms = 0, ma = 0;
    (void)hipEventElapsedTime(&ms, ev_step0, ev_step1);
    (void)hipEventElapsedTime(&ma, ev_step0, ev_asm1);
    S.t_step_ms = ms;
    S.t_assembly_ms = ma;
    S.t_solve_ms = ms - ma;
    S.lift_iters = ale_iters;
    if (out) *out = S;
    if (!S.converged)
        return fail(LX_ENOCONV, "step did not converge: rel. residual %.3e after %d iterations", S.rel_residual,
                    S.gmres_iters);
    if (nk >= 2) {
        // the best predictor among those scored; if it is the highest scored,
        // the next step (with one more level) may go one order higher
        int best = 2;
        double eb = h_gerr[0];
        for (int k = 1; k <= nk - 1; ++k)
            if (h_gerr[k] < eb) eb = h_gerr[k], best = k + 2;
        x_order = best == nk + 1 ? std::min(best + 1, 4) : best;
    }
    // commit: rotate history (u^n -> u^{n-1}, ...) and advance time
    const int Lh = std::max(L, 4);
    double *oldest = d_hist[Lh - 1];
    for (int l = Lh - 1; l > 0; --l) d_hist[l] = d_hist[l - 1];
    d_hist[0] = d_xs;
    d_xs = oldest;
    if (prob.ale) ale_commit();
    nlev = std::min(std::max(nlev, 1) + 1, L);
    nhist = std::min(nhist + 1, Lh);
    t = t1;
    ++step_index;
    return LX_OK;
}

// ------------------------------------------------------------------ checkpoint

namespace {
struct CkHead {
    char magic[8];
    int64_t bytes;
    int64_t nv, nt, nu, N, nblk, n_dir;
    int32_t fe, bdf_order, precision, ale, forcing, n_bc, precond, f_degree;
    int32_t levels, nlev, nhist, x_order;
    int32_t f_warm, ale_ext_valid, fv_elem, ale_nodal;
    int32_t proj_n, pad;
    double t;
    int64_t step_index;
};
const char kCkMagic[8] = {'L', 'X', 'N', 'S', 'C', 'K', '0', '2'};
}  // namespace

// The blob: header, then the solution levels, the nodal Dirichlet values, per
// nodal Neumann condition its flag and traction, the forcing, the ALE
// displacement history, lifting, shape and the lifting projection basis, and the
// power-iteration vector.
int64_t Sim::state_bytes() const
{
    const int L = prob.bdf_order, Lh = std::max(L, 4);
    int64_t b = sizeof(CkHead);
    b += (int64_t)Lh * N * 8;
    b += (int64_t)h_gnodal.size() * 8;
    for (const auto &bc : bcs)
        if (bc.d_hnodal) b += 8 + 3 * nu * 8;
    if (d_f) b += 3 * nu * 8;
    if (prob.ale) b += (int64_t)(L + 3 + kProjMax) * 3 * nv * 8;
    const bool f64 = solver.precision == LX_FP64;
    if (solver.precond == LX_PC_AMG && (f64 ? amg64.fv : (void *)amg32.fv))
        b += 4 * nu * (f64 ? 8 : 4) + kLamSlots * 8;   // the vector and the norm slots it is read with
    return b;
}

lx_status Sim::save_state(void *blob, int64_t bytes)
{
    const int64_t need = state_bytes();
    if (!blob || bytes != need) return fail(LX_EINVAL, "state blob needs exactly %lld bytes", (long long)need);
    LX_HIP(hipSetDevice(device));
    const int L = prob.bdf_order, Lh = std::max(L, 4);
    const bool f64 = solver.precision == LX_FP64;
    void *fv = solver.precond == LX_PC_AMG ? (f64 ? (void *)amg64.fv : (void *)amg32.fv) : nullptr;
    CkHead h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kCkMagic, 8);
    h.bytes = need;
    h.nv = nv, h.nt = nt, h.nu = nu, h.N = N, h.nblk = nblk, h.n_dir = n_dir;
    h.fe = prob.fe, h.bdf_order = L, h.precision = solver.precision, h.ale = prob.ale, h.forcing = prob.forcing;
    h.n_bc = (int32_t)bcs.size(), h.precond = solver.precond, h.f_degree = solver.f_degree;
    h.levels = Lh, h.nlev = nlev, h.nhist = nhist, h.x_order = x_order;
    h.f_warm = fv ? (f64 ? amg64.f_warm : amg32.f_warm) : 0;
    h.ale_ext_valid = ale_ext_valid;
    h.ale_nodal = ale_nodal;
    h.proj_n = proj_n;
    h.fv_elem = fv ? (f64 ? 8 : 4) : 0;
    h.t = t;
    h.step_index = step_index;
    char *o = (char *)blob;
    memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    auto d2h = [&](const void *src, int64_t n) -> lx_status {
        LX_HIP(hipMemcpyAsync(o, src, (size_t)n, hipMemcpyDeviceToHost, stream));
        o += n;
        return LX_OK;
    };
#define CK(x)                       \
    do {                            \
        lx_status _s = (x);         \
        if (_s != LX_OK) return _s; \
    } while (0)
    for (int l = 0; l < Lh; ++l) CK(d2h(d_hist[l], N * 8));
    memcpy(o, h_gnodal.data(), h_gnodal.size() * 8);
    o += h_gnodal.size() * 8;
    for (const auto &bc : bcs)
        if (bc.d_hnodal) {
            const double flag = bc.nodal_set ? 1.0 : 0.0;
            memcpy(o, &flag, 8);
            o += 8;
            CK(d2h(bc.d_hnodal, 3 * nu * 8));
        }
    if (d_f) CK(d2h(d_f, 3 * nu * 8));
    if (prob.ale) {
        for (int l = 0; l < L; ++l) CK(d2h(d_dhist[l], 3 * nv * 8));
        CK(d2h(d_cg, 3 * nv * 8));
        CK(d2h(d_ale_shape, 3 * nv * 8));
        CK(d2h(d_dbnd, 3 * nv * 8));
        CK(d2h(d_projQ, kProjMax * 3 * nv * 8));
    }
    if (fv) {
        CK(d2h(fv, 4 * nu * h.fv_elem));
        CK(d2h(f64 ? amg64.lam : amg32.lam, kLamSlots * 8));
    }
#undef CK
    LX_HIP(hipStreamSynchronize(stream));
    return LX_OK;
}

lx_status Sim::load_state(const void *blob, int64_t bytes)
{
    const int64_t need = state_bytes();
    if (!blob || bytes != need) return fail(LX_EINVAL, "state blob of %lld bytes, this simulation needs %lld",
                                            (long long)bytes, (long long)need);
    CkHead h;
    memcpy(&h, blob, sizeof(h));
    const int L = prob.bdf_order, Lh = std::max(L, 4);
    const bool f64 = solver.precision == LX_FP64;
    void *fv = solver.precond == LX_PC_AMG ? (f64 ? (void *)amg64.fv : (void *)amg32.fv) : nullptr;
    if (memcmp(h.magic, kCkMagic, 8) != 0 || h.bytes != need || h.nv != nv || h.nt != nt || h.nu != nu ||
        h.N != N || h.nblk != nblk || h.n_dir != n_dir || h.fe != prob.fe || h.bdf_order != L ||
        h.precision != solver.precision || h.ale != prob.ale || h.forcing != prob.forcing ||
        h.n_bc != (int32_t)bcs.size() || h.precond != solver.precond || h.f_degree != solver.f_degree ||
        h.levels != Lh || h.fv_elem != (fv ? (f64 ? 8 : 4) : 0))
        return fail(LX_EINVAL, "state blob was saved by a simulation of another mesh, problem or solver");
    if (h.nlev < 0 || h.nlev > L || h.nhist < 0 || h.nhist > Lh || h.x_order < 2 || h.x_order > 4 ||
        h.proj_n < 0 || h.proj_n > kProjMax)
        return fail(LX_EINVAL, "state blob holds invalid counters");
    LX_HIP(hipSetDevice(device));
    const char *o = (const char *)blob + sizeof(h);
    auto h2d = [&](void *dst, int64_t n) -> lx_status {
        LX_HIP(hipMemcpyAsync(dst, o, (size_t)n, hipMemcpyHostToDevice, stream));
        o += n;
        return LX_OK;
    };
#define CK(x)                       \
    do {                            \
        lx_status _s = (x);         \
        if (_s != LX_OK) return _s; \
    } while (0)
    for (int l = 0; l < Lh; ++l) CK(h2d(d_hist[l], N * 8));
    memcpy(h_gnodal.data(), o, h_gnodal.size() * 8);
    o += h_gnodal.size() * 8;
    dirty_gnodal = true;
    for (auto &bc : bcs)
        if (bc.d_hnodal) {
            double flag;
            memcpy(&flag, o, 8);
            o += 8;
            bc.nodal_set = flag != 0.0;
            CK(h2d(bc.d_hnodal, 3 * nu * 8));
        }
    if (d_f) CK(h2d(d_f, 3 * nu * 8));
    if (prob.ale) {
        for (int l = 0; l < L; ++l) CK(h2d(d_dhist[l], 3 * nv * 8));
        CK(h2d(d_cg, 3 * nv * 8));
        CK(h2d(d_ale_shape, 3 * nv * 8));
        CK(h2d(d_dbnd, 3 * nv * 8));
        CK(h2d(d_projQ, kProjMax * 3 * nv * 8));
        ale_ext_valid = h.ale_ext_valid != 0;
        ale_nodal = h.ale_nodal != 0;
        proj_n = h.proj_n;
    }
    if (fv) {
        CK(h2d(fv, 4 * nu * h.fv_elem));
        CK(h2d(f64 ? amg64.lam : amg32.lam, kLamSlots * 8));
        (f64 ? amg64.f_warm : amg32.f_warm) = h.f_warm != 0;
    }
#undef CK
    LX_HIP(hipStreamSynchronize(stream));
    t = h.t;
    step_index = h.step_index;
    nlev = h.nlev;
    nhist = h.nhist;
    x_order = h.x_order;
    return LX_OK;
}

}  // namespace lx
