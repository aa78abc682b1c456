// C ABI entry points for lx_sim (see include/lxns.h).
#include <cstring>
#include <new>
#include <vector>

#include "lx_sim.h"

using lx::fail;

#define LX_GUARD(sim)                                                   \
    do {                                                                \
        if (!(sim)) return fail(LX_EINVAL, "simulation handle is NULL"); \
    } while (0)

extern "C" lx_status lx_sim_create(const lx_device *dev, const lx_mesh *mesh, const lx_problem *problem,
                                   const lx_solver *solver, lx_sim **out)
{
    if (!out) return fail(LX_EINVAL, "out is NULL");
    *out = nullptr;
    lx_sim *s = new (std::nothrow) lx_sim();
    if (!s) return fail(LX_ENOMEM, "host allocation failed");
    lx_status st;
    try {
        st = s->create(dev, mesh, problem, solver);
    } catch (const std::bad_alloc &) {
        st = fail(LX_ENOMEM, "host allocation failed during setup");
    }
    if (st != LX_OK) {
        delete s;
        return st;
    }
    *out = s;
    return LX_OK;
}

extern "C" lx_status lx_sim_query(const lx_sim *s, lx_sizes *out)
{
    LX_GUARD(s);
    if (!out) return fail(LX_EINVAL, "out is NULL");
    out->n_vertices = s->nv;
    out->n_tets = s->nt;
    out->n_u_nodes = s->nu;
    out->n_dofs = 3 * s->nu + s->nv;
    out->n_blocks = s->p2 ? s->s64.nf + s->s64.ng + s->s64.nb + s->s64.nc : s->nblk;
    out->device_bytes = s->device_bytes;
    out->n_edges = s->nu - s->nv;
    out->n_scalar_nnz = s->p2 ? 9 * s->s64.nf + 3 * s->s64.ng + 3 * s->s64.nb + s->s64.nc : 16 * s->nblk;
    out->amg_levels = 0;
    out->amg_tail_level = 0;
    for (int l = 0; l < 8; ++l) out->amg_level_rows[l] = out->amg_level_nnz[l] = 0;
    if (s->solver.precond == LX_PC_AMG) {
        const bool f64 = s->solver.precision == LX_FP64;
        out->amg_levels = 1 + (f64 ? s->amg64.nlev : s->amg32.nlev);
        out->amg_tail_level = f64 ? s->amg64.tail.first : s->amg32.tail.first;
        for (int l = 0; l < out->amg_levels && l < 8; ++l) {
            out->amg_level_rows[l] = f64 ? s->amg64.L[l].n : s->amg32.L[l].n;
            out->amg_level_nnz[l] = f64 ? s->amg64.L[l].nnz : s->amg32.L[l].nnz;
        }
    }
    return LX_OK;
}

extern "C" lx_status lx_sim_get_edges(const lx_sim *s, int32_t *edges)
{
    LX_GUARD(s);
    if (!edges) return fail(LX_EINVAL, "edges is NULL");
    if (!s->p2) return LX_OK;
    for (int64_t k = 0; k < s->p2h.ne; ++k) {
        const uint64_t key = s->p2h.edge_key[k];
        edges[2 * k] = s->hs.perm_v[(int64_t)(key >> 32)];
        edges[2 * k + 1] = s->hs.perm_v[(int64_t)(key & 0xffffffffu)];
    }
    return LX_OK;
}

// caller u [nu][3] + p [nv] -> internal [nu][4]
static void to_internal(const lx_sim *s, const double *u, const double *p, std::vector<double> &x)
{
    x.assign(4 * s->nu, 0.0);
    for (int64_t i = 0; i < s->nu; ++i) {
        const int64_t o = s->caller_node(i);
        for (int c = 0; c < 3; ++c) x[4 * i + c] = u ? u[3 * o + c] : 0.0;
        if (i < s->nv) x[4 * i + 3] = p ? p[o] : 0.0;
    }
}

extern "C" lx_status lx_sim_set_state(lx_sim *s, int32_t level, const double *u, const double *p, const double *d)
{
    LX_GUARD(s);
    if (level < 0 || level >= s->prob.bdf_order) return fail(LX_EINVAL, "level must be in [0, bdf_order)");
    (void)hipSetDevice(s->device);
    std::vector<double> x;
    to_internal(s, u, p, x);
    LX_HIP(hipMemcpyAsync(s->d_hist[level], x.data(), sizeof(double) * x.size(), hipMemcpyHostToDevice, s->stream));
    if (d && s->prob.ale) {
        std::vector<double> dd(3 * s->nv);
        for (int64_t i = 0; i < s->nv; ++i)
            for (int c = 0; c < 3; ++c) dd[3 * i + c] = d[3 * (int64_t)s->hs.perm_v[i] + c];
        LX_HIP(hipMemcpyAsync(s->d_dhist[level], dd.data(), sizeof(double) * dd.size(), hipMemcpyHostToDevice,
                              s->stream));
        LX_HIP(hipStreamSynchronize(s->stream));
    }
    LX_HIP(hipStreamSynchronize(s->stream));
    s->nlev = std::max(s->nlev, level + 1);
    // guess history: only levels the caller can set count, stale deeper ones are dropped
    s->nhist = std::min(std::max(s->nhist, level + 1), (int)s->prob.bdf_order);
    return LX_OK;
}

extern "C" lx_status lx_sim_set_time(lx_sim *s, double t)
{
    LX_GUARD(s);
    s->t = t;
    return LX_OK;
}

extern "C" lx_status lx_sim_set_dirichlet_values(lx_sim *s, int32_t bc, const double *g)
{
    LX_GUARD(s);
    if (bc < 0 || bc >= (int32_t)s->bcs.size() || !g) return fail(LX_EINVAL, "bad bc index or NULL values");
    const lx_boundary &b = s->bcs[bc].spec;
    if (b.type != LX_BC_DIRICHLET || b.profile.kind != LX_PROFILE_NODAL)
        return fail(LX_EINVAL, "bc %d is not a Dirichlet condition with a nodal profile", bc);
    for (int64_t k = 0; k < s->n_dir; ++k) {
        if (s->h_dir_bc[k] != bc) continue;
        const int64_t o = s->caller_node(s->h_dir_node[k]);
        for (int c = 0; c < 3; ++c) s->h_gnodal[3 * k + c] = g[3 * o + c];
    }
    s->dirty_gnodal = true;
    return LX_OK;
}

// caller [n][3] over the velocity nodes (vertices only: n = nv) -> device
static lx_status upload_nodal3(lx_sim *s, const double *src, double *dst, bool vertices_only = false)
{
    const int64_t n = vertices_only ? s->nv : s->nu;
    std::vector<double> h(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) h[3 * i + c] = src[3 * s->caller_node(i) + c];
    LX_HIP(hipMemcpyAsync(dst, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s->stream));
    LX_HIP(hipStreamSynchronize(s->stream));
    return LX_OK;
}

extern "C" lx_status lx_sim_set_neumann_traction(lx_sim *s, int32_t bc, const double *h)
{
    LX_GUARD(s);
    if (bc < 0 || bc >= (int32_t)s->bcs.size() || !h) return fail(LX_EINVAL, "bad bc index or NULL values");
    auto &b = s->bcs[bc];
    if (b.spec.type != LX_BC_NEUMANN || b.spec.profile.kind != LX_PROFILE_NODAL)
        return fail(LX_EINVAL, "bc %d is not a Neumann condition with a nodal profile", bc);
    if (!b.d_hnodal) return LX_OK;   // no faces carry this tag
    (void)hipSetDevice(s->device);
    lx_status st = upload_nodal3(s, h, b.d_hnodal);
    if (st == LX_OK) b.nodal_set = true;
    return st;
}

extern "C" lx_status lx_sim_set_forcing(lx_sim *s, const double *f)
{
    LX_GUARD(s);
    if (!s->prob.forcing || !s->d_f) return fail(LX_ESTATE, "problem was created without nodal forcing");
    if (!f) return fail(LX_EINVAL, "f is NULL");
    (void)hipSetDevice(s->device);
    return upload_nodal3(s, f, s->d_f);
}

extern "C" lx_status lx_sim_set_ale_displacement(lx_sim *s, const double *d)
{
    LX_GUARD(s);
    if (!s->prob.ale) return fail(LX_ESTATE, "problem was created without ALE");
    if (!d) return fail(LX_EINVAL, "d is NULL");
    (void)hipSetDevice(s->device);
    lx_status st = upload_nodal3(s, d, s->d_ale_shape, true);
    if (st == LX_OK) {
        s->ale_ext_valid = false;
        s->ale_nodal = false;
    }
    return st;
}

extern "C" lx_status lx_sim_set_boundary_displacement(lx_sim *s, const double *d)
{
    LX_GUARD(s);
    if (!s->prob.ale) return fail(LX_ESTATE, "problem was created without ALE");
    if (!d) return fail(LX_EINVAL, "d is NULL");
    (void)hipSetDevice(s->device);
    lx_status st = upload_nodal3(s, d, s->d_dbnd, true);
    if (st == LX_OK) s->ale_nodal = true;
    return st;
}

extern "C" lx_status lx_sim_step(lx_sim *s, lx_step_stats *stats)
{
    LX_GUARD(s);
    try {
        return s->step(stats);
    } catch (const std::bad_alloc &) {
        return fail(LX_ENOMEM, "host allocation failed");
    }
}

extern "C" lx_status lx_sim_state_size(const lx_sim *s, int64_t *bytes)
{
    LX_GUARD(s);
    if (!bytes) return fail(LX_EINVAL, "bytes is NULL");
    *bytes = s->state_bytes();
    return LX_OK;
}

extern "C" lx_status lx_sim_get_state(const lx_sim *s, void *blob, int64_t bytes)
{
    LX_GUARD(s);
    try {
        return const_cast<lx_sim *>(s)->save_state(blob, bytes);
    } catch (const std::exception &e) {
        return fail(LX_ENOMEM, "checkpoint failed: %s", e.what());
    }
}

extern "C" lx_status lx_sim_restore_state(lx_sim *s, const void *blob, int64_t bytes)
{
    LX_GUARD(s);
    try {
        return s->load_state(blob, bytes);
    } catch (const std::exception &e) {
        return fail(LX_ENOMEM, "restore failed: %s", e.what());
    }
}

extern "C" lx_status lx_sim_get_solution(const lx_sim *s, double *u, double *p, double *t)
{
    LX_GUARD(s);
    (void)hipSetDevice(s->device);
    std::vector<double> x(4 * s->nu);
    LX_HIP(hipMemcpyAsync(x.data(), s->d_hist[0], sizeof(double) * x.size(), hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipStreamSynchronize(s->stream));
    for (int64_t i = 0; i < s->nu; ++i) {
        const int64_t o = s->caller_node(i);
        if (u)
            for (int c = 0; c < 3; ++c) u[3 * o + c] = x[4 * i + c];
        if (p && i < s->nv) p[o] = x[4 * i + 3];
    }
    if (t) *t = s->t;
    return LX_OK;
}

// 4x4 block entry (r, c) -> plane
static inline int plane_of(int r, int c)
{
    if (r < 3 && c < 3) return 3 * r + c;
    if (r < 3) return 9 + r;
    if (c < 3) return 12 + c;
    return 15;
}

extern "C" lx_status lx_sim_debug_export(lx_sim *s, int32_t *brow, int32_t *bcol, double *vals, double *rhs)
{
    LX_GUARD(s);
    if (s->p2) return fail(LX_EINVAL, "P2-P1 systems are exported by lx_sim_debug_export_p2");
    (void)hipSetDevice(s->device);
    lx::StepCoef C;
    lx_step_stats S;
    memset(&S, 0, sizeof(S));
    lx_status st;
    if (s->prob.semi_implicit) {
        st = s->build_system(s->t + s->prob.dt, C, S);
    } else {
        // implicit formulation: the Newton system at the last solution (Dirichlet rows set
        // to the update g - x)
        st = s->prepare(s->t + s->prob.dt, C);
        if (st == LX_OK) {
            LX_HIP(hipMemcpyAsync(s->d_xs, s->d_hist[0], sizeof(double) * s->N, hipMemcpyDeviceToDevice, s->stream));
            s->newton_system(s->t + s->prob.dt, C);
            LX_HIP(hipGetLastError());
        }
    }
    if (st != LX_OK) return st;
    const int64_t nb = s->nblk;
    std::vector<double> planes(16 * nb);
    const bool f64 = s->solver.precision == LX_FP64 || !s->prob.semi_implicit;   // the Newton system is FP64
    if (f64) {
        LX_HIP(hipMemcpyAsync(planes.data(), s->d_val64, sizeof(double) * 16 * nb, hipMemcpyDeviceToHost, s->stream));
    } else {
        std::vector<float> p32(16 * nb);
        LX_HIP(hipMemcpyAsync(p32.data(), s->d_val32, sizeof(float) * 16 * nb, hipMemcpyDeviceToHost, s->stream));
        LX_HIP(hipStreamSynchronize(s->stream));
        for (int64_t i = 0; i < 16 * nb; ++i) planes[i] = p32[i];
    }
    std::vector<double> r(4 * s->nv, 0.0);
    if (f64)
        LX_HIP(hipMemcpyAsync(r.data(), s->d_rhs64, sizeof(double) * r.size(), hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipStreamSynchronize(s->stream));
    for (int64_t i = 0; i < s->nv; ++i) {
        const int32_t oi = s->hs.perm_v[i];
        for (int32_t k = s->hs.rowptr[i]; k < s->hs.rowptr[i + 1]; ++k) {
            if (brow) brow[k] = oi;
            if (bcol) bcol[k] = s->hs.perm_v[s->hs.col[k]];
            if (vals)
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) vals[16 * (int64_t)k + 4 * a + b] = planes[plane_of(a, b) * nb + k];
        }
        if (rhs)
            for (int c = 0; c < 4; ++c) rhs[4 * (int64_t)oi + c] = r[4 * i + c];
    }
    return LX_OK;
}

// Scalar COO of the P2-P1 system in the caller's numbering: velocity dof 3 node + c
// (nodes: caller vertex ids, then nv + edge index), pressure dof 3 nu + vertex.
extern "C" lx_status lx_sim_debug_export_p2(lx_sim *s, int32_t *rows, int32_t *cols, double *vals, double *rhs)
{
    LX_GUARD(s);
    if (!s->p2) return fail(LX_EINVAL, "not a P2-P1 simulation");
    (void)hipSetDevice(s->device);
    lx::StepCoef C;
    lx_step_stats S;
    memset(&S, 0, sizeof(S));
    lx_status st = s->build_system(s->t + s->prob.dt, C, S);
    if (st != LX_OK) return st;
    const lx::P2Sys<double> &Y = s->s64;
    std::vector<double> F(9 * Y.nf), G(3 * Y.ng), B(3 * Y.nb), Cc(Y.nc), r(4 * s->nu);
    LX_HIP(hipMemcpyAsync(F.data(), Y.F, sizeof(double) * F.size(), hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipMemcpyAsync(G.data(), Y.G, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipMemcpyAsync(B.data(), Y.B, sizeof(double) * B.size(), hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipMemcpyAsync(Cc.data(), Y.C, sizeof(double) * Cc.size(), hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipMemcpyAsync(r.data(), s->d_rhs64, sizeof(double) * r.size(), hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipStreamSynchronize(s->stream));
    const lx::P2Setup &q = s->p2h;
    const int64_t pu = 3 * s->nu;
    int64_t o = 0;
    auto put = [&](int64_t rr, int64_t cc, double v) {
        if (rows) rows[o] = (int32_t)rr;
        if (cols) cols[o] = (int32_t)cc;
        if (vals) vals[o] = v;
        ++o;
    };
    for (int64_t i = 0; i < s->nu; ++i)
        for (int32_t k = q.fptr[i]; k < q.fptr[i + 1]; ++k)
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d)
                    put(3 * s->caller_node(i) + c, 3 * s->caller_node(q.fcol[k]) + d, F[(3 * c + d) * Y.nf + k]);
    for (int64_t i = 0; i < s->nu; ++i)
        for (int32_t k = q.gptr[i]; k < q.gptr[i + 1]; ++k)
            for (int c = 0; c < 3; ++c) put(3 * s->caller_node(i) + c, pu + s->hs.perm_v[q.gcol[k]], G[c * Y.ng + k]);
    for (int64_t i = 0; i < s->nv; ++i)
        for (int32_t k = q.bptr[i]; k < q.bptr[i + 1]; ++k)
            for (int d = 0; d < 3; ++d)
                put(pu + s->hs.perm_v[i], 3 * s->caller_node(q.bcol[k]) + d, B[d * Y.nb + k]);
    for (int64_t i = 0; i < s->nv; ++i)
        for (int32_t k = s->hs.rowptr[i]; k < s->hs.rowptr[i + 1]; ++k)
            put(pu + s->hs.perm_v[i], pu + s->hs.perm_v[s->hs.col[k]], Cc[k]);
    if (rhs)
        for (int64_t i = 0; i < s->nu; ++i) {
            const int64_t oc = s->caller_node(i);
            for (int c = 0; c < 3; ++c) rhs[3 * oc + c] = r[4 * i + c];
            if (i < s->nv) rhs[pu + oc] = r[4 * i + 3];
        }
    return LX_OK;
}

extern "C" lx_status lx_sim_debug_residual(lx_sim *s, const double *u, const double *p, double *r)
{
    LX_GUARD(s);
    if (!r) return fail(LX_EINVAL, "r is NULL");
    if (s->p2) return fail(LX_EINVAL, "the matrix-free residual is built for the P1-P1 pair");
    (void)hipSetDevice(s->device);
    if (!s->d_r64) {
        lx_status a = s->dalloc((void **)&s->d_r64, sizeof(double) * s->N);
        if (a != LX_OK) return a;
        a = s->dalloc((void **)&s->d_b64, sizeof(double) * s->N);
        if (a != LX_OK) return a;
    }
    if (!s->d_rrec) {
        lx_status a = s->dalloc((void **)&s->d_rrec, sizeof(double) * lx::kRRec * s->nt);
        if (a != LX_OK) return a;
    }
    lx::StepCoef C;
    lx_status st = s->prepare(s->t + s->prob.dt, C);
    if (st != LX_OK) return st;
    std::vector<double> x;
    to_internal(s, u, p, x);
    LX_HIP(hipMemcpyAsync(s->d_xs, x.data(), sizeof(double) * x.size(), hipMemcpyHostToDevice, s->stream));
    st = s->residual64(C, s->d_xs, true, s->t + s->prob.dt);
    if (st != LX_OK) return st;
    std::vector<double> h(4 * s->nv);
    LX_HIP(hipMemcpyAsync(h.data(), s->d_r64, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipStreamSynchronize(s->stream));
    for (int64_t i = 0; i < s->nv; ++i) {
        const int64_t o = s->hs.perm_v[i];
        for (int c = 0; c < 4; ++c) r[4 * o + c] = h[4 * i + c];
    }
    return LX_OK;
}

extern "C" lx_status lx_sim_boundary_integrals(lx_sim *s, int32_t bc, double *out)
{
    LX_GUARD(s);
    if (!out) return fail(LX_EINVAL, "out is NULL");
    if (s->p2) return fail(LX_EINVAL, "boundary integrals are built for the P1-P1 pair");
    if (bc < 0 || bc >= (int32_t)s->bcs.size()) return fail(LX_EINVAL, "bad boundary condition index %d", bc);
    const lx::BCDesc &B = s->bcs[bc];
    if (B.nf == 0 || !B.d_faces) {
        out[0] = out[1] = out[2] = 0.0;
        return LX_OK;
    }
    (void)hipSetDevice(s->device);
    lx::launch_boundary_integrals(B.nf, B.d_faces, s->d_x, B.spec.profile.normal, s->d_hist[0],
                                  s->prob.ale ? s->d_uA : nullptr, s->d_bint, s->stream);
    LX_HIP(hipGetLastError());
    LX_HIP(hipMemcpyAsync(out, s->d_bint, sizeof(double) * 3, hipMemcpyDeviceToHost, s->stream));
    LX_HIP(hipStreamSynchronize(s->stream));
    return LX_OK;
}

extern "C" void lx_sim_destroy(lx_sim *s) { delete s; }
