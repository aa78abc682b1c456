"""ctypes binding of liblxns.so (argument marshalling only; every step of the
time step runs in the HIP library).

The C entry points are exposed under their own names (lx_sim_create, ...)
through `lib()`, and wrapped by `Sim` and `Server`, which convert numpy
arrays and plain problem descriptions (objects with the attributes of the C
structs) into the C structs.  Loading fails loudly when the library has not
been built: there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblxns.so")

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P = ctypes.POINTER

LX_OK, LX_EINVAL, LX_ENOMEM, LX_EDEVICE, LX_ENOCONV, LX_EMESH, LX_EBUSY, LX_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "LX_OK", -1: "LX_EINVAL", -2: "LX_ENOMEM", -3: "LX_EDEVICE", -4: "LX_ENOCONV",
                -5: "LX_EMESH", -6: "LX_EBUSY", -7: "LX_ESTATE"}
LAW = {"constant": 0, "pulsatile": 1, "ramp": 2, "ramp2": 3, "linear": 4, "sine": 5}
PROFILE = {"uniform": 0, "parabolic": 1, "nodal": 2}
BC = {"noslip": 0, "dirichlet": 1, "neumann": 2, "resistance": 3}
LIFT = {"harmonic": 0, "elastic": 1}
STIFF = {"none": 0, "jacobian": 1, "boundary": 2}
FE = {"p1p1": 1, "p2p1": 2}
DIFF = {"gradgrad": 0, "symgrad": 1}
STAB = {"none": 0, "supg_pspg": 1, "vms_les": 2}
PREC = {"fp64": 0, "fp32_ir": 1}
PRECOND = {"amg": 0, "cheb_schur": 1}
REQ_STATE = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "setup"}


class LxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(c_vp, ctypes.c_size_t, c_vp)
FREE_FN = ctypes.CFUNCTYPE(None, c_vp, c_vp)


class lx_device(ctypes.Structure):
    _fields_ = [("device", c_i32), ("hip_stream", c_vp), ("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", c_vp)]


def torch_allocator(device=0, stream=None):
    """(alloc, free) callbacks that take device memory from PyTorch's caching allocator on
    `device` and `stream` (a hipStream_t as int, or None for the current stream).  Keep the
    returned pair alive as long as the object that uses it."""
    import torch

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except Exception:   # out of memory: the library reports LX_ENOMEM
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    return ALLOC_FN(_alloc), FREE_FN(_free)


class lx_mesh(ctypes.Structure):
    _fields_ = [("n_vertices", c_i64), ("n_tets", c_i64), ("n_bfaces", c_i64), ("coords", P(c_dbl)),
                ("tets", P(c_i32)), ("bfaces", P(c_i32)), ("bface_tag", P(c_i32))]


class lx_time_law(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("pad", c_i32), ("p", c_dbl * 8)]


class lx_profile(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("pad", c_i32), ("center", c_dbl * 3), ("normal", c_dbl * 3), ("radius", c_dbl)]


class lx_boundary(ctypes.Structure):
    _fields_ = [("type", c_i32), ("n_tags", c_i32), ("tags", P(c_i32)), ("theta", c_dbl), ("law", lx_time_law),
                ("profile", lx_profile), ("resistance", c_dbl), ("backflow", c_dbl)]


class lx_riis(ctypes.Structure):
    _fields_ = [("center", c_dbl * 3), ("normal", c_dbl * 3), ("outer_radius", c_dbl),
                ("orifice_radius", lx_time_law), ("R", c_dbl), ("eps", c_dbl)]


class lx_problem(ctypes.Structure):
    _fields_ = [("fe", c_i32), ("bdf_order", c_i32), ("dt", c_dbl), ("t0", c_dbl), ("rho", c_dbl), ("mu", c_dbl),
                ("diffusion", c_i32), ("stab", c_i32), ("C_r", c_dbl), ("semi_implicit", c_i32), ("ale", c_i32),
                ("forcing", c_i32), ("n_bc", c_i32), ("bc", P(lx_boundary)), ("n_riis", c_i32),
                ("n_ale_tags", c_i32), ("riis", P(lx_riis)), ("ale_tags", P(c_i32)), ("ale_law", lx_time_law),
                ("lifting", c_i32), ("stiffening", c_i32), ("lift_E", c_dbl), ("lift_nu", c_dbl),
                ("stiff_p", c_dbl * 2)]


class lx_solver(ctypes.Structure):
    _fields_ = [("precision", c_i32), ("restart", c_i32), ("max_iters", c_i32), ("max_ir", c_i32),
                ("rtol", c_dbl), ("ir_rtol", c_dbl), ("inner_rtol", c_dbl), ("deterministic", c_i32),
                ("collect_timing", c_i32), ("schur_degree", c_i32), ("asm_fp64", c_i32), ("schur_ratio", c_dbl),
                ("precond", c_i32), ("f_degree", c_i32), ("amg_degree", c_i32), ("amg_cycle", c_i32), ("f_ratio", c_dbl),
                ("amg_ratio", c_dbl), ("amg_coarse_cycle", c_i32)]


class lx_sizes(ctypes.Structure):
    _fields_ = [("n_vertices", c_i64), ("n_tets", c_i64), ("n_u_nodes", c_i64), ("n_dofs", c_i64),
                ("n_blocks", c_i64), ("device_bytes", c_i64), ("n_edges", c_i64), ("n_scalar_nnz", c_i64),
                ("amg_levels", c_i32), ("amg_tail_level", c_i32),
                ("amg_level_rows", c_i64 * 8), ("amg_level_nnz", c_i64 * 8)]


class lx_step_stats(ctypes.Structure):
    _fields_ = [("gmres_iters", c_i32), ("ir_iters", c_i32), ("restarts", c_i32), ("converged", c_i32),
                ("rel_residual", c_dbl), ("t_step_ms", c_dbl), ("t_assembly_ms", c_dbl), ("t_solve_ms", c_dbl),
                ("spmv_ms", c_dbl), ("spmv_calls", c_i64), ("asm_ms", c_dbl), ("asm_calls", c_i64),
                ("resid_ms", c_dbl), ("resid_calls", c_i64), ("newton_iters", c_i32), ("lift_iters", c_i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lx_server_cfg(ctypes.Structure):
    _fields_ = [("device", lx_device), ("hbm_budget_bytes", c_i64), ("max_active", c_i32), ("n_streams", c_i32)]


class lx_request(ctypes.Structure):
    _fields_ = [("mesh", lx_mesh), ("problem", lx_problem), ("solver", lx_solver), ("n_steps", c_i32),
                ("pad", c_i32)]


class lx_request_status(ctypes.Structure):
    _fields_ = [("state", c_i32), ("steps_done", c_i32), ("footprint_bytes", c_i64)]


class lx_latency_stats(ctypes.Structure):
    _fields_ = [("admit_wait_ms", c_dbl), ("setup_ms", c_dbl), ("total_ms", c_dbl), ("step_p50_ms", c_dbl), ("step_p99_ms", c_dbl),
                ("n_steps", c_i32), ("gmres_iters", c_i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SIGNATURES = {
    "lx_last_error": (ctypes.c_char_p, []),
    "lx_sim_create": (c_i32, [P(lx_device), P(lx_mesh), P(lx_problem), P(lx_solver), P(c_vp)]),
    "lx_sim_query": (c_i32, [c_vp, P(lx_sizes)]),
    "lx_sim_get_edges": (c_i32, [c_vp, c_vp]),
    "lx_sim_set_state": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    "lx_sim_set_time": (c_i32, [c_vp, c_dbl]),
    "lx_sim_set_dirichlet_values": (c_i32, [c_vp, c_i32, c_vp]),
    "lx_sim_set_neumann_traction": (c_i32, [c_vp, c_i32, c_vp]),
    "lx_sim_set_forcing": (c_i32, [c_vp, c_vp]),
    "lx_sim_set_ale_displacement": (c_i32, [c_vp, c_vp]),
    "lx_sim_set_boundary_displacement": (c_i32, [c_vp, c_vp]),
    "lx_sim_step": (c_i32, [c_vp, P(lx_step_stats)]),
    "lx_sim_get_solution": (c_i32, [c_vp, c_vp, c_vp, P(c_dbl)]),
    "lx_sim_state_size": (c_i32, [c_vp, P(c_i64)]),
    "lx_sim_get_state": (c_i32, [c_vp, c_vp, c_i64]),
    "lx_sim_restore_state": (c_i32, [c_vp, c_vp, c_i64]),
    "lx_sim_debug_export": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lx_sim_debug_export_p2": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lx_sim_debug_residual": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "lx_sim_boundary_integrals": (c_i32, [c_vp, c_i32, c_vp]),
    "lx_sim_residual_noalloc": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "lx_sim_destroy": (None, [c_vp]),
    "lx_server_create": (c_i32, [P(lx_server_cfg), P(c_vp)]),
    "lx_server_submit": (c_i32, [c_vp, P(lx_request), P(c_i64)]),
    "lx_server_tick": (c_i32, [c_vp, P(c_i32)]),
    "lx_server_poll": (c_i32, [c_vp, c_i64, P(lx_request_status)]),
    "lx_server_result": (c_i32, [c_vp, c_i64, c_vp, c_vp, P(lx_latency_stats)]),
    "lx_server_destroy": (None, [c_vp]),
}

_LIB = None


def lib():
    """Load liblxns.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblxns.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        # PyTorch ships its own HIP runtime under the same soname as ROCm's.  Loaded
        # first, it is the process's runtime and the library binds to it, so torch's
        # streams and memory are valid in the library; loaded after the library, it
        # would be a second runtime in the process, which then finds no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(status):
    if status != LX_OK:
        raise LxError(status, lib().lx_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(P(c_dbl))


def _ip(a):
    return a.ctypes.data_as(P(c_i32))


def _law(l):
    t = lx_time_law()
    t.kind = LAW[l.kind]
    for i, v in enumerate(l.p):
        t.p[i] = v
    return t


class _Marshal:
    """C structs for a mesh + problem + solver, holding the arrays they point to."""

    def __init__(self, mesh, prob, solver):
        self.keep = []
        co = np.ascontiguousarray(mesh.coords, dtype=np.float64)
        te = np.ascontiguousarray(mesh.tets, dtype=np.int32)
        bf = np.ascontiguousarray(mesh.bfaces, dtype=np.int32)
        bt = np.ascontiguousarray(mesh.btags, dtype=np.int32)
        self.keep += [co, te, bf, bt]
        self.mesh = lx_mesh(co.shape[0], te.shape[0], bt.shape[0], _dp(co), _ip(te), _ip(bf), _ip(bt))
        bcs = (lx_boundary * max(1, len(prob.bcs)))()
        for i, b in enumerate(prob.bcs):
            tags = np.ascontiguousarray(b.tags, dtype=np.int32)
            self.keep.append(tags)
            bcs[i].type = BC[b.type]
            bcs[i].n_tags = len(tags)
            bcs[i].tags = _ip(tags)
            bcs[i].theta = b.theta
            bcs[i].law = _law(b.law)
            pr = lx_profile()
            pr.kind = PROFILE[b.profile.kind]
            pr.center[:] = list(b.profile.center)
            pr.normal[:] = list(b.profile.normal)
            pr.radius = b.profile.radius
            bcs[i].profile = pr
            bcs[i].resistance = getattr(b, "resistance", 0.0)
            bcs[i].backflow = getattr(b, "backflow", 0.0)
        rs = (lx_riis * max(1, len(prob.valves)))()
        for i, v in enumerate(prob.valves):
            rs[i].center[:] = list(v.center)
            rs[i].normal[:] = list(v.normal)
            rs[i].outer_radius = v.outer_radius
            rs[i].orifice_radius = _law(v.orifice)
            rs[i].R = v.R
            rs[i].eps = v.eps
        at = np.ascontiguousarray(prob.ale_tags if prob.ale_tags else [0], dtype=np.int32)
        self.keep += [bcs, rs, at]
        p = lx_problem()
        p.fe = FE[prob.fe]
        p.bdf_order = prob.bdf_order
        p.dt, p.t0, p.rho, p.mu = prob.dt, prob.t0, prob.rho, prob.mu
        p.diffusion = DIFF[prob.diffusion]
        p.stab = STAB[prob.stab]
        p.C_r = prob.c_r() if hasattr(prob, "c_r") else prob.C_r
        p.semi_implicit = 0 if getattr(prob, "implicit", False) else 1
        p.ale = int(bool(prob.ale))
        p.forcing = int(bool(prob.forcing))
        p.n_bc = len(prob.bcs)
        p.bc = bcs
        p.n_riis = len(prob.valves)
        p.riis = rs
        p.n_ale_tags = len(prob.ale_tags) if prob.ale else 0
        p.ale_tags = _ip(at)
        p.ale_law = _law(prob.ale_law)
        p.lifting = LIFT[getattr(prob, "lifting", "harmonic")]
        p.stiffening = STIFF[getattr(prob, "stiffening", "none")]
        p.lift_E = float(getattr(prob, "lift_E", 1.0))
        p.lift_nu = float(getattr(prob, "lift_nu", 0.3))
        p.stiff_p[:] = [float(v) for v in getattr(prob, "stiff_p", (1.0, 1.0))]
        self.problem = p
        s = lx_solver()
        s.precision = PREC[solver.precision]
        s.restart = solver.restart
        s.max_iters = solver.max_iters
        s.max_ir = solver.max_ir
        s.rtol, s.ir_rtol, s.inner_rtol = solver.rtol, solver.ir_rtol, solver.inner_rtol
        s.deterministic = int(bool(getattr(solver, "deterministic", True)))
        s.collect_timing = max(0, int(getattr(solver, "collect_timing", 0)))
        s.schur_degree = int(getattr(solver, "schur_degree", 8))
        s.schur_ratio = float(getattr(solver, "schur_ratio", 100.0))
        s.asm_fp64 = int(bool(getattr(solver, "asm_fp64", False)))
        s.precond = PRECOND[getattr(solver, "precond", "amg")]
        s.f_degree = int(getattr(solver, "f_degree", 0))
        s.amg_degree = int(getattr(solver, "amg_degree", 0))
        s.amg_cycle = int(getattr(solver, "amg_cycle", 0))
        s.f_ratio = float(getattr(solver, "f_ratio", 0.0))
        s.amg_ratio = float(getattr(solver, "amg_ratio", 0.0))
        s.amg_coarse_cycle = int(getattr(solver, "amg_coarse_cycle", 0))
        self.solver = s


class Sim:
    """One simulation on one device (lx_sim_*)."""

    def __init__(self, mesh, prob, solver, device=0, stream=None, allocator=None):
        """allocator: None (the library's hipMalloc) or an (alloc, free) pair of callbacks such as
        torch_allocator(device, stream), kept alive with the object."""
        L = lib()
        self.m = _Marshal(mesh, prob, solver)
        self.nv = mesh.coords.shape[0]
        self._allocator = allocator
        dev = lx_device(device, stream)
        if allocator is not None:
            dev.alloc, dev.free = allocator
        h = c_vp()
        check(L.lx_sim_create(ctypes.byref(dev), ctypes.byref(self.m.mesh), ctypes.byref(self.m.problem),
                              ctypes.byref(self.m.solver), ctypes.byref(h)))
        self.h = h
        self.nu = self.query()["n_u_nodes"]   # velocity nodes (P2-P1: vertices, then edges())

    def close(self):
        if getattr(self, "h", None):
            lib().lx_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self):
        s = lx_sizes()
        check(lib().lx_sim_query(self.h, ctypes.byref(s)))
        out = {}
        for k, _ in s._fields_:
            v = getattr(s, k)
            out[k] = list(v) if isinstance(v, ctypes.Array) else v
        return out

    def set_state(self, level, u, p, d=None):
        u = np.ascontiguousarray(u, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        dd = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
        check(lib().lx_sim_set_state(self.h, level, u.ctypes.data, p.ctypes.data,
                                     None if dd is None else dd.ctypes.data))

    def set_time(self, t):
        check(lib().lx_sim_set_time(self.h, t))

    def set_dirichlet_values(self, bc, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        check(lib().lx_sim_set_dirichlet_values(self.h, bc, g.ctypes.data))

    def set_neumann_traction(self, bc, h):
        h = np.ascontiguousarray(h, dtype=np.float64)
        check(lib().lx_sim_set_neumann_traction(self.h, bc, h.ctypes.data))

    def set_forcing(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        check(lib().lx_sim_set_forcing(self.h, f.ctypes.data))

    def set_ale_displacement(self, d):
        d = np.ascontiguousarray(d, dtype=np.float64)
        check(lib().lx_sim_set_ale_displacement(self.h, d.ctypes.data))

    def set_boundary_displacement(self, d):
        d = np.ascontiguousarray(d, dtype=np.float64)
        check(lib().lx_sim_set_boundary_displacement(self.h, d.ctypes.data))

    def step(self, raise_on_fail=True):
        st = lx_step_stats()
        rc = lib().lx_sim_step(self.h, ctypes.byref(st))
        if rc != LX_OK and raise_on_fail:
            check(rc)
        d = st.as_dict()
        d["status"] = rc
        return d

    def edges(self):
        """[n_edges][2] caller vertex ids of the P2 edge nodes, in node order after the vertices."""
        ne = self.query()["n_edges"]
        e = np.zeros((ne, 2), dtype=np.int32)
        if ne:
            check(lib().lx_sim_get_edges(self.h, e.ctypes.data))
        return e

    def export_p2(self):
        """(rows, cols, vals, rhs) of the coming step's P2-P1 system, scalar COO in the caller's
        dof numbering (velocity 3 node + c, pressure 3 nu + vertex)."""
        q = self.query()
        n = q["n_scalar_nnz"]
        rows = np.zeros(n, dtype=np.int32)
        cols = np.zeros(n, dtype=np.int32)
        vals = np.zeros(n)
        rhs = np.zeros(q["n_dofs"])
        check(lib().lx_sim_debug_export_p2(self.h, rows.ctypes.data, cols.ctypes.data, vals.ctypes.data,
                                           rhs.ctypes.data))
        return rows, cols, vals, rhs

    def get_state(self):
        """Checkpoint blob (bytes) of the full time-stepping state."""
        n = c_i64()
        check(lib().lx_sim_state_size(self.h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        check(lib().lx_sim_get_state(self.h, buf, n.value))
        return buf.raw

    def restore_state(self, blob):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        check(lib().lx_sim_restore_state(self.h, buf, len(blob)))

    def solution(self):
        u = np.zeros((self.nu, 3))
        p = np.zeros(self.nv)
        t = c_dbl()
        check(lib().lx_sim_get_solution(self.h, u.ctypes.data, p.ctypes.data, ctypes.byref(t)))
        return u, p, t.value

    def export(self):
        """(brow, bcol, vals[nblk][4][4], rhs[nv][4]) of the coming step, caller numbering."""
        nb = self.query()["n_blocks"]
        br = np.zeros(nb, dtype=np.int32)
        bc = np.zeros(nb, dtype=np.int32)
        vals = np.zeros((nb, 4, 4))
        rhs = np.zeros((self.nv, 4))
        check(lib().lx_sim_debug_export(self.h, br.ctypes.data, bc.ctypes.data, vals.ctypes.data, rhs.ctypes.data))
        return br, bc, vals, rhs

    def boundary_integrals(self, bc_index):
        """(int (u - u_ALE) . n, int p, area) over condition bc_index's faces, last step."""
        out = np.zeros(3)
        check(lib().lx_sim_boundary_integrals(self.h, int(bc_index), out.ctypes.data))
        return out

    def residual(self, u, p):
        u = np.ascontiguousarray(u, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        r = np.zeros((self.nv, 4))
        check(lib().lx_sim_debug_residual(self.h, u.ctypes.data, p.ctypes.data, r.ctypes.data))
        return r


def residual_noalloc(sim, u_dev, p_dev, r_dev):
    """lx_sim_residual_noalloc on device pointers (ints): u [nv][3], p [nv], r [nv][4], caller
    numbering; queued on the simulation's stream."""
    check(lib().lx_sim_residual_noalloc(sim.h, c_vp(u_dev), c_vp(p_dev), c_vp(r_dev)))


class Server:
    """Continuous-batching request server (lx_server_*)."""

    def __init__(self, hbm_budget_bytes, max_active=16, n_streams=8, device=0):
        cfg = lx_server_cfg(lx_device(device, None), int(hbm_budget_bytes), int(max_active), int(n_streams))
        h = c_vp()
        check(lib().lx_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self._keep = {}
        self._nv = {}

    def submit(self, mesh, prob, solver, n_steps):
        m = _Marshal(mesh, prob, solver)
        req = lx_request(m.mesh, m.problem, m.solver, int(n_steps), 0)
        t = c_i64()
        check(lib().lx_server_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = m
        self._nv[t.value] = mesh.coords.shape[0]
        return t.value

    def tick(self):
        n = c_i32()
        check(lib().lx_server_tick(self.h, ctypes.byref(n)))
        return n.value

    def poll(self, ticket):
        st = lx_request_status()
        check(lib().lx_server_poll(self.h, ticket, ctypes.byref(st)))
        return {"state": REQ_STATE[st.state], "steps_done": st.steps_done, "footprint_bytes": st.footprint_bytes}

    def result(self, ticket):
        nv = self._nv[ticket]
        u = np.zeros((nv, 3))
        p = np.zeros(nv)
        lat = lx_latency_stats()
        check(lib().lx_server_result(self.h, ticket, u.ctypes.data, p.ctypes.data, ctypes.byref(lat)))
        self._keep.pop(ticket, None)
        return u, p, lat.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib().lx_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
