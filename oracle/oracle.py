"""FP64 CPU oracle: time loop, boundary data and linear solve around the C element
routines in lxo.c.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU baseline, never by the device library or its binding.

What it computes per step (paper Sec. 2.3 and 2.4; readings listed in lxo.c):
  1. t^{n+1} = t^n + dt; BDF order min(sigma, number of stored levels); alpha,
     u_BDF = sum beta_i u^{n-i}, u_EXT = sum gamma_i u^{n-i}, p_EXT likewise.
  2. ALE (if on): boundary displacement at t^{n+1}, harmonic extension on the
     reference mesh, x^{n+1} = x^ + d^{n+1}, u_ALE = (alpha d^{n+1} - d_BDF)/dt.
  3. Element assembly on x^{n+1} (lxo.c), Neumann face terms, backflow
     stabilisation and resistance conditions (the latter a rank-1 term
     C_R w w^T kept beside the sparse matrix), Dirichlet rows.
  4. Solve A x = b exactly (dense LU, or sparse LU), or by the oracle's own
     GMRES + SIMPLE for large systems; rotate the history.
  Fully implicit formulation (Sec. 2.3, u* = u^{n+1} - u_ALE, implicit LES term):
  steps 3-4 become Newton's method (Sec. 2.4) on the nonlinear residual, its
  Jacobian by the complex step, each update solved exactly, from the step's
  starting state until ||R|| <= newton_rtol ||R_0||.  Outflow conditions are
  linear in the new state as in step 3 (backflow coefficient at u_EXT): their
  matrix terms join the Jacobian and -R gains b_out - (B + C_R w w^T) x.
"""
import ctypes
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

# BDF tables (constant step): alpha, beta (u_BDF weights), gamma (u_EXT weights)
BDF = {
    1: (1.0, [1.0], [1.0]),
    2: (1.5, [2.0, -0.5], [2.0, -1.0]),
    3: (11.0 / 6.0, [3.0, -1.5, 1.0 / 3.0], [3.0, -3.0, 1.0]),
}

STAB = {"none": 0, "supg_pspg": 1, "vms_les": 2}


class OrcParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("sigma", ctypes.c_double), ("dt", ctypes.c_double),
                ("rho", ctypes.c_double), ("mu", ctypes.c_double), ("C_r", ctypes.c_double),
                ("stab", ctypes.c_int32), ("symgrad", ctypes.c_int32), ("n_riis", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("riis", ctypes.POINTER(ctypes.c_double))]


def lib_path():
    return os.path.join(_HERE, "liblxo.so")


def build(quiet=True):
    """Compile lxo.c into liblxo.so with gcc (plain C, -O2, OpenMP loops)."""
    import subprocess
    src = os.path.join(_HERE, "lxo.c")
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared", "-o", lib_path(), src,
           "-lm"]
    subprocess.check_call(cmd)


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path()):
            build()
        L = ctypes.CDLL(lib_path())
        P, D, I64, I32 = ctypes.POINTER, ctypes.c_double, ctypes.c_int64, ctypes.c_int32
        vp = ctypes.c_void_p
        L.orc_element_p1.restype = D
        L.orc_element_p1.argtypes = [vp] * 7 + [P(OrcParams), vp, vp]
        L.orc_vertex_graph.restype = I64
        L.orc_vertex_graph.argtypes = [I64, I64, I64, vp, vp, vp]
        L.orc_pattern_p1.restype = None
        L.orc_pattern_p1.argtypes = [I64, vp, vp, vp, vp]
        L.orc_assemble_p1.restype = I64
        L.orc_assemble_p1.argtypes = [I64, I64] + [vp] * 8 + [P(OrcParams)] + [vp] * 4
        L.orc_neumann_p1.restype = None
        L.orc_neumann_p1.argtypes = [I64, I64, vp, vp, vp, vp]
        L.orc_flux_weights.restype = None
        L.orc_flux_weights.argtypes = [I64, vp, vp, vp, vp]
        L.orc_backflow_p1.restype = None
        L.orc_backflow_p1.argtypes = [I64, vp, vp, vp, vp, D, vp, vp, vp, vp]
        L.orc_boundary_integrals.restype = None
        L.orc_boundary_integrals.argtypes = [I64, vp, vp, vp, vp, vp, vp, vp]
        L.orc_newton_element_p1.restype = D
        L.orc_newton_element_p1.argtypes = [vp] * 7 + [P(OrcParams), D, vp, vp]
        L.orc_assemble_p1_newton.restype = I64
        L.orc_assemble_p1_newton.argtypes = [I64, I64] + [vp] * 8 + [P(OrcParams)] + [vp] * 4
        L.orc_dirichlet_rows.restype = None
        L.orc_dirichlet_rows.argtypes = [I64, vp, vp, vp, vp, vp, vp]
        L.orc_gmres_simple.restype = I64
        L.orc_gmres_simple.argtypes = [I64, vp, vp, vp, vp, vp, I32, D, I64, I32, D, P(D)]
        L.orc_tau.restype = None
        L.orc_tau.argtypes = [P(OrcParams), vp, vp, vp, D, P(D), P(D)]
        L.orc_delta.restype = D
        L.orc_delta.argtypes = [D, D]
        L.orc_valve_distance.restype = D
        L.orc_valve_distance.argtypes = [vp, vp]
        L.orc_quad_p1.restype = None
        L.orc_quad_p1.argtypes = [vp, vp]
        L.orc_lifting_element.restype = D
        L.orc_lifting_element.argtypes = [vp, I32, D, D, D, vp]
        L.orc_lifting_matrix.restype = None
        L.orc_lifting_matrix.argtypes = [I64, vp, vp, I32, D, D, vp, vp, vp, vp]
        L.orc_point_triangle_distance.restype = D
        L.orc_point_triangle_distance.argtypes = [vp, vp, vp, vp]
        L.orc_boundary_distance.restype = None
        L.orc_boundary_distance.argtypes = [I64, vp, vp, I64, vp, vp]
        L.orc_set_threads.restype = I32
        L.orc_set_threads.argtypes = [I32]
        _LIB = L
    return _LIB


def _p(a):
    """Pointer argument for the C routines; the pointer object holds a reference to the
    array, so a temporary passed inline stays alive for the duration of the call."""
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def set_threads(n):
    """Threads of the oracle's parallel loops (0: leave as is); returns the count in effect.
    Results do not depend on it."""
    return int(lib().orc_set_threads(int(n)))


# ---------------------------------------------------------------- boundary data

def time_law(law, t):
    """g(t) of Sec. 2.2.1: constant, pulsatile, sinusoidal ramp, and an open-then-close
    pair of ramps (optionally periodic) for valve schedules; also linear g0 + g1 t and
    sine A sin(w t + phi), the time factors of the rigid-translation and ALE-Beltrami
    mesh motions (Appendix A)."""
    k, p = law.kind, law.p
    if k == "constant":
        return p[0]
    if k == "linear":
        return p[0] + p[1] * t
    if k == "sine":
        return p[0] * np.sin(p[1] * t + p[2])
    if k == "pulsatile":
        gmin, gmax, T = p[:3]
        return gmin + (gmax - gmin) * 0.5 * (1.0 - np.cos(2.0 * np.pi * t / T))
    if k == "ramp":
        g0, g1, t0, tL = p[:4]
        if t < t0:
            return g0
        if t < t0 + tL:
            return g0 + 0.5 * (g1 - g0) * (1.0 - np.cos(np.pi * (t - t0) / tL))
        return g1
    if k == "ramp2":
        g0, g1, to, do, tc, dc, per = p[:7]
        tau = np.fmod(t, per) if per > 0 else t
        if tau < to:
            return g0
        if tau < to + do:
            return g0 + 0.5 * (g1 - g0) * (1.0 - np.cos(np.pi * (tau - to) / do))
        if tau < tc:
            return g1
        if tau < tc + dc:
            return g1 + 0.5 * (g0 - g1) * (1.0 - np.cos(np.pi * (tau - tc) / dc))
        return g0
    raise ValueError(k)


def profile_values(prof, X):
    """s(x) at points X (Sec. 2.2.1): parabolic -2 (R^2 - r^2)/(pi R^4) n with r the
    distance to the profile centre, or uniform -n."""
    n = np.asarray(prof.normal, float)
    if prof.kind == "uniform":
        return np.broadcast_to(-n, X.shape).copy()
    if prof.kind == "parabolic":
        R = prof.radius
        r2 = np.sum((X - np.asarray(prof.center, float)) ** 2, axis=1)
        return (-2.0 * (R * R - r2) / (np.pi * R ** 4))[:, None] * n[None, :]
    raise ValueError(prof.kind)


def dirichlet_sets(mesh, prob):
    """Vertex -> boundary-condition index for Dirichlet-type conditions.  No-slip wins
    over other Dirichlet data on shared vertices; otherwise the first listed wins."""
    owner = np.full(mesh.nv, -1, dtype=np.int64)
    order = [i for i, b in enumerate(prob.bcs) if b.type == "noslip"] + \
            [i for i, b in enumerate(prob.bcs) if b.type == "dirichlet"]
    for i in order:
        b = prob.bcs[i]
        faces = mesh.bfaces[np.isin(mesh.btags, b.tags)]
        vs = np.unique(faces.reshape(-1))
        vs = vs[owner[vs] < 0]
        owner[vs] = i
    return owner


# ---------------------------------------------------------------- the oracle

class OracleSim:
    """The oracle's time stepper for the P1-P1 system."""

    def __init__(self, mesh, prob, solve="auto", gmres_rtol=1e-13, restart=30, max_iters=100000,
                 schur_degree=16, schur_ratio=300.0):
        assert prob.fe == "p1p1", "P2-P1 oracle lives in OracleSimP2"
        self.mesh, self.prob = mesh, prob
        self.nv = mesh.nv
        self.xhat = np.ascontiguousarray(mesh.coords, dtype=np.float64)
        self.x = self.xhat.copy()
        self.tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
        self.solve_mode = solve
        self.gmres_rtol, self.restart, self.max_iters = gmres_rtol, restart, max_iters
        self.schur_degree, self.schur_ratio = schur_degree, schur_ratio
        self.t = prob.t0
        self.step_index = 0
        nv = self.nv
        self.u_hist = [np.zeros((nv, 3))]
        self.p_hist = [np.zeros(nv)]
        self.d_hist = [np.zeros((nv, 3))]
        self.n_levels = 0            # valid history levels (0: start from rest, counts as 1)
        self.owner = dirichlet_sets(mesh, prob)
        self.dir_nodal = {}          # bc index -> [nv][3] values at t^{n+1}
        self.neu_nodal = {}          # bc index -> [nv][3] traction at t^{n+1}
        self.forcing = None
        self.ale_shape = np.zeros((nv, 3))
        self.ale_nodal = None
        L = lib()
        self.vptr = np.zeros(nv + 1, dtype=np.int64)
        nadj = L.orc_vertex_graph(nv, mesh.nt, 4, _p(self.tets), None, None)
        self.vadj = np.zeros(nadj, dtype=np.int32)
        L.orc_vertex_graph(nv, mesh.nt, 4, _p(self.tets), _p(self.vptr), _p(self.vadj))
        nnz = 16 * nadj
        self.rowptr = np.zeros(4 * nv + 1, dtype=np.int64)
        self.col = np.zeros(nnz, dtype=np.int32)
        L.orc_pattern_p1(nv, _p(self.vptr), _p(self.vadj), _p(self.rowptr), _p(self.col))
        self.val = np.zeros(nnz)
        self.rhs = np.zeros(4 * nv)
        self.last_iters = 0
        self.last_res = 0.0

    # ---- state
    def set_state(self, level, u, p, d=None):
        while len(self.u_hist) <= level:
            self.u_hist.append(np.zeros((self.nv, 3)))
            self.p_hist.append(np.zeros(self.nv))
            self.d_hist.append(np.zeros((self.nv, 3)))
        self.u_hist[level] = np.array(u, dtype=np.float64).reshape(self.nv, 3)
        self.p_hist[level] = np.array(p, dtype=np.float64).reshape(self.nv)
        if d is not None:
            self.d_hist[level] = np.array(d, dtype=np.float64).reshape(self.nv, 3)
        self.n_levels = max(self.n_levels, level + 1)
        if level == 0 and self.prob.ale:
            self.x = self.xhat + self.d_hist[0]

    def set_dirichlet_values(self, bc_index, g):
        self.dir_nodal[bc_index] = np.array(g, dtype=np.float64).reshape(self.nv, 3)

    def set_neumann_traction(self, bc_index, h):
        self.neu_nodal[bc_index] = np.array(h, dtype=np.float64).reshape(self.nv, 3)

    def set_forcing(self, f):
        self.forcing = np.array(f, dtype=np.float64).reshape(self.nv, 3)

    def set_ale_displacement(self, d):
        self.ale_shape = np.array(d, dtype=np.float64).reshape(self.nv, 3)
        self.ale_nodal = None

    def set_boundary_displacement(self, d):
        """Boundary displacement at t^{n+1} (used from now on instead of law(t) * shape)."""
        self.ale_nodal = np.array(d, dtype=np.float64).reshape(self.nv, 3)

    # ---- one step
    def _coeffs(self):
        order = min(self.prob.bdf_order, max(self.n_levels, 1))
        alpha, beta, gamma = BDF[order]
        return order, alpha, beta, gamma

    def _combo(self, hist, w):
        out = np.zeros_like(hist[0])
        for i, wi in enumerate(w):
            out += wi * hist[i]
        return out

    def _ale_update(self, t1, alpha, beta):
        """Lifting of the boundary displacement on the reference mesh (Sec. 2.1.1, eq.
        (lifting)): harmonic extension or linear elasticity, with the stiffening
        coefficient per element; Dirichlet rows on the vertices of the ale_tags faces.
        Returns d^{n+1} and u_ALE."""
        from scipy.sparse.linalg import spsolve
        prob, m = self.prob, self.mesh
        dB = self.ale_nodal if self.ale_nodal is not None else time_law(prob.ale_law, t1) * self.ale_shape
        faces = m.bfaces[np.isin(m.btags, prob.ale_tags)]
        bnodes = np.unique(faces.reshape(-1))
        K = self.lifting_matrix().tolil()
        rhs = np.zeros(3 * self.nv)
        diag = K.diagonal()
        for v in bnodes:
            for c in range(3):
                r = 3 * v + c
                K.rows[r] = [r]
                K.data[r] = [diag[r]]
                rhs[r] = diag[r] * dB[v, c]
        d = spsolve(K.tocsc(), rhs).reshape(self.nv, 3)
        dbdf = self._combo(self.d_hist, beta)
        uale = (alpha * d - dbdf) / prob.dt
        return d, uale

    def lifting_alpha(self):
        """Stiffening coefficient per element (Sec. 2.1.1): 1, (J0 / J)^chi with J the
        Jacobian determinant of the map from the unit simplex to the element (6 times
        its volume), or max(d, beta)^-gamma with d the distance from the element's
        centroid to the ale_tags faces, all on the reference mesh."""
        prob, m = self.prob, self.mesh
        if prob.stiffening == "none":
            return np.ones(m.nt)
        if prob.stiffening == "jacobian":
            J0, chi = prob.stiff_p
            X = self.xhat[self.tets]
            J = np.abs(np.linalg.det(np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)))
            return (J0 / J) ** chi
        if prob.stiffening == "boundary":
            beta, gamma = prob.stiff_p
            return np.maximum(self.boundary_distance(), beta) ** (-gamma)
        raise ValueError(prob.stiffening)

    def boundary_distance(self):
        m = self.mesh
        faces = np.ascontiguousarray(m.bfaces[np.isin(m.btags, self.prob.ale_tags)], dtype=np.int32)
        dist = np.zeros(m.nt)
        lib().orc_boundary_distance(m.nt, _p(self.xhat), _p(self.tets), len(faces), _p(faces), _p(dist))
        return dist

    def lifting_matrix(self):
        """[3 nv]^2 stiffness of the lifting problem, index 3v+c, on the reference mesh."""
        from scipy.sparse import coo_matrix
        prob, m = self.prob, self.mesh
        kind = {"harmonic": 0, "elastic": 1}[prob.lifting]
        a = np.ascontiguousarray(self.lifting_alpha(), dtype=np.float64)
        n = 144 * m.nt
        rows, cols, vals = np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64), np.zeros(n)
        lib().orc_lifting_matrix(m.nt, _p(self.xhat), _p(self.tets), kind, prob.lift_E, prob.lift_nu, _p(a),
                                 _p(rows), _p(cols), _p(vals))
        return coo_matrix((vals, (rows, cols)), shape=(3 * self.nv, 3 * self.nv)).tocsr()

    def laplacian(self):
        """P1 stiffness matrix on the reference mesh: int grad phi_a . grad phi_b."""
        from scipy.sparse import coo_matrix
        X = self.xhat[self.tets]                                  # [nt][4][3]
        J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        Jinv = np.linalg.inv(J)
        vol = np.abs(np.linalg.det(J)) / 6.0
        grads = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)  # [nt][4][3]
        Ke = vol[:, None, None] * np.einsum("eaj,ebj->eab", grads, grads)
        rows = np.repeat(self.tets, 4, axis=1).reshape(-1)
        cols = np.tile(self.tets, (1, 4)).reshape(-1)
        return coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(self.nv, self.nv)).tocsr()

    def params(self, order, alpha, t1):
        prob = self.prob
        riis = []
        for v in prob.valves:
            nrm = np.asarray(v.normal, float)
            nrm = nrm / np.linalg.norm(nrm)
            riis += list(v.center) + list(nrm) + [time_law(v.orifice, t1), v.outer_radius, v.R, v.eps]
        self._riis = np.array(riis if riis else [0.0], dtype=np.float64)
        P = OrcParams(alpha=alpha, sigma=float(order), dt=prob.dt, rho=prob.rho, mu=prob.mu,
                      C_r=prob.c_r(), stab=STAB[prob.stab], symgrad=int(prob.diffusion == "symgrad"),
                      n_riis=len(prob.valves), pad=0,
                      riis=self._riis.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return P

    def assemble(self):
        """Build (A, b) of the coming step without solving.  Returns t^{n+1}."""
        L = lib()
        prob = self.prob
        t1 = self.t + prob.dt
        order, alpha, beta, gamma = self._coeffs()
        uE = self._combo(self.u_hist, gamma)
        pE = self._combo(self.p_hist, gamma)
        uB = self._combo(self.u_hist, beta)
        if prob.ale:
            d1, uA = self._ale_update(t1, alpha, beta)
            x = self.xhat + d1
        else:
            d1, uA = None, np.zeros((self.nv, 3))
            x = self.xhat
        self._pending_d = d1
        self.x_next = x
        self.uA = uA
        P = self.params(order, alpha, t1)
        self.val[:] = 0.0
        self.rhs[:] = 0.0
        f = self.forcing if prob.forcing else None
        rc = L.orc_assemble_p1(self.nv, self.mesh.nt, _p(np.ascontiguousarray(x)), _p(self.xhat),
                               _p(self.tets), _p(np.ascontiguousarray(uE)), _p(np.ascontiguousarray(uB)),
                               _p(np.ascontiguousarray(uA)), _p(np.ascontiguousarray(pE)),
                               _p(None if f is None else np.ascontiguousarray(f)), ctypes.byref(P),
                               _p(self.rowptr), _p(self.col), _p(self.val), _p(self.rhs))
        if rc != 0:
            raise RuntimeError("oracle assembly failed at element %d" % (-rc - 1))
        # Neumann terms
        for i, b in enumerate(prob.bcs):
            if b.type != "neumann":
                continue
            faces = np.ascontiguousarray(self.mesh.bfaces[np.isin(self.mesh.btags, b.tags)], dtype=np.int32)
            if b.profile.kind == "nodal":
                h = self.neu_nodal.get(i)
                if h is None:
                    continue
            else:
                hv = b.theta * time_law(b.law, t1)
                if hv == 0.0:
                    continue
                h = np.broadcast_to(-hv * np.asarray(b.profile.normal, float), (self.nv, 3))
            h = np.ascontiguousarray(h, dtype=np.float64)
            L.orc_neumann_p1(self.nv, len(faces), _p(np.ascontiguousarray(x)), _p(faces), _p(h), _p(self.rhs))
        # outflow conditions: backflow stabilisation (into the matrix) and resistance
        # conditions (right-hand side here, the rank-1 term in matrix())
        skip = np.ascontiguousarray((self.owner >= 0).astype(np.int8))
        self.rank1 = []
        for i, b in enumerate(prob.bcs):
            if b.type not in ("neumann", "resistance"):
                continue
            faces = self.bc_faces(i)
            dirv = np.ascontiguousarray(b.profile.normal, dtype=np.float64)
            xc = np.ascontiguousarray(x)
            if b.backflow > 0.0:
                L.orc_backflow_p1(len(faces), _p(xc), _p(faces), _p(dirv), _p(np.ascontiguousarray(uE)),
                                  0.5 * b.backflow * prob.rho, _p(skip), _p(self.rowptr), _p(self.col),
                                  _p(self.val))
            if b.type == "resistance":
                w = np.zeros(3 * self.nv)
                L.orc_flux_weights(len(faces), _p(xc), _p(faces), _p(dirv), _p(w))
                w_row = w.reshape(self.nv, 3).copy()
                w_row[self.owner >= 0] = 0.0
                w_row = w_row.reshape(-1)
                p0 = b.theta * time_law(b.law, t1)
                self.rhs[:3 * self.nv] += w_row * (-p0 + b.resistance * float(w @ uA.reshape(-1)))
                self.rank1.append((b.resistance, w_row, w))
        # Dirichlet rows
        rows, gvals = self.dirichlet_rows(t1, x, uA)
        L.orc_dirichlet_rows(len(rows), _p(rows), _p(gvals), _p(self.rowptr), _p(self.col),
                             _p(self.val), _p(self.rhs))
        self.dir_rows, self.dir_vals = rows, gvals
        return t1

    def dirichlet_values(self, t1, x, uA):
        """[nv][3] Dirichlet data at t^{n+1} (rows of non-Dirichlet vertices are 0)."""
        g = np.zeros((self.nv, 3))
        for i, b in enumerate(self.prob.bcs):
            vs = np.nonzero(self.owner == i)[0]
            if len(vs) == 0:
                continue
            if b.type == "noslip":
                g[vs] = uA[vs]
            elif b.profile.kind == "nodal":
                g[vs] = self.dir_nodal[i][vs]
            else:
                g[vs] = b.theta * time_law(b.law, t1) * profile_values(b.profile, x[vs])
        return g

    def dirichlet_rows(self, t1, x, uA):
        g = self.dirichlet_values(t1, x, uA)
        vs = np.nonzero(self.owner >= 0)[0]
        rows = (3 * vs[:, None] + np.arange(3)[None, :]).reshape(-1).astype(np.int64)
        return np.ascontiguousarray(rows), np.ascontiguousarray(g[vs].reshape(-1))

    def bc_faces(self, i):
        b = self.prob.bcs[i]
        return np.ascontiguousarray(self.mesh.bfaces[np.isin(self.mesh.btags, b.tags)], dtype=np.int32)

    def matrix(self, rank1=True):
        """The assembled sparse matrix; rank1: plus C_R w_row w^T of every resistance
        condition (velocity rows and columns; w_row is w with Dirichlet rows zeroed)."""
        from scipy.sparse import csr_matrix, coo_matrix
        N = 4 * self.nv
        A = csr_matrix((self.val.copy(), self.col.copy(), self.rowptr.copy()), shape=(N, N))
        if rank1:
            for cr, w_row, w in getattr(self, "rank1", []):
                r = np.nonzero(w_row)[0]
                c = np.nonzero(w)[0]
                R, Cc = np.meshgrid(r, c, indexing="ij")
                A = A + coo_matrix((cr * np.outer(w_row[r], w[c]).reshape(-1), (R.reshape(-1), Cc.reshape(-1))),
                                   shape=(N, N)).tocsr()
        return A

    def boundary_integrals(self, bc_index):
        """(int (u - u_ALE) . n, int p, area) over condition bc_index's faces on the
        configuration and with the solution of the last step."""
        b = self.prob.bcs[bc_index]
        faces = self.bc_faces(bc_index)
        out = np.zeros(3)
        uA = getattr(self, "uA", None) if self.prob.ale else None
        lib().orc_boundary_integrals(len(faces), _p(np.ascontiguousarray(self.x)), _p(faces),
                                     _p(np.ascontiguousarray(b.profile.normal, dtype=np.float64)),
                                     _p(np.ascontiguousarray(self.u_hist[0])),
                                     _p(None if uA is None else np.ascontiguousarray(uA)),
                                     _p(np.ascontiguousarray(self.p_hist[0])), _p(out))
        return out

    def solve(self, x0=None):
        N = 4 * self.nv
        mode = self.solve_mode
        if mode == "auto":
            mode = "dense" if N <= 6000 else ("direct" if N <= 150000 else "gmres")
        if mode == "dense":
            A = self.matrix().toarray()
            sol = np.linalg.solve(A, self.rhs)
            self.last_iters, self.last_res = 0, 0.0
        elif mode == "direct":
            from scipy.sparse.linalg import spsolve
            sol = spsolve(self.matrix().tocsc(), self.rhs)
            self.last_iters, self.last_res = 0, 0.0
        else:
            if getattr(self, "rank1", []):
                raise ValueError("the oracle's GMRES takes the sparse matrix only: resistance conditions need "
                                 "solve='dense' or 'direct'")
            sol = np.ascontiguousarray(x0.copy() if x0 is not None else np.zeros(N))
            res = ctypes.c_double(0.0)
            it = lib().orc_gmres_simple(self.nv, _p(self.rowptr), _p(self.col), _p(self.val),
                                        _p(self.rhs), _p(sol), self.restart, self.gmres_rtol,
                                        self.max_iters, self.schur_degree, self.schur_ratio,
                                        ctypes.byref(res))
            if it < 0:
                raise RuntimeError("oracle GMRES did not converge (res %.3e)" % res.value)
            self.last_iters, self.last_res = int(it), res.value
        return sol

    def newton_system(self, u, p):
        """Newton system at the state (u, p) of the coming step (implicit formulation): the
        Jacobian in self.val and -R in self.rhs, Neumann data included, Dirichlet rows as
        a_ii dx_i = a_ii (g_i - u_i).  Returns t^{n+1}."""
        L = lib()
        prob = self.prob
        t1 = self.t + prob.dt
        order, alpha, beta, gamma = self._coeffs()
        uB = self._combo(self.u_hist, beta)
        if getattr(self, "_newton_t1", None) != t1:
            if prob.ale:
                d1, uA = self._ale_update(t1, alpha, beta)
                x = self.xhat + d1
            else:
                d1, uA = None, np.zeros((self.nv, 3))
                x = self.xhat
            self._pending_d, self.x_next, self.uA, self._newton_t1 = d1, x, uA, t1
        x, uA = self.x_next, self.uA
        P = self.params(order, alpha, t1)
        self.val[:] = 0.0
        self.rhs[:] = 0.0
        f = self.forcing if prob.forcing else None
        rc = L.orc_assemble_p1_newton(self.nv, self.mesh.nt, _p(np.ascontiguousarray(x)), _p(self.xhat),
                                      _p(self.tets), _p(np.ascontiguousarray(u)), _p(np.ascontiguousarray(p)),
                                      _p(np.ascontiguousarray(uB)), _p(np.ascontiguousarray(uA)),
                                      _p(None if f is None else np.ascontiguousarray(f)), ctypes.byref(P),
                                      _p(self.rowptr), _p(self.col), _p(self.val), _p(self.rhs))
        if rc != 0:
            raise RuntimeError("oracle Newton assembly failed at element %d" % (-rc - 1))
        for i, b in enumerate(prob.bcs):
            if b.type != "neumann":
                continue
            faces = self.bc_faces(i)
            if b.profile.kind == "nodal":
                h = self.neu_nodal.get(i)
                if h is None:
                    continue
            else:
                hv = b.theta * time_law(b.law, t1)
                if hv == 0.0:
                    continue
                h = np.broadcast_to(-hv * np.asarray(b.profile.normal, float), (self.nv, 3))
            L.orc_neumann_p1(self.nv, len(faces), _p(np.ascontiguousarray(x)), _p(faces),
                             _p(np.ascontiguousarray(h, dtype=np.float64)), _p(self.rhs))
        # outflow conditions, both linear in u^{n+1} (the backflow coefficient is taken at
        # u_EXT, as in the semi-implicit system): the backflow matrix Bf and the resistance
        # term C_R w_row w^T join the Jacobian, and -R gains b_out - (Bf + C_R w_row w^T) x
        self.rank1 = []
        skip = np.ascontiguousarray((self.owner >= 0).astype(np.int8))
        xu = np.concatenate([u.reshape(-1), p])
        uE = self._combo(self.u_hist, gamma)
        for i, b in enumerate(prob.bcs):
            if b.type not in ("neumann", "resistance"):
                continue
            faces = self.bc_faces(i)
            dirv = np.ascontiguousarray(b.profile.normal, dtype=np.float64)
            xc = np.ascontiguousarray(x)
            if b.backflow > 0.0:
                bf = np.zeros_like(self.val)
                L.orc_backflow_p1(len(faces), _p(xc), _p(faces), _p(dirv), _p(np.ascontiguousarray(uE)),
                                  0.5 * b.backflow * prob.rho, _p(skip), _p(self.rowptr), _p(self.col), _p(bf))
                self.val += bf
                from scipy.sparse import csr_matrix
                N = 4 * self.nv
                self.rhs -= csr_matrix((bf, self.col.copy(), self.rowptr.copy()), shape=(N, N)) @ xu
            if b.type == "resistance":
                w = np.zeros(3 * self.nv)
                L.orc_flux_weights(len(faces), _p(xc), _p(faces), _p(dirv), _p(w))
                w_row = w.reshape(self.nv, 3).copy()
                w_row[self.owner >= 0] = 0.0
                w_row = w_row.reshape(-1)
                p0 = b.theta * time_law(b.law, t1)
                self.rhs[:3 * self.nv] += w_row * (-p0 + b.resistance * float(w @ uA.reshape(-1)) -
                                                   b.resistance * float(w @ u.reshape(-1)))
                self.rank1.append((b.resistance, w_row, w))
        rows, gvals = self.dirichlet_rows(t1, x, uA)
        cur = np.concatenate([u.reshape(-1), p])[rows]
        L.orc_dirichlet_rows(len(rows), _p(rows), _p(np.ascontiguousarray(gvals - cur)), _p(self.rowptr),
                             _p(self.col), _p(self.val), _p(self.rhs))
        return t1

    def step_implicit(self, newton_rtol=1e-12, max_newton=30, x0=None):
        """One step of the fully implicit formulation by Newton's method from x0 (default:
        the previous solution); the updates are solved directly.  Stops when ||R|| <=
        newton_rtol ||R_0|| or the last update is below newton_rtol ||x||.  Records the
        nonlinear residual norms in self.newton_norms."""
        nv = self.nv
        x = np.concatenate([self.u_hist[0].reshape(-1), self.p_hist[0]]) if x0 is None else np.array(x0, float)
        self._newton_t1 = None
        norms, dx = [], None
        for it in range(max_newton + 1):
            t1 = self.newton_system(x[:3 * nv].reshape(nv, 3), x[3 * nv:])
            norms.append(float(np.linalg.norm(self.rhs)))
            # converged: the residual fell by newton_rtol, or the last update was that small
            # against the state (a start already at the solution leaves only rounding)
            if norms[-1] <= newton_rtol * norms[0] or norms[-1] == 0.0 or \
                    (dx is not None and np.linalg.norm(dx) <= newton_rtol * np.linalg.norm(x)):
                break
            if it == max_newton:
                raise RuntimeError("oracle Newton did not converge: %s" % norms)
            dx = self.solve()
            x = x + dx
        self.newton_norms = norms
        u = x[:3 * nv].reshape(nv, 3).copy()
        p = x[3 * nv:].copy()
        self._commit(u, p, t1)
        return u, p

    def _commit(self, u, p, t1):
        self.u_hist = [u] + self.u_hist[: self.prob.bdf_order - 1]
        self.p_hist = [p] + self.p_hist[: self.prob.bdf_order - 1]
        if self.prob.ale:
            self.d_hist = [self._pending_d] + self.d_hist[: self.prob.bdf_order - 1]
            self.x = self.x_next
        self.n_levels = min(max(self.n_levels, 1) + 1, self.prob.bdf_order)
        self.t = t1
        self.step_index += 1

    def step(self):
        if getattr(self.prob, "implicit", False):
            return self.step_implicit()
        t1 = self.assemble()
        x0 = np.concatenate([self.u_hist[0].reshape(-1), self.p_hist[0]])
        sol = self.solve(x0)
        u = sol[:3 * self.nv].reshape(self.nv, 3).copy()
        p = sol[3 * self.nv:].copy()
        self._commit(u, p, t1)
        return u, p

    def solution(self):
        return self.u_hist[0].copy(), self.p_hist[0].copy(), self.t


def element_p1(X, Xh, uE, uB, uA, pE, f, alpha=1.0, sigma=1.0, dt=0.01, rho=1.0, mu=0.01, C_r=30.0,
               stab="vms_les", symgrad=False, valves=()):
    """Element matrix (16x16) and vector (16) of one P1 element, for unit tests.
    valves: sequence of 10-tuples (center3, normal3, r_in, r_out, R, eps)."""
    riis = np.array([x for v in valves for x in v] or [0.0], dtype=np.float64)
    P = OrcParams(alpha=alpha, sigma=sigma, dt=dt, rho=rho, mu=mu, C_r=C_r, stab=STAB[stab],
                  symgrad=int(symgrad), n_riis=len(valves), pad=0,
                  riis=riis.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (X, Xh, uE, uB, uA, pE, f)]
    Ke = np.zeros((16, 16))
    Fe = np.zeros(16)
    det = lib().orc_element_p1(*[_p(a) for a in arrs], ctypes.byref(P), _p(Ke), _p(Fe))
    return Ke, Fe, det


def newton_element_p1(X, Xh, u, p, uB, uA, f, alpha=1.0, sigma=1.0, dt=0.01, rho=1.0, mu=0.01, C_r=30.0,
                      stab="vms_les", symgrad=False, valves=(), h=0.0):
    """Residual (16) and Jacobian (16x16) of the implicit formulation on one P1 element at the
    state (u, p), for unit tests.  h: complex-step size (0: the default)."""
    riis = np.array([x for v in valves for x in v] or [0.0], dtype=np.float64)
    P = OrcParams(alpha=alpha, sigma=sigma, dt=dt, rho=rho, mu=mu, C_r=C_r, stab=STAB[stab],
                  symgrad=int(symgrad), n_riis=len(valves), pad=0,
                  riis=riis.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (X, Xh, u, p, uB, uA, f)]
    Ke = np.zeros((16, 16))
    Re = np.zeros(16)
    lib().orc_newton_element_p1(*[_p(a) for a in arrs], ctypes.byref(P), float(h), _p(Ke), _p(Re))
    return Re, Ke
