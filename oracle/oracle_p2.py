"""FP64 CPU oracle for the P2-P1 (Taylor-Hood) pair (test infrastructure only).

Same time loop as oracle.py (paper Sec. 2.3), with quadratic velocity on the
vertices and edge midpoints of each tetrahedron and linear pressure on the
vertices.  Element matrices come from orc_element_p2 in lxo.c (every entry
evaluated at every quadrature point of a 27-point conical-product rule, exact
to degree 5); they are summed into a sparse matrix with scipy.  Global
numbering: velocity node n (vertices first, then edges in the order of
`edges()`) has DOFs 3n + c; pressure vertex v has DOF 3 n_u + v.
Supported: Dirichlet/no-slip data (profiles or nodal values at P2 nodes),
constant Neumann tractions, RIIS valves; not ALE.
"""
import ctypes

import numpy as np

from .oracle import lib, _p, OrcParams, BDF, STAB, time_law, profile_values
from .errors import tet_rule

LOCAL_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def edges(tets, nv):
    """Unique edges as sorted vertex pairs (lexicographic order) and the element ->
    edge map [nt][6] in the local edge order."""
    pairs = np.stack([np.sort(tets[:, [i, j]], axis=1) for i, j in LOCAL_EDGES], axis=1)   # [nt][6][2]
    key = pairs[:, :, 0].astype(np.int64) * nv + pairs[:, :, 1]
    uniq, inv = np.unique(key.reshape(-1), return_inverse=True)
    E = np.stack([uniq // nv, uniq % nv], axis=1).astype(np.int64)
    return E, inv.reshape(-1, 6).astype(np.int64)


def _lib_p2():
    L = lib()
    if not hasattr(L, "_p2_ready"):
        vp = ctypes.c_void_p
        L.orc_elements_p2.restype = ctypes.c_int64
        L.orc_elements_p2.argtypes = [ctypes.c_int64] + [vp] * 9 + [ctypes.POINTER(OrcParams), ctypes.c_int32,
                                                                   vp, vp, vp, vp]
        L._p2_ready = True
    return L


class OracleSimP2:
    def __init__(self, mesh, prob, solve="auto"):
        assert prob.fe == "p2p1" and not prob.ale
        self.mesh, self.prob = mesh, prob
        self.nv = mesh.nv
        self.x = np.ascontiguousarray(mesh.coords, dtype=np.float64)
        self.tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
        self.E, self.tedge = edges(mesh.tets, mesh.nv)
        self.ne = len(self.E)
        self.nu = self.nv + self.ne
        self.nodes = np.ascontiguousarray(np.concatenate([mesh.tets, self.nv + self.tedge], axis=1), dtype=np.int32)
        self.xnode = np.concatenate([self.x, 0.5 * (self.x[self.E[:, 0]] + self.x[self.E[:, 1]])])
        self.qlam, self.qw = tet_rule(3)
        self.qlam = np.ascontiguousarray(self.qlam)
        self.qw = np.ascontiguousarray(self.qw)
        self.solve_mode = solve
        self.t = prob.t0
        self.u_hist = [np.zeros((self.nu, 3))]
        self.p_hist = [np.zeros(self.nv)]
        self.n_levels = 0
        self.dir_nodal = {}
        self.neu_nodal = {}
        self.forcing = None
        self._dirichlet_nodes()

    # ---- boundary node sets (vertices + edges of boundary faces)
    def face_nodes(self, tags):
        m = self.mesh
        faces = m.bfaces[np.isin(m.btags, tags)]
        if len(faces) == 0:
            return np.zeros(0, dtype=np.int64)
        key_all = self.E[:, 0] * self.nv + self.E[:, 1]
        fe = []
        for i, j in ((0, 1), (0, 2), (1, 2)):
            pr = np.sort(faces[:, [i, j]], axis=1).astype(np.int64)
            fe.append(np.searchsorted(key_all, pr[:, 0] * self.nv + pr[:, 1]))
        return np.unique(np.concatenate([faces.reshape(-1).astype(np.int64), self.nv + np.concatenate(fe)]))

    def _dirichlet_nodes(self):
        owner = np.full(self.nu, -1, dtype=np.int64)
        order = [i for i, b in enumerate(self.prob.bcs) if b.type == "noslip"] + \
                [i for i, b in enumerate(self.prob.bcs) if b.type == "dirichlet"]
        for i in order:
            ns = self.face_nodes(self.prob.bcs[i].tags)
            ns = ns[owner[ns] < 0]
            owner[ns] = i
        self.owner = owner

    # ---- state
    def set_state(self, level, u, p):
        while len(self.u_hist) <= level:
            self.u_hist.append(np.zeros((self.nu, 3)))
            self.p_hist.append(np.zeros(self.nv))
        self.u_hist[level] = np.array(u, dtype=np.float64).reshape(self.nu, 3)
        self.p_hist[level] = np.array(p, dtype=np.float64).reshape(self.nv)
        self.n_levels = max(self.n_levels, level + 1)

    def set_dirichlet_values(self, bc_index, g):
        self.dir_nodal[bc_index] = np.array(g, dtype=np.float64).reshape(self.nu, 3)

    def set_neumann_traction(self, bc_index, h):
        self.neu_nodal[bc_index] = np.array(h, dtype=np.float64).reshape(self.nu, 3)

    def set_forcing(self, f):
        self.forcing = np.array(f, dtype=np.float64).reshape(self.nu, 3)

    def _combo(self, hist, w):
        out = np.zeros_like(hist[0])
        for i, wi in enumerate(w):
            out += wi * hist[i]
        return out

    def assemble(self):
        from scipy.sparse import coo_matrix
        prob = self.prob
        t1 = self.t + prob.dt
        order = min(prob.bdf_order, max(self.n_levels, 1))
        alpha, beta, gamma = BDF[order]
        uE = np.ascontiguousarray(self._combo(self.u_hist, gamma))
        pE = np.ascontiguousarray(self._combo(self.p_hist, gamma))
        uB = np.ascontiguousarray(self._combo(self.u_hist, beta))
        riis = []
        for v in prob.valves:
            nrm = np.asarray(v.normal, float)
            nrm = nrm / np.linalg.norm(nrm)
            riis += list(v.center) + list(nrm) + [time_law(v.orifice, t1), v.outer_radius, v.R, v.eps]
        riis = np.array(riis if riis else [0.0])
        P = OrcParams(alpha=alpha, sigma=float(order), dt=prob.dt, rho=prob.rho, mu=prob.mu, C_r=prob.c_r(),
                      stab=STAB[prob.stab], symgrad=int(prob.diffusion == "symgrad"), n_riis=len(prob.valves),
                      pad=0, riis=riis.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        nt = self.mesh.nt
        Ke = np.zeros((nt, 34, 34))
        Fe = np.zeros((nt, 34))
        f = np.ascontiguousarray(self.forcing) if (prob.forcing and self.forcing is not None) else None
        rc = _lib_p2().orc_elements_p2(nt, _p(self.x), _p(self.x), _p(self.tets), _p(self.nodes), _p(uE), _p(uB),
                                       None, _p(pE), _p(f), ctypes.byref(P), len(self.qw), _p(self.qlam),
                                       _p(self.qw), _p(Ke), _p(Fe))
        if rc != 0:
            raise RuntimeError("P2 oracle: degenerate element %d" % (-rc - 1))
        dof = np.concatenate([(3 * self.nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(nt, 30),
                              3 * self.nu + self.tets], axis=1)
        N = 3 * self.nu + self.nv
        R = np.repeat(dof[:, :, None], 34, axis=2)
        C = np.repeat(dof[:, None, :], 34, axis=1)
        A = coo_matrix((Ke.reshape(-1), (R.reshape(-1), C.reshape(-1))), shape=(N, N)).tocsr()
        b = np.bincount(dof.reshape(-1), weights=Fe.reshape(-1), minlength=N)
        # constant Neumann tractions sigma n = -theta h(t) n: int phi over a face is 0
        # at its vertices and area/3 at its edge midpoints
        for i, bc in enumerate(prob.bcs):
            if bc.type != "neumann":
                continue
            if bc.profile.kind == "nodal":
                self._neumann_nodal(bc, self.neu_nodal.get(i), b)
                continue
            h = bc.theta * time_law(bc.law, t1)
            if h == 0.0:
                continue
            tr = -h * np.asarray(bc.profile.normal, float)
            faces = self.mesh.bfaces[np.isin(self.mesh.btags, bc.tags)]
            key_all = self.E[:, 0] * self.nv + self.E[:, 1]
            for fi in faces:
                a = self.x[fi[1]] - self.x[fi[0]]
                c = self.x[fi[2]] - self.x[fi[0]]
                area = 0.5 * np.linalg.norm(np.cross(a, c))
                for i0, j0 in ((0, 1), (0, 2), (1, 2)):
                    pr = sorted((fi[i0], fi[j0]))
                    n = self.nv + np.searchsorted(key_all, pr[0] * self.nv + pr[1])
                    b[3 * n:3 * n + 3] += area / 3.0 * tr
        # Dirichlet rows
        g = self.dirichlet_values(t1)
        rows = np.nonzero(self.owner >= 0)[0]
        A = A.tolil()
        for n in rows:
            for c in range(3):
                r = 3 * n + c
                aii = A[r, r]
                A.rows[r] = [r]
                A.data[r] = [aii]
                b[r] = aii * g[n, c]
        self.A = A.tocsr()
        self.b = b
        return t1

    # symmetric 6-point degree-4 rule on the triangle (Dunavant 1985), barycentric
    # (a, a, 1-2a) and permutations; weights relative to the area
    _TRI_A = (0.445948490915965, 0.091576213509771)
    _TRI_W = (0.223381589678011, 0.109951743655322)

    def _neumann_nodal(self, bc, h, b):
        """(h, v) on the faces of `bc` with h interpolated by P2 on each face."""
        if h is None:
            return
        faces = self.mesh.bfaces[np.isin(self.mesh.btags, bc.tags)]
        key_all = self.E[:, 0] * self.nv + self.E[:, 1]
        pts = []
        for a, wgt in zip(self._TRI_A, self._TRI_W):
            c = 1.0 - 2.0 * a
            for l in ((a, a, c), (a, c, a), (c, a, a)):
                pts.append((np.array(l), wgt))
        for fi in faces:
            a = self.x[fi[1]] - self.x[fi[0]]
            c = self.x[fi[2]] - self.x[fi[0]]
            area = 0.5 * np.linalg.norm(np.cross(a, c))
            en = []
            for i0, j0 in ((0, 1), (0, 2), (1, 2)):
                pr = sorted((fi[i0], fi[j0]))
                en.append(self.nv + np.searchsorted(key_all, pr[0] * self.nv + pr[1]))
            nodes = list(fi) + en                      # 3 vertices, edges (0,1), (0,2), (1,2)
            for L, wgt in pts:
                phi = np.array([L[0] * (2 * L[0] - 1), L[1] * (2 * L[1] - 1), L[2] * (2 * L[2] - 1),
                                4 * L[0] * L[1], 4 * L[0] * L[2], 4 * L[1] * L[2]])
                hq = phi @ h[nodes]
                for k, n in enumerate(nodes):
                    b[3 * n:3 * n + 3] += wgt * area * phi[k] * hq

    def dirichlet_values(self, t1):
        g = np.zeros((self.nu, 3))
        for i, bc in enumerate(self.prob.bcs):
            ns = np.nonzero(self.owner == i)[0]
            if len(ns) == 0:
                continue
            if bc.type == "noslip":
                g[ns] = 0.0
            elif bc.profile.kind == "nodal":
                g[ns] = self.dir_nodal[i][ns]
            else:
                g[ns] = bc.theta * time_law(bc.law, t1) * profile_values(bc.profile, self.xnode[ns])
        return g

    def step(self):
        t1 = self.assemble()
        N = 3 * self.nu + self.nv
        mode = self.solve_mode
        if mode == "auto":
            mode = "dense" if N <= 6000 else "direct"
        if mode == "dense":
            sol = np.linalg.solve(self.A.toarray(), self.b)
        else:
            from scipy.sparse.linalg import spsolve
            sol = spsolve(self.A.tocsc(), self.b)
        u = sol[:3 * self.nu].reshape(self.nu, 3).copy()
        p = sol[3 * self.nu:].copy()
        self.u_hist = [u] + self.u_hist[: self.prob.bdf_order - 1]
        self.p_hist = [p] + self.p_hist[: self.prob.bdf_order - 1]
        self.n_levels = min(max(self.n_levels, 1) + 1, self.prob.bdf_order)
        self.t = t1
        return u, p

    def solution(self):
        return self.u_hist[0].copy(), self.p_hist[0].copy(), self.t
