"""Shared problem set-ups for the device-vs-oracle parity tests.

Each case returns (mesh, problem, drive) where drive(sim, t1) pushes the nodal
data of the step ending at t1 into any object with the simulation interface
(the device binding or the oracle), and init(sim) sets the history.
"""
import numpy as np

from inputs import tube, cube_kuhn, exact
from inputs.meshes import TUBE_TAGS
from inputs.problem import (Boundary, Profile, Problem, TimeLaw, Valve, beltrami_cube_problem,
                            tube_problem)


class Case:
    def __init__(self, mesh, prob, init, drive, name):
        self.mesh, self.prob, self.init, self.drive, self.name = mesh, prob, init, drive, name


def beltrami(n=4, dt=0.01, bdf=1, stab="vms_les"):
    mesh, prob = beltrami_cube_problem(n, dt=dt, bdf_order=bdf, stab=stab)
    ex = exact.Beltrami(mu=prob.mu)
    X = mesh.coords

    def init(s):
        for lev in range(bdf):
            s.set_state(lev, ex.velocity(X, -lev * dt), ex.pressure(X, -lev * dt))

    def drive(s, t1):
        s.set_dirichlet_values(0, ex.velocity(X, t1))
        s.set_neumann_traction(1, ex.traction(X, t1, (-1, 0, 0)))

    return Case(mesh, prob, init, drive, "beltrami%d" % n)


def tube_valve(nxy=4, nz=8, length=2.0, bdf=2, stab="vms_les", diffusion="gradgrad", seed=7, random_hist=True,
               forcing=False, R=300.0, eps=0.3, peak=50.0):
    """Jittered, shuffled tube with pulsatile parabolic inflow, no-slip wall, zero-traction
    outlet and a mid-length RIIS disc; random (seeded) history so that every term is active."""
    mesh = tube(nxy=nxy, nz=nz, radius=1.0, length=length, seed=seed)
    prob = tube_problem(mesh, dt=2e-3, bdf_order=bdf, peak=peak, R=R, eps=eps, t0=0.1)
    prob.stab = stab
    prob.diffusion = diffusion
    prob.forcing = forcing
    rng = np.random.default_rng(seed)
    hist = [(rng.normal(size=(mesh.nv, 3)) * 10.0, rng.normal(size=mesh.nv) * 100.0) for _ in range(bdf)]
    f = rng.normal(size=(mesh.nv, 3)) * 5.0

    def init(s):
        if random_hist:
            for lev in range(bdf):
                s.set_state(lev, *hist[lev])

    def drive(s, t1):
        if forcing:
            s.set_forcing(f)

    return Case(mesh, prob, init, drive, "tube%dx%d_%s_bdf%d" % (nxy, nz, stab, bdf))


def oracle_matrix_from_blocks(br, bc, vals, nv):
    """Block COO (caller numbering) -> scipy CSR in the oracle's DOF numbering
    (velocity 3v+c, pressure 3nv+v)."""
    from scipy.sparse import coo_matrix
    r = np.arange(4)
    rowoff = np.where(r < 3, r, 0)
    rows = np.where(r[None, :] < 3, 3 * br[:, None] + r[None, :], 3 * nv + br[:, None])      # [nb][4]
    cols = np.where(r[None, :] < 3, 3 * bc[:, None] + r[None, :], 3 * nv + bc[:, None])
    R = np.repeat(rows[:, :, None], 4, axis=2)
    Cc = np.repeat(cols[:, None, :], 4, axis=1)
    del rowoff
    return coo_matrix((vals.reshape(-1), (R.reshape(-1), Cc.reshape(-1))), shape=(4 * nv, 4 * nv)).tocsr()


def rowwise_rel_err(A, Bm):
    """max over rows of max|A_r - B_r| / max|B_r|."""
    D = (A - Bm).tocsr()
    Bc = Bm.tocsr()
    n = Bc.shape[0]
    worst = 0.0
    dmax = np.zeros(n)
    bmax = np.zeros(n)
    for M, out in ((D, dmax), (Bc, bmax)):
        Mabs = abs(M).tocsr()
        nz = np.diff(Mabs.indptr) > 0
        out[nz] = np.maximum.reduceat(Mabs.data, Mabs.indptr[:-1][nz])
    mask = bmax > 0
    if mask.any():
        worst = float((dmax[mask] / bmax[mask]).max())
    if (~mask).any():
        worst = max(worst, float(dmax[~mask].max()))
    return worst


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def tube_ale(nxy=4, nz=8, length=2.0, bdf=2, seed=5):
    """Tube whose whole boundary contracts radially (d^ = law(t) * (-0.1 x^, -0.1 y^, 0),
    pulsatile law), no-slip wall u = u_ALE, parabolic inflow, zero-traction outlet and an
    annular RIIS valve whose orifice opens during the run."""
    mesh = tube(nxy=nxy, nz=nz, radius=1.0, length=length, seed=seed)
    prob = tube_problem(mesh, dt=2e-3, bdf_order=bdf, peak=30.0, R=200.0, eps=0.3, t0=0.0)
    prob.valves = [Valve(center=(0.0, 0.0, length / 2), normal=(0.0, 0.0, 1.0), outer_radius=10.0,
                         orifice=TimeLaw("ramp2", (0.0, 0.6, 0.0, 0.004, 1.0, 0.1, 0.0)), R=200.0, eps=0.3)]
    prob.ale = True
    prob.ale_tags = (TUBE_TAGS["wall"], TUBE_TAGS["inlet"], TUBE_TAGS["outlet"])
    prob.ale_law = TimeLaw("pulsatile", (0.0, 1.0, 0.02))
    shape = np.zeros_like(mesh.coords)
    shape[:, 0] = -0.1 * mesh.coords[:, 0]
    shape[:, 1] = -0.1 * mesh.coords[:, 1]

    def init(s):
        s.set_ale_displacement(shape)

    def drive(s, t1):
        pass

    return Case(mesh, prob, init, drive, "tube_ale%dx%d" % (nxy, nz))


def tube_ale_curved(nxy=4, nz=6, length=1.5, seed=2):
    """ALE with a non-linear boundary displacement (sinusoidal bulge), so that the
    harmonic extension is not trivially exact."""
    mesh = tube(nxy=nxy, nz=nz, radius=1.0, length=length, seed=seed)
    prob = tube_problem(mesh, dt=2e-3, bdf_order=2, peak=20.0, valve=False)
    prob.ale = True
    prob.ale_tags = (TUBE_TAGS["wall"],)
    prob.ale_law = TimeLaw("ramp", (0.0, 1.0, 0.0, 0.01))
    X = mesh.coords
    shape = np.zeros_like(X)
    bump = 0.05 * np.sin(np.pi * X[:, 2] / length)
    shape[:, 0] = bump * X[:, 0]
    shape[:, 1] = bump * X[:, 1]

    def init(s):
        s.set_ale_displacement(shape)

    def drive(s, t1):
        pass

    return Case(mesh, prob, init, drive, "tube_ale_curved")


def beltrami_ale(n=4, c=0.5, dt=0.01, nodal=True):
    """The paper's ALE verification (Appendix A) on the unit cube: Beltrami flow on a mesh
    moved by the harmonic extension of d^ = c sin(t) (sin pi x^, sin pi y^, sin pi z^)
    (tangential on every face).  nodal: the boundary displacement is set for every step
    (the lifting problem is solved each step); otherwise the sine law scales the shape."""
    from inputs.meshes import CUBE_TAGS
    mesh, prob = beltrami_cube_problem(n, dt=dt)
    prob.ale = True
    prob.ale_tags = tuple(CUBE_TAGS.values())
    prob.ale_law = TimeLaw("constant", (1.0,)) if nodal else TimeLaw("sine", (c, 1.0, 0.0))
    ex = exact.Beltrami(mu=prob.mu)
    X = mesh.coords
    D = np.sin(np.pi * X)

    def init(s):
        if not nodal:
            s.set_ale_displacement(D)
        s.set_state(0, ex.velocity(X, 0.0), ex.pressure(X, 0.0), np.zeros_like(X))

    def drive(s, t1):
        Xb = X + c * np.sin(t1) * D
        if nodal:
            s.set_boundary_displacement(c * np.sin(t1) * D)
        s.set_dirichlet_values(0, ex.velocity(Xb, t1))
        s.set_neumann_traction(1, ex.traction(Xb, t1, (-1, 0, 0)))

    return Case(mesh, prob, init, drive, "beltrami_ale%d%s" % (n, "_nodal" if nodal else ""))


def tube_outflow(nxy=4, nz=8, length=2.0, kind="resistance", cr=40.0, beta=1.0, p0=2.0, ale=False, seed=13,
                 bdf=2):
    """Tube whose outlet carries a resistance condition (p0 constant, C_R = cr) or a plain
    Neumann one, with inertial backflow stabilisation (beta); random history whose axial
    velocity is negative over part of the outlet, so that the backflow term is active;
    optional ALE with an axially stretching outlet."""
    from inputs.problem import Boundary, Profile, TimeLaw
    mesh = tube(nxy=nxy, nz=nz, radius=1.0, length=length, seed=seed)
    prob = tube_problem(mesh, dt=2e-3, bdf_order=bdf, peak=30.0, valve=False)
    prob.bcs[2] = Boundary(kind, (TUBE_TAGS["outlet"],), law=TimeLaw("constant", (p0,)),
                           profile=Profile("uniform", normal=(0.0, 0.0, 1.0)), resistance=cr, backflow=beta)
    rng = np.random.default_rng(seed)
    X = mesh.coords
    hist = []
    for _ in range(bdf):
        u = rng.normal(size=(mesh.nv, 3))
        u[:, 2] += 3.0 * np.sin(2.0 * X[:, 0]) + 1.0      # inflow and outflow across the outlet
        hist.append((u, rng.normal(size=mesh.nv) * 10.0))
    shape = np.zeros_like(X)
    shape[:, 2] = 0.05 * X[:, 2] * (1.0 + 0.3 * X[:, 0])
    if ale:
        prob.ale = True
        prob.ale_tags = (TUBE_TAGS["outlet"], TUBE_TAGS["inlet"], TUBE_TAGS["wall"])
        prob.ale_law = TimeLaw("linear", (0.0, 5.0))

    def init(s):
        for lev in range(bdf):
            s.set_state(lev, *hist[lev])
        if ale:
            s.set_ale_displacement(shape)

    def drive(s, t1):
        pass

    return Case(mesh, prob, init, drive, "tube_%s%s" % (kind, "_ale" if ale else ""))


def tube_lifting(lifting="elastic", stiffening="none", stiff_p=(1.0, 1.0), nxy=4, nz=6, length=1.5, seed=6):
    """ALE tube whose wall bulges non-linearly (d^ = law(t) 0.05 sin(pi z/L) (x, y, 0), plus an
    axial shift of the outlet) lifted by the chosen operator and stiffening; every boundary
    face carries the displacement."""
    mesh = tube(nxy=nxy, nz=nz, radius=1.0, length=length, seed=seed)
    prob = tube_problem(mesh, dt=2e-3, bdf_order=2, peak=20.0, valve=False)
    prob.ale = True
    prob.ale_tags = (TUBE_TAGS["wall"], TUBE_TAGS["inlet"], TUBE_TAGS["outlet"])
    prob.ale_law = TimeLaw("ramp", (0.0, 1.0, 0.0, 0.01))
    prob.lifting, prob.lift_E, prob.lift_nu = lifting, 2.0, 0.3
    prob.stiffening, prob.stiff_p = stiffening, stiff_p
    X = mesh.coords
    shape = np.zeros_like(X)
    bump = 0.05 * np.sin(np.pi * X[:, 2] / length)
    shape[:, 0] = bump * X[:, 0]
    shape[:, 1] = bump * X[:, 1]
    shape[:, 2] = 0.03 * X[:, 2] * X[:, 2] / length

    def init(s):
        s.set_ale_displacement(shape)

    def drive(s, t1):
        pass

    return Case(mesh, prob, init, drive, "tube_lift_%s_%s" % (lifting, stiffening))
