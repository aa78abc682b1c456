"""Pins of the oracle's outflow boundary terms: the resistance condition's flux
functional and rank-1 coupling, the inertial backflow stabilisation and the
flow-rate / pressure integrals, against closed forms, exactness properties, an
equivalent Neumann problem and the resistance law of a developed tube flow.
None of them touches the device library."""
import numpy as np
import pytest

from inputs import tube
from inputs.meshes import TUBE_TAGS
from inputs.problem import Boundary, Profile, SolverCfg, TimeLaw, tube_problem
from oracle import OracleSim, lib
from oracle.oracle import _p


def _tube(nxy=4, nz=8, length=2.0, seed=3):
    return tube(nxy=nxy, nz=nz, radius=1.0, length=length, seed=seed)


def _outlet(mesh):
    return np.ascontiguousarray(mesh.bfaces[mesh.btags == TUBE_TAGS["outlet"]], dtype=np.int32)


def _areas_centroids(X, faces):
    """Triangle areas and centroids by numpy cross products (independent of lxo.c)."""
    P = X[faces]
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    return 0.5 * np.linalg.norm(cr, axis=1), P.mean(axis=1)


def _with_outlet(mesh, kind, p0=0.0, cr=0.0, beta=0.0, **kw):
    prob = tube_problem(mesh, valve=False, **kw)
    prob.bcs[2] = Boundary(kind, (TUBE_TAGS["outlet"],), law=TimeLaw("constant", (p0,)),
                           profile=Profile("uniform", normal=(0.0, 0.0, 1.0)), resistance=cr, backflow=beta)
    return prob


def test_flux_weights_exact_for_linear_fields():
    """w . u = int_Gamma u . n exactly for a linear field u = a + B x on the flat outlet
    (P1 holds it), whatever the orientation of the listed triangles; every w_v is normal
    to the outlet, and sum_v w_v = |Gamma| n."""
    m = _tube()
    faces = _outlet(m)
    flip = faces.copy()
    flip[::2, 1], flip[::2, 2] = faces[::2, 2], faces[::2, 1]
    X = np.ascontiguousarray(m.coords)
    area, cen = _areas_centroids(X, faces)
    r = np.random.default_rng(4)
    a, B = r.normal(size=3), r.normal(size=(3, 3))
    u = a[None, :] + X @ B.T
    exact = np.sum(area * (a[2] + (cen @ B.T)[:, 2]))
    for F in (faces, np.ascontiguousarray(flip)):
        w = np.zeros(3 * m.nv)
        lib().orc_flux_weights(len(F), _p(X), _p(F), _p(np.array([0.0, 0.0, 1.0])), _p(w))
        W = w.reshape(-1, 3)
        assert abs(W[:, :2]).max() < 1e-15
        assert abs(W[:, 2].sum() - area.sum()) < 1e-13
        assert abs(w @ u.reshape(-1) - exact) < 1e-12 * max(1.0, abs(exact))


def _assembled(prob, mesh, uE):
    o = OracleSim(mesh, prob, solve="dense")
    o.set_state(0, uE, np.zeros(mesh.nv))
    o.assemble()
    return o


@pytest.mark.parametrize("sign", [-1.0, 1.0])
def test_backflow_closed_form(sign):
    """With u_EXT = sign c n on the outlet, the backflow term adds beta rho c/2 times the
    P1 face mass matrix (|F|/12 (1 + delta_ab) per triangle, computed here by hand) to
    every velocity component of the non-Dirichlet outlet rows for inflow (sign -1), and
    nothing at all for outflow (sign +1)."""
    m = _tube()
    c, beta, rho = 0.7, 0.8, 1.0
    uE = np.zeros((m.nv, 3))
    uE[:, 2] = sign * c
    A0 = _assembled(_with_outlet(m, "neumann"), m, uE).matrix(rank1=False)
    o1 = _assembled(_with_outlet(m, "neumann", beta=beta), m, uE)
    D = (o1.matrix(rank1=False) - A0).tocoo()
    if sign > 0:
        assert abs(D).max() == 0.0
        return
    faces = _outlet(m)
    area, _ = _areas_centroids(np.asarray(m.coords), faces)
    M = np.zeros((m.nv, m.nv))
    for f, ar in zip(faces, area):
        for i in f:
            for j in f:
                M[i, j] += ar / 12.0 * (2.0 if i == j else 1.0)
    dirichlet = o1.owner >= 0
    M[dirichlet, :] = 0.0
    expect = np.zeros((4 * m.nv, 4 * m.nv))
    for comp in range(3):
        expect[comp:3 * m.nv:3, comp:3 * m.nv:3] = 0.5 * beta * rho * c * M
    # the difference of two assembled matrices: rounding of the larger entries
    assert abs(D.toarray() - expect).max() < 1e-14 * abs(A0).max()
    assert abs(expect).max() > 0


@pytest.mark.parametrize("ale", [False, True])
def test_resistance_equals_neumann_at_its_pressure(ale):
    """A step with the resistance condition sigma n = -(p0 + C_R Q) n has the solution of
    the same step with the plain Neumann condition sigma n = -h n, h = p0 + C_R Q, where
    Q = int (u - u_ALE) . n is the flux of the resistance solution itself: pins the sign,
    the rank-1 coupling, the Dirichlet rows and the face orientation together.  With
    ALE, the outlet moves axially and Q is taken through the moving surface."""
    m = _tube()
    p0, cr = 3.0, 40.0
    r = np.random.default_rng(9)
    hist = r.normal(size=(m.nv, 3)), r.normal(size=m.nv)
    out = []
    for kind in ("resistance", "neumann"):
        prob = _with_outlet(m, kind, p0=p0, cr=cr, peak=30.0, dt=2e-3)
        if ale:
            prob.ale = True
            prob.ale_tags = (TUBE_TAGS["outlet"],)
            prob.ale_law = TimeLaw("linear", (0.0, 5.0))
        o = OracleSim(m, prob, solve="dense")
        if ale:
            shape = np.zeros((m.nv, 3))
            shape[:, 2] = 0.05 * m.coords[:, 2]
            o.set_ale_displacement(shape)
        o.set_state(0, *hist)
        if kind == "neumann":
            o.prob.bcs[2].law = TimeLaw("constant", (p0 + cr * q,))
        u, p = o.step()
        out.append((u, p))
        if kind == "resistance":
            q, pint, area = o.boundary_integrals(2)
    (u1, p1), (u2, p2) = out
    assert abs(q) > 1e-3
    assert np.abs(u1 - u2).max() < 1e-10 * np.abs(u1).max()
    assert np.abs(p1 - p2).max() < 1e-10 * np.abs(p1).max()


def test_resistance_law_of_developed_flow():
    """Steady inflow rate g through a tube whose outlet carries the resistance
    condition: once the flow has settled, the outlet's mean pressure is p0 + C_R Q_out
    (the normal viscous stress of a developed flow vanishes; 3% here) and Q_out is the
    inflow; a wrong sign of the coupling would give -C_R Q."""
    m = _tube(nxy=4, nz=10, length=3.0)
    p0, cr, g = 1.0, 30.0, 0.5
    prob = _with_outlet(m, "resistance", p0=p0, cr=cr, mu=0.5, dt=0.05)
    prob.bcs[1].law = TimeLaw("constant", (g,))
    prob.bdf_order = 1
    o = OracleSim(m, prob, solve="direct")
    for _ in range(12):
        o.step()
    q, pint, area = o.boundary_integrals(2)
    qin, _, _ = o.boundary_integrals(1)
    pbar = pint / area
    print("Q_out %.5f (inflow %.5f), mean outlet pressure %.5f vs p0 + C_R Q %.5f"
          % (q, -qin, pbar, p0 + cr * q))
    assert abs(q + qin) < 1e-3 * abs(qin)        # what comes in goes out
    assert abs(pbar - (p0 + cr * q)) < 0.03 * (p0 + cr * q)


def test_boundary_integrals_exact_and_convergent():
    """int p and the area are exact for a linear pressure; the inflow flux of the
    interpolated unit-flow-rate parabolic profile converges to -1 at second order."""
    errs = []
    for nxy, nz in ((4, 4), (8, 4)):
        m = _tube(nxy=nxy, nz=nz)
        X = np.ascontiguousarray(m.coords)
        faces = np.ascontiguousarray(m.bfaces[m.btags == TUBE_TAGS["inlet"]], dtype=np.int32)
        area, cen = _areas_centroids(X, faces)
        p = 2.0 + X @ np.array([0.3, -0.2, 0.1])
        rr = X[:, 0] ** 2 + X[:, 1] ** 2
        u = np.zeros((m.nv, 3))
        u[:, 2] = 2.0 * (1.0 - rr) / np.pi          # unit flow rate along +z
        out = np.zeros(3)
        lib().orc_boundary_integrals(len(faces), _p(X), _p(faces), _p(np.array([0.0, 0.0, -1.0])),
                                     _p(np.ascontiguousarray(u)), None, _p(p), _p(out))
        assert abs(out[2] - area.sum()) < 1e-13
        assert abs(out[1] - np.sum(area * (2.0 + cen @ np.array([0.3, -0.2, 0.1])))) < 1e-12
        errs.append(abs(out[0] + 1.0))
    rate = np.log2(errs[0] / errs[1])
    print("inflow flux errors %s, rate %.2f" % (errs, rate))
    assert rate > 1.8
