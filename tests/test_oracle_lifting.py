"""Pins of the oracle's lifting variants (harmonic and linear-elastic extension of the
boundary displacement, Jacobian- and boundary-based stiffening): element energies in
closed form, rigid-body kernels, exact reproduction of linear and rigid boundary
motions, the stiffening laws against independent geometry, and the point-to-triangle
distance against brute force.  None of them touches the device library."""
import numpy as np
import pytest

from inputs import cube_kuhn, tube
from inputs.meshes import CUBE_TAGS, TUBE_TAGS
from inputs.problem import TimeLaw, beltrami_cube_problem
from oracle import OracleSim, lib
from oracle.oracle import _p

rng = np.random.default_rng(2024)


def rand_tet():
    while True:
        X = rng.normal(size=(4, 3))
        if abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1))) > 0.1:
            return X


def element(X, kind, E, nu, alpha):
    K = np.zeros((12, 12))
    vol = lib().orc_lifting_element(_p(np.ascontiguousarray(X)), kind, E, nu, alpha, _p(K))
    return K, vol


@pytest.mark.parametrize("kind", [0, 1])
def test_element_energy_of_linear_fields(kind):
    """d = B x on one element: d^T K d = alpha vol |B|^2 (harmonic) or
    alpha vol (E/(1+nu) |sym B|^2 + E nu/((1+nu)(1-2nu)) (tr B)^2) (elasticity)."""
    for _ in range(20):
        X = rand_tet()
        B = rng.normal(size=(3, 3))
        E, nu, alpha = rng.uniform(0.5, 3.0), rng.uniform(0.0, 0.45), rng.uniform(0.2, 5.0)
        K, vol = element(X, kind, E, nu, alpha)
        d = (X @ B.T).reshape(-1)
        vol_ref = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1))) / 6.0
        assert abs(vol - vol_ref) < 1e-13 * vol_ref
        if kind == 0:
            expect = alpha * vol_ref * np.sum(B * B)
        else:
            S = 0.5 * (B + B.T)
            expect = alpha * vol_ref * (E / (1 + nu) * np.sum(S * S) + E * nu / ((1 + nu) * (1 - 2 * nu)) * np.trace(B) ** 2)
        assert abs(d @ K @ d - expect) < 1e-11 * abs(expect)
        assert np.abs(K - K.T).max() < 1e-12 * np.abs(K).max()


def test_elastic_element_rigid_kernel():
    """Translations and infinitesimal rotations (omega x x) cost no elastic energy:
    K r = 0 for all six modes (the harmonic operator keeps only the translations)."""
    X = rand_tet()
    Ke, _ = element(X, 1, 2.0, 0.3, 1.7)
    Kh, _ = element(X, 0, 2.0, 0.3, 1.7)
    for c in range(3):
        t = np.zeros((4, 3))
        t[:, c] = 1.0
        assert np.abs(Ke @ t.reshape(-1)).max() < 1e-12 * np.abs(Ke).max()
        assert np.abs(Kh @ t.reshape(-1)).max() < 1e-12 * np.abs(Kh).max()
        w = np.zeros(3)
        w[c] = 1.0
        r = np.cross(w[None, :], X).reshape(-1)
        assert np.abs(Ke @ r).max() < 1e-12 * np.abs(Ke).max()
        assert np.abs(Kh @ r).max() > 1e-3 * np.abs(Kh).max()


def _lift(mesh, prob, shape):
    o = OracleSim(mesh, prob, solve="dense")
    o.set_ale_displacement(shape)
    d, _ = o._ale_update(prob.t0 + prob.dt, 1.0, [1.0])
    return o, d


def _cube_ale(n, lifting, stiffening="none", stiff_p=(1.0, 1.0)):
    mesh, prob = beltrami_cube_problem(n)
    prob.ale = True
    prob.ale_tags = tuple(CUBE_TAGS.values())
    prob.ale_law = TimeLaw("constant", (1.0,))
    prob.lifting, prob.lift_E, prob.lift_nu = lifting, 2.5, 0.35
    prob.stiffening, prob.stiff_p = stiffening, stiff_p
    return mesh, prob


@pytest.mark.parametrize("lifting", ["harmonic", "elastic"])
@pytest.mark.parametrize("stiffening", ["none", "jacobian"])
def test_linear_boundary_motion_lifted_exactly(lifting, stiffening):
    """With a constant stiffening coefficient (none, or Jacobian-based on the uniform
    Kuhn cube, whose elements all have one volume) a linear boundary displacement is
    lifted exactly: the interior follows the same linear map."""
    mesh, prob = _cube_ale(4, lifting, stiffening, (0.5, 1.5))
    B = rng.normal(size=(3, 3)) * 0.05
    shape = mesh.coords @ B.T
    _, d = _lift(mesh, prob, shape)
    assert np.abs(d - shape).max() < 1e-12


@pytest.mark.parametrize("lifting", ["harmonic", "elastic"])
def test_rigid_boundary_motion_lifted_exactly_with_boundary_stiffening(lifting):
    """On the jittered tube with boundary-based stiffening (a coefficient varying by
    orders of magnitude across elements), a rigid translation is lifted exactly by both
    operators and an infinitesimal rotation by the elastic one."""
    m = tube(nxy=4, nz=6, radius=1.0, length=2.0, seed=4)
    mesh, _ = m, None
    from inputs.problem import tube_problem
    prob = tube_problem(m, valve=False)
    prob.ale = True
    prob.ale_tags = (TUBE_TAGS["wall"], TUBE_TAGS["inlet"], TUBE_TAGS["outlet"])
    prob.lifting, prob.lift_E, prob.lift_nu = lifting, 1.0, 0.3
    prob.stiffening, prob.stiff_p = "boundary", (0.05, 2.0)
    o = OracleSim(m, prob, solve="dense")
    a = o.lifting_alpha()
    assert a.max() / a.min() > 10.0
    shapes = [np.tile([0.1, -0.2, 0.05], (m.nv, 1))]
    if lifting == "elastic":
        shapes.append(np.cross(np.array([0.02, -0.01, 0.03])[None, :], m.coords))
    for shape in shapes:
        _, d = _lift(m, prob, shape)
        assert np.abs(d - shape).max() < 1e-11


def test_jacobian_stiffening_law():
    """alpha = (J0 / J)^chi with J = 6 |element volume|, volumes from the coordinates."""
    m = tube(nxy=3, nz=4, radius=1.0, length=1.0, seed=8)
    from inputs.problem import tube_problem
    prob = tube_problem(m, valve=False)
    prob.stiffening, prob.stiff_p = "jacobian", (0.01, 1.3)
    o = OracleSim(m, prob, solve="dense")
    X = m.coords[m.tets]
    vol = np.abs(np.einsum("ei,ei->e", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]))) / 6.0
    assert np.abs(o.lifting_alpha() - (0.01 / (6.0 * vol)) ** 1.3).max() < 1e-12 * (0.01 / (6.0 * vol.min())) ** 1.3


def test_boundary_distance_on_the_cube():
    """With every face of the unit cube as the moving boundary, the distance of a centroid
    is its distance to the nearest of the six planes; alpha follows max(d, beta)^-gamma."""
    mesh, prob = _cube_ale(4, "harmonic", "boundary", (0.1, 1.5))
    o = OracleSim(mesh, prob, solve="dense")
    c = mesh.coords[mesh.tets].mean(axis=1)
    expect = np.minimum(c, 1.0 - c).min(axis=1)
    assert np.abs(o.boundary_distance() - expect).max() < 1e-14
    assert np.abs(o.lifting_alpha() - np.maximum(expect, 0.1) ** -1.5).max() < 1e-12


def test_point_triangle_distance_brute_force():
    """Against the minimum over a fine barycentric grid of the triangle (grid spacing
    h: the true minimum is below and within h times the longest edge)."""
    n = 400
    s, t = np.meshgrid(np.arange(n + 1) / n, np.arange(n + 1) / n)
    keep = s + t <= 1.0
    s, t = s[keep], t[keep]
    for _ in range(30):
        T = rng.normal(size=(3, 3))
        P = rng.normal(size=3) * 1.5
        pts = T[0] + s[:, None] * (T[1] - T[0]) + t[:, None] * (T[2] - T[0])
        brute = np.linalg.norm(pts - P, axis=1).min()
        d = lib().orc_point_triangle_distance(_p(P), _p(np.ascontiguousarray(T[0])), _p(np.ascontiguousarray(T[1])),
                                              _p(np.ascontiguousarray(T[2])))
        edge = max(np.linalg.norm(T[1] - T[0]), np.linalg.norm(T[2] - T[0]), np.linalg.norm(T[2] - T[1]))
        assert d <= brute + 1e-12
        assert brute - d <= 2.0 * edge / n
