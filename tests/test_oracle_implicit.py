"""Pins of the oracle's fully implicit formulation (u* = u^{n+1} - u_ALE, implicit LES
term) and its Newton's method: the residual against the independently pinned
semi-implicit element where the two coincide, the complex-step Jacobian against central
differences and (Galerkin) against the exact second difference of a quadratic residual,
exact affine solutions, and Newton's quadratic convergence.  None of them touches the
device library."""
import numpy as np
import pytest

from inputs import exact, tube
from inputs.meshes import TUBE_TAGS
from inputs.problem import tube_problem
from oracle import OracleSim, element_p1
from oracle.oracle import newton_element_p1

rng = np.random.default_rng(77)
VALVE = (0.1, 0.0, 0.2, 0.0, 0.0, 1.0, 0.3, 5.0, 50.0, 0.4)   # center, normal, r_in, r_out, R, eps


def rand_tet():
    while True:
        X = rng.normal(size=(4, 3))
        if abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1))) > 0.2:
            return X


def state():
    X = rand_tet()
    return dict(X=X, Xh=X + 0.05 * rng.normal(size=(4, 3)), u=rng.normal(size=(4, 3)), p=rng.normal(size=4),
                uB=rng.normal(size=(4, 3)), uA=0.3 * rng.normal(size=(4, 3)), f=rng.normal(size=(4, 3)))


KW = dict(alpha=1.5, sigma=2.0, dt=0.01, rho=1.1, mu=0.03, C_r=30.0)


@pytest.mark.parametrize("stab", ["none", "supg_pspg", "vms_les"])
@pytest.mark.parametrize("symgrad", [False, True])
def test_residual_equals_semi_implicit_system_at_the_extrapolated_state(stab, symgrad):
    """At (u, p) = (u_EXT, p_EXT) the implicit residual is the semi-implicit system's
    Ke x - Fe: u*, tau and the LES factor are the same there."""
    for _ in range(5):
        s = state()
        R, _ = newton_element_p1(s["X"], s["Xh"], s["u"], s["p"], s["uB"], s["uA"], s["f"], stab=stab,
                                 symgrad=symgrad, valves=(VALVE,), **KW)
        Ke, Fe, _ = element_p1(s["X"], s["Xh"], s["u"], s["uB"], s["uA"], s["p"], s["f"], stab=stab,
                               symgrad=symgrad, valves=(VALVE,), **KW)
        x = np.concatenate([s["u"].reshape(-1), s["p"]])
        ref = Ke @ x - Fe
        assert np.abs(R - ref).max() < 1e-12 * (np.abs(Ke).max() * np.abs(x).max() + np.abs(Fe).max())


@pytest.mark.parametrize("stab", ["none", "supg_pspg", "vms_les"])
def test_complex_step_jacobian_against_central_differences(stab):
    s = state()
    args = (s["X"], s["Xh"], s["u"], s["p"], s["uB"], s["uA"], s["f"])
    R, K = newton_element_p1(*args, stab=stab, valves=(VALVE,), **KW)
    h = 1e-6
    x = np.concatenate([s["u"].reshape(-1), s["p"]])
    for j in range(16):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        Rp, _ = newton_element_p1(s["X"], s["Xh"], xp[:12].reshape(4, 3), xp[12:], s["uB"], s["uA"], s["f"],
                                  stab=stab, valves=(VALVE,), **KW)
        Rm, _ = newton_element_p1(s["X"], s["Xh"], xm[:12].reshape(4, 3), xm[12:], s["uB"], s["uA"], s["f"],
                                  stab=stab, valves=(VALVE,), **KW)
        fd = (Rp - Rm) / (2 * h)
        assert np.abs(K[:, j] - fd).max() < 1e-6 * max(1.0, np.abs(K).max())


def test_galerkin_residual_is_quadratic():
    """Without stabilisation R is quadratic in the state, so R(x+v) - R(x-v) = 2 J(x) v
    exactly (to rounding) for any v."""
    s = state()
    x = np.concatenate([s["u"].reshape(-1), s["p"]])
    _, K = newton_element_p1(s["X"], s["Xh"], s["u"], s["p"], s["uB"], s["uA"], s["f"], stab="none", **KW)
    for _ in range(3):
        v = rng.normal(size=16)
        Rp, _ = newton_element_p1(s["X"], s["Xh"], (x + v)[:12].reshape(4, 3), (x + v)[12:], s["uB"], s["uA"],
                                  s["f"], stab="none", **KW)
        Rm, _ = newton_element_p1(s["X"], s["Xh"], (x - v)[:12].reshape(4, 3), (x - v)[12:], s["uB"], s["uA"],
                                  s["f"], stab="none", **KW)
        assert np.abs(Rp - Rm - 2 * K @ v).max() < 1e-11 * np.abs(Rp).max()


@pytest.mark.parametrize("name", ["couette", "stagnation", "general"])
def test_implicit_patch_affine_exact(name):
    """Exact affine Navier-Stokes solutions (with their forcing) are reproduced by the
    implicit formulation: every strong residual vanishes on them."""
    from tests.test_oracle_pins import _patch_run
    f = {"couette": exact.couette(), "stagnation": exact.stagnation(),
         "general": exact.Affine([[0.3, 0.5, -0.2], [0.1, -0.7, 0.4], [0.6, 0.2, 0.4]],
                                 u0=(0.2, -0.1, 0.3), q=(0.3, -0.2, 0.5), p0=1.0, mu=0.04)}[name]
    eu, ep = _patch_run(f, implicit=True)
    assert eu < 1e-10
    if name == "general":
        assert ep < 1e-9


def test_newton_converges_quadratically():
    """A VMS-LES tube step (RIIS valve, pulsatile inflow, random history): from the
    previous solution the nonlinear residual falls quadratically to 1e-12 of its start."""
    m = tube(nxy=4, nz=8, radius=1.0, length=2.0, seed=21)
    prob = tube_problem(m, dt=2e-3, peak=40.0, R=300.0, eps=0.3, t0=0.1)
    prob.implicit = True
    o = OracleSim(m, prob, solve="direct")
    r = np.random.default_rng(5)
    for lev in range(2):
        o.set_state(lev, r.normal(size=(m.nv, 3)) * 10.0, r.normal(size=m.nv) * 100.0)
    o.step_implicit(newton_rtol=1e-12)
    n = np.array(o.newton_norms) / o.newton_norms[0]
    print("relative Newton residuals", n)
    assert n[-1] <= 1e-12 and len(n) <= 7
    # quadratic: C_k = n[k+1] / n[k]^2 stays bounded (a linear rate q gives C_k ~ q^(1-k),
    # growing by 1/q per iteration)
    C = [n[k + 1] / n[k] ** 2 for k in range(1, len(n) - 1) if n[k + 1] > 1e-14]
    assert len(C) >= 2
    assert all(C[k + 1] <= 10.0 * C[k] for k in range(len(C) - 1)), C


def _outflow_sims(ale, stab):
    from tests._cases import tube_outflow
    case = tube_outflow(nxy=3, nz=5, kind="resistance", cr=40.0, beta=1.0, ale=ale)
    case.prob.stab = stab
    semi = OracleSim(case.mesh, case.prob, solve="dense")
    case.prob.implicit = True
    impl = OracleSim(case.mesh, case.prob, solve="dense")
    for s in (semi, impl):
        case.init(s)
    return case, semi, impl


@pytest.mark.parametrize("ale", [False, True])
def test_outflow_residual_equals_semi_implicit_system_at_the_extrapolated_state(ale):
    """Resistance (C_R w w^T, data -p0 + C_R w . u_ALE) and backflow (coefficient at u_EXT)
    are linear in the new state, so at (u_EXT, p_EXT) the implicit -R is b - A x of the
    semi-implicit system with its rank-1 term, on every row that is not a Dirichlet row
    (those hold a_ii (g_i - x_i) with each formulation's own diagonal)."""
    case, semi, impl = _outflow_sims(ale, "vms_les")
    order, alpha, beta, gamma = semi._coeffs()
    uE, pE = semi._combo(semi.u_hist, gamma), semi._combo(semi.p_hist, gamma)
    semi.assemble()
    x = np.concatenate([uE.reshape(-1), pE])
    ref = semi.rhs - semi.matrix() @ x
    impl.newton_system(uE, pE)
    free = np.ones(len(x), bool)
    free[semi.dir_rows] = False
    # the outflow terms are a visible part of these rows
    rows = np.zeros(len(x), bool)
    for i, b in enumerate(case.prob.bcs):
        if b.type == "resistance":
            rows[:3 * semi.nv] |= np.repeat(np.isin(np.arange(semi.nv), semi.bc_faces(i).reshape(-1)), 3)
    out = (semi.matrix() - semi.matrix(rank1=False)) @ x
    assert np.abs(out[rows & free]).max() > 1e-3 * np.abs(ref[rows & free]).max()
    err = np.abs(impl.rhs - ref)[free].max()
    assert err < 1e-11 * np.abs(ref).max(), err


@pytest.mark.parametrize("stab", ["none", "vms_les"])
def test_outflow_jacobian_against_differences_of_the_residual(stab):
    """The assembled Jacobian with the outflow terms (backflow block, C_R w_row w^T) is
    the derivative of -R: without stabilisation R is quadratic and the central second
    difference is exact (to rounding); with VMS-LES central differences to O(h^2).
    Rows of Dirichlet vertices are left out (their diagonal moves with the state)."""
    case, _, o = _outflow_sims(True, stab)
    r = np.random.default_rng(3)
    nv = o.nv
    x = np.concatenate([o.u_hist[0].reshape(-1), o.p_hist[0]]) + r.normal(size=4 * nv)
    o.newton_system(x[:3 * nv].reshape(nv, 3), x[3 * nv:])
    J = o.matrix()
    rows, _ = o.dirichlet_rows(o._newton_t1, o.x_next, o.uA)
    free = np.ones(4 * nv, bool)
    free[rows] = False

    def mR(y):
        o.newton_system(y[:3 * nv].reshape(nv, 3), y[3 * nv:])
        return o.rhs.copy()

    h = 1.0 if stab == "none" else 1e-6
    for _ in range(3):
        v = r.normal(size=4 * nv)
        d = -(mR(x + h * v) - mR(x - h * v)) / (2 * h)
        Jv = J @ v
        tol = (1e-11 if stab == "none" else 1e-6) * np.abs(Jv).max()
        assert np.abs(d - Jv)[free].max() < tol


def test_newton_converges_with_outflow_terms():
    """A VMS-LES tube with a resistance outlet, backflow and ALE: Newton's method with
    the outflow terms in the Jacobian still converges quadratically, to 1e-12."""
    case, _, o = _outflow_sims(True, "vms_les")
    o.step_implicit(newton_rtol=1e-12)
    n = np.array(o.newton_norms) / o.newton_norms[0]
    assert n[-1] <= 1e-12 and len(n) <= 7, n
    C = [n[k + 1] / n[k] ** 2 for k in range(1, len(n) - 1) if n[k + 1] > 1e-14]
    assert all(C[k + 1] <= 10.0 * C[k] for k in range(len(C) - 1)), C
