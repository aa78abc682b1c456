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
