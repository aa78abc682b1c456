"""Device (HIP, through the C ABI) versus oracle parity.

Tolerances: FP64 matrices and residuals row-wise relative <= 1e-12; FP64 steps
(device GMRES at rtol 1e-14, oracle dense LU) relative L2 <= 1e-10 for u and p
separately (the pressure error is the solve tolerance times a conditioning
factor of about 1e3, hence the tight solve); FP32 matrices <= 2e-5 row-wise;
FP32 + FP64 refinement steps (refined to 1e-13) <= 1e-8.
"""
import numpy as np
import pytest

from inputs.problem import SolverCfg
from oracle import OracleSim
from tests._cases import beltrami, tube_valve, oracle_matrix_from_blocks, rowwise_rel_err, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


def _gpu(case, stream, precision="fp64", rtol=1e-12, **kw):
    from paper_2304_12032_amd import Sim
    sv = SolverCfg(precision=precision, rtol=rtol, ir_rtol=rtol, max_iters=20000, **kw)
    return Sim(case.mesh, case.prob, sv, device=0, stream=stream)


CASES = [
    lambda: beltrami(4),
    lambda: tube_valve(4, 8),
    lambda: tube_valve(8, 16, length=4.0, bdf=3, stab="supg_pspg", diffusion="symgrad", forcing=True),
    lambda: tube_valve(6, 10, bdf=1, stab="none"),
]
IDS = ["beltrami4", "tube_vms_bdf2", "tube8x16_supg_symgrad_bdf3_forcing", "tube_galerkin_bdf1"]


@pytest.mark.parametrize("mk", CASES, ids=IDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_matrix_parity(mk, precision, stream):
    case = mk()
    print("case", case.name, precision, flush=True)
    g = _gpu(case, stream, precision)
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
        case.drive(s, case.prob.t0 + case.prob.dt)
    br, bc, vals, rhs = g.export()
    o.assemble()
    Ag = oracle_matrix_from_blocks(br, bc, vals, case.mesh.nv)
    Ao = o.matrix()
    err = rowwise_rel_err(Ag, Ao)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert err < tol, err
    if precision == "fp64":
        nv = case.mesh.nv
        rg = np.concatenate([rhs[:, :3].reshape(-1), rhs[:, 3]])
        assert rel_l2(rg, o.rhs) < 1e-12
    g.close()


@pytest.mark.parametrize("mk", CASES, ids=IDS)
def test_matrix_free_residual(mk, stream):
    """The FP64 element-wise residual equals b - A x of the oracle's assembled system."""
    case = mk()
    print("case", case.name, flush=True)
    g = _gpu(case, stream, "fp32_ir")
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
        case.drive(s, case.prob.t0 + case.prob.dt)
    rng = np.random.default_rng(3)
    nv = case.mesh.nv
    u = rng.normal(size=(nv, 3))
    p = rng.normal(size=nv) * 10
    r = g.residual(u, p)
    o.assemble()
    x = np.concatenate([u.reshape(-1), p])
    ro = o.rhs - o.matrix() @ x
    rg = np.concatenate([r[:, :3].reshape(-1), r[:, 3]])
    scale = np.abs(o.rhs).max() + np.abs(o.matrix()).max() * np.abs(x).max()
    assert np.abs(rg - ro).max() < 1e-12 * scale
    g.close()


@pytest.mark.parametrize("mk,steps", [(CASES[0], 10), (CASES[1], 4), (CASES[2], 3)], ids=IDS[:3])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_steps_parity(mk, steps, precision, stream):
    case = mk()
    print("case", case.name, precision, flush=True)
    g = _gpu(case, stream, precision, rtol=1e-14 if precision == "fp64" else 1e-13)
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
    tol = 1e-10 if precision == "fp64" else 1e-8
    worst = (0.0, 0.0)
    for k in range(steps):
        t1 = o.t + case.prob.dt
        for s in (g, o):
            case.drive(s, t1)
        st = g.step()
        uo, po = o.step()
        ug, pg, tg = g.solution()
        assert abs(tg - o.t) < 1e-12
        eu, ep = rel_l2(ug, uo), rel_l2(pg, po)
        worst = (max(worst[0], eu), max(worst[1], ep))
        print("step", k, "iters", st["gmres_iters"], "ir", st["ir_iters"], "res %.2e" % st["rel_residual"],
              "err u %.2e p %.2e" % (eu, ep), flush=True)
    assert worst[0] < tol and worst[1] < tol, worst
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_restart_matches_continuation(precision, stream):
    """A simulation restarted from two stored levels (set_state, set_time) continues the
    uninterrupted trajectory to the solver's tolerance.  The restarted one holds only the
    levels it was given, so its first steps start from the BDF extrapolation while the
    uninterrupted one, with five and more steps behind it, extrapolates from four levels:
    the stopping test, not the start, fixes the solution."""
    case = tube_valve(4, 8)
    print("case", case.name, precision, flush=True)
    rtol = 1e-14 if precision == "fp64" else 1e-13
    a = _gpu(case, stream, precision, rtol=rtol)
    case.init(a)
    traj = []
    for k in range(9):
        t1 = a.solution()[2] + case.prob.dt
        case.drive(a, t1)
        a.step()
        traj.append(a.solution())
    a.close()
    b = _gpu(case, stream, precision, rtol=rtol)
    (u4, p4, _), (u5, p5, t5) = traj[4], traj[5]
    b.set_state(0, u5, p5)
    b.set_state(1, u4, p4)
    b.set_time(t5)
    worst = 0.0
    for k in range(6, 9):
        t1 = t5 + (k - 5) * case.prob.dt
        case.drive(b, t1)
        st = b.step()
        ub, pb, tb = b.solution()
        ua, pa, ta = traj[k]
        assert abs(tb - ta) < 1e-12
        e = max(rel_l2(ub, ua), rel_l2(pb, pa))
        worst = max(worst, e)
        print("step %d: %d iterations, difference %.2e" % (k, st["gmres_iters"], e), flush=True)
    b.close()
    assert worst < (1e-10 if precision == "fp64" else 1e-8), worst


# ------------------------------------------------------------------ C1 exactly

def test_c1_beltrami_cube_fp64(stream):
    """The Beltrami unit cube exactly as configured: 8^3 hexahedra Kuhn-split into 3,072
    tets (729 vertices, N = 2,916), P1-P1 VMS-LES, nu = 0.01, BDF1, dt = 0.01, 10 steps.
    Device GMRES at rtol 1e-14 against the oracle's dense LU, every step <= 1e-10 for u and
    p separately; the device's final errors against the exact solution equal the oracle's."""
    from oracle.errors import p1_errors
    from inputs import exact
    case = beltrami(8)
    assert case.mesh.nt == 3072 and case.mesh.nv == 729
    g = _gpu(case, stream, "fp64", rtol=1e-14)
    o = OracleSim(case.mesh, case.prob, solve="dense")
    for s in (g, o):
        case.init(s)
    worst = (0.0, 0.0)
    for k in range(10):
        t1 = o.t + case.prob.dt
        for s in (g, o):
            case.drive(s, t1)
        st = g.step()
        uo, po = o.step()
        ug, pg, _ = g.solution()
        eu, ep = rel_l2(ug, uo), rel_l2(pg, po)
        worst = (max(worst[0], eu), max(worst[1], ep))
        print("step", k, "iters", st["gmres_iters"], "res %.2e" % st["rel_residual"], "err u %.2e p %.2e" % (eu, ep),
              flush=True)
    g.close()
    assert worst[0] < 1e-10 and worst[1] < 1e-10, worst
    ex = exact.Beltrami(mu=case.prob.mu)
    eg = np.array(p1_errors(case.mesh.coords, case.mesh.tets, ug, pg, ex, o.t))
    eo = np.array(p1_errors(case.mesh.coords, case.mesh.tets, uo, po, ex, o.t))
    print("errors vs exact (u L2, u H1, p L2): device", eg, "oracle", eo, flush=True)
    assert np.abs(eg - eo).max() < 1e-8 * np.abs(eo).max()


def test_beltrami_rates_on_device(stream):
    """The device alone reproduces the expected space orders of the paper's Test I between
    h = 1/4 and h = 1/8 (e_L2^u ~ 2, e_H1^u ~ 1, e_L2^p ~ 2)."""
    import json
    import os
    from oracle.errors import p1_errors
    from inputs import exact
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "convergence_orders.json")))["p1p1"]
    errs = []
    for n in (4, 8):
        case = beltrami(n)
        g = _gpu(case, stream, "fp32_ir", rtol=1e-10)
        case.init(g)
        for _ in range(10):
            t1 = g.solution()[2] + case.prob.dt
            case.drive(g, t1)
            g.step()
        u, p, t = g.solution()
        g.close()
        errs.append(np.array(p1_errors(case.mesh.coords, case.mesh.tets, u, p, exact.Beltrami(mu=case.prob.mu), t)))
    rates = np.log2(errs[0] / errs[1])
    print("device rates", rates, flush=True)
    assert rates[0] > golden["u_L2"] - 0.15 and rates[1] > golden["u_H1"] - 0.1 and rates[2] > golden["p_L2"] - 0.2


# ------------------------------------------------- the other preconditioners / assembly

@pytest.mark.parametrize("schur_degree", [0, 16], ids=["plain_simple", "chebyshev_schur"])
@pytest.mark.parametrize("mk", [CASES[0], CASES[1]], ids=IDS[:2])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_steps_parity_cheb_schur(mk, schur_degree, precision, stream):
    """LX_PC_CHEB_SCHUR: block-Jacobi F~ with diag(S~)^{-1} (schur_degree 0, the plain
    block-Jacobi SIMPLE of Sec. 2.4) or a Chebyshev iteration on S~."""
    case = mk()
    print("case", case.name, precision, "schur_degree", schur_degree, flush=True)
    g = _gpu(case, stream, precision, rtol=1e-14 if precision == "fp64" else 1e-13, precond="cheb_schur",
             schur_degree=schur_degree, schur_ratio=300.0)
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
    worst = (0.0, 0.0)
    for k in range(3):
        t1 = o.t + case.prob.dt
        for s in (g, o):
            case.drive(s, t1)
        st = g.step()
        uo, po = o.step()
        ug, pg, _ = g.solution()
        eu, ep = rel_l2(ug, uo), rel_l2(pg, po)
        worst = (max(worst[0], eu), max(worst[1], ep))
        print("step", k, "iters", st["gmres_iters"], "err u %.2e p %.2e" % (eu, ep), flush=True)
    g.close()
    tol = 1e-10 if precision == "fp64" else 1e-8
    assert worst[0] < tol and worst[1] < tol, worst


@pytest.mark.parametrize("mk", CASES[:3], ids=IDS[:3])
def test_asm_fp64_parity(mk, stream):
    """FP32 + refinement with the FP32 matrix built by FP64 element arithmetic and rounded
    (asm_fp64): the matrix is the oracle's rounded to FP32 (<= 1e-7 row-wise) and the
    refined steps match the oracle to <= 1e-8."""
    case = mk()
    print("case", case.name, flush=True)
    g = _gpu(case, stream, "fp32_ir", rtol=1e-13, asm_fp64=True)
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
        case.drive(s, case.prob.t0 + case.prob.dt)
    br, bc, vals, _ = g.export()
    o.assemble()
    err = rowwise_rel_err(oracle_matrix_from_blocks(br, bc, vals, case.mesh.nv), o.matrix())
    print("FP32 matrix from FP64 arithmetic: row-wise %.2e" % err, flush=True)
    assert err < 1e-7, err
    worst = (0.0, 0.0)
    for k in range(3):
        t1 = o.t + case.prob.dt
        for s in (g, o):
            case.drive(s, t1)
        g.step()
        uo, po = o.step()
        ug, pg, _ = g.solution()
        worst = (max(worst[0], rel_l2(ug, uo)), max(worst[1], rel_l2(pg, po)))
    g.close()
    print("steps: worst err u %.2e p %.2e" % worst, flush=True)
    assert worst[0] < 1e-8 and worst[1] < 1e-8, worst
