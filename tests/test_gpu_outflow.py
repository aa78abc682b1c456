"""Device parity for the outflow conditions: resistance (rank-1 coupling) and
inertial backflow stabilisation on P1-P1, and the boundary flow-rate / pressure
integrals, against the oracle.  Tolerances as in the other parity tests: FP64
matrices and residuals <= 1e-12 row-wise / of scale; FP64 steps (device rtol
1e-14, oracle dense LU) <= 1e-10; FP32 + FP64 refinement steps <= 1e-8;
boundary integrals <= 1e-12 relative."""
import numpy as np
import pytest

from inputs.problem import SolverCfg
from oracle import OracleSim
from tests._cases import tube_outflow, oracle_matrix_from_blocks, rowwise_rel_err, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


def _gpu(case, stream, precision="fp64", rtol=1e-12):
    from paper_2304_12032_amd import Sim
    sv = SolverCfg(precision=precision, rtol=rtol, ir_rtol=rtol, max_iters=20000)
    return Sim(case.mesh, case.prob, sv, device=0, stream=stream)


CASES = [lambda: tube_outflow(kind="neumann", cr=0.0, beta=1.0),
         lambda: tube_outflow(kind="resistance", cr=40.0, beta=0.0),
         lambda: tube_outflow(kind="resistance", cr=40.0, beta=1.5),
         lambda: tube_outflow(kind="resistance", cr=25.0, beta=1.0, ale=True)]
IDS = ["neumann_backflow", "resistance", "resistance_backflow", "resistance_backflow_ale"]


@pytest.mark.parametrize("mk", CASES, ids=IDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_outflow_matrix_parity(mk, precision, stream):
    """The assembled matrix (backflow term included, the rank-1 term left out on both
    sides) and, in FP64, the right-hand side (resistance data included)."""
    case = mk()
    print("case", case.name, precision, flush=True)
    g = _gpu(case, stream, precision)
    o = OracleSim(case.mesh, case.prob, solve="dense")
    for s in (g, o):
        case.init(s)
    br, bc, vals, rhs = g.export()
    o.assemble()
    err = rowwise_rel_err(oracle_matrix_from_blocks(br, bc, vals, case.mesh.nv), o.matrix(rank1=False))
    assert err < (1e-12 if precision == "fp64" else 2e-5), err
    if precision == "fp64":
        rg = np.concatenate([rhs[:, :3].reshape(-1), rhs[:, 3]])
        assert rel_l2(rg, o.rhs) < 1e-12
    g.close()


@pytest.mark.parametrize("mk", CASES, ids=IDS)
def test_outflow_matrix_free_residual(mk, stream):
    """The FP64 matrix-free residual equals b - (A + C_R w_row w^T) x of the oracle."""
    case = mk()
    g = _gpu(case, stream, "fp32_ir")
    o = OracleSim(case.mesh, case.prob, solve="dense")
    for s in (g, o):
        case.init(s)
    rng = np.random.default_rng(5)
    nv = case.mesh.nv
    u = rng.normal(size=(nv, 3))
    p = rng.normal(size=nv) * 10
    r = g.residual(u, p)
    o.assemble()
    x = np.concatenate([u.reshape(-1), p])
    A = o.matrix()
    ro = o.rhs - A @ x
    rg = np.concatenate([r[:, :3].reshape(-1), r[:, 3]])
    scale = np.abs(o.rhs).max() + np.abs(A).max() * np.abs(x).max()
    assert np.abs(rg - ro).max() < 1e-12 * scale
    g.close()


@pytest.mark.parametrize("mk", CASES, ids=IDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_outflow_steps_parity(mk, precision, stream):
    """Three steps against the oracle's dense solves; then the outlet's flux, pressure
    integral and area against the oracle's."""
    case = mk()
    print("case", case.name, precision, flush=True)
    g = _gpu(case, stream, precision, rtol=1e-14 if precision == "fp64" else 1e-13)
    o = OracleSim(case.mesh, case.prob, solve="dense")
    for s in (g, o):
        case.init(s)
    tol = 1e-10 if precision == "fp64" else 1e-8
    for k in range(3):
        st = g.step()
        uo, po = o.step()
        ug, pg, _ = g.solution()
        eu, ep = rel_l2(ug, uo), rel_l2(pg, po)
        print("step", k, "iters", st["gmres_iters"], "err u %.2e p %.2e" % (eu, ep), flush=True)
        assert eu < tol and ep < tol, (eu, ep)
    for bc in (1, 2):
        bg, bo = g.boundary_integrals(bc), o.boundary_integrals(bc)
        print("bc", bc, "device", bg, "oracle", bo, flush=True)
        assert np.abs(bg - bo).max() <= tol * np.abs(bo).max()
    g.close()
