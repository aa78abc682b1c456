"""Device parity for the fully implicit formulation (u* = u^{n+1} - u_ALE, implicit LES
term) and its Newton's method, against the oracle: the Newton system (Jacobian by
forward-mode dual numbers on the device, by the complex step in the oracle, both exact
to rounding) at a given state, row-wise <= 1e-12 and its right-hand side -R <= 1e-12
(outflow conditions included: the backflow block in the planes, the rank-1 resistance
term applied beside them and left out of the export);
and three implicit steps (device Newton to 1e-13 with each update solved to 1e-14,
oracle Newton with dense solves) <= 1e-10 for u and p; with FP32 updates <= 1e-8."""
import numpy as np
import pytest

from inputs.problem import SolverCfg
from oracle import OracleSim
from tests._cases import (beltrami, tube_valve, tube_ale, tube_outflow, oracle_matrix_from_blocks, rowwise_rel_err,
                          rel_l2)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


def _implicit(case):
    case.prob.implicit = True
    return case


CASES = [lambda: _implicit(tube_valve(4, 8)),
         lambda: _implicit(tube_valve(6, 10, bdf=3, stab="supg_pspg", diffusion="symgrad", forcing=True)),
         lambda: _implicit(tube_valve(4, 8, bdf=1, stab="none")),
         lambda: _implicit(beltrami(4)),
         lambda: _implicit(tube_ale()),
         lambda: _implicit(tube_outflow(kind="resistance", cr=40.0, beta=1.0, ale=True)),
         lambda: _implicit(tube_outflow(kind="neumann", cr=0.0, beta=2.0, p0=1.0))]
IDS = ["tube_vms_valve", "tube_supg_symgrad_bdf3_forcing", "tube_galerkin_bdf1", "beltrami4", "tube_ale",
       "tube_resistance_backflow_ale", "tube_neumann_backflow"]


def _gpu(case, stream, rtol=1e-14, newton_rtol=1e-13, precision="fp64"):
    from paper_2304_12032_amd import Sim
    sv = SolverCfg(precision=precision, rtol=rtol, ir_rtol=newton_rtol, max_ir=20, max_iters=50000)
    return Sim(case.mesh, case.prob, sv, device=0, stream=stream)


@pytest.mark.parametrize("mk", CASES, ids=IDS)
def test_newton_system_parity(mk, stream):
    case = mk()
    g = _gpu(case, stream)
    o = OracleSim(case.mesh, case.prob, solve="dense")
    for s in (g, o):
        case.init(s)
        case.drive(s, case.prob.t0 + case.prob.dt)
    br, bc, vals, rhs = g.export()
    o._newton_t1 = None
    o.newton_system(o.u_hist[0], o.p_hist[0])
    err = rowwise_rel_err(oracle_matrix_from_blocks(br, bc, vals, case.mesh.nv), o.matrix(rank1=False))
    rg = np.concatenate([rhs[:, :3].reshape(-1), rhs[:, 3]])
    erhs = rel_l2(rg, o.rhs)
    print(case.name, "Jacobian row-wise %.2e, -R %.2e" % (err, erhs), flush=True)
    assert err < 1e-12 and erhs < 1e-12
    g.close()


# Steps: the stabilised cases, plus a VMS-LES tube from rest.  The unstabilised (Galerkin) P1-P1
# Jacobian is compared above but not stepped: equal-order P1-P1 without stabilisation has spurious
# pressure modes (the oracle's dense Jacobian is singular from rest), and at the large random
# states of these cases its velocity block is indefinite, which stalls the SIMPLE-preconditioned
# GMRES (its Chebyshev velocity block assumes a positive spectrum).
STEP_CASES = [CASES[0], CASES[1], CASES[3], CASES[4], CASES[5], CASES[6],
              lambda: _implicit(tube_valve(4, 8, random_hist=False))]
STEP_IDS = [IDS[0], IDS[1], IDS[3], IDS[4], IDS[5], IDS[6], "tube_vms_from_rest"]


@pytest.mark.parametrize("mk", STEP_CASES, ids=STEP_IDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_implicit_steps_parity(mk, precision, stream):
    """FP64: Newton to 1e-13, u and p <= 1e-10.  FP32 updates (the FP64 Jacobian and
    residual rounded, each update to inner_rtol): Newton to 1e-12, <= 1e-8, the bar of
    the refined FP32 semi-implicit steps."""
    case = mk()
    f64 = precision == "fp64"
    g = _gpu(case, stream, precision=precision, newton_rtol=1e-13 if f64 else 1e-12)
    o = OracleSim(case.mesh, case.prob, solve="dense")
    for s in (g, o):
        case.init(s)
    for k in range(3):
        t1 = o.t + case.prob.dt
        for s in (g, o):
            case.drive(s, t1)
        st = g.step()
        uo, po = o.step_implicit(newton_rtol=1e-13)
        ug, pg, _ = g.solution()
        eu, ep = rel_l2(ug, uo), rel_l2(pg, po)
        print(case.name, precision, "step", k, "newton", st["newton_iters"],
              "(oracle %d)" % (len(o.newton_norms) - 1), "gmres", st["gmres_iters"],
              "err u %.2e p %.2e" % (eu, ep), flush=True)
        assert 1 <= st["newton_iters"] <= (10 if f64 else 16)
        tol = 1e-10 if f64 else 1e-8
        assert eu < tol and ep < tol, (eu, ep)
    g.close()
