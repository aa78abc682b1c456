"""The one-workgroup coarse AMG cycle and the sliced-ELL finest level, against
the oracle and against the plain layouts (every level cycled by its own
launches; the finest level in CSR), and the tabulated operator of the coarse
cycle against cycling it at every visit.

The small parity cases have a two-level Schur hierarchy (one smoothed level
and the dense one), where the coarse cycle does not apply.  This tube is large
enough for three levels whose middle one fits one workgroup's LDS, so the
device runs it; the oracle solves by sparse LU.  Tolerances as in the other
step tests: FP64 steps (device GMRES to 1e-14) <= 1e-10, FP32 + FP64
refinement (refined to 1e-13) <= 1e-8; with the coarse cycle switched off
(LXNS_AMG_TAIL=0) the FP64 fields agree with it to <= 1e-10 and the GMRES
iteration counts within 2 (the cycle sums in another order).
"""
import os

import numpy as np
import pytest

from inputs.problem import SolverCfg
from oracle import OracleSim
from tests._cases import rel_l2, tube_valve

pytestmark = pytest.mark.gpu

STEPS = 1


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


def _case():
    return tube_valve(12, 60, length=6.0, seed=11)


def _gpu(case, stream, precision, tail=True, sell=True, op=True):
    from paper_2304_12032_amd import Sim
    rtol = 1e-14 if precision == "fp64" else 1e-13
    sv = SolverCfg(precision=precision, rtol=rtol, ir_rtol=rtol, max_iters=20000)
    env = {"LXNS_AMG_TAIL": tail, "LXNS_AMG_SELL": sell, "LXNS_TAIL_OP": op}
    old = {k: os.environ.get(k) for k in env}
    for k, on in env.items():
        if not on:
            os.environ[k] = "0"
    try:
        g = Sim(case.mesh, case.prob, sv, device=0, stream=stream)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    q = g.query()
    print("%s: %d vertices, AMG levels %d, coarse cycle from level %d" % (precision, case.mesh.nv, q["amg_levels"],
                                                                         q["amg_tail_level"]), flush=True)
    return g, q


def _run(g, case, steps):
    case.init(g)
    out = []
    for k in range(steps):
        case.drive(g, case.prob.t0 + (k + 1) * case.prob.dt)
        st = g.step()
        u, p, _ = g.solution()
        out.append((u, p, st["gmres_iters"]))
    return out


@pytest.fixture(scope="module")
def oracle_steps():
    """The oracle's steps of the case (sparse LU; about half a minute per step on one core)."""
    case = _case()
    o = OracleSim(case.mesh, case.prob)
    case.init(o)
    out = []
    for k in range(STEPS):
        case.drive(o, o.t + case.prob.dt)
        out.append(o.step())
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_coarse_cycle_steps_parity(precision, stream, oracle_steps):
    case = _case()
    g, q = _gpu(case, stream, precision)
    assert q["amg_levels"] >= 3 and q["amg_tail_level"] >= 1
    dev = _run(g, case, STEPS)
    g.close()
    tol = 1e-10 if precision == "fp64" else 1e-8
    for k in range(STEPS):
        uo, po = oracle_steps[k]
        ug, pg, it = dev[k]
        eu, ep = rel_l2(ug, uo), rel_l2(pg, po)
        print("step %d: %d iterations, err u %.2e p %.2e" % (k, it, eu, ep), flush=True)
        assert eu < tol and ep < tol, (eu, ep)


def test_coarse_cycle_matches_level_kernels(stream):
    case = _case()
    g1, q1 = _gpu(case, stream, "fp64", tail=True)
    a = _run(g1, case, STEPS)
    g1.close()
    g0, q0 = _gpu(case, stream, "fp64", tail=False)
    b = _run(g0, case, STEPS)
    g0.close()
    assert q1["amg_tail_level"] >= 1 and q0["amg_tail_level"] == 0
    assert q1["amg_levels"] == q0["amg_levels"]
    for k in range(STEPS):
        (u1, p1, i1), (u0, p0, i0) = a[k], b[k]
        eu, ep = rel_l2(u1, u0), rel_l2(p1, p0)
        print("step %d: iterations %d (one workgroup) / %d (level kernels), diff u %.2e p %.2e" % (k, i1, i0, eu, ep),
              flush=True)
        assert abs(i1 - i0) <= 2
        assert eu < 1e-10 and ep < 1e-10, (eu, ep)


def test_sell_matches_csr(stream):
    """The finest level in sliced-ELL order against the same level in CSR."""
    case = _case()
    g1, _ = _gpu(case, stream, "fp64")
    a = _run(g1, case, STEPS)
    g1.close()
    g0, _ = _gpu(case, stream, "fp64", sell=False)
    b = _run(g0, case, STEPS)
    g0.close()
    for k in range(STEPS):
        (u1, p1, i1), (u0, p0, i0) = a[k], b[k]
        eu, ep = rel_l2(u1, u0), rel_l2(p1, p0)
        print("step %d: iterations %d (sliced ELL) / %d (CSR), diff u %.2e p %.2e" % (k, i1, i0, eu, ep), flush=True)
        assert abs(i1 - i0) <= 2
        assert eu < 1e-10 and ep < 1e-10, (eu, ep)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_tail_operator_matches_cycle(precision, stream):
    """The coarse cycle's operator, tabulated once per step by cycling the unit vectors and
    applied as one dense product per visit, against running the cycle at every visit: the
    same linear map in another summation order, so the same iteration counts (within 1) and
    fields that agree to the solve tolerance."""
    case = _case()
    g1, q1 = _gpu(case, stream, precision, op=True)
    a = _run(g1, case, 2)
    g1.close()
    g0, _ = _gpu(case, stream, precision, op=False)
    b = _run(g0, case, 2)
    g0.close()
    assert q1["amg_tail_level"] >= 1
    tol = 1e-10 if precision == "fp64" else 1e-8
    for k in range(2):
        (u1, p1, i1), (u0, p0, i0) = a[k], b[k]
        eu, ep = rel_l2(u1, u0), rel_l2(p1, p0)
        print("step %d: iterations %d (tabulated) / %d (cycled), diff u %.2e p %.2e" % (k, i1, i0, eu, ep),
              flush=True)
        assert abs(i1 - i0) <= 1
        assert eu < tol and ep < tol, (eu, ep)
