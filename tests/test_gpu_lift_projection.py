"""The lifting's initial guess projected onto earlier lifting solutions (nodal
boundary displacement set every step): the projection changes where the CG starts,
never what it converges to, so every step must still match the oracle's direct
lifting solve (FP64 steps <= 1e-10), with and without the projection
(LXNS_LIFT_PROJ=0).  For a motion that is one shape times a time law the new
solution lies in the span of the first one, and the CG must find the projected
guess already converged; for a travelling wave (no finite set of shapes) the
projection must not cost iterations.  A checkpoint taken mid-run must carry the
basis: 6 steps = 3 + save/restore + 3, bitwise."""
import os

import numpy as np
import pytest

from inputs.problem import SolverCfg
from oracle import OracleSim
from tests._cases import rel_l2, tube_lifting

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


def _shape(mesh, length):
    X = mesh.coords
    s = np.zeros_like(X)
    bump = 0.05 * np.sin(np.pi * X[:, 2] / length)
    s[:, 0], s[:, 1] = bump * X[:, 0], bump * X[:, 1]
    return s


def _separable(mesh, length, t):
    return np.sin(60.0 * t) * _shape(mesh, length)


def _wave(mesh, length, t):
    X = mesh.coords
    s = np.zeros_like(X)
    amp = 0.05 * np.sin(np.pi * X[:, 2] / length - 80.0 * t)
    s[:, 0], s[:, 1] = amp * X[:, 0], amp * X[:, 1]
    s[:, 2] = 0.02 * np.cos(2.0 * np.pi * X[:, 2] / length + 50.0 * t) * X[:, 0]
    return s


def _sim(case, stream, proj):
    from paper_2304_12032_amd import Sim
    old = os.environ.get("LXNS_LIFT_PROJ")
    if not proj:
        os.environ["LXNS_LIFT_PROJ"] = "0"
    try:
        sv = SolverCfg(precision="fp64", rtol=1e-14, max_iters=20000)
        return Sim(case.mesh, case.prob, sv, device=0, stream=stream)
    finally:
        if old is None:
            os.environ.pop("LXNS_LIFT_PROJ", None)
        else:
            os.environ["LXNS_LIFT_PROJ"] = old


def _run(case, motion, sim, steps, oracle=None):
    length = 1.5
    iters, fields = [], []
    for k in range(steps):
        t1 = case.prob.t0 + (k + 1) * case.prob.dt
        d = motion(case.mesh, length, t1)
        sim.set_boundary_displacement(d)
        st = sim.step()
        iters.append(st["lift_iters"])
        ug, pg, _ = sim.solution()
        fields.append((ug, pg))
        if oracle is not None:
            oracle.set_boundary_displacement(d)
            uo, po = oracle.step()
            eu, ep = rel_l2(ug, uo), rel_l2(pg, po)
            assert eu < 1e-10 and ep < 1e-10, (k, eu, ep)
    return iters, fields


@pytest.mark.parametrize("lifting", ["harmonic", "elastic"])
@pytest.mark.parametrize("motion", ["separable", "wave"])
def test_projection_keeps_parity_and_saves_iterations(lifting, motion, stream):
    case = tube_lifting(lifting, "none", (1.0, 1.0), nxy=6, nz=10)
    fn = _separable if motion == "separable" else _wave
    res = {}
    for proj in (True, False):
        g = _sim(case, stream, proj)
        o = OracleSim(case.mesh, case.prob, solve="dense")
        for s in (g, o):
            case.init(s)
        res[proj] = _run(case, fn, g, 6, o)[0]
        g.close()
    print("%s %s: lifting CG iterations with projection %s, without %s" % (lifting, motion, res[True], res[False]),
          flush=True)
    assert res[True][0] == res[False][0]            # the first step has no basis yet
    assert sum(res[True][2:]) <= sum(res[False][2:])
    if motion == "separable":
        assert max(res[True][1:]) <= 2


def test_checkpoint_carries_the_basis(stream):
    case = tube_lifting("harmonic", "none", (1.0, 1.0), nxy=6, nz=10)
    a = _sim(case, stream, True)
    case.init(a)
    _, fa = _run(case, _wave, a, 6)
    b = _sim(case, stream, True)
    case.init(b)
    _run(case, _wave, b, 3)
    blob = b.get_state()
    b.close()
    c = _sim(case, stream, True)
    case.init(c)
    c.restore_state(blob)
    # continue the same motion from step 4 on
    length = 1.5
    fc = []
    for k in range(3, 6):
        t1 = case.prob.t0 + (k + 1) * case.prob.dt
        c.set_boundary_displacement(_wave(case.mesh, length, t1))
        c.step()
        ug, pg, _ = c.solution()
        fc.append((ug, pg))
    for (ua, pa), (uc, pc) in zip(fa[3:], fc):
        assert np.array_equal(ua, uc) and np.array_equal(pa, pc)
    a.close()
    c.close()
