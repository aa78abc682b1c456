"""The allocation-free residual entry point (lx_sim_residual_noalloc) against the
entry point it varies (lx_sim_debug_residual) and against the oracle.

Two calls in a row on one device, the second on a smaller mesh, so that the
shared static scratch holds the first call's larger contents when the second
runs: each output equals lx_sim_debug_residual's bitwise and the oracle's
b - A x to 1e-12 of the scale.  A mesh beyond the scratch limit is rejected.
"""
import numpy as np
import pytest

from inputs import tube
from inputs.problem import SolverCfg, tube_problem
from oracle import OracleSim
from tests._cases import tube_valve, tube_ale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


def _check(case, precision, stream, seed):
    import torch
    from paper_2304_12032_amd import Sim
    from paper_2304_12032_amd.lxns import residual_noalloc
    g = Sim(case.mesh, case.prob, SolverCfg(precision=precision, rtol=1e-12, ir_rtol=1e-12, max_iters=20000),
            stream=stream)
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
        case.drive(s, case.prob.t0 + case.prob.dt)
    rng = np.random.default_rng(seed)
    nv = case.mesh.nv
    u = rng.normal(size=(nv, 3))
    p = rng.normal(size=nv) * 10
    ref = g.residual(u, p)
    ud = torch.tensor(u, dtype=torch.float64, device="cuda:0")
    pd = torch.tensor(p, dtype=torch.float64, device="cuda:0")
    rd = torch.full((nv, 4), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    residual_noalloc(g, ud.data_ptr(), pd.data_ptr(), rd.data_ptr())
    torch.cuda.synchronize()
    r = rd.cpu().numpy()
    o.assemble()
    x = np.concatenate([u.reshape(-1), p])
    A = o.matrix()
    ro = o.rhs - A @ x
    rg = np.concatenate([r[:, :3].reshape(-1), r[:, 3]])
    scale = np.abs(o.rhs).max() + abs(A).max() * np.abs(x).max()
    print("%s %s: nv %d, nt %d; equal to the allocating entry point: %s; vs oracle %.2e of %.2e" %
          (case.name, precision, nv, case.mesh.nt, np.array_equal(r, ref), np.abs(rg - ro).max(), scale), flush=True)
    g.close()
    assert np.array_equal(r, ref)
    assert np.abs(rg - ro).max() < 1e-12 * scale


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_noalloc_residual_two_calls_second_smaller(precision, stream):
    _check(tube_valve(8, 16, length=4.0, bdf=3, stab="supg_pspg", diffusion="symgrad", forcing=True), precision,
           stream, 1)
    _check(tube_valve(4, 8), precision, stream, 2)


def test_noalloc_residual_moving_mesh(stream):
    _check(tube_ale(6, 10), "fp64", stream, 3)
    _check(tube_ale(4, 8), "fp64", stream, 4)


def test_noalloc_residual_rejects_large_mesh(stream):
    import torch
    from paper_2304_12032_amd import Sim, LxError
    from paper_2304_12032_amd.lxns import residual_noalloc
    m = tube(nxy=24, nz=60, seed=1)
    assert m.nt > 170000
    g = Sim(m, tube_problem(m), SolverCfg(), stream=stream)
    d = torch.zeros((m.nv, 4), dtype=torch.float64, device="cuda:0")
    with pytest.raises(LxError) as ei:
        residual_noalloc(g, d.data_ptr(), d.data_ptr(), d.data_ptr())
    assert ei.value.status == -1 and "scratch" in str(ei.value)
    g.close()
