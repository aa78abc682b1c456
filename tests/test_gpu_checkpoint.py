"""Checkpoint and restore through the C ABI (lx_sim_state_size / get_state /
restore_state), and device memory from the caller's allocator (lx_device.alloc).

Ten steps in one go equal five steps, a checkpoint, a fresh simulation restored
from it and five more steps, bitwise, in FP64 and in FP32 + FP64 refinement, on
the tube with a valve and on the moving-mesh tube.  A simulation whose device
memory comes from PyTorch's caching allocator computes bitwise the same steps
as one that allocates with hipMalloc.
"""
import numpy as np
import pytest

from inputs.problem import SolverCfg
from tests._cases import tube_valve, tube_ale, tube_ale_curved

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


def _sim(case, stream, precision, **kw):
    from paper_2304_12032_amd import Sim
    sv = SolverCfg(precision=precision, rtol=1e-12, ir_rtol=1e-12, max_iters=20000)
    return Sim(case.mesh, case.prob, sv, device=0, stream=stream, **kw)


def _run(sim, case, steps):
    for _ in range(steps):
        t1 = sim.solution()[2] + case.prob.dt
        case.drive(sim, t1)
        sim.step()


CASES = {"tube_valve": lambda: tube_valve(4, 8), "tube_ale": tube_ale, "tube_ale_curved": tube_ale_curved}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_checkpoint_restore_bitwise(name, precision, stream):
    case = CASES[name]()
    print("case", case.name, precision, flush=True)
    a = _sim(case, stream, precision)
    case.init(a)
    _run(a, case, 10)
    ua, pa, ta = a.solution()
    a.close()
    b = _sim(case, stream, precision)
    case.init(b)
    _run(b, case, 5)
    blob = b.get_state()
    ub5, pb5, tb5 = b.solution()
    b.close()
    c = _sim(case, stream, precision)
    c.restore_state(blob)
    uc5, pc5, tc5 = c.solution()
    assert np.array_equal(uc5, ub5) and np.array_equal(pc5, pb5) and tc5 == tb5
    _run(c, case, 5)
    uc, pc, tc = c.solution()
    c.close()
    print("state %d bytes; 5 + restore + 5 vs 10: max |du| %.3e |dp| %.3e" %
          (len(blob), np.abs(uc - ua).max(), np.abs(pc - pa).max()), flush=True)
    assert tc == ta
    assert np.array_equal(uc, ua) and np.array_equal(pc, pa)


def test_restore_rejects_other_problem(stream):
    from paper_2304_12032_amd import LxError
    a = _sim(tube_valve(4, 8), stream, "fp64")
    blob = a.get_state()
    a.close()
    b = _sim(tube_valve(4, 9), stream, "fp64")
    with pytest.raises(LxError):
        b.restore_state(blob)
    with pytest.raises(LxError):
        b.restore_state(blob[:-8])
    b.close()


def test_caller_allocator_bitwise(stream):
    """Device memory from torch's caching allocator (through lx_device.alloc / free): the
    same results, bitwise, and the memory returns to torch when the simulation ends."""
    import torch
    from paper_2304_12032_amd import torch_allocator
    case = tube_valve(4, 8)
    ref = _sim(case, stream, "fp32_ir")
    case.init(ref)
    _run(ref, case, 4)
    ur, pr, _ = ref.solution()
    ref.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    alloc = torch_allocator(0, stream)
    s = _sim(case, stream, "fp32_ir", allocator=alloc)
    held = torch.cuda.memory_allocated(0) - before
    q = s.query()
    case.init(s)
    _run(s, case, 4)
    us, ps, _ = s.solution()
    s.close()
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated(0)
    print("torch allocator held %d bytes (library count %d); released to %d" % (held, q["device_bytes"], after - before),
          flush=True)
    assert held >= q["device_bytes"] > 0
    assert after == before
    assert np.array_equal(us, ur) and np.array_equal(ps, pr)
