"""Device parity for ALE mesh motion and the continuous-batching server.

ALE: the mesh moves by the harmonic extension of a prescribed boundary
displacement; assembly, no-slip data u = u_ALE and the valve distance all
follow the mesh, compared with the oracle at the FP64 step tolerance.
Serving: every request's result in a mixed batch equals the same request run
alone, and admission respects the device-memory budget in arrival order.
"""
import numpy as np
import pytest

from inputs import tube
from inputs.problem import SolverCfg, tube_problem
from oracle import OracleSim
from tests._cases import (tube_ale, tube_ale_curved, beltrami_ale, oracle_matrix_from_blocks, rowwise_rel_err,
                          rel_l2)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


ALE_CASES = [tube_ale, tube_ale_curved, lambda: beltrami_ale(4, nodal=True), lambda: beltrami_ale(4, nodal=False)]
ALE_IDS = ["linear_shape_valve", "curved_shape", "beltrami_nodal_every_step", "beltrami_sine_law"]


@pytest.mark.parametrize("mk", ALE_CASES, ids=ALE_IDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_ale_steps_parity(mk, precision, stream):
    """Steps on the moving mesh against the oracle: FP64 (device rtol 1e-14) <= 1e-10, FP32 +
    FP64 refinement (refined to 1e-13) <= 1e-8, u and p separately."""
    from paper_2304_12032_amd import Sim
    case = mk()
    print("case", case.name, precision, flush=True)
    rtol = 1e-14 if precision == "fp64" else 1e-13
    g = Sim(case.mesh, case.prob, SolverCfg(precision=precision, rtol=rtol, ir_rtol=rtol, max_iters=20000),
            stream=stream)
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
    worst = (0.0, 0.0)
    for k in range(4):
        t1 = o.t + case.prob.dt
        for s in (g, o):
            case.drive(s, t1)
        st = g.step()
        uo, po = o.step()
        ug, pg, _ = g.solution()
        eu, ep = rel_l2(ug, uo), rel_l2(pg, po)
        worst = (max(worst[0], eu), max(worst[1], ep))
        print("step", k, "iters", st["gmres_iters"], "ir", st["ir_iters"], "err u %.2e p %.2e" % (eu, ep),
              flush=True)
    tol = 1e-10 if precision == "fp64" else 1e-8
    assert worst[0] < tol and worst[1] < tol, worst
    g.close()


@pytest.mark.parametrize("mk", ALE_CASES[:3], ids=ALE_IDS[:3])
def test_ale_matrix_free_residual(mk, stream):
    """The FP64 matrix-free residual of the refinement loop on the moved mesh (x^{n+1},
    u_ALE, no-slip = u_ALE) equals b - A x of the oracle's assembled system to 1e-12, after
    two steps have moved the mesh and filled the displacement history."""
    from paper_2304_12032_amd import Sim
    case = mk()
    print("case", case.name, flush=True)
    g = Sim(case.mesh, case.prob, SolverCfg(precision="fp32_ir", rtol=1e-13, ir_rtol=1e-13, max_iters=20000),
            stream=stream)
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
    for k in range(2):
        t1 = o.t + case.prob.dt
        for s in (g, o):
            case.drive(s, t1)
        g.step()
        o.step()
    t1 = o.t + case.prob.dt
    for s in (g, o):
        case.drive(s, t1)
    rng = np.random.default_rng(4)
    nv = case.mesh.nv
    u = rng.normal(size=(nv, 3))
    p = rng.normal(size=nv) * 10
    r = g.residual(u, p)
    o.assemble()
    x = np.concatenate([u.reshape(-1), p])
    A = o.matrix()
    ro = o.rhs - A @ x
    rg = np.concatenate([r[:, :3].reshape(-1), r[:, 3]])
    scale = np.abs(o.rhs).max() + abs(A).max() * np.abs(x).max()
    print("residual difference %.2e of scale %.2e" % (np.abs(rg - ro).max(), scale), flush=True)
    assert np.abs(rg - ro).max() < 1e-12 * scale
    g.close()


def test_ale_matrix_parity(stream):
    """The matrix of a step on the moved mesh (x^{n+1}, u_ALE) matches the oracle's."""
    from paper_2304_12032_amd import Sim
    case = tube_ale()
    g = Sim(case.mesh, case.prob, SolverCfg(precision="fp64", rtol=1e-14, max_iters=20000), stream=stream)
    o = OracleSim(case.mesh, case.prob)
    for s in (g, o):
        case.init(s)
    g.step()
    o.step()
    br, bc, vals, rhs = g.export()
    o.assemble()
    assert rowwise_rel_err(oracle_matrix_from_blocks(br, bc, vals, case.mesh.nv), o.matrix()) < 1e-11
    g.close()


def _requests():
    out = []
    for i, (nxy, nz, mu, peak) in enumerate([(4, 10, 0.03, 40.0), (6, 8, 0.045, 25.0), (3, 12, 0.02, 70.0)]):
        m = tube(nxy=nxy, nz=nz, radius=1.0, length=3.0, seed=10 + i)
        p = tube_problem(m, mu=mu, peak=peak, dt=1e-3, R=500.0, eps=0.3)
        out.append((m, p))
    return out


def test_serving_mix_equals_alone(stream):
    """Three requests of different sizes and parameters served together: each result is
    bitwise the one the same request gives alone (every reduction has a fixed order, so
    nothing depends on what else runs), and each matches the oracle's run of the request
    (FP32 + FP64 refinement to 1e-12 against dense LU: <= 1e-8 for u and p)."""
    from paper_2304_12032_amd import Server, Sim
    sv = SolverCfg(precision="fp32_ir", ir_rtol=1e-12, max_iters=20000)
    reqs = _requests()
    steps = 4
    srv = Server(hbm_budget_bytes=1 << 34, max_active=8, n_streams=4)
    tickets = [srv.submit(m, p, sv, steps) for m, p in reqs]
    for _ in range(100):
        if srv.tick() == 0 and all(srv.poll(t)["state"] in ("done", "failed") for t in tickets):
            break
    results = [srv.result(t) for t in tickets]
    srv.close()
    for (m, p), (u, pr, lat) in zip(reqs, results):
        alone = Sim(m, p, sv, stream=stream)
        for _ in range(steps):
            alone.step()
        ua, pa, _ = alone.solution()
        alone.close()
        o = OracleSim(m, p, solve="dense")
        for _ in range(steps):
            uo, po = o.step()
        eo = (rel_l2(u, uo), rel_l2(pr, po))
        print("request nv=%d: mix vs alone max |du| %.2e |dp| %.2e; vs oracle u %.2e p %.2e; p50 %.2f ms p99 %.2f ms"
              % (m.nv, np.abs(u - ua).max(), np.abs(pr - pa).max(), eo[0], eo[1], lat["step_p50_ms"],
                 lat["step_p99_ms"]), flush=True)
        assert lat["n_steps"] == steps
        assert np.array_equal(u, ua) and np.array_equal(pr, pa)
        assert eo[0] < 1e-8 and eo[1] < 1e-8, eo


def test_serving_admission_by_budget(stream):
    """With a budget that holds one request at a time (equal-size requests, budget 1.05x
    one footprint estimate), requests run one after another in arrival order and each
    waits for the previous one's memory."""
    from paper_2304_12032_amd import Server
    sv = SolverCfg(precision="fp32_ir", ir_rtol=1e-8)
    reqs = []
    for i, (mu, peak) in enumerate([(0.03, 40.0), (0.045, 25.0), (0.02, 60.0)]):
        m = tube(nxy=4, nz=10, radius=1.0, length=3.0, seed=20 + i)
        reqs.append((m, tube_problem(m, mu=mu, peak=peak, dt=1e-3, R=500.0, eps=0.3)))
    probe = Server(hbm_budget_bytes=1 << 34)
    est = max(probe.poll(probe.submit(m, p, sv, 1))["footprint_bytes"] for m, p in reqs)
    probe.close()
    srv = Server(hbm_budget_bytes=int(est * 1.05), max_active=8, n_streams=2)
    tickets = [srv.submit(m, p, sv, 2) for m, p in reqs]
    order, seen = [], set()
    for _ in range(100):
        srv.tick()
        states = [srv.poll(t)["state"] for t in tickets]
        assert sum(s == "running" for s in states) <= 1
        for t, s in zip(tickets, states):
            if s == "done" and t not in seen:
                seen.add(t)
                order.append(t)
        if len(seen) == len(tickets):
            break
    assert order == tickets
    lats = [srv.result(t)[2] for t in tickets]
    assert lats[2]["admit_wait_ms"] >= lats[1]["admit_wait_ms"] >= lats[0]["admit_wait_ms"]
    assert lats[1]["admit_wait_ms"] > 0
    srv.close()
