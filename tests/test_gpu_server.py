"""Server mechanics on the device: the footprint estimate against what a simulation
allocates, the budget check once a simulation exists (a short estimate is corrected,
the request queued again), set-up reported apart from stepping, and results bitwise
equal to the same request run alone."""
import os

import numpy as np
import pytest

from inputs import tube
from inputs.problem import SolverCfg, tube_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def stream():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch.cuda.current_stream(0).cuda_stream


def _req(seed, nxy=4, nz=10, mu=0.03, peak=40.0):
    m = tube(nxy=nxy, nz=nz, radius=1.0, length=3.0, seed=seed)
    return m, tube_problem(m, mu=mu, peak=peak, dt=1e-3, R=500.0, eps=0.3)


def _drain(srv, tickets, limit=2000):
    seen = []
    for _ in range(limit):
        n = srv.tick()
        states = [srv.poll(t)["state"] for t in tickets]
        seen.append(states)
        if n == 0 and all(s in ("done", "failed") for s in states):
            return seen
    raise AssertionError("server did not drain: %s" % seen[-1])


def _alone(m, p, sv, steps, stream):
    from paper_2304_12032_amd import Sim
    s = Sim(m, p, sv, stream=stream)
    for _ in range(steps):
        s.step()
    u, pr, _ = s.solution()
    s.close()
    return u, pr


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_estimate_bounds_measured_footprint(precision):
    """For tubes of several sizes and both precisions the admission estimate is an upper
    bound of what the simulation allocates, and not a loose one (within 2x plus the
    estimate's fixed 6 MB allowance for small levels and tables)."""
    from paper_2304_12032_amd import Server
    sv = SolverCfg(precision=precision)
    for nxy, nz in ((3, 6), (6, 12), (10, 24)):
        m, p = _req(1, nxy=nxy, nz=nz)
        srv = Server(hbm_budget_bytes=1 << 36, max_active=2, n_streams=1)
        t = srv.submit(m, p, sv, 1)
        est = srv.poll(t)["footprint_bytes"]
        real = None
        for _ in range(2000):
            srv.tick()
            st = srv.poll(t)
            if st["state"] in ("running", "done"):
                real = st["footprint_bytes"]
            if st["state"] in ("done", "failed"):
                break
        assert srv.poll(t)["state"] == "done"
        srv.result(t)
        srv.close()
        print("%s nv=%d nt=%d: estimate %d B, measured %d B, ratio %.3f"
              % (precision, m.nv, m.nt, est, real, est / real), flush=True)
        assert real <= est < 2 * real + (8 << 20)


def test_short_estimate_is_corrected(stream):
    """With the estimates scaled to 20% (at most 0.4 of a measured footprint), two equal
    requests are admitted together into a budget of 1.5 measured footprints; once set up, the second breaks the budget, is
    released and queued again with its measured footprint, and runs after the first.
    Both results are bitwise the requests' results alone; at no time do two run."""
    from paper_2304_12032_amd import Server
    sv = SolverCfg(precision="fp32_ir", ir_rtol=1e-10)
    reqs = [_req(31), _req(32, mu=0.045, peak=25.0)]
    probe = Server(hbm_budget_bytes=1 << 36, max_active=2, n_streams=1)
    t0 = probe.submit(*reqs[0], sv, 0)
    _drain(probe, [t0])
    real = probe.poll(t0)["footprint_bytes"]
    probe.result(t0)
    probe.close()
    os.environ["LXNS_SERVER_EST_SCALE"] = "0.2"
    try:
        srv = Server(hbm_budget_bytes=int(1.5 * real), max_active=4, n_streams=2)
    finally:
        del os.environ["LXNS_SERVER_EST_SCALE"]
    tickets = [srv.submit(m, p, sv, 3) for m, p in reqs]
    seen = _drain(srv, tickets)
    assert all(sum(s == "running" for s in states) <= 1 for states in seen)
    out = [srv.result(t) for t in tickets]
    srv.close()
    for (m, p), (u, pr, lat) in zip(reqs, out):
        assert lat["n_steps"] == 3
        ua, pa = _alone(m, p, sv, 3, stream)
        assert np.array_equal(u, ua) and np.array_equal(pr, pa)
    # the one set up second was admitted again when the other retired
    early, late = sorted((lat for _, _, lat in out), key=lambda l: l["admit_wait_ms"])
    assert late["admit_wait_ms"] >= early["total_ms"] - 5.0


def test_measured_footprint_over_budget_fails():
    """A request whose estimate (scaled to 30%) fits but whose simulation alone breaks the
    budget ends FAILED with the reason, and the server goes on with the next one."""
    from paper_2304_12032_amd import Server, LxError
    sv = SolverCfg(precision="fp32_ir")
    big, small = _req(41, nxy=8, nz=20), _req(42, nxy=3, nz=6)
    probe = Server(hbm_budget_bytes=1 << 36, max_active=2, n_streams=1)
    tb = probe.submit(*big, sv, 0)
    _drain(probe, [tb])
    real = probe.poll(tb)["footprint_bytes"]
    probe.result(tb)
    probe.close()
    os.environ["LXNS_SERVER_EST_SCALE"] = "0.3"
    try:
        srv = Server(hbm_budget_bytes=int(0.8 * real), max_active=4, n_streams=1)
    finally:
        del os.environ["LXNS_SERVER_EST_SCALE"]
    t1 = srv.submit(*big, sv, 2)
    t2 = srv.submit(*small, sv, 2)
    _drain(srv, [t1, t2])
    assert srv.poll(t1)["state"] == "failed"
    with pytest.raises(LxError, match="exceeds the budget"):
        srv.result(t1)
    assert srv.poll(t2)["state"] == "done"
    srv.result(t2)
    srv.close()


def test_setup_reported_apart_from_steps(stream):
    """Eight requests on two streams: every request's set-up time is reported as
    setup_ms, apart from the admission wait and the step latencies; each runs its steps,
    and the results equal the requests alone."""
    from paper_2304_12032_amd import Server
    sv = SolverCfg(precision="fp32_ir", ir_rtol=1e-10)
    reqs = [_req(50 + i, nxy=3 + i % 3, nz=6 + 2 * i, mu=0.02 + 0.004 * i, peak=20.0 + 7.0 * i) for i in range(8)]
    srv = Server(hbm_budget_bytes=1 << 36, max_active=8, n_streams=2)
    tickets = [srv.submit(m, p, sv, 3) for m, p in reqs]
    _drain(srv, tickets)
    out = [srv.result(t) for t in tickets]
    srv.close()
    for (m, p), (u, pr, lat) in zip(reqs, out):
        assert lat["n_steps"] == 3 and lat["setup_ms"] > 0
        assert lat["total_ms"] >= lat["admit_wait_ms"] + lat["setup_ms"]
        ua, pa = _alone(m, p, sv, 3, stream)
        assert np.array_equal(u, ua) and np.array_equal(pr, pa)
