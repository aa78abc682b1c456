"""Device P2-P1 (Taylor-Hood) path against the P2-P1 oracle.

The device numbers its edge nodes in its own order (lx_sim_get_edges); the
oracle in another.  Inputs are evaluated at each side's node coordinates;
outputs are compared after mapping device nodes onto oracle nodes by their
vertex pairs.
"""
import numpy as np
import pytest

from inputs import exact
from inputs.problem import SolverCfg, beltrami_cube_problem
from tests._cases import rel_l2, rowwise_rel_err, tube_valve

pytestmark = pytest.mark.gpu


def _sim(mesh, prob, **kw):
    from paper_2304_12032_amd import Sim
    return Sim(mesh, prob, SolverCfg(**kw))


def _node_map(dev, orc):
    """device node -> oracle node"""
    key = {(int(a), int(b)): k for k, (a, b) in enumerate(orc.E)}
    m = np.arange(orc.nu)
    for k, (a, b) in enumerate(dev.edges()):
        m[orc.nv + k] = orc.nv + key[(min(a, b), max(a, b))]
    return m


def _dof_map(nmap, nu, nv):
    d = np.empty(3 * nu + nv, dtype=np.int64)
    for c in range(3):
        d[3 * np.arange(nu) + c] = 3 * nmap + c
    d[3 * nu:] = 3 * nu + np.arange(nv)
    return d


def _dev_xnode(dev, mesh):
    e = dev.edges()
    return np.concatenate([mesh.coords, 0.5 * (mesh.coords[e[:, 0]] + mesh.coords[e[:, 1]])])


class P2Case:
    """Problem + per-side drivers (each side evaluates data at its own nodes)."""

    def __init__(self, name, mesh, prob, init, drive):
        self.name, self.mesh, self.prob, self.init, self.drive = name, mesh, prob, init, drive


def beltrami_p2(n=3, dt=0.01, bdf=1):
    mesh, prob = beltrami_cube_problem(n, dt=dt, bdf_order=bdf)
    prob.fe = "p2p1"
    ex = exact.Beltrami(mu=prob.mu)

    def init(s, X):
        for lev in range(bdf):
            s.set_state(lev, ex.velocity(X, -lev * dt), ex.pressure(mesh.coords, -lev * dt))

    def drive(s, X, t1):
        s.set_dirichlet_values(0, ex.velocity(X, t1))
        s.set_neumann_traction(1, ex.traction(X, t1, (-1, 0, 0)))

    return P2Case("beltrami%d_p2" % n, mesh, prob, init, drive)


def tube_p2(seed=3):
    """Small jittered tube with pulsatile inflow, RIIS disc, BDF2 and a random
    (seeded) history so that every stabilisation term is active."""
    base = tube_valve(nxy=4, nz=6, length=1.5, bdf=2, seed=seed, random_hist=False)
    mesh, prob = base.mesh, base.prob
    prob.fe = "p2p1"
    rng = np.random.default_rng(seed)
    # history as smooth-plus-noise functions of position, so each side evaluates it at its own nodes
    coef = rng.normal(size=(2, 4, 3))

    def field(X, lev):
        u = 10.0 * np.sin(X @ coef[lev, :3]) + coef[lev, 3]
        p = 100.0 * np.cos(X @ coef[lev, :3, 0])
        return u, p

    def init(s, X):
        for lev in range(2):
            u, _ = field(X, lev)
            _, p = field(mesh.coords, lev)
            s.set_state(lev, u, p)

    def drive(s, X, t1):
        pass

    return P2Case("tube_p2", mesh, prob, init, drive)


CASES = [beltrami_p2, tube_p2]


def _oracle(case):
    from oracle.oracle_p2 import OracleSimP2
    o = OracleSimP2(case.mesh, case.prob, solve="dense")
    case.init(o, o.xnode)
    return o


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("make", CASES, ids=lambda f: f.__name__)
def test_p2_matrix_parity(make, precision):
    from scipy.sparse import coo_matrix
    case = make()
    dev = _sim(case.mesh, case.prob, precision=precision)
    X = _dev_xnode(dev, case.mesh)
    case.init(dev, X)
    case.drive(dev, X, case.prob.t0 + case.prob.dt)
    rows, cols, vals, rhs = dev.export_p2()
    orc = _oracle(case)
    case.drive(orc, orc.xnode, case.prob.t0 + case.prob.dt)
    orc.assemble()
    d = _dof_map(_node_map(dev, orc), orc.nu, orc.nv)
    N = 3 * orc.nu + orc.nv
    A = coo_matrix((vals, (d[rows], d[cols])), shape=(N, N)).tocsr()
    b = np.zeros(N)
    b[d] = rhs
    err = rowwise_rel_err(A, orc.A)
    print("%s %s: matrix row-wise rel. error %.3e" % (case.name, precision, err))
    assert err <= 1e-12
    assert rel_l2(b, orc.b) <= 1e-12
    dev.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("make", CASES, ids=lambda f: f.__name__)
def test_p2_steps_parity(make, precision):
    case = make()
    kw = dict(precision=precision, rtol=1e-14, ir_rtol=1e-13, max_iters=4000)
    dev = _sim(case.mesh, case.prob, **kw)
    X = _dev_xnode(dev, case.mesh)
    case.init(dev, X)
    orc = _oracle(case)
    nmap = _node_map(dev, orc)
    tol = 1e-10 if precision == "fp64" else 1e-8
    for k in range(2):
        t1 = case.prob.t0 + (k + 1) * case.prob.dt
        case.drive(dev, X, t1)
        st = dev.step()
        case.drive(orc, orc.xnode, t1)
        uo, po = orc.step()
        ud, pd, _ = dev.solution()
        u_err = rel_l2(ud, uo[nmap])
        p_err = rel_l2(pd, po)
        print("%s %s step %d: %d iterations, u %.2e p %.2e" % (case.name, precision, k, st["gmres_iters"], u_err,
                                                                p_err))
        assert u_err <= tol and p_err <= tol
    dev.close()
