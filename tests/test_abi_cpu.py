"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point that include/lxns.h declares, and rejects bad input before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from inputs import cube_kuhn, tube
from inputs.problem import SolverCfg, beltrami_cube_problem, tube_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lxns.h")).read()
    return sorted(set(re.findall(r"^\s*(?:lx_status|void|const char \*)\s*\*?\s*(lx_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2304_12032_amd import lib
    L = lib()
    syms = declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(L, s), s


def test_binding_loads_torch_before_the_library():
    """The library must bind to the HIP runtime PyTorch ships (same soname as ROCm's):
    loading the library first would bring a second runtime into the process, and
    torch would then find no device.  A fresh interpreter that only loads the library
    has torch loaded before it."""
    import subprocess
    import sys
    code = ("import sys; from paper_2304_12032_amd import lxns; assert 'torch' not in sys.modules; "
            "lxns.lib(); assert 'torch' in sys.modules")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr


def test_binding_signatures_cover_header():
    from paper_2304_12032_amd.lxns import SIGNATURES
    assert set(declared_symbols()) == set(SIGNATURES)


def _create(mesh, prob, solver):
    from paper_2304_12032_amd import Sim
    return Sim(mesh, prob, solver)


def test_degenerate_tet_rejected():
    from paper_2304_12032_amd import LxError
    mesh, prob = beltrami_cube_problem(2)
    mesh.coords = mesh.coords.copy()
    t = mesh.tets[5]
    # collapse one tet: move a vertex onto the plane of the other three
    mesh.coords[t[3]] = mesh.coords[t[0]] + 0.3 * (mesh.coords[t[1]] - mesh.coords[t[0]]) \
        + 0.3 * (mesh.coords[t[2]] - mesh.coords[t[0]])
    with pytest.raises(LxError) as ei:
        _create(mesh, prob, SolverCfg())
    assert ei.value.status == -5


def test_vertex_out_of_range_rejected():
    from paper_2304_12032_amd import LxError
    mesh, prob = beltrami_cube_problem(2)
    mesh.tets = mesh.tets.copy()
    mesh.tets[0, 0] = mesh.nv + 3
    with pytest.raises(LxError) as ei:
        _create(mesh, prob, SolverCfg())
    assert ei.value.status == -5


@pytest.mark.parametrize("field,value", [("bdf_order", 4), ("dt", 0.0), ("stab", "bogus")])
def test_bad_problem_rejected(field, value):
    from paper_2304_12032_amd import LxError
    mesh, prob = beltrami_cube_problem(2)
    setattr(prob, field, value)
    with pytest.raises((LxError, KeyError)) as ei:
        _create(mesh, prob, SolverCfg())
    if isinstance(ei.value, LxError):
        assert ei.value.status == -1


@pytest.mark.parametrize("what", ["ale", "cheb_schur"])
def test_p2p1_unsupported_options_rejected(what):
    """P2-P1 is built without ALE and with the AMG preconditioner only: both are
    rejected during validation, before any device call."""
    from paper_2304_12032_amd import LxError
    mesh, prob = beltrami_cube_problem(2)
    prob.fe = "p2p1"
    sv = SolverCfg()
    if what == "ale":
        prob.ale = True
    else:
        sv.precond = "cheb_schur"
    with pytest.raises(LxError) as ei:
        _create(mesh, prob, sv)
    assert ei.value.status == -1


def test_server_rejects_p2p1_request():
    from paper_2304_12032_amd import Server, LxError
    m = tube(nxy=4, nz=8, length=2.0)
    prob = tube_problem(m)
    prob.fe = "p2p1"
    srv = Server(hbm_budget_bytes=1 << 34, max_active=4)
    with pytest.raises(LxError) as ei:
        srv.submit(m, prob, SolverCfg(), 5)
    assert ei.value.status == -1
    srv.close()


def test_bad_restart_rejected():
    from paper_2304_12032_amd import LxError
    mesh, prob = beltrami_cube_problem(2)
    with pytest.raises(LxError) as ei:
        _create(mesh, prob, SolverCfg(restart=65))
    assert ei.value.status == -1


@pytest.mark.parametrize("field,value", [("amg_coarse_cycle", 7), ("amg_coarse_cycle", -1), ("amg_cycle", 4),
                                         ("amg_degree", 9), ("f_degree", 17), ("amg_ratio", 0.5)])
def test_bad_amg_parameters_rejected(field, value):
    """The solver checks the multigrid parameters before touching a device."""
    from paper_2304_12032_amd import LxError
    mesh, prob = beltrami_cube_problem(2)
    with pytest.raises(LxError) as ei:
        _create(mesh, prob, SolverCfg(**{field: value}))
    assert ei.value.status == -1


def test_server_rejects_request_over_budget():
    from paper_2304_12032_amd import Server, LxError
    m = tube(nxy=4, nz=8, length=2.0)
    srv = Server(hbm_budget_bytes=1 << 20, max_active=4)
    with pytest.raises(LxError) as ei:
        srv.submit(m, tube_problem(m), SolverCfg(precision="fp32_ir"), 5)
    assert ei.value.status == -6
    srv2 = Server(hbm_budget_bytes=1 << 34, max_active=4)
    t = srv2.submit(m, tube_problem(m), SolverCfg(precision="fp32_ir"), 5)
    assert srv2.poll(t)["state"] == "queued"
    assert srv2.poll(t)["footprint_bytes"] > 0
    srv.close()
    srv2.close()


@pytest.mark.parametrize("what", ["p2_resistance", "p2_backflow", "negative_resistance", "backflow_on_dirichlet"])
def test_bad_outflow_conditions_rejected(what):
    """Resistance and backflow terms are built for P1-P1 Neumann-type conditions with
    non-negative coefficients; anything else is rejected during validation."""
    from paper_2304_12032_amd import LxError
    from inputs.meshes import TUBE_TAGS
    from inputs.problem import Boundary, Profile, TimeLaw
    m = tube(nxy=3, nz=4, length=1.0)
    prob = tube_problem(m, valve=False)
    out = Boundary("resistance", (TUBE_TAGS["outlet"],), law=TimeLaw("constant", (0.0,)),
                   profile=Profile("uniform", normal=(0.0, 0.0, 1.0)), resistance=10.0)
    if what == "p2_resistance":
        prob.fe = "p2p1"
    elif what == "p2_backflow":
        prob.fe = "p2p1"
        out.type, out.resistance, out.backflow = "neumann", 0.0, 1.0
    elif what == "negative_resistance":
        out.resistance = -1.0
    else:
        prob.bcs[1].backflow = 1.0
    prob.bcs[2] = out
    with pytest.raises(LxError) as ei:
        _create(m, prob, SolverCfg())
    assert ei.value.status == -1


@pytest.mark.parametrize("what", ["nu_half", "E_zero", "stiff_negative"])
def test_bad_lifting_parameters_rejected(what):
    """The lifting moduli and stiffening parameters are checked before any device call."""
    from paper_2304_12032_amd import LxError
    from inputs.meshes import TUBE_TAGS
    m = tube(nxy=3, nz=4, length=1.0)
    prob = tube_problem(m, valve=False)
    prob.ale = True
    prob.ale_tags = (TUBE_TAGS["wall"],)
    prob.lifting = "elastic"
    if what == "nu_half":
        prob.lift_nu = 0.5
    elif what == "E_zero":
        prob.lift_E = 0.0
    else:
        prob.stiffening, prob.stiff_p = "boundary", (0.1, -1.0)
    with pytest.raises(LxError) as ei:
        _create(m, prob, SolverCfg())
    assert ei.value.status == -1


@pytest.mark.parametrize("what", ["p2", "no_newton_updates"])
def test_implicit_unsupported_options_rejected(what):
    """The implicit formulation runs P1-P1 (FP64 or FP32 updates, outflow terms included)
    with at least one Newton update; anything else is rejected during validation."""
    from paper_2304_12032_amd import LxError
    m = tube(nxy=3, nz=4, length=1.0)
    prob = tube_problem(m, valve=False)
    prob.implicit = True
    sv = SolverCfg()
    if what == "p2":
        prob.fe = "p2p1"
    else:
        sv.max_ir = 0
    with pytest.raises(LxError) as ei:
        _create(m, prob, sv)
    assert ei.value.status == -1
