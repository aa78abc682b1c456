"""Plain data containers describing a problem (no evaluation logic).

They mirror the C ABI's structs field for field; the device binding marshals
them into those structs and the oracle interprets them on its own.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from .meshes import Mesh, cube_kuhn, tube, spheroid, TUBE_TAGS, SPHEROID_TAGS, CUBE_TAGS


@dataclass
class TimeLaw:
    """constant: p=(v,)  pulsatile: p=(gmin, gmax, period)  ramp: p=(g0, g1, t0, tL)
    ramp2 (open then close): p=(g0, g1, t_open, dur_open, t_close, dur_close, period)
    linear: p=(g0, g1) -> g0 + g1 t   sine: p=(A, w, phi) -> A sin(w t + phi)."""
    kind: str = "constant"
    p: Tuple[float, ...] = (0.0,)


@dataclass
class Profile:
    """uniform (s = -n), parabolic (unit flow rate, radius), or nodal (values set per step)."""
    kind: str = "uniform"
    center: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    normal: Tuple[float, float, float] = (0.0, 0.0, -1.0)   # outward unit normal
    radius: float = 1.0


@dataclass
class Boundary:
    """type: noslip | dirichlet | neumann | resistance.  Dirichlet: u = theta g(t) s(x).
    Neumann: sigma n = -theta h(t) n (profile.kind == 'nodal' means a nodal traction
    vector is supplied per step instead).  Resistance: sigma n = -(theta p0(t) +
    resistance * int (u - u_ALE) . n) n with p0 = law; profile.normal orients the face
    normals outward.  backflow > 0 (neumann, resistance): inertial backflow
    stabilisation, the traction gains backflow * rho/2 min(u . n, 0) u."""
    type: str
    tags: Tuple[int, ...]
    theta: float = 1.0
    law: TimeLaw = field(default_factory=TimeLaw)
    profile: Profile = field(default_factory=Profile)
    resistance: float = 0.0
    backflow: float = 0.0


@dataclass
class Valve:
    """RIIS surface: an annular disc (center, unit normal, outer radius) whose central
    orifice radius follows `orifice` in time; resistance R, half-thickness eps."""
    center: Tuple[float, float, float]
    normal: Tuple[float, float, float]
    outer_radius: float
    orifice: TimeLaw
    R: float
    eps: float


@dataclass
class Problem:
    fe: str = "p1p1"                 # p1p1 | p2p1
    bdf_order: int = 1
    dt: float = 0.01
    t0: float = 0.0
    rho: float = 1.0
    mu: float = 0.01
    diffusion: str = "gradgrad"      # gradgrad | symgrad
    stab: str = "vms_les"            # none | supg_pspg | vms_les
    C_r: Optional[float] = None      # None -> 30 (P1) / 60 (P2)
    implicit: bool = False           # fully implicit formulation (u* = u^{n+1} - u_ALE, implicit
                                     # LES term) solved by Newton's method; else semi-implicit
    ale: bool = False
    ale_tags: Tuple[int, ...] = ()
    ale_law: TimeLaw = field(default_factory=lambda: TimeLaw("constant", (1.0,)))
    # lifting problem of the ALE displacement: harmonic | elastic (E, nu); stiffening
    # alpha per element: none | jacobian (J0, chi): (J0/J)^chi | boundary (beta, gamma):
    # max(d, beta)^-gamma with d the distance of the element's centroid to the faces
    # tagged ale_tags (reference configuration)
    lifting: str = "harmonic"
    lift_E: float = 1.0
    lift_nu: float = 0.3
    stiffening: str = "none"
    stiff_p: Tuple[float, float] = (1.0, 1.0)
    forcing: bool = False
    bcs: List[Boundary] = field(default_factory=list)
    valves: List[Valve] = field(default_factory=list)

    def c_r(self):
        if self.C_r is not None:
            return self.C_r
        return 30.0 if self.fe == "p1p1" else 60.0


@dataclass
class SolverCfg:
    precision: str = "fp64"          # fp64 | fp32_ir
    restart: int = 30
    max_iters: int = 3000
    max_ir: int = 30
    rtol: float = 1e-8
    ir_rtol: float = 1e-8
    inner_rtol: float = 1e-4
    deterministic: bool = True
    collect_timing: int = 0          # n >= 1: time every n-th in-cycle SpMV launch (and every assembly pass)
    schur_degree: int = 16           # precond = "cheb_schur" only
    schur_ratio: float = 300.0
    asm_fp64: bool = False
    precond: str = "amg"             # amg | cheb_schur
    f_degree: int = 0                # amg: Chebyshev degree on the velocity block (1 = block Jacobi;
    f_ratio: float = 0.0             #   0 = library default: 3 / ratio 5 for P1-P1, 12 / 300 for P2-P1)
    amg_degree: int = 2              # amg: Chebyshev smoothing degree per level
    amg_cycle: int = 2               # amg: coarse corrections per level below the finest (2 = W)
    amg_ratio: float = 30.0
    amg_coarse_cycle: int = 0        # amg: coarse corrections per level on the levels held in LDS (0 = 3)


# ----------------------------------------------------------------- configs

def beltrami_cube_problem(n=8, mu=0.01, dt=0.01, bdf_order=1, stab="vms_les"):
    """Unit cube with Beltrami data: Dirichlet (nodal, exact) on five faces and the exact
    traction (nodal) on the face x = 0."""
    mesh = cube_kuhn(n)
    T = CUBE_TAGS
    bcs = [Boundary("dirichlet", (T["x1"], T["y0"], T["y1"], T["z0"], T["z1"]),
                    profile=Profile("nodal")),
           Boundary("neumann", (T["x0"],), profile=Profile("nodal", normal=(-1.0, 0.0, 0.0)))]
    prob = Problem(fe="p1p1", bdf_order=bdf_order, dt=dt, rho=1.0, mu=mu, stab=stab, bcs=bcs)
    return mesh, prob


def tube_problem(mesh, mu=0.035, dt=1e-3, bdf_order=2, peak=50.0, period=1.0, valve=True,
                 R=1e4, eps=0.05, t0=0.0, fe="p1p1"):
    """Pulsatile parabolic inflow at z=0 (flow-rate law g(t) = gmax (1 - cos 2 pi t / T)/2
    with gmax = peak pi r^2 / 2), no-slip wall, zero-traction outlet, optional RIIS disc
    filling the section at mid-length."""
    r = mesh.info.get("radius", 1.0)
    L = mesh.info.get("length", 10.0)
    gmax = peak * np.pi * r * r / 2.0
    bcs = [Boundary("noslip", (TUBE_TAGS["wall"],)),
           Boundary("dirichlet", (TUBE_TAGS["inlet"],), law=TimeLaw("pulsatile", (0.0, gmax, period)),
                    profile=Profile("parabolic", center=(0.0, 0.0, 0.0), normal=(0.0, 0.0, -1.0),
                                    radius=r)),
           Boundary("neumann", (TUBE_TAGS["outlet"],), law=TimeLaw("constant", (0.0,)),
                    profile=Profile("uniform", normal=(0.0, 0.0, 1.0)))]
    valves = []
    if valve:
        valves.append(Valve(center=(0.0, 0.0, L / 2.0), normal=(0.0, 0.0, 1.0),
                            outer_radius=10.0 * r, orifice=TimeLaw("constant", (0.0,)), R=R, eps=eps))
    return Problem(fe=fe, bdf_order=bdf_order, dt=dt, t0=t0, rho=1.0, mu=mu, stab="vms_les",
                   bcs=bcs, valves=valves)


def tube_poiseuille_state(mesh, prob, t):
    """Steady Poiseuille field of the tube at the inflow rate of time t (an initial
    condition, not a solution of the stabilised discrete problem): u_z = 2 g(t) / (pi r^2)
    (1 - rho^2 / r^2) with g the pulsatile flow-rate law of the inlet, and the matching
    linear pressure drop 8 mu g(t) / (pi r^4) (L - z) to a zero outlet pressure."""
    r = mesh.info.get("radius", 1.0)
    L = mesh.info.get("length", 10.0)
    inlet = [b for b in prob.bcs if b.type == "dirichlet"][0]
    gmin, gmax, period = inlet.law.p
    g = gmin + (gmax - gmin) * 0.5 * (1.0 - np.cos(2.0 * np.pi * t / period))
    x = mesh.coords
    rr = np.minimum((x[:, 0] ** 2 + x[:, 1] ** 2) / (r * r), 1.0)
    u = np.zeros_like(x)
    u[:, 2] = 2.0 * g / (np.pi * r * r) * (1.0 - rr)
    p = 8.0 * prob.mu * g / (np.pi * r ** 4) * (L - x[:, 2])
    return u, p


def chamber_problem(mesh, mu=0.035, dt=5e-4, R=1e4, eps=0.1, cycle=0.8):
    """Truncated spheroid with a prescribed 10% radial contraction of the whole boundary
    (d = -0.1 (1 - cos 2 pi t / cycle)/2 (0, y, z), harmonically extended), no-slip wall,
    zero-traction caps, two RIIS annular valves at x = -3 (inlet) and x = +3 (outlet)."""
    xcut = mesh.info.get("xcut", 3.5)
    a, b, _ = mesh.info.get("semi", (4.0, 3.0, 3.0))
    bcs = [Boundary("noslip", (SPHEROID_TAGS["wall"],)),
           Boundary("neumann", (SPHEROID_TAGS["cap_lo"],), law=TimeLaw("constant", (0.0,)),
                    profile=Profile("uniform", normal=(-1.0, 0.0, 0.0))),
           Boundary("neumann", (SPHEROID_TAGS["cap_hi"],), law=TimeLaw("constant", (0.0,)),
                    profile=Profile("uniform", normal=(1.0, 0.0, 0.0)))]
    valves = []
    for xv, (t_open, t_close) in ((3.0, (0.0, 0.35)), (-3.0, (0.40, 0.75))):
        rr = 0.8 * b * np.sqrt(1.0 - xv * xv / (a * a))
        valves.append(Valve(center=(xv, 0.0, 0.0), normal=(1.0, 0.0, 0.0), outer_radius=10.0,
                            orifice=TimeLaw("ramp2", (0.0, rr, t_open, 0.05, t_close, 0.05, cycle)),
                            R=R, eps=eps))
    prob = Problem(fe="p1p1", bdf_order=2, dt=dt, rho=1.0, mu=mu, stab="vms_les", bcs=bcs,
                   valves=valves, ale=True,
                   ale_tags=(SPHEROID_TAGS["wall"], SPHEROID_TAGS["cap_lo"], SPHEROID_TAGS["cap_hi"]),
                   ale_law=TimeLaw("pulsatile", (0.0, 1.0, cycle)))
    return prob


def chamber_displacement_shape(mesh):
    """Nodal shape D(x^) = -0.1 (0, y^, z^) of the chamber's wall motion (linear, hence
    exactly harmonic)."""
    d = np.zeros_like(mesh.coords)
    d[:, 1] = -0.1 * mesh.coords[:, 1]
    d[:, 2] = -0.1 * mesh.coords[:, 2]
    return d
