"""Writes tube983k_poiseuille_oracle.json: sampled oracle solutions of the first
three steps of the 983,040-tet tube (the benchmark's mesh and problem) started
from the Poiseuille field of the inflow rate at t0 = 0.25 s.

Calls only the oracle (its assembly and its own GMRES + SIMPLE solve to a
relative residual of 1e-14) and the seeded input generators.  A direct solve at
this size is out of reach, so the oracle's iterative solve at 1e-14 stands in
for x = A^{-1} b (Sec. 2.4 solver, run to a tolerance far below the parity
bound).  Stored per step: the values at 2048 seeded vertices (u and p), the full
L2 norms of u and p, the oracle's iteration count and final residual.

Run:  python tests/golden/make_tube983k_oracle.py   (about an hour on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from inputs import tube                                        # noqa: E402
from inputs.problem import tube_problem, tube_poiseuille_state  # noqa: E402
from inputs.rng import permutation                             # noqa: E402
from oracle import OracleSim                                   # noqa: E402

T0, STEPS, NSAMPLE, SAMPLE_SEED, RTOL = 0.25, 3, 2048, 77, 1e-14


def main():
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tube983k_poiseuille_oracle.json")
    mesh = tube(nxy=32, nz=160, seed=0)
    prob = tube_problem(mesh, t0=T0)
    sim = OracleSim(mesh, prob, solve="gmres", gmres_rtol=RTOL, max_iters=200000)
    for lev in range(prob.bdf_order):
        sim.set_state(lev, *tube_poiseuille_state(mesh, prob, T0 - lev * prob.dt))
    sample = np.sort(permutation(SAMPLE_SEED, mesh.nv)[:NSAMPLE])
    steps = []
    for k in range(STEPS):
        t0 = time.time()
        u, p = sim.step()
        print("step %d: %d oracle iterations, residual %.2e, %.0f s" % (k, sim.last_iters, sim.last_res,
                                                                        time.time() - t0), flush=True)
        steps.append({"t": sim.t, "iters": sim.last_iters, "rel_residual": sim.last_res,
                      "u_norm": float(np.linalg.norm(u)), "p_norm": float(np.linalg.norm(p)),
                      "u": [[float(c) for c in u[v]] for v in sample], "p": [float(p[v]) for v in sample]})
    doc = {"_source": "oracle only: make_tube983k_oracle.py (tube 32x32x160 seed 0, tube_problem(t0=0.25), "
                      "Poiseuille history at t0 and t0 - dt, oracle GMRES+SIMPLE to rtol 1e-14)",
           "mesh": {"nxy": 32, "nz": 160, "seed": 0, "n_tets": int(mesh.nt), "n_vertices": int(mesh.nv)},
           "t0": T0, "oracle_rtol": RTOL, "sample_seed": SAMPLE_SEED,
           "vertices": [int(v) for v in sample], "steps": steps}
    with open(out_path, "w") as fh:
        json.dump(doc, fh)
    print("wrote", out_path)


if __name__ == "__main__":
    main()
