"""FP64 CPU oracle (test infrastructure only; see oracle.py)."""
from .oracle import (OracleSim, element_p1, time_law, profile_values, dirichlet_sets, BDF, lib, build)
