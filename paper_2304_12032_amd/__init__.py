"""MI355X (gfx950) library for one semi-implicit BDF time step of the VMS-LES
Navier-Stokes equations on tetrahedra with RIIS valves and ALE motion.

The numerical work runs in the HIP library liblxns.so (C ABI in
include/lxns.h); this package holds its sources, the build script and a
ctypes binding.
"""
from .lxns import Sim, Server, LxError, lib, check, LIB_PATH, torch_allocator

__all__ = ["Sim", "Server", "LxError", "lib", "check", "LIB_PATH", "torch_allocator"]
