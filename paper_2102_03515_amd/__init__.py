"""MI355X-native AMG-preconditioned CG for the reduced optimality system.

Solves the P1 finite element system (rho*K + M) u = f of the singularly
perturbed reaction-diffusion equation -rho*Lap(u) + u = ubar (the reduced
first-order optimality condition of elliptic optimal control with energy
regularization) on one gfx950 GPU.  The work runs in ``libocpamg.so``
(hand-written HIP); ``capi`` is its ctypes binding.
"""
from .capi import (Context, DeviceMesh, Hierarchy, OcpError, SolveInfo, System, amg_setup,  # noqa: F401
                   fe_assemble, fe_derive, lib, pcg_begin, pcg_solve, pcg_solve_batch, pcg_solve_multi, pcg_solve_noalloc,
                   upload_mesh)
from . import capi  # noqa: F401
