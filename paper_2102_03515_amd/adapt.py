"""Adaptive solve loop of Sections 4.2 and 4.3: solve, estimate, mark, refine.

Each step assembles A = rho K + M and f on the current mesh (fe_assemble),
builds the AMG hierarchy (amg_setup), solves by PCG (pcg_solve), evaluates
the residual error indicator on the device (fe_error_indicator), and refines
the host mesh by bisection of the tetrahedra Doerfler's criterion marks
(ocp_refiner_refine).  All arithmetic runs in the library; this module only
sequences the calls and moves the mesh and the indicator between host and
device.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import capi


@dataclass
class Step:
    n_vertices: int
    n_tets: int
    n_dofs: int
    iterations: int
    true_rel_res: float
    eta: float               # sqrt of the summed indicators
    marked: int
    levels: int


@dataclass
class AdaptiveResult:
    steps: List[Step] = field(default_factory=list)
    mesh: Optional[object] = None       # the last mesh (ocp_inputs.Mesh-like, host arrays)
    u: Optional[object] = None          # the last state on its vertices (torch, device)
    system: Optional[object] = None
    eta2: Optional[np.ndarray] = None   # the last indicators


class HostMesh:
    """A mesh in host memory (the fields the library's upload reads)."""

    def __init__(self, xyz, tets, dirichlet, N=0):
        self.xyz = xyz
        self.tets = tets
        self.dirichlet = dirichlet
        self.N = N

    @property
    def n_vertices(self):
        return int(self.xyz.shape[0])

    @property
    def n_tets(self):
        return int(self.tets.shape[0])


def adaptive_solve(ctx, mesh, rho: float, target, steps: int, theta: float = 0.5, rtol: float = 1e-8,
                   precision: int = capi.PREC_FP64, amg_kw: Optional[dict] = None, stop=capi.STOP_L2):
    """Run `steps` solve-estimate-mark-refine cycles from `mesh` (Kuhn-ordered
    tetrahedra); the last step solves without refining."""
    import torch
    ref = capi.Refiner(mesh.xyz, mesh.tets)
    res = AdaptiveResult()
    try:
        for k in range(steps):
            xyz, tets, dirichlet = ref.get()
            hm = HostMesh(xyz, tets, dirichlet, getattr(mesh, "N", 0))
            dm = capi.upload_mesh(hm)
            s = capi.fe_assemble(ctx, dm, rho, target)
            h = capi.amg_setup(ctx, s, precision=precision, **(amg_kw or {}))
            u, info, rc = capi.pcg_solve(ctx, s, h, rtol=rtol, stop=stop)
            if rc != capi.OK:
                raise capi.OcpError(rc, f"adaptive step {k}: solve status {rc}")
            eta2_dev = s.error_indicator(target, u)
            eta2 = eta2_dev.cpu().numpy()
            marked = 0
            if k + 1 < steps:
                marked = ref.refine(eta2, theta)
            res.steps.append(Step(n_vertices=hm.n_vertices, n_tets=hm.n_tets, n_dofs=s.n,
                                  iterations=info.iterations, true_rel_res=info.true_rel_res,
                                  eta=float(np.sqrt(eta2.sum())), marked=marked, levels=h.n_levels))
            h.close()
            if k + 1 < steps:
                s.close()
                del u
                torch.cuda.synchronize()
            else:
                res.mesh, res.u, res.system, res.eta2 = hm, u, s, eta2
    finally:
        ref.close()
    return res
