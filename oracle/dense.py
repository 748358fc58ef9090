"""Dense numpy assembly and Cholesky solve for tiny meshes -- TEST INFRASTRUCTURE.

An element-by-element restatement of system (linsys) of Section 2,
independent of ``oracle.c``: per tetrahedron the barycentric gradients come
from ``numpy.linalg.inv`` of the edge matrix, K_e = |tau| G G^T, M_e is the
exact integral of lambda_a lambda_b (|tau|/20 (1 + delta_ab)), and f_e uses the
same 4-point degree-2 rule as the C oracle (the paper fixes no load rule).
The global matrix is a dense numpy array, the solve is a Cholesky
factorisation (``scipy.linalg.cho_factor``).  Only for meshes with a few
hundred unknowns.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

QA = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
QB = (5.0 - np.sqrt(5.0)) / 20.0


def eval_target(target, pts: np.ndarray) -> np.ndarray:
    """ubar at points pts[..., 3]."""
    if target.kind == "sine":
        out = np.full(pts.shape[:-1], float(target.offset))
        for km, am in zip(np.asarray(target.k), np.asarray(target.amp)):
            out = out + am * np.prod(np.sin(km * np.pi * pts), axis=-1)
        return out
    if target.kind == "box":
        lo = np.asarray(target.lo)
        hi = np.asarray(target.hi)
        return np.all((pts > lo) & (pts < hi), axis=-1).astype(np.float64)
    raise ValueError(target.kind)


def element_arrays(xyz: np.ndarray, tets: np.ndarray):
    """Per-element volume, barycentric gradients [ne,4,3], K_e and M_e [ne,4,4]."""
    p = xyz[tets]                                  # [ne, 4, 3]
    B = np.transpose(p[:, 1:, :] - p[:, :1, :], (0, 2, 1))   # columns = edges
    det = np.linalg.det(B)
    vol = np.abs(det) / 6.0
    Binv = np.linalg.inv(B)                        # rows = grad lambda_1..3
    G = np.empty((tets.shape[0], 4, 3))
    G[:, 1:, :] = Binv
    G[:, 0, :] = -Binv.sum(axis=1)
    Ke = vol[:, None, None] * np.einsum("eac,ebc->eab", G, G)
    Me = vol[:, None, None] / 20.0 * (np.ones((4, 4)) + np.eye(4))[None]
    return vol, G, Ke, Me


def element_load(xyz: np.ndarray, tets: np.ndarray, target) -> np.ndarray:
    """f_e[a] = sum_q |tau|/4 ubar(x_q) lambda_a(x_q), 4-point rule [ne, 4]."""
    p = xyz[tets]
    vol = np.abs(np.linalg.det(np.transpose(p[:, 1:, :] - p[:, :1, :], (0, 2, 1)))) / 6.0
    lam = np.full((4, 4), QB) + np.eye(4) * (QA - QB)   # lam[q, a]
    xq = np.einsum("qa,ead->eqd", lam, p)              # [ne, 4 points, 3]
    u = eval_target(target, xq)                         # [ne, 4]
    return (vol[:, None] / 4.0) * np.einsum("eq,qa->ea", u, lam)


def assemble_dense(mesh, rho: float, target):
    """Dense A (interior x interior) and f."""
    interior = np.flatnonzero(mesh.dirichlet == 0)
    dof = -np.ones(mesh.n_vertices, dtype=np.int64)
    dof[interior] = np.arange(interior.size)
    _, _, Ke, Me = element_arrays(mesh.xyz, mesh.tets)
    fe = element_load(mesh.xyz, mesh.tets, target)
    n = interior.size
    A = np.zeros((n, n))
    f = np.zeros(n)
    d = dof[mesh.tets]                              # [ne, 4]
    Ae = rho * Ke + Me
    for a in range(4):
        ia = d[:, a]
        ok = ia >= 0
        np.add.at(f, ia[ok], fe[ok, a])
        for b in range(4):
            jb = d[:, b]
            okb = ok & (jb >= 0)
            np.add.at(A, (ia[okb], jb[okb]), Ae[okb, a, b])
    return A, f


def assemble_full_dense(mesh, rho: float, target=None):
    """Dense K, M over all vertices (before the boundary is eliminated)."""
    nv = mesh.n_vertices
    _, _, Ke, Me = element_arrays(mesh.xyz, mesh.tets)
    K = np.zeros((nv, nv))
    M = np.zeros((nv, nv))
    for a in range(4):
        for b in range(4):
            np.add.at(K, (mesh.tets[:, a], mesh.tets[:, b]), Ke[:, a, b])
            np.add.at(M, (mesh.tets[:, a], mesh.tets[:, b]), Me[:, a, b])
    return K, M


def solve_dense(A: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Cholesky solve of the SPD system."""
    c = sla.cho_factor(A, lower=True)
    return sla.cho_solve(c, f)
