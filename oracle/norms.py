"""Error norms against the closed-form solutions -- TEST INFRASTRUCTURE.

For a target that is a finite sum of Dirichlet eigenfunctions of the unit cube,
ubar = sum_m a_m prod_d sin(k_{m,d} pi x_d), equation (6) is solved mode by
mode: u_rho = sum_m a_m / (1 + rho pi^2 |k_m|^2) prod_d sin(k_{m,d} pi x_d).
With a single mode k = (1,1,1) this is the manufactured solution of
Section 4.1.  The errors ||u_rho - u_rho,h||_L2 and ||grad(u_rho - u_rho,h)||_L2
of Tables 1 and 2 are integrated element by element with a conical-product
(collapsed Gauss-Jacobi) rule built from ``scipy.special.roots_jacobi``.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi


def conical_rule(n: int = 4):
    """Points (barycentric lambda_1..3) and weights on the unit tetrahedron.

    x = s1, y = (1-s1) s2, z = (1-s1)(1-s2) s3 with Jacobian (1-s1)^2 (1-s2);
    s1 uses Gauss-Jacobi with weight (1-s)^2, s2 weight (1-s), s3 Legendre.
    Exact for polynomials of degree 2n-1; weights sum to 1/6.
    """
    pts, wts = [], []
    for a in (2, 1, 0):
        xi, w = roots_jacobi(n, a, 0)
        pts.append((1.0 + xi) / 2.0)
        wts.append(w / 2.0 ** (a + 1))
    s1, s2, s3 = np.meshgrid(*pts, indexing="ij")
    w = np.einsum("i,j,k->ijk", *wts)
    x = s1
    y = (1 - s1) * s2
    z = (1 - s1) * (1 - s2) * s3
    return np.stack([x.ravel(), y.ravel(), z.ravel()], -1), w.ravel()


def closed_form(target, rho: float):
    """Callables u(x) and grad u(x) of the exact solution of eq. (5)."""
    if target.kind != "sine" or float(target.offset) != 0.0:
        raise ValueError("closed form needs a homogeneous sine-mode target")
    ks = np.asarray(target.k, dtype=np.float64)
    amps = np.asarray(target.amp, dtype=np.float64)
    coef = amps / (1.0 + rho * np.pi ** 2 * (ks ** 2).sum(axis=1))

    def u(p):
        out = np.zeros(p.shape[:-1])
        for k, c in zip(ks, coef):
            out = out + c * np.prod(np.sin(k * np.pi * p), axis=-1)
        return out

    def grad(p):
        out = np.zeros(p.shape)
        for k, c in zip(ks, coef):
            s = np.sin(k * np.pi * p)
            co = np.cos(k * np.pi * p) * k * np.pi
            out[..., 0] += c * co[..., 0] * s[..., 1] * s[..., 2]
            out[..., 1] += c * s[..., 0] * co[..., 1] * s[..., 2]
            out[..., 2] += c * s[..., 0] * s[..., 1] * co[..., 2]
        return out

    return u, grad


def fe_errors(mesh, u_vertices: np.ndarray, target, rho: float, n_quad: int = 4,
              chunk: int = 200_000):
    """(||u - u_h||_L2, ||grad(u - u_h)||_L2) for nodal values u_vertices."""
    u_ex, g_ex = closed_form(target, rho)
    bary, w = conical_rule(n_quad)
    lam = np.concatenate([1.0 - bary.sum(axis=1, keepdims=True), bary], axis=1)  # [nq, 4]
    e2 = 0.0
    g2 = 0.0
    for s in range(0, mesh.n_tets, chunk):
        t = mesh.tets[s:s + chunk]
        p = mesh.xyz[t]                                     # [ne,4,3]
        B = np.transpose(p[:, 1:, :] - p[:, :1, :], (0, 2, 1))
        det = np.abs(np.linalg.det(B))
        Binv = np.linalg.inv(B)
        G = np.concatenate([-Binv.sum(axis=1, keepdims=True), Binv], axis=1)   # [ne,4,3]
        uh = u_vertices[t]                                  # [ne,4]
        xq = np.einsum("qa,ead->eqd", lam, p)               # [ne,nq,3]
        uhq = uh @ lam.T                                    # [ne,nq]
        diff = u_ex(xq) - uhq
        e2 += float(np.sum(det[:, None] * w[None, :] * diff ** 2))
        guh = np.einsum("ea,ead->ed", uh, G)                # [ne,3]
        gd = g_ex(xq) - guh[:, None, :]
        g2 += float(np.sum(det[:, None] * w[None, :] * np.sum(gd ** 2, axis=-1)))
    return np.sqrt(e2), np.sqrt(g2)


def target_error_l2(mesh, u_vertices: np.ndarray, target, n_quad: int = 4,
                    chunk: int = 200_000) -> float:
    """||ubar - u_h||_L2 (Table 3's L2 column, squared there)."""
    bary, w = conical_rule(n_quad)
    lam = np.concatenate([1.0 - bary.sum(axis=1, keepdims=True), bary], axis=1)
    from .dense import eval_target
    e2 = 0.0
    for s in range(0, mesh.n_tets, chunk):
        t = mesh.tets[s:s + chunk]
        p = mesh.xyz[t]
        B = np.transpose(p[:, 1:, :] - p[:, :1, :], (0, 2, 1))
        det = np.abs(np.linalg.det(B))
        xq = np.einsum("qa,ead->eqd", lam, p)
        diff = eval_target(target, xq) - u_vertices[t] @ lam.T
        e2 += float(np.sum(det[:, None] * w[None, :] * diff ** 2))
    return float(np.sqrt(e2))
