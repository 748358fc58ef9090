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


def control_and_adjoint(mesh, u_vertices: np.ndarray, target, rho: float, nodal_target=None):
    """Adjoint p = -rho u (gradient equation (4), Section 1) and control
    z = (ubar - u) / rho (state equation (2) with the reduced equation (5)),
    both at the vertices of the mesh from the nodal state u.  ubar is taken at
    the vertices (its values there for a P1 target)."""
    from .dense import eval_target
    u = np.asarray(u_vertices, dtype=np.float64)
    ub = np.asarray(nodal_target, dtype=np.float64) if nodal_target is not None else eval_target(target, mesh.xyz)
    return -rho * u, (ub - u) / rho


def closed_form_control(target, rho: float):
    """z_rho(x) = (ubar - u_rho)/rho of a homogeneous sine-mode target: mode m
    contributes a_m pi^2 |k_m|^2 / (1 + rho pi^2 |k_m|^2) prod_d sin(k_md pi x_d)
    (-Lap of the mode-by-mode state)."""
    ks = np.asarray(target.k, dtype=np.float64)
    amps = np.asarray(target.amp, dtype=np.float64)
    lam = np.pi ** 2 * (ks ** 2).sum(axis=1)
    coef = amps * lam / (1.0 + rho * lam)

    def z(p):
        out = np.zeros(p.shape[:-1])
        for k, c in zip(ks, coef):
            out = out + c * np.prod(np.sin(k * np.pi * p), axis=-1)
        return out

    return z


def box_series_coefficient(k: int, lo: float = 0.25, hi: float = 0.75) -> float:
    """b_k = 2 int_lo^hi sin(k pi x) dx = (2/(k pi)) (cos(k pi lo) - cos(k pi hi)):
    the sine-series coefficient of the indicator of (lo, hi) on (0, 1)."""
    return 2.0 / (k * np.pi) * (np.cos(k * np.pi * lo) - np.cos(k * np.pi * hi))


def box_indicator_state_on_grid(N: int, rho: float, K: int = 63, lo: float = 0.25, hi: float = 0.75):
    """u_rho of eq. (5) for the box indicator target, truncated to wave
    numbers <= K in every direction, at the lattice points (i/N, j/N, k/N):
    u_rho = sum_k b_k1 b_k2 b_k3 / (1 + rho pi^2 |k|^2) prod_d sin(k_d pi x_d)
    (the target's sine series solved mode by mode).  Returns [N+1]^3 indexed
    [i, j, k] with x = i/N.  A truncation-limited reference (loose for small
    rho, where u_rho approaches the discontinuous target)."""
    ks = np.arange(1, K + 1)
    b = box_series_coefficient(ks, lo, hi)
    k2 = ks[:, None, None] ** 2 + ks[None, :, None] ** 2 + ks[None, None, :] ** 2
    C = b[:, None, None] * b[None, :, None] * b[None, None, :] / (1.0 + rho * np.pi ** 2 * k2)
    x = np.arange(N + 1) / N
    S = np.sin(np.pi * ks[:, None] * x[None, :])       # [K, N+1]
    return np.einsum("abc,ai,bj,ck->ijk", C, S, S, S, optimize=True)


def error_indicator(mesh, u_vertices: np.ndarray, target, rho: float, nodal_target=None) -> np.ndarray:
    """Residual error indicator per tetrahedron for -rho Lap u + u = ubar and a
    P1 state u_h (the robust weighting of Verfuerth's estimators for
    reaction-diffusion problems):
        eta_T^2 = a_T^2 ||ubar - u_h||^2_T
                + 1/2 sum over interior faces F of T of rho^(-1/2) a_F |F| (rho [grad u_h . n_F])^2,
        a_S = min(1, h_S / sqrt(rho)), h_S the longest edge of S.
    ||ubar - u_h||^2_T by the 4-point degree-2 rule (barycentric (a, b, b, b)
    and permutations, a = (5 + 3 sqrt5)/20, b = (5 - sqrt5)/20, weights
    |T|/4); faces with one tetrahedron lie on the boundary and add nothing."""
    from .dense import eval_target
    xyz = np.asarray(mesh.xyz, dtype=np.float64)
    tets = np.asarray(mesh.tets, dtype=np.int64)
    u = np.asarray(u_vertices, dtype=np.float64)
    p = xyz[tets]                                              # [nt,4,3]
    B = np.transpose(p[:, 1:, :] - p[:, :1, :], (0, 2, 1))     # columns: edges from vertex 0
    vol = np.abs(np.linalg.det(B)) / 6.0
    Gi = np.linalg.inv(B)                                      # rows: grad lambda_1..3
    uh = u[tets]
    grad = np.einsum("ea,ead->ed", uh[:, 1:] - uh[:, :1], Gi)
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    h = np.max([np.linalg.norm(p[:, a] - p[:, b], axis=1) for a, b in edges], axis=0)
    a_ = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
    b_ = (5.0 - np.sqrt(5.0)) / 20.0
    r2 = np.zeros(len(tets))
    for q in range(4):
        lam = np.full(4, b_)
        lam[q] = a_
        xq = np.einsum("a,ead->ed", lam, p)
        uq = uh @ lam
        if nodal_target is not None:
            tq = np.asarray(nodal_target)[tets] @ lam
        else:
            tq = eval_target(target, xq)
        r2 += (tq - uq) ** 2
    r2 *= vol / 4.0
    srho = np.sqrt(rho)
    eta = np.minimum(1.0, h / srho) ** 2 * r2
    # interior faces: the same sorted vertex triple in two tetrahedra
    faces = np.concatenate([np.sort(np.delete(tets, a, axis=1), axis=1) for a in range(4)])
    owner = np.tile(np.arange(len(tets)), 4)
    order = np.lexsort(faces.T[::-1])
    fs, ow = faces[order], owner[order]
    same = np.all(fs[1:] == fs[:-1], axis=1)
    i1 = np.flatnonzero(same)
    t1, t2, f = ow[i1], ow[i1 + 1], fs[i1]
    e1 = xyz[f[:, 1]] - xyz[f[:, 0]]
    e2 = xyz[f[:, 2]] - xyz[f[:, 0]]
    nrm = np.cross(e1, e2)
    nn = np.linalg.norm(nrm, axis=1)
    area = 0.5 * nn
    hf = np.max([np.linalg.norm(e1, axis=1), np.linalg.norm(e2, axis=1), np.linalg.norm(e2 - e1, axis=1)], axis=0)
    jump = rho * np.sum((grad[t1] - grad[t2]) * nrm, axis=1) / nn
    c = 0.5 / srho * np.minimum(1.0, hf / srho) * area * jump ** 2
    np.add.at(eta, t1, c)
    np.add.at(eta, t2, c)
    return eta
