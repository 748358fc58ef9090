"""Seeded synthetic inputs for the reduced optimal-control equation.

This module produces *inputs only*: the tetrahedral mesh of the unit cube
Omega = (0,1)^3 used in the paper's experiments (Section 4), the homogeneous
Dirichlet boundary marker, and descriptors of the target functions ubar
(Sections 4.1 and 4.2).  It holds none of the method's arithmetic: no element
matrices, no quadrature, no target evaluation, no solver.  Both the CPU
oracle and the GPU library consume what is produced here.

Mesh recipe (the paper does not state its tetrahedral split; this is the
reading used throughout): N^3 cubes of edge h = 1/N, each cut into the six
Kuhn tetrahedra that share the diagonal from the cube's (0,0,0) corner to its
(1,1,1) corner.  Vertex (i,j,k) has id i + (N+1)*(j + (N+1)*k) and coordinates
(i,j,k)*h.  Tetrahedron 6*c + p of cube c = ci + N*(cj + N*ck) walks from the
cube's base vertex along the three axes in the order given by the p-th
permutation of KUHN_PERMS.  Optional jitter moves every interior vertex
independently by U(-a*h, a*h) per coordinate, drawn in vertex-id order from
numpy.random.default_rng(seed).

Target recipes:
  * sine modes  ubar = offset + sum_m amp_m prod_d sin(k_{m,d} pi x_d); the
    random recipe draws k ~ U{1..8}^3 (duplicates allowed) and then
    amp ~ N(0,1)/|k|^2 from default_rng(seed), in that order;
  * open-box indicator ubar = 1 on (lo,hi) componentwise, 0 elsewhere
    (points on the box faces get 0);
  * nodal  ubar given by its values at the mesh vertices (device or host
    array supplied by the caller).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


@dataclass
class Mesh:
    """A tetrahedral mesh: vertex coordinates, 4-vertex tets, Dirichlet mask."""

    N: int                      # cubes per edge (h = 1/N)
    xyz: np.ndarray             # float64 [n_vertices, 3]
    tets: np.ndarray            # int32   [n_tets, 4]
    dirichlet: np.ndarray       # uint8   [n_vertices], 1 on Gamma
    jitter: float = 0.0
    seed: Optional[int] = None

    @property
    def n_vertices(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def h(self) -> float:
        return 1.0 / self.N

    @property
    def n_interior(self) -> int:
        return int(self.n_vertices - int(self.dirichlet.sum(dtype=np.int64)))


def kuhn_mesh(N: int, jitter: float = 0.0, seed: Optional[int] = None) -> Mesh:
    """Kuhn 6-tet split of the N^3 cube lattice of the unit cube."""
    if N < 1:
        raise ValueError("N must be >= 1")
    n1 = N + 1
    g = np.arange(n1, dtype=np.float64) / N
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.empty((n1 ** 3, 3), dtype=np.float64)
    xyz[:, 0] = ii.reshape(-1)
    xyz[:, 1] = jj.reshape(-1)
    xyz[:, 2] = kk.reshape(-1)
    del ii, jj, kk

    ib = np.arange(n1, dtype=np.int64)
    on_b = (ib == 0) | (ib == N)
    bk, bj, bi = np.meshgrid(on_b, on_b, on_b, indexing="ij")
    dirichlet = (bi | bj | bk).reshape(-1).astype(np.uint8)
    del bi, bj, bk

    c = np.arange(N, dtype=np.int32)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    base = (ci + n1 * (cj + n1 * ck)).reshape(-1).astype(np.int32)
    del ci, cj, ck
    step = (1, n1, n1 * n1)
    offs = np.zeros((6, 4), dtype=np.int32)
    for p, perm in enumerate(KUHN_PERMS):
        acc = 0
        for s, axis in enumerate(perm):
            acc += step[axis]
            offs[p, s + 1] = acc
    tets = (base[:, None, None] + offs[None, :, :]).reshape(-1, 4)
    del base

    if jitter:
        rng = np.random.default_rng(seed)
        interior = np.flatnonzero(dirichlet == 0)
        h = 1.0 / N
        d = rng.uniform(-jitter * h, jitter * h, size=(interior.size, 3))
        xyz[interior] += d
    return Mesh(N=N, xyz=xyz, tets=np.ascontiguousarray(tets), dirichlet=dirichlet,
                jitter=float(jitter), seed=seed)


@dataclass
class SineModes:
    """ubar = offset + sum_m amp[m] * prod_d sin(k[m,d] * pi * x_d)."""

    k: np.ndarray                 # int32 [n_modes, 3]
    amp: np.ndarray               # float64 [n_modes]
    offset: float = 0.0
    kind: str = field(default="sine", init=False)


@dataclass
class BoxIndicator:
    """ubar = 1 on the open box (lo, hi), 0 elsewhere."""

    lo: Tuple[float, float, float] = (0.25, 0.25, 0.25)
    hi: Tuple[float, float, float] = (0.75, 0.75, 0.75)
    kind: str = field(default="box", init=False)


@dataclass
class Nodal:
    """ubar given by its values at the mesh vertices."""

    values: np.ndarray            # float64 [n_vertices]
    kind: str = field(default="nodal", init=False)


def single_sine(offset: float = 0.0) -> SineModes:
    """ubar = offset + sin(pi x) sin(pi y) sin(pi z) (Sections 4.1 and 4.3)."""
    return SineModes(k=np.array([[1, 1, 1]], dtype=np.int32),
                     amp=np.array([1.0]), offset=float(offset))


def random_sine_modes(seed: int, n_modes: int = 64, kmax: int = 8) -> SineModes:
    """Seeded superposition of sine modes with amplitudes N(0,1)/|k|^2."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, size=(n_modes, 3)).astype(np.int32)
    amp = rng.standard_normal(n_modes) / (k.astype(np.float64) ** 2).sum(axis=1)
    return SineModes(k=k, amp=amp)


def box_indicator() -> BoxIndicator:
    """Discontinuous target of Section 4.2: 1 on (0.25, 0.75)^3."""
    return BoxIndicator()


# --------------------------------------------------------------------------
# Named workloads (sizes and seeds of the synthetic runs)
# --------------------------------------------------------------------------

WORKLOADS = {
    # 16^3 cubes, rho = h^2, the eigenfunction target of Section 4.1
    "cube16_sine111": dict(N=16, jitter=0.0, seed=None, rhos=[1.0 / 256], target="sine111"),
    # 128^3 cubes, jittered interior, three rho values, discontinuous target
    "cube128_jitter_box": dict(N=128, jitter=0.15, seed=1, rhos=[1e-6, 1.0 / 16384, 1e-2],
                               target="box"),
    # 256^3 cubes, rho = h^2, 64 seeded sine modes, mixed precision
    "cube256_modes64": dict(N=256, jitter=0.0, seed=None, rhos=[1.0 / 65536],
                            target=("modes", 1000)),
    # 128^3 cubes, rho = h^2, 32 targets with seeds 2000..2031
    "cube128_modes64_x32": dict(N=128, jitter=0.0, seed=None, rhos=[1.0 / 16384],
                                target=("modes_batch", 2000, 32)),
}


def make_target(spec):
    if spec == "sine111":
        return single_sine()
    if spec == "box":
        return box_indicator()
    if isinstance(spec, tuple) and spec[0] == "modes":
        return random_sine_modes(spec[1])
    if isinstance(spec, tuple) and spec[0] == "modes_batch":
        return [random_sine_modes(spec[1] + j) for j in range(spec[2])]
    raise ValueError(f"unknown target spec {spec!r}")


@dataclass
class Request:
    """One solve request of the serving stream."""

    rid: int
    t_arrival: float      # seconds from stream start
    N: int
    rho: float
    target_seed: int


SERVE_SIZES = (32, 48, 64, 96, 128, 160)


def serving_requests(n_requests: int, rate: float = 200.0, seed: int = 3000,
                     sizes=SERVE_SIZES) -> List[Request]:
    """Poisson arrival stream of solve requests.

    Arrivals: exponential gaps with mean 1/rate from default_rng(seed).
    Per request r: default_rng(seed + 1 + r) draws N uniformly from `sizes`,
    then a coin for rho = h^2 (probability 1/2), else rho = 10^U(-8,-2).
    The target is random_sine_modes(seed + 1 + r).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(n_requests):
        rr = np.random.default_rng(seed + 1 + r)
        N = int(sizes[int(rr.integers(0, len(sizes)))])
        if rr.random() < 0.5:
            rho = 1.0 / (N * N)
        else:
            rho = float(10.0 ** rr.uniform(-8.0, -2.0))
        out.append(Request(rid=r, t_arrival=float(t[r]), N=N, rho=rho, target_seed=seed + 1 + r))
    return out
