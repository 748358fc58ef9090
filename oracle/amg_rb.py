"""The red-black AMG of Section 3.1 written out from its definitions -- TEST INFRASTRUCTURE.

Only the test suite may import this module; the product package never does.

Section 3.1 coarsens by a red-black colouring of the matrix graph: pick an
unmarked dof, mark it black (coarse) and its unmarked neighbours red (fine),
repeat until every dof is marked; a fine dof is interpolated by the average
of its coarse neighbours (the operator P); the coarse operator is Galerkin's
A_c = P^T A P; one V-cycle applies a forward Gauss-Seidel sweep before and a
backward sweep after the coarse correction (with the coarse problem solved
the same way, recursively, from a zero initial guess).

The paper leaves the visiting order open.  Here (as on the GPU, where the
same set comes out of parallel rounds) the dofs are picked in decreasing
order of the key (lowbias32(i XOR salt) >> 2, i) of the aggregation module,
salt = 0x9E3779B9 (level + 1).  Gauss-Seidel visits the dofs colour by colour
in a colouring of the graph of A (every off-diagonal entry of the pattern
couples): colour c holds every still uncoloured dof whose key
(lowbias32(i XOR salt') >> 2, i), salt' = salt XOR 0x5bd1e995, exceeds the
keys of all its uncoloured neighbours.  Inside one colour no two dofs are
coupled, so the order within a colour does not matter.  Loops are plain Python (small
problems only); scipy.sparse does the products.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .amg import level_salt, priority, structural_product

COLOUR_SALT = 0x5BD1E995


def key(i: int, salt: int):
    return (priority(i, salt), i)


def neighbours(A: sp.csr_matrix, theta: float = 0.0):
    """Strong neighbours as in the aggregation module (theta = 0: every
    off-diagonal pattern entry)."""
    from .amg import strong_neighbours
    return strong_neighbours(A, theta)


def red_black_split(nbrs, salt: int) -> np.ndarray:
    """Sequential red-black colouring in decreasing key: True = black (coarse)."""
    n = len(nbrs)
    order = sorted(range(n), key=lambda i: key(i, salt), reverse=True)
    mark = np.zeros(n, dtype=np.int8)        # 0 unmarked, 1 black, 2 red
    for i in order:
        if mark[i] != 0:
            continue
        mark[i] = 1
        for j in nbrs[i]:
            if mark[j] == 0:
                mark[j] = 2
    return mark == 1


def averaging_prolongator(nbrs, coarse: np.ndarray) -> sp.csr_matrix:
    """P[i, c(i)] = 1 for a coarse dof; P[i, c(j)] = 1 / #coarse neighbours
    for each coarse neighbour j of a fine dof."""
    n = len(nbrs)
    cidx = -np.ones(n, dtype=np.int64)
    cidx[coarse] = np.arange(int(coarse.sum()))
    rows, cols, vals = [], [], []
    for i in range(n):
        if coarse[i]:
            rows.append(i)
            cols.append(cidx[i])
            vals.append(1.0)
            continue
        cn = sorted(j for j in nbrs[i] if coarse[j])
        if not cn:
            raise RuntimeError(f"fine dof {i} has no coarse neighbour")
        for j in cn:
            rows.append(i)
            cols.append(cidx[j])
            vals.append(1.0 / len(cn))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, int(coarse.sum())))


def colouring(A: sp.csr_matrix, salt: int) -> np.ndarray:
    """Colour of every dof (see the module docstring)."""
    A = A.tocsr()
    n = A.shape[0]
    adj = [[int(j) for j in A.indices[A.indptr[i]:A.indptr[i + 1]] if j != i] for i in range(n)]
    keys = [key(i, salt) for i in range(n)]
    colour = -np.ones(n, dtype=np.int64)
    c = 0
    while (colour < 0).any():
        taken = [i for i in range(n) if colour[i] < 0 and
                 all(keys[i] > keys[j] for j in adj[i] if colour[j] < 0)]
        colour[taken] = c
        c += 1
    return colour


def build_hierarchy(A: sp.csr_matrix, theta: float = 0.0, coarse_max: int = 512, max_levels: int = 10):
    """Levels as dicts {A, coarse, P, colour}; the last has A only (colour too
    when it has more than 2048 rows)."""
    levels = []
    A = A.tocsr()
    for lev in range(max_levels):
        n = A.shape[0]
        salt = level_salt(lev)
        if n <= coarse_max or lev + 1 >= max_levels:
            levels.append({"A": A})
            break
        colour = colouring(A, salt ^ COLOUR_SALT)
        nbrs = neighbours(A, theta)
        coarse = red_black_split(nbrs, salt)
        nc = int(coarse.sum())
        if nc <= 0 or 2 * nc > n:
            levels.append({"A": A, "colour": colour})
            break
        P = averaging_prolongator(nbrs, coarse)
        levels.append({"A": A, "coarse": coarse, "P": P, "colour": colour})
        A = structural_product(P.T.tocsr(), A, P)
    return levels


def gs_sweep(A: sp.csr_matrix, b: np.ndarray, x: np.ndarray, colour: np.ndarray, forward: bool) -> np.ndarray:
    """One Gauss-Seidel sweep in colour order: for each colour, every dof of
    that colour takes x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii."""
    A = A.tocsr()
    d = A.diagonal()
    x = x.copy()
    cols = range(int(colour.max()) + 1)
    for c in (cols if forward else reversed(cols)):
        rows = np.flatnonzero(colour == c)
        off = A[rows] @ x - d[rows] * x[rows]
        x[rows] = (b[rows] - off) / d[rows]
    return x


def vcycle(levels, b: np.ndarray, lev: int = 0) -> np.ndarray:
    """B b: forward sweep from zero, restriction of the residual with P^T,
    the coarse problem by this cycle again (the last level exactly), the
    correction P x_c, a backward sweep."""
    L = levels[lev]
    A = L["A"]
    if lev == len(levels) - 1:
        return np.linalg.solve(A.toarray(), b)
    x = gs_sweep(A, b, np.zeros_like(b), L["colour"], True)
    bc = L["P"].T @ (b - A @ x)
    x = x + L["P"] @ vcycle(levels, bc, lev + 1)
    return gs_sweep(A, b, x, L["colour"], False)
