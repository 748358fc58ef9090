"""Smoothed-aggregation hierarchy written out from its definitions -- TEST INFRASTRUCTURE.

Only the test suite may import this module; the product package never does.

Section 3.1 of the paper builds its AMG from three ingredients: a greedy
colouring of the matrix graph that picks coarse dofs and marks their
neighbours, an interpolation P from the coarse dofs, and the Galerkin coarse
operator A_c = P^T A P, applied recursively.  The GPU library realises these
as smoothed aggregation; this module states that construction plainly, one
definition per function, so that the GPU setup can be compared with it:

  strength     j is a strong neighbour of i  iff  j != i, a_ij != 0 and
               |a_ij| >= theta * sqrt(a_ii * a_jj); for theta = 0 every
               off-diagonal entry of the sparsity pattern is strong
  priority     p(i) = lowbias32(i XOR salt) >> 2, where lowbias32 is the
               published 32-bit integer hash  x ^= x>>16; x *= 0x7feb352d;
               x ^= x>>15; x *= 0x846ca68b; x ^= x>>16  (C. Wellons), and the
               salt of level l is 0x9E3779B9 * (l+1) mod 2^32; ties by index
  roots        greedy distance-2 independent set: visit nodes by decreasing
               (p(i), i); take i if no taken node is within two strong steps
  aggregates   a root forms aggregate number = rank of the root by index;
               a non-root adjacent to roots joins the one of largest
               (p, index); any other node joins the aggregate of its adjacent
               node (adjacent to a root) of largest (p, index)
  P_tent       P_tent[i, agg(i)] = 1/sqrt(|agg(i)|)
  lambda       max_i sum_j |a_ij| / a_ii   (Gershgorin bound of D^-1 A)
  P            (I - (omega/lambda) D^-1 A) P_tent
  A_c          P^T A P
  pattern      P and A_c keep every structural entry of the product (an
               entry some product term reaches), also one whose terms cancel
               to 0.0: the sparsity pattern of the next level, and with
               theta = 0 its strength, depend on the patterns only
  levels       stop at n <= coarse_max, at max_levels, or where the
               aggregation leaves more than half of the nodes
The paper fixes none of the parameters (strength threshold, stopping rule,
coarsest size); the defaults here are this build's choices, and the tests
pass them explicitly.  The sparse products use scipy.sparse (a library
primitive).  Only for small problems: the loops are plain Python.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MASK = 0xFFFFFFFF


def lowbias32(x: int) -> int:
    x &= MASK
    x ^= x >> 16
    x = (x * 0x7FEB352D) & MASK
    x ^= x >> 15
    x = (x * 0x846CA68B) & MASK
    x ^= x >> 16
    return x


def level_salt(level: int) -> int:
    return (0x9E3779B9 * (level + 1)) & MASK


def priority(i: int, salt: int) -> int:
    return lowbias32(i ^ salt) >> 2


def strong_neighbours(A: sp.csr_matrix, theta: float):
    d = A.diagonal()
    out = []
    for i in range(A.shape[0]):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        nb = []
        for j, a in zip(A.indices[lo:hi], A.data[lo:hi]):
            if j == i:
                continue
            if theta == 0.0 or (a != 0.0 and abs(a) >= theta * np.sqrt(d[i] * d[j])):
                nb.append(int(j))
        out.append(nb)
    return out


def greedy_mis2(nbrs, salt: int):
    n = len(nbrs)
    order = sorted(range(n), key=lambda i: (priority(i, salt), i), reverse=True)
    blocked = np.zeros(n, dtype=bool)
    root = np.zeros(n, dtype=bool)
    for i in order:
        if blocked[i]:
            continue
        root[i] = True
        blocked[i] = True
        for j in nbrs[i]:
            blocked[j] = True
            for k in nbrs[j]:
                blocked[k] = True
    return root


def aggregate(nbrs, root, salt: int):
    n = len(nbrs)
    root_id = -np.ones(n, dtype=np.int64)
    root_id[root] = np.arange(int(root.sum()))
    agg = -np.ones(n, dtype=np.int64)
    step1 = np.zeros(n, dtype=bool)
    key = [(priority(i, salt), i) for i in range(n)]
    for i in range(n):
        if root[i]:
            agg[i] = root_id[i]
            continue
        cands = [j for j in nbrs[i] if root[j]]
        if cands:
            best = max(cands, key=lambda j: key[j])
            agg[i] = root_id[best]
            step1[i] = True
    for i in range(n):
        if agg[i] >= 0:
            continue
        cands = [j for j in nbrs[i] if step1[j]]
        if not cands:
            raise RuntimeError(f"node {i} is not within two strong steps of a root")
        best = max(cands, key=lambda j: key[j])
        agg[i] = agg[best]
    return agg, int(root.sum())


def tentative_prolongator(agg, nc: int) -> sp.csr_matrix:
    n = agg.size
    sizes = np.bincount(agg, minlength=nc)
    vals = 1.0 / np.sqrt(sizes[agg].astype(np.float64))
    return sp.csr_matrix((vals, (np.arange(n), agg)), shape=(n, nc))


def gershgorin(A: sp.csr_matrix) -> float:
    d = A.diagonal()
    return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel() / d))


def _ones(M: sp.csr_matrix) -> sp.csr_matrix:
    """The sparsity pattern of M (every stored entry) with value 1."""
    M = M.tocsr()
    return sp.csr_matrix((np.ones(M.indices.size), M.indices.copy(), M.indptr.copy()), shape=M.shape)


def structural_product(*mats) -> sp.csr_matrix:
    """M1 M2 ... with the structural pattern of the product: scipy drops
    entries whose sum is exactly 0.0, so the pattern comes from the product
    of the 0/1 patterns (positive terms cannot cancel) and the values from
    the ordinary product, entries missing there being explicit zeros."""
    V = mats[0]
    S = _ones(mats[0])
    for M in mats[1:]:
        V = V @ M
        S = S @ _ones(M)
    V = V.tocsr()
    S = S.tocsr()
    S.sort_indices()
    V.sort_indices()
    ncol = S.shape[1]
    srow = np.repeat(np.arange(S.shape[0], dtype=np.int64), np.diff(S.indptr))
    vrow = np.repeat(np.arange(V.shape[0], dtype=np.int64), np.diff(V.indptr))
    skey = srow * ncol + S.indices
    vkey = vrow * ncol + V.indices
    pos = np.searchsorted(skey, vkey)
    assert np.all(skey[pos] == vkey), "a value entry outside the structural pattern"
    data = np.zeros(skey.size)
    data[pos] = V.data
    return sp.csr_matrix((data, S.indices.copy(), S.indptr.copy()), shape=S.shape)


def smoothed_prolongator(A: sp.csr_matrix, Pt: sp.csr_matrix, omega: float) -> sp.csr_matrix:
    """(I - (omega/lambda) D^-1 A) P_tent on A's pattern (its diagonal is
    stored: A is SPD)."""
    A = A.tocsr()
    lam = gershgorin(A)
    d = A.diagonal()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    vals = -(omega / lam) * A.data / d[rows]
    vals = vals + (A.indices == rows)
    S = sp.csr_matrix((vals, A.indices.copy(), A.indptr.copy()), shape=A.shape)
    return structural_product(S, Pt)


def build_hierarchy(A: sp.csr_matrix, theta: float = 0.0, omega: float = 1.9,
                    coarse_max: int = 512, max_levels: int = 10):
    """Levels as dicts {A, agg, P, nc}; the last has only A."""
    levels = []
    A = A.tocsr()
    for lev in range(max_levels):
        n = A.shape[0]
        if n <= coarse_max or lev + 1 >= max_levels:
            levels.append({"A": A})
            break
        salt = level_salt(lev)
        nbrs = strong_neighbours(A, theta)
        root = greedy_mis2(nbrs, salt)
        agg, nc = aggregate(nbrs, root, salt)
        if nc <= 0 or 2 * nc > n:
            levels.append({"A": A})
            break
        Pt = tentative_prolongator(agg, nc)
        P = smoothed_prolongator(A, Pt, omega)
        levels.append({"A": A, "agg": agg, "nc": nc, "P": P})
        A = structural_product(P.T.tocsr(), A, P)
    return levels


def strength_margin(A: sp.csr_matrix, theta: float) -> float:
    """Smallest relative distance of |a_ij|/sqrt(a_ii a_jj) from theta over
    off-diagonal nonzeros (how far every strength decision is from a tie)."""
    A = A.tocoo()
    d = A.tocsr().diagonal()
    off = A.row != A.col
    r = np.abs(A.data[off]) / np.sqrt(d[A.row[off]] * d[A.col[off]])
    if theta == 0.0 or r.size == 0:
        return np.inf
    return float(np.min(np.abs(r - theta)) / theta)
