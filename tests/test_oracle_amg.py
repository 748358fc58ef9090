"""Pins of the oracle's smoothed-aggregation construction (oracle/amg.py),
on the CPU, against what graph theory and linear algebra fix independently of
its code (Section 3.1: a coarsening of the matrix graph, an interpolation P,
Galerkin coarse operators A_c = P^T A P):

  * the independent set is checked by breadth-first distances, not by the
    oracle's marking: a node is a root iff no root of larger priority key
    lies within two strong steps (this characterizes the greedy set in key
    order uniquely), so roots are pairwise more than two steps apart and
    every node is within two steps of a root;
  * aggregates partition the nodes, one root each, the root within two steps;
  * P_tent has orthonormal columns and reproduces constants;
  * the Gershgorin bound is >= the largest eigenvalue of D^-1 A from a dense
    generalized eigensolver, with equality where the bound is attained;
  * the smoothed prolongator reproduces constants on a graph Laplacian
    (A 1 = 0), equals (1 - omega) P_tent for a diagonal A, and keeps an entry
    that cancels exactly as a stored zero;
  * every coarse operator is symmetric positive definite and satisfies the
    Galerkin identity v^T A_c w = (P v)^T A (P w), evaluated by matrix-vector
    products; each level at least halves the unknowns.
"""
from collections import deque

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import ocp_inputs as I
import oracle as O
from oracle import amg as OA


# ---------------------------------------------------------------- graphs
def _graph_from_edges(n, edges):
    nb = [set() for _ in range(n)]
    for a, b in edges:
        nb[a].add(b)
        nb[b].add(a)
    return [sorted(s) for s in nb]


def _path(n):
    return _graph_from_edges(n, [(i, i + 1) for i in range(n - 1)])


def _grid5(m):
    idx = lambda i, j: i * m + j
    e = []
    for i in range(m):
        for j in range(m):
            if i + 1 < m:
                e.append((idx(i, j), idx(i + 1, j)))
            if j + 1 < m:
                e.append((idx(i, j), idx(i, j + 1)))
    return _graph_from_edges(m * m, e)


def _kuhn_pattern(N):
    o = O.assemble(I.kuhn_mesh(N), 1.0, I.single_sine())
    return OA.strong_neighbours(o.csr(), 0.0)


def _random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    e = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]
    return _graph_from_edges(n, e)


GRAPHS = {"path40": lambda: _path(40), "grid9": lambda: _grid5(9), "kuhn4": lambda: _kuhn_pattern(4),
          "random60": lambda: _random_graph(60, 0.06, 3)}


def _dist_le2(nbrs):
    """For every node, the set of nodes at breadth-first distance 1 or 2."""
    out = []
    for s in range(len(nbrs)):
        seen = {s: 0}
        q = deque([s])
        while q:
            u = q.popleft()
            if seen[u] == 2:
                continue
            for v in nbrs[u]:
                if v not in seen:
                    seen[v] = seen[u] + 1
                    q.append(v)
        out.append({v for v, d in seen.items() if d in (1, 2)})
    return out


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("level", [0, 3])
def test_mis2_is_the_key_ordered_distance2_independent_set(name, level):
    nbrs = GRAPHS[name]()
    salt = OA.level_salt(level)
    root = OA.greedy_mis2(nbrs, salt)
    near = _dist_le2(nbrs)
    key = [(OA.priority(i, salt), i) for i in range(len(nbrs))]
    for i in range(len(nbrs)):
        blocked_by_higher = any(root[j] and key[j] > key[i] for j in near[i])
        assert bool(root[i]) == (not blocked_by_higher), (name, i)
    roots = np.flatnonzero(root)
    for r in roots:
        assert not any(root[j] for j in near[r])                 # independent at distance 2
    for i in range(len(nbrs)):
        assert root[i] or any(root[j] for j in near[i])           # maximal


@pytest.mark.parametrize("name", list(GRAPHS))
def test_aggregates_partition_with_one_root_each(name):
    nbrs = GRAPHS[name]()
    salt = OA.level_salt(1)
    root = OA.greedy_mis2(nbrs, salt)
    agg, nc = OA.aggregate(nbrs, root, salt)
    n = len(nbrs)
    assert nc == int(root.sum())
    assert agg.min() == 0 and agg.max() == nc - 1
    roots = np.flatnonzero(root)
    # aggregate number = rank of its root by index, one root per aggregate
    np.testing.assert_array_equal(agg[roots], np.arange(nc))
    near = _dist_le2(nbrs)
    key = [(OA.priority(i, salt), i) for i in range(n)]
    for i in range(n):
        if root[i]:
            continue
        r = roots[agg[i]]
        adjacent_roots = [j for j in nbrs[i] if root[j]]
        # roots are more than two steps apart: at most one is adjacent
        assert len(adjacent_roots) <= 1
        if adjacent_roots:
            assert r == adjacent_roots[0]
        else:
            assert r in near[i]                                       # two steps from its root
            # it joins through its neighbour of largest key among those
            # adjacent to a root
            via = [j for j in nbrs[i] if any(root[k] for k in nbrs[j]) and not root[j]]
            assert via and agg[i] == agg[max(via, key=lambda j: key[j])]


def test_tentative_prolongator_orthonormal_and_reproduces_constants():
    nbrs = _kuhn_pattern(5)
    salt = OA.level_salt(0)
    root = OA.greedy_mis2(nbrs, salt)
    agg, nc = OA.aggregate(nbrs, root, salt)
    Pt = OA.tentative_prolongator(agg, nc)
    assert np.all(np.diff(Pt.indptr) == 1) and np.all(Pt.data > 0)
    np.testing.assert_allclose((Pt.T @ Pt).toarray(), np.eye(nc), atol=1e-15)
    c = np.sqrt(np.bincount(agg, minlength=nc))
    np.testing.assert_allclose(Pt @ c, np.ones(len(nbrs)), rtol=1e-15)


def test_gershgorin_bounds_the_spectrum_and_is_attained():
    o = O.assemble(I.kuhn_mesh(6, jitter=0.15, seed=9), 1e-2, I.single_sine())
    A = o.csr()
    d = A.diagonal()
    lam_max = sla.eigh(A.toarray(), np.diag(d), eigvals_only=True)[-1]
    g = OA.gershgorin(A)
    assert g >= lam_max * (1 - 1e-13)
    assert g < 2.5 * lam_max   # a bound, not an arbitrary large number
    assert OA.gershgorin(sp.csr_matrix(np.array([[2.0, -1.0], [-1.0, 2.0]]))) == 1.5   # D^-1 A has 1/2, 3/2
    assert OA.gershgorin(sp.diags([3.0, 5.0, 7.0]).tocsr()) == 1.0


def test_smoothed_prolongator_properties():
    # graph Laplacian of a 2D grid: A 1 = 0, so P c = 1 where P_tent c = 1
    m = 8
    nbrs = _grid5(m)
    n = m * m
    rows, cols, vals = [], [], []
    for i in range(n):
        rows.append(i); cols.append(i); vals.append(float(len(nbrs[i])) + 0.0)
        for j in nbrs[i]:
            rows.append(i); cols.append(j); vals.append(-1.0)
    L = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    salt = OA.level_salt(0)
    root = OA.greedy_mis2(nbrs, salt)
    agg, nc = OA.aggregate(nbrs, root, salt)
    Pt = OA.tentative_prolongator(agg, nc)
    P = OA.smoothed_prolongator(L, Pt, 4.0 / 3.0)
    c = np.sqrt(np.bincount(agg, minlength=nc))
    np.testing.assert_allclose(P @ c, np.ones(n), atol=1e-14)
    assert abs(P - Pt).max() > 0.1   # smoothing changed it
    # diagonal A: D^-1 A = I, lambda = 1, P = (1 - omega) P_tent
    D = sp.diags(np.linspace(1.0, 3.0, n)).tocsr()
    P2 = OA.smoothed_prolongator(D, Pt, 0.6)
    np.testing.assert_allclose(P2.toarray(), 0.4 * Pt.toarray(), rtol=1e-15, atol=0)
    # an entry whose two terms cancel stays in the pattern as a stored 0
    A = sp.csr_matrix(np.array([[2.0, 0.5, -0.5], [0.5, 2.0, 0.0], [-0.5, 0.0, 2.0]]))
    Pt3 = OA.tentative_prolongator(np.array([0, 1, 1]), 2)
    P3 = OA.smoothed_prolongator(A, Pt3, 1.0)
    P3.sort_indices()
    assert P3.indptr[1] - P3.indptr[0] == 2 and P3[0, 1] == 0.0


@pytest.mark.parametrize("N,jit,theta", [(10, 0.15, 0.0), (10, 0.0, 0.08)])
def test_hierarchy_is_galerkin_and_spd(N, jit, theta):
    o = O.assemble(I.kuhn_mesh(N, jitter=jit, seed=5), 1.0 / N ** 2, I.single_sine())
    levels = OA.build_hierarchy(o.csr(), theta=theta, coarse_max=16)
    assert len(levels) >= 2
    rng = np.random.default_rng(1)
    for l in range(len(levels) - 1):
        A, P, nc = levels[l]["A"], levels[l]["P"], levels[l]["nc"]
        Ac = levels[l + 1]["A"]
        assert 2 * nc <= A.shape[0]
        v, w = rng.standard_normal(nc), rng.standard_normal(nc)
        lhs = v @ (Ac @ w)
        rhs = (P @ v) @ (A @ (P @ w))
        assert abs(lhs - rhs) <= 1e-12 * abs(Ac).max() * np.abs(v).sum() * np.abs(w).sum()
        Acd = Ac.toarray()
        np.testing.assert_allclose(Acd, Acd.T, rtol=0, atol=1e-15 * np.abs(Acd).max())
        sla.cho_factor(Acd)   # positive definite
    last = levels[-1]["A"].shape[0]
    assert last <= 16 or "agg" not in levels[-1]


def test_strength_threshold():
    A = sp.csr_matrix((np.array([4.0, -1.0, -0.1, -1.0, 4.0, 0.0, -0.1, 0.0, 4.0]),
                       np.array([0, 1, 2, 0, 1, 2, 0, 1, 2]), np.array([0, 3, 6, 9])), shape=(3, 3))
    assert OA.strong_neighbours(A, 0.1) == [[1], [0], []]        # |a_02| = 0.1 < 0.1 * 4; a_12 = 0
    assert OA.strong_neighbours(A, 0.0) == [[1, 2], [0, 2], [0, 1]]   # theta = 0: the stored pattern
    assert OA.strong_neighbours(A, 0.025) == [[1, 2], [0], [0]]


def test_priority_hash_is_a_permutation():
    """lowbias32 is a composition of invertible steps (xor-shifts, odd
    multipliers): inverting each step from its definition recovers x."""
    M = 0xFFFFFFFF

    def unxorshift(y, s):
        x = y
        for _ in range(32 // s + 1):
            x = y ^ (x >> s)
        return x & M

    def inverse(y):
        y = unxorshift(y, 16)
        y = (y * pow(0x846CA68B, -1, 1 << 32)) & M
        y = unxorshift(y, 15)
        y = (y * pow(0x7FEB352D, -1, 1 << 32)) & M
        return unxorshift(y, 16)

    rng = np.random.default_rng(0)
    for x in rng.integers(0, 1 << 32, size=2000, dtype=np.uint64):
        assert inverse(OA.lowbias32(int(x))) == int(x)


# ------------------------------------------------- red-black method (Section 3.1)
from oracle import amg_rb as RB  # noqa: E402


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_red_black_split_is_the_greedy_independent_set(name):
    """Black dofs are pairwise non-adjacent, every red dof has a black
    neighbour, and a dof is black iff no neighbour of larger key is black
    (the characterization of the greedy set visited in decreasing key,
    checked here on the final sets, not by replaying the marking)."""
    nbrs = GRAPHS[name]()
    salt = OA.level_salt(0)
    black = RB.red_black_split(nbrs, salt)
    for i, nb in enumerate(nbrs):
        if black[i]:
            assert not any(black[j] for j in nb)
        else:
            assert any(black[j] for j in nb)
        higher_black = any(black[j] and RB.key(j, salt) > RB.key(i, salt) for j in nb)
        assert black[i] == (not higher_black)


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_averaging_prolongator(name):
    """P 1 = 1 (an average reproduces constants), a black dof's row is a unit
    vector on its own coarse number, a red dof's row is uniform over exactly
    its black neighbours."""
    nbrs = GRAPHS[name]()
    black = RB.red_black_split(nbrs, OA.level_salt(1))
    P = RB.averaging_prolongator(nbrs, black).tocsr()
    np.testing.assert_allclose(P @ np.ones(P.shape[1]), 1.0, rtol=0, atol=1e-15)
    cnum = np.cumsum(black) - 1
    for i in range(len(nbrs)):
        cols = P.indices[P.indptr[i]:P.indptr[i + 1]]
        vals = P.data[P.indptr[i]:P.indptr[i + 1]]
        if black[i]:
            assert list(cols) == [cnum[i]] and vals[0] == 1.0
        else:
            want = sorted(cnum[j] for j in nbrs[i] if black[j])
            assert sorted(cols) == want
            assert np.all(vals == vals[0])


def test_colouring_is_proper_and_local_maximal():
    """No two coupled dofs share a colour; a dof of colour c has, for every
    earlier colour c' < c, a neighbour of colour c' with a larger key or it
    had a larger-key neighbour still uncoloured at round c' (it lost that
    round), i.e. colour c is exactly the set of local key maxima among the
    dofs not coloured before c."""
    o = O.assemble(I.kuhn_mesh(5, jitter=0.15, seed=2), 1.0, I.single_sine())
    A = o.csr()
    salt = OA.level_salt(0) ^ RB.COLOUR_SALT
    col = RB.colouring(A, salt)
    n = A.shape[0]
    adj = [[int(j) for j in A.indices[A.indptr[i]:A.indptr[i + 1]] if j != i] for i in range(n)]
    for i in range(n):
        assert all(col[j] != col[i] for j in adj[i])
        for c in range(col[i] + 1):
            alive = [j for j in adj[i] if col[j] >= c]
            is_max = all(RB.key(i, salt) > RB.key(j, salt) for j in alive)
            assert is_max == (c == col[i])


def test_gauss_seidel_sweep_is_a_triangular_solve():
    """A forward sweep from zero in colour order solves (D + L) x = b where L
    is the strictly lower part of A with the dofs ordered by colour; a
    backward sweep from x0 equals x0 + (D + U)^-1 (b - A x0) (U the strictly
    upper part): both by a dense triangular solve, not by the sweep code."""
    m = I.kuhn_mesh(4, jitter=0.15, seed=5)
    A = O.assemble(m, 1e-2, I.single_sine()).csr()
    col = RB.colouring(A, 123)
    perm = np.argsort(col, kind="stable")
    Ad = A.toarray()[np.ix_(perm, perm)]
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    x = RB.gs_sweep(A, b, np.zeros_like(b), col, True)
    xl = sla.solve_triangular(np.tril(Ad), b[perm], lower=True)
    np.testing.assert_allclose(x[perm], xl, rtol=1e-12, atol=1e-12 * np.abs(xl).max())
    x0 = np.random.default_rng(1).standard_normal(A.shape[0])
    xb = RB.gs_sweep(A, b, x0, col, False)
    corr = sla.solve_triangular(np.triu(Ad), (b - A @ x0)[perm], lower=False)
    np.testing.assert_allclose(xb[perm], x0[perm] + corr, rtol=1e-12, atol=1e-12 * np.abs(corr).max())


def test_red_black_vcycle_is_the_two_grid_operator():
    """With two levels the cycle is I - B A = (I - U^-1 A)(I - P A_c^-1 P^T A)
    (I - L^-1 A), L = D + lower part, U = D + upper part in colour order
    (the two-grid operator of Section 3.1 with m = 1 and the backward sweep
    after the correction); B is symmetric positive definite; every coarse
    operator satisfies v^T A_c w = (P v)^T A (P w)."""
    m = I.kuhn_mesh(6, jitter=0.15, seed=6)
    A = O.assemble(m, 1e-2, I.single_sine()).csr()
    lv = RB.build_hierarchy(A, coarse_max=60, max_levels=2)
    assert len(lv) == 2
    n = A.shape[0]
    B = np.array([RB.vcycle(lv, e) for e in np.eye(n)]).T
    Ad = A.toarray()
    perm = np.argsort(lv[0]["colour"], kind="stable")
    Pm = np.eye(n)[perm]                     # Pm @ v reorders v by colour
    Ap = Pm @ Ad @ Pm.T
    Lo = Pm.T @ np.tril(Ap) @ Pm
    Up = Pm.T @ np.triu(Ap) @ Pm
    P = lv[0]["P"].toarray()
    Ac = P.T @ Ad @ P
    E = (np.eye(n) - np.linalg.solve(Up, Ad)) @ (np.eye(n) - P @ np.linalg.solve(Ac, P.T @ Ad)) @ \
        (np.eye(n) - np.linalg.solve(Lo, Ad))
    np.testing.assert_allclose(np.eye(n) - B @ Ad, E, atol=1e-10)
    np.testing.assert_allclose(B, B.T, atol=1e-12 * np.abs(B).max())
    assert np.linalg.eigvalsh((B + B.T) / 2).min() > 0
    lv3 = RB.build_hierarchy(O.assemble(I.kuhn_mesh(9), 1.0, I.single_sine()).csr(), coarse_max=20)
    rng = np.random.default_rng(7)
    for a, b in zip(lv3[:-1], lv3[1:]):
        v, w = rng.standard_normal((2, b["A"].shape[0]))
        lhs = v @ (b["A"] @ w)
        rhs = (a["P"] @ v) @ (a["A"] @ (a["P"] @ w))
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs) + 1e-14
        assert 2 * b["A"].shape[0] <= a["A"].shape[0]
