"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test ties an oracle function to something other than itself: exact
integrals, textbook stencils, invariants, a library Cholesky solve, the
closed-form solution of Section 4.1 and the rates of Tables 1-3.
"""
import numpy as np
import pytest

import ocp_inputs as I
import oracle as O
from oracle import dense, norms
from conftest import golden


def _rand_tet(rng, scale=1.0):
    while True:
        p = rng.standard_normal((4, 3)) * scale
        B = (p[1:] - p[0]).T
        if abs(np.linalg.det(B)) > 0.05 * scale ** 3:
            return p


class _Callable:
    """A target given by a python function (test-only, for the numpy path)."""

    kind = "callable"

    def __init__(self, fn):
        self.fn = fn


def _eval(target, pts):
    if target.kind == "callable":
        return target.fn(pts)
    return dense.eval_target(target, pts)


# ---------------------------------------------------------------- elements

def test_mass_matrix_exact_integrals():
    """M_e[a,b] = int lambda_a lambda_b, checked with an independent degree-7 rule."""
    rng = np.random.default_rng(0)
    bary, w = norms.conical_rule(4)
    lam = np.concatenate([1 - bary.sum(1, keepdims=True), bary], 1)
    for _ in range(5):
        p = _rand_tet(rng)
        Ke, Me, fe, vol = O.element(p, I.single_sine())
        det = abs(np.linalg.det((p[1:] - p[0]).T))
        Mq = det * np.einsum("q,qa,qb->ab", w, lam, lam)
        np.testing.assert_allclose(Me, Mq, rtol=1e-13, atol=0)
        assert vol == pytest.approx(det / 6.0, rel=1e-14)


def test_stiffness_energy_of_linear_functions():
    """v^T K_e v = |tau| |c|^2 for v the nodal values of l(x) = c.x + d.

    The nodal values of affine functions span R^4 on a nondegenerate tet, so
    this fixes every entry of K_e (and implies K_e 1 = 0)."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        p = _rand_tet(rng)
        Ke, _, _, vol = O.element(p, I.single_sine())
        np.testing.assert_allclose(Ke, Ke.T, rtol=0, atol=1e-13 * np.abs(Ke).max())
        np.testing.assert_allclose(Ke @ np.ones(4), 0.0, atol=1e-12 * np.abs(Ke).max())
        for _ in range(6):
            c = rng.standard_normal(3)
            d = rng.standard_normal()
            v = p @ c + d
            assert v @ Ke @ v == pytest.approx(vol * c @ c, rel=1e-12)


def test_load_rule_exact_for_quadratics():
    """The 4-point rule integrates ubar*lambda_a exactly for linear ubar
    (degree-2 integrand): check against monomial integrals over the unit
    simplex, int x^i y^j z^k = i! j! k! / (i+j+k+3)!."""
    from math import factorial
    ref = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    tets = np.arange(4, dtype=np.int32)[None]
    for (i, j, k) in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 0, 0)]:
        tgt = _Callable(lambda P, i=i, j=j, k=k: P[..., 0] ** i * P[..., 1] ** j * P[..., 2] ** k)
        lamq = np.full((4, 4), dense.QB) + np.eye(4) * (dense.QA - dense.QB)
        xq = lamq @ ref
        u = _eval(tgt, xq)
        fe = (1.0 / 6.0 / 4.0) * (u @ lamq)
        # lambda_0 = 1-x-y-z, lambda_1 = x, lambda_2 = y, lambda_3 = z
        def mono(a, b, c):
            return factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
        exact = [mono(i, j, k) - mono(i + 1, j, k) - mono(i, j + 1, k) - mono(i, j, k + 1),
                 mono(i + 1, j, k), mono(i, j + 1, k), mono(i, j, k + 1)]
        np.testing.assert_allclose(fe, exact, rtol=1e-14, atol=1e-16)
    # and the numpy element_load uses the same points
    fe2 = dense.element_load(ref, tets, I.single_sine())
    lamq = np.full((4, 4), dense.QB) + np.eye(4) * (dense.QA - dense.QB)
    np.testing.assert_allclose(fe2[0], (1 / 24) * (dense.eval_target(I.single_sine(), lamq @ ref) @ lamq),
                               rtol=1e-14)


def test_c_and_numpy_elements_agree():
    rng = np.random.default_rng(2)
    tgt = I.random_sine_modes(7, n_modes=5, kmax=3)
    for _ in range(5):
        p = _rand_tet(rng, 0.3) + 0.5
        Ke, Me, fe, vol = O.element(p, tgt)
        v2, _, K2, M2 = dense.element_arrays(p, np.arange(4, dtype=np.int32)[None])
        f2 = dense.element_load(p, np.arange(4, dtype=np.int32)[None], tgt)
        np.testing.assert_allclose(Ke, K2[0], rtol=1e-12, atol=1e-13 * abs(Ke).max())
        np.testing.assert_allclose(Me, M2[0], rtol=1e-13)
        np.testing.assert_allclose(fe, f2[0], rtol=1e-12, atol=1e-15)


# ------------------------------------------------------- global invariants

@pytest.mark.parametrize("jitter", [0.0, 0.15])
def test_mass_sums_to_volume_and_stiffness_rows_vanish(jitter):
    m = I.kuhn_mesh(3, jitter=jitter, seed=5)
    K, M = dense.assemble_full_dense(m, 1.0)
    assert M.sum() == pytest.approx(1.0, rel=1e-13)
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-13 * np.abs(K).max())
    # patch test: K applied to an affine function vanishes at interior vertices
    rng = np.random.default_rng(3)
    c = rng.standard_normal(3)
    v = m.xyz @ c + 0.7
    interior = m.dirichlet == 0
    np.testing.assert_allclose((K @ v)[interior], 0.0, atol=1e-12 * np.abs(K).max())


def test_kuhn_stencil_is_textbook():
    """Unjittered Kuhn mesh: K = h * 7-point Laplacian stencil, and the mass
    row is h^3 * {2/5 diag; 1/20 axis; 1/30 face diagonal; 1/20 body diagonal}."""
    N = 4
    h = 1.0 / N
    m = I.kuhn_mesh(N)
    s = O.assemble(m, 1.0, I.single_sine(), keep_km=True)
    vid = 2 + (N + 1) * (2 + (N + 1) * 2)
    i = s.dof_of_vertex[vid]
    cols = s.col[s.row_ptr[i]:s.row_ptr[i + 1]]
    K = dict(zip(cols, s.valK[s.row_ptr[i]:s.row_ptr[i + 1]]))
    Mv = dict(zip(cols, s.valM[s.row_ptr[i]:s.row_ptr[i + 1]]))
    assert len(cols) == 15
    def d(di, dj, dk):
        return s.dof_of_vertex[vid + di + (N + 1) * (dj + (N + 1) * dk)]
    assert K[i] == pytest.approx(6 * h, rel=1e-13)
    assert Mv[i] == pytest.approx(0.4 * h ** 3, rel=1e-13)
    axis = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    face = [(1, 1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, -1, -1)]
    body = [(1, 1, 1), (-1, -1, -1)]
    for o in axis:
        assert K[d(*o)] == pytest.approx(-h, rel=1e-13)
        assert Mv[d(*o)] == pytest.approx(h ** 3 / 20, rel=1e-13)
    for o in face:
        assert abs(K[d(*o)]) < 1e-15
        assert Mv[d(*o)] == pytest.approx(h ** 3 / 30, rel=1e-13)
    for o in body:
        assert abs(K[d(*o)]) < 1e-15
        assert Mv[d(*o)] == pytest.approx(h ** 3 / 20, rel=1e-13)


def test_constant_target_gives_dual_volumes():
    """ubar = 1: f_i = int phi_i = sum_j M_ij = h^3 on the unjittered mesh."""
    N = 5
    m = I.kuhn_mesh(N)
    one = I.SineModes(k=np.array([[1, 1, 1]], dtype=np.int32), amp=np.array([0.0]), offset=1.0)
    s = O.assemble(m, 0.3, one)
    np.testing.assert_allclose(s.f, 1.0 / N ** 3, rtol=1e-13)


def test_nodal_target_gives_mass_times_values():
    """A P1 target (NODAL) is integrated exactly: f = M_{I,all} ubar."""
    m = I.kuhn_mesh(3, jitter=0.15, seed=9)
    rng = np.random.default_rng(4)
    vals = rng.standard_normal(m.n_vertices)
    s = O.assemble(m, 0.5, I.Nodal(values=vals))
    _, M = dense.assemble_full_dense(m, 1.0)
    interior = np.flatnonzero(m.dirichlet == 0)
    np.testing.assert_allclose(s.f, (M @ vals)[interior], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("N,jitter,tgt", [(3, 0.0, "sine"), (4, 0.15, "box"), (5, 0.15, "modes")])
def test_c_assembly_matches_dense_numpy(N, jitter, tgt):
    m = I.kuhn_mesh(N, jitter=jitter, seed=11)
    target = {"sine": I.single_sine(), "box": I.box_indicator(),
              "modes": I.random_sine_modes(3, n_modes=8)}[tgt]
    rho = 0.01
    s = O.assemble(m, rho, target)
    A, f = dense.assemble_dense(m, rho, target)
    Ac = s.csr().toarray()
    np.testing.assert_allclose(Ac, A, rtol=0, atol=1e-14 * np.abs(A).max())
    np.testing.assert_allclose(s.f, f, rtol=0, atol=1e-14 * np.abs(f).max())
    # sampled rows equal full-assembly rows
    vids = s.vertex_of_dof[[0, s.n // 2, s.n - 1]]
    cols, vals, cnt, fs = O.sample_rows(m, rho, target, vids)
    for r, i in enumerate(s.dof_of_vertex[vids]):
        a, b = s.row_ptr[i], s.row_ptr[i + 1]
        np.testing.assert_array_equal(cols[r, :cnt[r]], s.col[a:b])
        np.testing.assert_array_equal(vals[r, :cnt[r]], s.val[a:b])
        assert fs[r] == s.f[i]


def test_nnz_formula_kuhn():
    """Exact interior nnz of the 15-point Kuhn pattern."""
    for N in (4, 7, 16):
        s = O.assemble(I.kuhn_mesh(N), 1.0, I.single_sine())
        nnz = (N - 1) ** 3 + 2 * (3 * (N - 2) * (N - 1) ** 2 + 3 * (N - 2) ** 2 * (N - 1) + (N - 2) ** 3)
        assert s.nnz == nnz


# ------------------------------------------------------------------ solve

@pytest.mark.parametrize("N,jitter,rho", [(2, 0.0, 1.0), (4, 0.15, 1e-2), (6, 0.15, 1e-6), (7, 0.0, 1.0 / 49)])
def test_pcg_matches_cholesky(N, jitter, rho):
    m = I.kuhn_mesh(N, jitter=jitter, seed=N)
    tgt = I.random_sine_modes(N, n_modes=6)
    A, f = dense.assemble_dense(m, rho, tgt)
    u_chol = dense.solve_dense(A, f)
    s = O.assemble(m, rho, tgt)
    x, it, rr = O.pcg(s, rtol=1e-15)
    np.testing.assert_allclose(x, u_chol, rtol=0, atol=1e-12 * np.abs(u_chol).max())


# ------------------------------------------------- discretization (Sec. 5.1)

def _errors(N, rho, tgt):
    m = I.kuhn_mesh(N)
    x, s, it, rr = O.solve(m, rho, tgt, rtol=1e-13)
    u = O.to_vertices(s, x, m.n_vertices)
    return norms.fe_errors(m, u, tgt, rho)


def test_closed_form_solution_single_mode():
    """At the vertices of a fine mesh the discrete solution approaches
    u_rho = ubar / (1 + 3 pi^2 rho) (Section 4.1)."""
    rho = 1e-2
    errs = []
    for N in (12, 24):
        m = I.kuhn_mesh(N)
        x, s, it, rr = O.solve(m, rho, I.single_sine())
        p = m.xyz[s.vertex_of_dof]
        exact = np.prod(np.sin(np.pi * p), axis=1) / (1 + 3 * np.pi ** 2 * rho)
        errs.append(np.abs(x - exact).max())
        assert errs[-1] < 3.0 / N ** 2
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.slow
def test_eoc_matches_tables_1_and_2():
    """L2 eoc -> 2 and H1 eoc -> 1 for fixed rho, as in Tables 1 and 2;
    the eoc columns of the paper are matched within 0.06 for h <= 1/16."""
    t1 = golden("table1_l2_errors.txt")
    t2 = golden("table2_h1_errors.txt")
    tgt = I.single_sine()
    for col, rho in zip((2, 4, 6), (1.0, 1e-2, 1e-4)):
        e = [_errors(N, rho, tgt) for N in (8, 16, 32)]
        l2 = np.array([a for a, _ in e])
        h1 = np.array([b for _, b in e])
        eoc_l2 = np.log2(l2[:-1] / l2[1:])
        eoc_h1 = np.log2(h1[:-1] / h1[1:])
        # paper rows h = 1/16 and 1/32 hold the eoc of the step from the row above
        np.testing.assert_allclose(eoc_l2, t1[2:4, col], atol=0.06)
        np.testing.assert_allclose(eoc_h1, t2[2:4, col], atol=0.06)
        assert abs(eoc_l2[-1] - 2.0) < 0.07
        assert abs(eoc_h1[-1] - 1.0) < 0.03


@pytest.mark.slow
def test_theorem1_rate_with_rho_h2():
    """Theorem 1: with rho = h^2 the error to the target decays like O(h^2)."""
    tgt = I.single_sine()
    errs = []
    for N in (16, 32, 64):
        m = I.kuhn_mesh(N)
        rho = 1.0 / N ** 2
        x, s, it, rr = O.solve(m, rho, tgt, rtol=1e-13)
        u = O.to_vertices(s, x, m.n_vertices)
        errs.append(norms.target_error_l2(m, u, tgt))
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert eoc[0] > 1.85 and eoc[1] > eoc[0] and abs(eoc[1] - 2.0) < 0.05


def test_table3_l2_column():
    """Table 3's L2 column is the regularization error (1/8)(3pi^2 rho/(1+3pi^2 rho))^2;
    the oracle on a 32^3 mesh reproduces it."""
    t3 = golden("table3_target_l2.txt")
    tgt = I.single_sine()
    m = I.kuhn_mesh(32)
    for rho, printed in t3[:3]:
        closed = 0.125 * (3 * np.pi ** 2 * rho / (1 + 3 * np.pi ** 2 * rho)) ** 2
        assert printed == pytest.approx(closed, rel=3e-4)
        x, s, it, rr = O.solve(m, rho, tgt, rtol=1e-13)
        u = O.to_vertices(s, x, m.n_vertices)
        e = norms.target_error_l2(m, u, tgt)
        # triangle inequality: | ||ubar-u_h|| - ||ubar-u_rho|| | <= ||u_rho-u_h||
        delta = norms.fe_errors(m, u, tgt, rho)[0]
        assert abs(e - np.sqrt(closed)) <= delta * (1 + 1e-6)
        assert delta < 0.05 * np.sqrt(closed)


def test_mode_superposition():
    """Multi-mode target: the discrete error against the mode-by-mode closed
    form decays at second order."""
    tgt = I.SineModes(k=np.array([[1, 2, 1], [2, 1, 3]], dtype=np.int32), amp=np.array([1.0, -0.5]))
    rho = 1e-3
    e = [_errors(N, rho, tgt)[0] for N in (8, 16, 32)]
    eoc = np.log2(e[1] / e[2])
    assert 1.85 < eoc < 2.2


def test_control_and_adjoint_recovery():
    """Section 1: p = -rho u and z = (ubar - u)/rho.  For the eigenfunction
    target z_rho = 3 pi^2 ubar / (1 + 3 pi^2 rho) (= -Lap u_rho, independently
    of the recovery formula); the recovered nodal control converges to it at
    second order in h for fixed rho, and p + rho u vanishes."""
    tgt = I.single_sine()
    rho = 1e-2
    zc = norms.closed_form_control(tgt, rho)
    errs = []
    for N in (8, 16, 32):
        m = I.kuhn_mesh(N)
        x, s, it, rr = O.solve(m, rho, tgt, rtol=1e-13)
        u = O.to_vertices(s, x, m.n_vertices)
        p, z = norms.control_and_adjoint(m, u, tgt, rho)
        assert np.abs(p + rho * u).max() == 0.0
        exact = 3 * np.pi ** 2 * np.prod(np.sin(np.pi * m.xyz), axis=-1) / (1 + 3 * np.pi ** 2 * rho)
        np.testing.assert_allclose(zc(m.xyz), exact, rtol=1e-13, atol=1e-13)
        errs.append(np.abs(z - exact).max() / np.abs(exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)
    assert errs[-1] < 1e-2


def test_box_series_reference():
    """The sine-series coefficients of the box indicator equal 2 int sin(k pi x)
    over the box edge interval (Gauss-Legendre quadrature), vanish for even k,
    and by Parseval the squared L2 norm of the truncated series tends to the
    box volume 1/8; the series state at rho -> 0 approaches the indicator at
    interior lattice points away from the box faces."""
    from numpy.polynomial.legendre import leggauss
    xg, wg = leggauss(40)
    for k in range(1, 12):
        xs = 0.25 + 0.25 * (xg + 1.0)
        quad = 2.0 * 0.25 * float(np.sum(wg * np.sin(k * np.pi * xs)))
        assert norms.box_series_coefficient(k) == pytest.approx(quad, abs=1e-14)
        if k % 2 == 0:
            assert abs(norms.box_series_coefficient(k)) < 1e-15
    ks = np.arange(1, 400)
    one_d = 0.5 * np.sum(norms.box_series_coefficient(ks) ** 2)   # ||1_(1/4,3/4)||^2 = 1/2 in 1D
    assert one_d == pytest.approx(0.5, abs=2e-3)
    g = norms.box_indicator_state_on_grid(16, 1e-8, K=127)
    assert g[8, 8, 8] == pytest.approx(1.0, abs=0.03)      # box centre (the partial sums converge like 1/K)
    assert abs(g[2, 8, 8]) < 0.02                           # outside the box
    assert g[4, 8, 8] == pytest.approx(0.5, abs=0.03)      # on a face: the series gives the mean


def test_error_indicator_closed_forms():
    """The indicator's two terms against closed forms on the unjittered Kuhn
    mesh (N = 4, the box faces on grid planes):
      * u_h = 0 and the box target with h >= sqrt(rho): no flux jump, and the
        element terms add up to the box volume 1/8 (each tetrahedron lies
        inside or outside the box);
      * u_h = the interpolant of |x - 1/2| with that interpolant as a P1
        target: no element residual; the normal flux jumps by 2 rho across
        the plane x = 1/2 only, whose faces (area 1 in total, longest edge
        h sqrt2) give 4 rho^(3/2) min(1, h sqrt2 / sqrt(rho))."""
    m = I.kuhn_mesh(4)
    h = 0.25
    rho = 1e-3
    eta = norms.error_indicator(m, np.zeros(m.n_vertices), I.box_indicator(), rho)
    assert eta.sum() == pytest.approx(0.125, rel=1e-13)
    v = np.abs(m.xyz[:, 0] - 0.5)
    for rho in (1e-3, 1.0):
        eta = norms.error_indicator(m, v, None, rho, nodal_target=v)
        want = 4 * rho ** 1.5 * min(1.0, h * np.sqrt(2.0) / np.sqrt(rho))
        assert eta.sum() == pytest.approx(want, rel=1e-12)
        # only tetrahedra touching the plane x = 1/2 carry a jump
        xs = m.xyz[m.tets][:, :, 0]
        touching = np.sum(np.abs(xs - 0.5) < 1e-14, axis=1) == 3
        assert np.all(eta[~touching] == 0.0)
    # a linear state and target: zero up to rounding
    lin = 0.3 + m.xyz @ np.array([1.0, -2.0, 0.5])
    assert norms.error_indicator(m, lin, None, 1e-2, nodal_target=lin).max() < 1e-26
