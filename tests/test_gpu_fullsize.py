"""Full-size GPU checks at the benchmark configurations, on sampled rows.

At 127^3 and 255^3 unknowns the oracle cannot solve the system, but it
builds any single row of A and entry of f by itself from the mesh and the
element formulas.  These tests call the library as bench.py does (same entry
points, default AMG parameters, the same precision) and compare, at a few
thousand sampled rows spread over the domain (including rows next to the
boundary):
  * the CSR pattern of each sampled row: bit-exact;
  * its values and load entry: to rounding of the row scale;
  * the residual f - A u of the returned solution computed with the
    oracle's rows against the same residual computed on the GPU, and its
    norm against the 1e-8 relative-residual stop (a sample of the residual
    cannot exceed the whole).
"""
import numpy as np
import pytest

import ocp_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_03515_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context()


def _sample_vertices(N, count, seed):
    rng = np.random.default_rng(seed)
    ijk = rng.integers(1, N, size=(count, 3))
    edge = np.array([[1, 1, 1], [N - 1, N - 1, N - 1], [1, N - 1, 1], [N - 1, 1, N - 1], [N // 2, 1, N - 1]])
    ijk = np.vstack([ijk, edge])
    v = ijk[:, 0] + (N + 1) * (ijk[:, 1] + (N + 1) * ijk[:, 2])
    return np.unique(v).astype(np.int32)


def _gpu_rows(s, dofs):
    """CSR rows of the given dofs, gathered on the device."""
    import torch
    rp, col, val = s.csr()
    d = torch.from_numpy(dofs.astype(np.int64)).cuda()
    b = rp[d].long()
    e = rp[d + 1].long()
    cnt = (e - b).cpu().numpy()
    idx = torch.cat([torch.arange(int(x), int(y), device="cuda") for x, y in zip(b.cpu(), e.cpu())])
    return cnt, col[idx].cpu().numpy(), val[idx].cpu().numpy()


def _check_rows(s, mesh, rho, target, verts, x_gpu, f_gpu, Ax_gpu, rtol_stop):
    """Pattern, values, loads and residual at the sampled rows."""
    dof_of_vertex = s.dof_of_vertex().cpu().numpy()
    dofs = dof_of_vertex[verts]
    assert (dofs >= 0).all()
    ocols, ovals, ocnt, of = O.sample_rows(mesh, rho, target, verts)
    cnt, gcol, gval = _gpu_rows(s, dofs)
    np.testing.assert_array_equal(cnt, ocnt)
    scale = np.abs(ovals).max()
    pos = 0
    r_o = np.empty(len(verts))
    bound = np.empty(len(verts))
    for q in range(len(verts)):
        c = int(cnt[q])
        np.testing.assert_array_equal(gcol[pos:pos + c], ocols[q, :c])
        np.testing.assert_allclose(gval[pos:pos + c], ovals[q, :c], rtol=0, atol=1e-14 * scale)
        xs = x_gpu[ocols[q, :c]]
        r_o[q] = of[q] - float(np.dot(ovals[q, :c], xs))
        bound[q] = float(np.dot(np.abs(ovals[q, :c]), np.abs(xs))) + abs(of[q])
        pos += c
    np.testing.assert_allclose(f_gpu[dofs], of, rtol=0, atol=1e-13 * np.abs(of).max())
    r_g = f_gpu[dofs] - Ax_gpu[dofs]
    assert np.all(np.abs(r_g - r_o) <= 1e-13 * bound + 1e-300)
    fn = float(np.linalg.norm(f_gpu))
    assert float(np.linalg.norm(r_o)) <= rtol_stop * fn
    return float(np.linalg.norm(r_o) / fn)


def _interior(s, u):
    return u[s.vertex_of_dof().long()].contiguous()


def test_cube256_modes64_mixed_and_fp64(P, ctx):
    """The headline configuration: 255^3 unknowns, rho = h^2, 64 sine modes,
    FP32 hierarchy with FP64 CG to 1e-8; the FP64 hierarchy alongside."""
    print("[fullsize] cube256 modes64 mixed + fp64", flush=True)
    N, rho = 256, 1.0 / 65536
    mesh = I.kuhn_mesh(N)
    target = I.random_sine_modes(1000)
    dm = P.upload_mesh(mesh)
    s = P.fe_assemble(ctx, dm, rho, target)
    assert s.n == 255 ** 3 and s.nnz == 247163083
    verts = _sample_vertices(N, 2000, 41)
    res = {}
    for prec in (P.capi.PREC_MIXED, P.capi.PREC_FP64):
        h = P.amg_setup(ctx, s, precision=prec)
        u, info, rc = P.pcg_solve(ctx, s, h, rtol=1e-8, maxit=500)
        assert rc == 0 and info.true_rel_res <= 1.0001e-8 and info.iterations <= 30, info.as_dict()
        x = _interior(s, u)
        Ax = s.spmv(x)
        rs = _check_rows(s, mesh, rho, target, verts, x.cpu().numpy(), s.f().cpu().numpy(), Ax.cpu().numpy(),
                         1.0001e-8)
        res[prec] = (x, info.iterations, rs)
        print(f"    precision={prec} its={info.iterations} true_res={info.true_rel_res:.2e} "
              f"sampled_res={rs:.2e}", flush=True)
        h.close()
    xm, xd = res[P.capi.PREC_MIXED][0], res[P.capi.PREC_FP64][0]
    diff = float((xm - xd).norm() / xd.norm())
    print(f"    mixed vs fp64 relative difference {diff:.2e}")
    assert diff < 1e-6


def _kappa_bound(o, mesh):
    """An upper bound of the condition number of the oracle's A: lambda_max
    <= the largest absolute row sum (Gershgorin), and lambda_min >= min over
    interior vertices of (volume of the tets around it) / 20, because each
    element mass matrix is at least |tau|/20 times the identity on its
    vertices (its eigenvalues are |tau|/20 {5, 1, 1, 1}) and rho K >= 0."""
    rows = np.repeat(np.arange(o.n), np.diff(o.row_ptr))
    lmax = float(np.bincount(rows, weights=np.abs(o.val), minlength=o.n).max())
    p = mesh.xyz[mesh.tets]
    B = np.transpose(p[:, 1:, :] - p[:, :1, :], (0, 2, 1))
    vol = np.abs(np.linalg.det(B)) / 6.0
    patch = np.zeros(mesh.n_vertices)
    for a in range(4):
        np.add.at(patch, mesh.tets[:, a], vol)
    lmin = float(patch[~mesh.dirichlet.astype(bool)].min()) / 20.0
    return lmax / lmin


@pytest.mark.parametrize("rho", [1e-6, 1.0 / 16384, 1e-2])
def test_cube128_jitter_box_vs_oracle(P, ctx, rho):
    """127^3 unknowns, interior vertices jittered by 0.15h (seed 1), the box
    indicator target.  The oracle solves the whole system (its own assembly,
    Jacobi-PCG to 1e-14): the FP64 AMG-PCG solution at rtol 1e-13 is within
    1e-10 of it; the FP64 and mixed solutions at the 1e-8 stop are within
    kappa(A) times their true residual of it (error printed); sampled rows
    match the oracle's rows."""
    print(f"[fullsize] cube128 jitter box rho={rho:g} vs oracle", flush=True)
    N = 128
    mesh = I.kuhn_mesh(N, jitter=0.15, seed=1)
    target = I.box_indicator()
    o = O.assemble(mesh, rho, target)
    xo, it_o, rr_o = O.pcg(o, rtol=1e-14)
    print(f"    oracle: {it_o} Jacobi-PCG iterations, residual {rr_o:.1e}", flush=True)
    uo = O.to_vertices(o, xo, mesh.n_vertices)
    kappa = _kappa_bound(o, mesh)
    dm = P.upload_mesh(mesh)
    s = P.fe_assemble(ctx, dm, rho, target)
    h = P.amg_setup(ctx, s)
    u, info, rc = P.pcg_solve(ctx, s, h, rtol=1e-13, maxit=500)
    assert rc == 0
    err = float(np.linalg.norm(u.cpu().numpy() - uo) / np.linalg.norm(uo))
    print(f"    fp64 rtol 1e-13: its={info.iterations} error vs oracle {err:.2e}", flush=True)
    assert err < 1e-10
    for prec in (P.capi.PREC_FP64, P.capi.PREC_MIXED):
        hp = h if prec == P.capi.PREC_FP64 else P.amg_setup(ctx, s, precision=prec)
        u, info, rc = P.pcg_solve(ctx, s, hp, rtol=1e-8, maxit=500)
        assert rc == 0 and info.true_rel_res <= 1.0001e-8 and info.iterations <= 40, info.as_dict()
        err = float(np.linalg.norm(u.cpu().numpy() - uo) / np.linalg.norm(uo))
        print(f"    precision={prec} rtol 1e-8: levels={hp.n_levels} its={info.iterations} "
              f"true_res={info.true_rel_res:.2e} error vs oracle {err:.2e} (bound {kappa * info.true_rel_res:.1e}, "
              f"kappa <= {kappa:.1f})", flush=True)
        assert err <= kappa * info.true_rel_res * 1.001 + 1e-13
        if prec == P.capi.PREC_FP64:
            x = _interior(s, u)
            rs = _check_rows(s, mesh, rho, target, _sample_vertices(N, 1500, 43), x.cpu().numpy(),
                             s.f().cpu().numpy(), s.spmv(x).cpu().numpy(), 1.0001e-8)
            print(f"    sampled_res={rs:.2e}", flush=True)


def test_cube128_block_32_targets(P, ctx):
    """127^3 unknowns, rho = h^2, 32 sine-mode targets (seeds 2000..2031) in
    one block PCG (FP32 hierarchy, FP64 CG); every seventh column checked on
    sampled rows against the oracle's rows and loads of its own target."""
    print("[fullsize] cube128 block k=32 mixed", flush=True)
    N, k = 128, 32
    rho = 1.0 / N ** 2
    mesh = I.kuhn_mesh(N)
    targets = [I.random_sine_modes(2000 + j) for j in range(k)]
    dm = P.upload_mesh(mesh)
    s = P.fe_assemble(ctx, dm, rho, targets[0])
    h = P.amg_setup(ctx, s, precision=P.capi.PREC_MIXED)
    F = s.load_multi(targets)
    U, infos, rc = P.pcg_solve_multi(ctx, s, h, F, rtol=1e-8, maxit=500)
    assert rc == 0
    assert all(i.true_rel_res <= 1.0001e-8 for i in infos), [i.as_dict() for i in infos]
    verts = _sample_vertices(N, 800, 47)
    vod = s.vertex_of_dof().long()
    for j in range(0, k, 7):
        x = U[:, j][vod].contiguous()
        f = F[:, j].contiguous()
        rs = _check_rows(s, mesh, rho, targets[j], verts, x.cpu().numpy(), f.cpu().numpy(),
                         s.spmv(x).cpu().numpy(), 1.0001e-8)
        print(f"    column {j}: its={infos[j].iterations} true_res={infos[j].true_rel_res:.2e} "
              f"sampled_res={rs:.2e}", flush=True)
    # the block equals the single-vector solve of a column to the stop tolerance
    u1, info1, _ = P.pcg_solve(ctx, s, h, f=F[:, 0].contiguous(), rtol=1e-8)
    d = float((U[:, 0] - u1).norm() / u1.norm())
    print(f"    column 0 vs single solve: {d:.2e} (its {infos[0].iterations} vs {info1.iterations})")
    assert d < 1e-6
