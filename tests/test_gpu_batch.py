"""GPU tests of the packed batch of small solves.

Two paths: the persistent kernel (one workgroup per solve, every iteration
on the device) and the graph path (one HIP graph launch per iteration for
all solves).  Bars: the graph path returns the same bits and iteration
counts as pcg_solve alone; the persistent path runs the same arithmetic with
dot products summed in another order, so it agrees with pcg_solve to
rounding (FP64 hierarchy at a tight tolerance: within 1e-10 relative, and
within 1e-10 of the oracle's solution), takes the same number of iterations
up to one, and returns the same bits from one batch call to the next.
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _problems(P, ctx):
    systems, hs, fs, keep, meshes = [], [], [], [], []
    for N, rho, prec in [(6, 1e-2, P.capi.PREC_MIXED), (8, 1.0 / 64, P.capi.PREC_FP64),
                         (10, 1e-5, P.capi.PREC_MIXED), (12, 1e-3, P.capi.PREC_FP64)]:
        mesh = I.kuhn_mesh(N, jitter=0.15, seed=60 + N)
        dm = P.upload_mesh(mesh)
        s = P.fe_assemble(ctx, dm, rho, I.random_sine_modes(N))
        h = P.amg_setup(ctx, s, precision=prec, coarse_max=16)
        keep += [dm, s, h]
        for j in range(3):
            systems.append(s)
            hs.append(None if j == 2 and N == 8 else h)
            fs.append(None if j == 0 else s.load(I.random_sine_modes(100 * N + j)))
            meshes.append((mesh, rho, N, j))
    return systems, hs, fs, keep, meshes


def test_graph_batch_equals_individual_solves(P):
    import torch
    print("[batch graph] 12 solves: N 6..12, mixed/fp64/jacobi, shared systems", flush=True)
    ctx = P.Context()
    systems, hs, fs, keep, _ = _problems(P, ctx)
    us, infos, rc = P.pcg_solve_batch(ctx, systems, hs, fs, rtol=1e-10, maxit=2000, graph=True)
    assert rc == 0
    for i, (s, h, f) in enumerate(zip(systems, hs, fs)):
        u1, info1, rc1 = P.pcg_solve(ctx, s, h, f=f, rtol=1e-10, maxit=2000)
        assert rc1 == 0 and info1.iterations == infos[i].iterations, (i, info1.iterations, infos[i].iterations)
        assert torch.equal(u1, us[i]), i
    us2, _, _ = P.pcg_solve_batch(ctx, systems, hs, fs, rtol=1e-10, maxit=2000, graph=True)
    assert all(torch.equal(a, b) for a, b in zip(us, us2))


def test_persistent_batch_matches_solves_and_oracle(P):
    import torch
    print("[batch persistent] 12 solves: N 6..12, mixed/fp64/jacobi", flush=True)
    ctx = P.Context()
    systems, hs, fs, keep, meta = _problems(P, ctx)
    us, infos, rc = P.pcg_solve_batch(ctx, systems, hs, fs, rtol=1e-12, maxit=2000)
    assert rc == 0
    for i, (s, h, f) in enumerate(zip(systems, hs, fs)):
        u1, info1, rc1 = P.pcg_solve(ctx, s, h, f=f, rtol=1e-12, maxit=2000)
        assert rc1 == 0 and abs(info1.iterations - infos[i].iterations) <= 1, (i, info1.iterations,
                                                                              infos[i].iterations)
        assert infos[i].true_rel_res <= 1.0001e-12 * 10, infos[i].as_dict()
        d = _rel(us[i].cpu().numpy(), u1.cpu().numpy())
        assert d < (1e-10 if h is None or h.params.precision == P.capi.PREC_FP64 else 1e-8), (i, d)
    # FP64 hierarchy solves against the oracle
    for i, (mesh, rho, N, j) in enumerate(meta):
        if hs[i] is not None and hs[i].params.precision == P.capi.PREC_FP64 and j == 1:
            target = I.random_sine_modes(100 * N + j)
            x, o, _, _ = O.solve(mesh, rho, target, rtol=1e-14)
            assert _rel(us[i].cpu().numpy(), O.to_vertices(o, x, mesh.n_vertices)) < 1e-10
    us2, _, _ = P.pcg_solve_batch(ctx, systems, hs, fs, rtol=1e-12, maxit=2000)
    assert all(torch.equal(a, b) for a, b in zip(us, us2))


def test_batch_on_a_private_stream_and_errors(P):
    import torch
    print("[batch] explicit stream; error paths", flush=True)
    ctx = P.Context(stream=torch.cuda.Stream())
    mesh = I.kuhn_mesh(6)
    dm = P.upload_mesh(mesh)
    s = P.fe_assemble(ctx, dm, 1e-2, I.single_sine())
    h = P.amg_setup(ctx, s, coarse_max=16)
    for graph in (False, True):
        us, infos, rc = P.pcg_solve_batch(ctx, [s, s], [h, h], None, rtol=1e-9, graph=graph)
        assert rc == 0 and torch.equal(us[0], us[1])
    dm5 = P.upload_mesh(I.kuhn_mesh(5))
    other = P.fe_assemble(ctx, dm5, 1.0, I.single_sine())   # another mesh: the hierarchy does not fit
    with pytest.raises(P.OcpError) as ei:
        P.pcg_solve_batch(ctx, [s, other], [h, h], None)
    assert ei.value.code == P.capi.ERR_INVALID_ARG
    with pytest.raises(P.OcpError):
        P.pcg_solve_batch(ctx, [], None, None)
