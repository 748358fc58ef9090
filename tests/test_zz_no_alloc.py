"""The allocation-free solve (pcg_solve_noalloc) against pcg_solve, through
the C interface.

Bar: the same kernels run on the same inputs, so the solution, iteration
count and residuals equal pcg_solve's bit for bit; no allocator callback runs
during the call; two calls in a row (the second on a smaller problem, which
finds the first call's data in the scratch region) both match; a problem
whose work memory exceeds the scratch region is refused before any work.
"""
import numpy as np
import pytest

import ocp_inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_03515_amd as P
    return P


def _case(P, ctx, N, rho, target, seed):
    mesh = I.kuhn_mesh(N, jitter=0.15, seed=seed)
    dm = P.upload_mesh(mesh)
    return P.fe_assemble(ctx, dm, rho, target), dm


@pytest.mark.parametrize("precision", ["fp64", "mixed", "jacobi"])
def test_noalloc_equals_pcg_solve_twice(P, precision):
    import torch
    print(f"[pcg_solve_noalloc] {precision}: cube40 then cube18", flush=True)
    allocs = []
    ctx = P.Context(on_alloc=allocs.append)
    cases = []
    for N, seed in ((40, 81), (18, 82)):
        s, dm = _case(P, ctx, N, 1.0 / N ** 2, I.random_sine_modes(seed), seed)
        h = None
        if precision != "jacobi":
            prec = P.capi.PREC_MIXED if precision == "mixed" else P.capi.PREC_FP64
            h = P.amg_setup(ctx, s, precision=prec, coarse_max=64)
        rtol = 1e-8 if precision == "mixed" else 1e-12
        u_ref, info_ref, rc_ref = P.pcg_solve(ctx, s, h, rtol=rtol, maxit=2000)
        assert rc_ref == 0
        cases.append((N, s, dm, h, rtol, u_ref, info_ref))
    for N, s, dm, h, rtol, u_ref, info_ref in cases:   # larger first, then smaller
        u = torch.full_like(u_ref, float("nan"))
        torch.cuda.synchronize()
        before = len(allocs)
        u, info, rc = P.pcg_solve_noalloc(ctx, s, h, u=u, rtol=rtol, maxit=2000)
        assert len(allocs) == before, "the allocation-free solve called the allocator"
        assert rc == 0
        assert torch.equal(u, u_ref), f"N={N}: solution differs from pcg_solve"
        assert info.iterations == info_ref.iterations
        assert info.true_rel_res == info_ref.true_rel_res
        assert info.rel_res_l2 == info_ref.rel_res_l2
        print(f"    N={N} its={info.iterations} true_res={info.true_rel_res:.2e}", flush=True)


def test_noalloc_with_a_right_hand_side_and_repeat(P):
    import torch
    print("[pcg_solve_noalloc] explicit f, repeated call", flush=True)
    allocs = []
    ctx = P.Context(on_alloc=allocs.append)
    s, dm = _case(P, ctx, 24, 1e-2, I.box_indicator(), 83)
    h = P.amg_setup(ctx, s, precision=P.capi.PREC_MIXED, coarse_max=64)
    f = s.load(I.random_sine_modes(84))
    u_ref, info_ref, _ = P.pcg_solve(ctx, s, h, f=f, rtol=1e-9)
    u = torch.empty_like(u_ref)
    torch.cuda.synchronize()
    before = len(allocs)
    for _ in range(2):
        u, info, rc = P.pcg_solve_noalloc(ctx, s, h, f=f, u=u, rtol=1e-9)
        assert rc == 0 and torch.equal(u, u_ref) and info.iterations == info_ref.iterations
    assert len(allocs) == before


def test_noalloc_refuses_a_problem_beyond_the_scratch_region(P):
    import torch
    print("[pcg_solve_noalloc] cube128 FP64 hierarchy: refused", flush=True)
    ctx = P.Context()
    s, dm = _case(P, ctx, 128, 1.0 / 128 ** 2, I.single_sine(), 85)
    h = P.amg_setup(ctx, s, coarse_max=512)
    u = torch.zeros(s.view().n_vertices, dtype=torch.float64, device="cuda")
    with pytest.raises(P.OcpError) as ei:
        P.pcg_solve_noalloc(ctx, s, h, u=u, rtol=1e-8)
    assert ei.value.code == P.capi.ERR_UNSUPPORTED and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert float(u.abs().max()) == 0.0   # nothing was enqueued
