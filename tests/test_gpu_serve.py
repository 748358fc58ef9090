"""GPU tests of the serving path: the step interface of PCG, systems derived
from stored K and M, and the continuous-batching server.

Bars: a solve driven in steps returns the same bits as the blocking solve;
solves that run at the same time on several streams with one shared
hierarchy return the same bits as each alone; a derived system's matrix
matches the oracle's assembly at the new rho to rounding; every served
result reaches the 1e-8 relative residual, is the same in the mix as alone,
and matches the oracle's solution to the accuracy that residual allows.
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


def test_step_api_matches_blocking_solve(P):
    import torch
    print("[step api] cube12 mixed, steps of 3; two contexts sharing a hierarchy", flush=True)
    ctx = P.Context()
    mesh = I.kuhn_mesh(12, jitter=0.15, seed=51)
    dm = P.upload_mesh(mesh)
    s = P.fe_assemble(ctx, dm, 1.0 / 144, I.random_sine_modes(9))
    h = P.amg_setup(ctx, s, precision=P.capi.PREC_MIXED, coarse_max=32)
    u1, info1, rc1 = P.pcg_solve(ctx, s, h, rtol=1e-10)
    hd = P.pcg_begin(ctx, s, h, rtol=1e-10)
    with pytest.raises(P.OcpError) as ei:      # the context is held by the step solve
        P.pcg_solve(ctx, s, h, rtol=1e-10)
    assert ei.value.code == P.capi.ERR_INVALID_ARG
    steps = 0
    while True:
        st, inf = hd.poll()
        if st == 0:
            break
        if st == 1:
            hd.advance(3)
            steps += 1
            assert steps < 200
    u2, info2, rc2 = hd.end()
    assert inf.status == 0 and inf.iterations == info1.iterations
    assert rc1 == rc2 == 0 and info1.iterations == info2.iterations
    assert torch.equal(u1, u2)
    # two solves in flight on two streams with the same hierarchy
    f_a = s.load(I.random_sine_modes(10))
    f_b = s.load(I.random_sine_modes(11))
    ua, _, _ = P.pcg_solve(ctx, s, h, f=f_a, rtol=1e-10)
    ub, _, _ = P.pcg_solve(ctx, s, h, f=f_b, rtol=1e-10)
    ca = P.Context(stream=torch.cuda.Stream())
    cb = P.Context(stream=torch.cuda.Stream())
    ha = P.pcg_begin(ca, s, h, f=f_a, rtol=1e-10)
    hb = P.pcg_begin(cb, s, h, f=f_b, rtol=1e-10)
    active = [ha, hb]
    for _ in range(100000):
        states = [hnd.poll()[0] for hnd in active]
        if all(x == 0 for x in states):
            break
        for hnd, x in zip(active, states):
            if x == 1:
                hnd.advance(2)
    ua2, _, _ = ha.end()
    ub2, _, _ = hb.end()
    assert torch.equal(ua, ua2) and torch.equal(ub, ub2)


def test_concurrent_first_solves_on_a_fresh_system(P):
    """Two host threads, each with its own context and stream, start the
    first Jacobi-PCG solves on one freshly assembled system at the same time
    (the Jacobi diagonal is built by whichever comes first and published only
    when complete), then the first block solves of one shape (whose panel
    width is timed and published once).  Every result matches the oracle, and
    the two threads' results are the same bits."""
    import threading
    import torch
    print("[concurrent first solves] cube14 Jacobi + block k=8 on two threads", flush=True)
    N, rho = 14, 1e-2
    mesh = I.kuhn_mesh(N, jitter=0.15, seed=61)
    target = I.random_sine_modes(61)
    ctx0 = P.Context()
    dm = P.upload_mesh(mesh)
    s = P.fe_assemble(ctx0, dm, rho, target)
    h = P.amg_setup(ctx0, s, coarse_max=32)
    torch.cuda.synchronize()
    ctxs = [P.Context(stream=torch.cuda.Stream()) for _ in range(2)]
    targets = [I.random_sine_modes(70 + j) for j in range(8)]
    with torch.cuda.stream(ctxs[0].stream):
        F = s.load_multi(targets, ctx=ctxs[0])
    ctxs[0].stream.synchronize()
    out = [None, None]
    errors = []
    barrier = threading.Barrier(2)

    def run(i):
        try:
            with torch.cuda.stream(ctxs[i].stream):
                barrier.wait()
                u, info, rc = P.pcg_solve(ctxs[i], s, None, rtol=1e-13, maxit=5000)
                barrier.wait()
                U, infos, rcm = P.pcg_solve_multi(ctxs[i], s, h, F, rtol=1e-12, maxit=200)
                ctxs[i].stream.synchronize()
            out[i] = (u.cpu(), rc, U.cpu(), rcm)
        except BaseException as exc:
            errors.append(exc)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    assert out[0][1] == out[1][1] == 0 and out[0][3] == out[1][3] == 0
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][2], out[1][2])
    x, o, it, rr = O.solve(mesh, rho, target, rtol=1e-14)
    uo = O.to_vertices(o, x, mesh.n_vertices)
    assert _rel(out[0][0].numpy(), uo) < 1e-10
    for j in (0, 7):
        xj, oj, _, _ = O.solve(mesh, rho, targets[j], rtol=1e-14)
        uj = O.to_vertices(oj, xj, mesh.n_vertices)
        assert _rel(out[0][2][:, j].numpy(), uj) < 1e-9


def test_fe_derive_matches_oracle_assembly(P):
    print("[fe_derive] cube10 jitter rho 1e-3 -> 0.37", flush=True)
    ctx = P.Context()
    mesh = I.kuhn_mesh(10, jitter=0.15, seed=53)
    dm = P.upload_mesh(mesh)
    base = P.fe_assemble(ctx, dm, 1e-3, I.single_sine(), P.capi.KEEP_KM)
    d = P.fe_derive(ctx, base, 0.37)
    rp, col, val = (t.cpu().numpy() for t in d.csr())
    o = O.assemble(mesh, 0.37, I.single_sine())
    np.testing.assert_array_equal(rp, o.row_ptr)
    np.testing.assert_array_equal(col, o.col)
    np.testing.assert_allclose(val, o.val, rtol=0, atol=1e-14 * np.abs(o.val).max())
    np.testing.assert_array_equal(d.f().cpu().numpy(), base.f().cpu().numpy())
    with pytest.raises(P.OcpError):
        P.fe_derive(ctx, d, 1.0)     # a derived system keeps no K and M


def test_hierarchy_of_a_nearby_rho_preconditions(P):
    print("[compatible hierarchy] cube10 jitter: hierarchy at rho 1e-3 for rho 1.5e-3", flush=True)
    ctx = P.Context()
    mesh = I.kuhn_mesh(10, jitter=0.15, seed=55)
    dm = P.upload_mesh(mesh)
    base = P.fe_assemble(ctx, dm, 1e-3, I.single_sine(), P.capi.KEEP_KM)
    s1 = P.fe_derive(ctx, base, 1e-3)
    s2 = P.fe_derive(ctx, base, 1.5e-3)
    h1 = P.amg_setup(ctx, s1, coarse_max=32)
    target = I.random_sine_modes(12)
    u, info, rc = P.pcg_solve(ctx, s2, h1, f=s2.load(target), rtol=1e-12)
    assert rc == 0 and info.true_rel_res <= 1.0001e-11, info.as_dict()
    x, o, _, _ = O.solve(mesh, 1.5e-3, target, rtol=1e-14)
    assert _rel(u.cpu().numpy(), O.to_vertices(o, x, mesh.n_vertices)) < 1e-9
    dm8 = P.upload_mesh(I.kuhn_mesh(8))
    s3 = P.fe_assemble(ctx, dm8, 1e-3, I.single_sine())
    with pytest.raises(P.OcpError) as ei:
        P.pcg_solve(ctx, s3, h1)
    assert ei.value.code == P.capi.ERR_INVALID_ARG


def _requests():
    reqs = []
    specs = [(8, None), (10, 1e-3), (12, None), (8, 1e-5), (10, None), (12, 1e-3), (8, None), (10, 1e-3),
             (12, 2e-2), (10, None), (8, 1e-5), (12, None)]
    for r, (N, rho) in enumerate(specs):
        reqs.append(I.Request(rid=r, t_arrival=0.002 * r, N=N, rho=rho if rho else 1.0 / (N * N),
                              target_seed=4000 + r))
    return reqs


def test_server_mix_equals_alone_and_oracle(P):
    import torch
    from paper_2102_03515_amd import serve
    print("[serve] 12 requests on 4 slots vs alone", flush=True)
    reqs = _requests()
    srv = serve.Server(slots=4, precision=P.capi.PREC_MIXED, keep_solutions=True, amg_kw={"coarse_max": 32})
    mix, makespan = srv.run(reqs, realtime=False)
    stats = dict(srv.stats)
    srv.close()
    assert stats["hits"] >= 4
    for r in mix:
        assert r.status == 0 and r.true_rel_res <= 1.0001e-8, (r.rid, r.true_rel_res)
    alone = serve.Server(slots=1, precision=P.capi.PREC_MIXED, keep_solutions=True, amg_kw={"coarse_max": 32})
    for q in reqs:
        (res,), _ = alone.run([q], realtime=False)
        assert torch.equal(res.u, mix[q.rid].u), q.rid
    alone.close()
    q = reqs[5]
    x, o, _, _ = O.solve(I.kuhn_mesh(q.N), q.rho, I.random_sine_modes(q.target_seed), rtol=1e-14)
    err = _rel(mix[q.rid].u.cpu().numpy(), O.to_vertices(o, x, (q.N + 1) ** 3))
    print(f"    makespan {makespan:.3f}s hits {stats['hits']} err vs oracle {err:.2e}")
    assert err < 1e-6


def test_server_admission_under_a_small_budget(P):
    import torch
    from paper_2102_03515_amd import serve
    print("[serve] budget for one cache entry at a time", flush=True)
    reqs = [I.Request(rid=r, t_arrival=0.0, N=10, rho=10.0 ** (-2 - r), target_seed=4100 + r) for r in range(6)]
    fp = serve.footprint(10, P.capi.PREC_MIXED)
    budget = fp["base"] + fp["mesh"] + int(1.5 * (fp["entry"] + fp["solve"]))
    small = serve.Server(slots=3, precision=P.capi.PREC_MIXED, hbm_budget=budget, keep_solutions=True,
                         amg_kw={"coarse_max": 32}, rho_bucket=None)
    res, _ = small.run(reqs, realtime=False)
    st = dict(small.stats)
    small.close()
    big = serve.Server(slots=3, precision=P.capi.PREC_MIXED, keep_solutions=True, amg_kw={"coarse_max": 32},
                       rho_bucket=None)
    ref, _ = big.run(reqs, realtime=False)
    big.close()
    assert st["evictions"] >= 4 and st["admission_waits"] >= 1, st
    for a, b in zip(res, ref):
        assert a.true_rel_res <= 1.0001e-8 and torch.equal(a.u, b.u)
