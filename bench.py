#!/usr/bin/env python3
"""AMG-PCG throughput benchmark (DOF/s to a 1e-8 relative residual).

Workload (default "cube256_modes64"): the unit cube cut into 256^3 Kuhn
cubes (6 tets each), 255^3 = 16,581,375 interior unknowns, rho = h^2, target
ubar = 64 seeded sine modes (seed 1000).  One step is the whole hot path on
that input: assembly of A = rho*K + M and f, smoothed-aggregation setup with
an FP32 hierarchy, and mixed-precision PCG (FP32 V-cycle, FP64 CG) to
||r|| <= 1e-8 ||f||.  The mesh and target are resident on the GPU before the
timed region starts.  `value` = unknowns x steps / wall time of the timed steps.

Also reported: the same step with an FP64 hierarchy, solve-only DOF/s,
iterations, per-phase times, the live-measured duration of the dominant
kernel against the HBM roofline, and the CPU oracle timed on a bounded sample
of the same workload family.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "cube256_modes64": dict(N=256, jitter=0.0, seed=None, rho=1.0 / 65536, target=("modes", 1000)),
    "cube128_jitter_box": dict(N=128, jitter=0.15, seed=1, rho=1.0 / 16384, target="box"),
    "cube16_sine111": dict(N=16, jitter=0.0, seed=None, rho=1.0 / 256, target="sine111"),
}


def kernel_bytes(kernel: int, n: int, entries: int, coded: bool, mixed: bool) -> float:
    """Algorithmic HBM bytes of one launch of a fine-level kernel on the
    sliced-ELL matrix as stored: every stored entry read once (its value and
    either a 4-bit column code or a 4-byte column), the per-slice metadata
    once (width and offset; with codes also the code offset and the 16-entry
    offset table), and every vector read or written once (a gathered vector
    counts once).  CG vectors are double; V-cycle values and vectors are float
    in mixed precision."""
    vs = 4 if mixed else 8
    slices = (n + 63) // 64
    col_b = 0.5 if coded else 4.0
    meta = (8.0 + (68.0 if coded else 0.0)) * slices

    def mat(v):
        return (v + col_b) * entries + meta

    if kernel == 0:    # q = A p, p.q: 8-byte values, p gathered, q written
        return mat(8) + 16.0 * n
    if kernel == 1:    # x2 = D^-1 (c1 b + c2 r1), r1 = b - A y0: y0 (gathered), b(8), d, x2
        return mat(vs) + 8.0 * n + 3.0 * vs * n
    if kernel == 5:    # r2 = b - A x2: x2 b(8) r2
        return mat(vs) + 8.0 * n + 2.0 * vs * n
    if kernel == 6:    # r0 = b - A xp, x1 = xp + a D^-1 r0: xp b(8) d r0 x1
        return mat(vs) + 8.0 * n + 4.0 * vs * n
    if kernel == 2:    # r1 = b - A x1, z = xp + D^-1 (c1 r0 + c2 r1), b.z: x1 b(8) xp r0 d z(8)
        return mat(vs) + 16.0 * n + 4.0 * vs * n
    raise ValueError(kernel)


def csr_bytes(kernel: int, n: int, nnz: int, mixed: bool) -> float:
    """Algorithmic HBM bytes of one launch as the method defines them, on the
    CSR matrix (a value and a 4-byte column per nonzero, 4(n+1) bytes of row
    pointers) with the vectors of kernel_bytes: for the CG SpMV
    12 nnz + 4(n+1) + 16 n.  The kernels read the sliced-ELL copy with 4-bit
    column codes instead, which moves fewer bytes (kernel_bytes)."""
    vs = 4 if mixed else 8

    def mat(v):
        return (v + 4.0) * nnz + 4.0 * (n + 1)

    if kernel == 0:
        return mat(8) + 16.0 * n
    if kernel == 1:
        return mat(vs) + 8.0 * n + 3.0 * vs * n
    if kernel == 5:
        return mat(vs) + 8.0 * n + 2.0 * vs * n
    if kernel == 6:
        return mat(vs) + 8.0 * n + 4.0 * vs * n
    if kernel == 2:
        return mat(vs) + 16.0 * n + 4.0 * vs * n
    raise ValueError(kernel)


def kappa_bound(system, dmesh):
    """Upper bound of the condition number of A (diagnostic, outside the timed
    region): lambda_max <= the largest absolute row sum, lambda_min >= the
    smallest volume of the tetrahedra around an interior vertex over 20 (each
    element mass matrix is at least |tau|/20 times the identity on its
    vertices; rho K is positive semidefinite)."""
    import torch
    rp, col, val = system.csr()
    n = rp.numel() - 1
    rows = torch.repeat_interleave(torch.arange(n, device=val.device), (rp[1:] - rp[:-1]).long())
    lmax = float(torch.zeros(n, dtype=torch.float64, device=val.device).index_add_(0, rows, val.abs()).max())
    del rows, rp, col, val
    xyz, tets = dmesh.xyz, dmesh.tets.long()
    patch = torch.zeros(xyz.shape[0], dtype=torch.float64, device=xyz.device)
    for s in range(0, tets.shape[0], 1 << 24):
        t = tets[s:s + (1 << 24)]
        p = xyz[t]                                   # [m,4,3]
        e = p[:, 1:, :] - p[:, :1, :]                # rows: edge vectors from vertex 0
        det = (e[:, 0, 0] * (e[:, 1, 1] * e[:, 2, 2] - e[:, 1, 2] * e[:, 2, 1])
               - e[:, 0, 1] * (e[:, 1, 0] * e[:, 2, 2] - e[:, 1, 2] * e[:, 2, 0])
               + e[:, 0, 2] * (e[:, 1, 0] * e[:, 2, 1] - e[:, 1, 1] * e[:, 2, 0]))
        vol = det.abs() / 6.0
        for a in range(4):
            patch.index_add_(0, t[:, a], vol)
    interior = dmesh.dirichlet == 0
    lmin = float(patch[interior].min()) / 20.0
    return lmax / lmin


# HBM bytes per launch of the fine-level kernels from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE) of `bench.py --calibrate-copy`, each scaled
# by what the same counter reads for the 1 GiB elementwise copy of that run.
# Only kernels measured as they stand are listed (None otherwise).
MEASURED_TRAFFIC = {
    # k_cg_spmv_pq_sell at 255^3 (coded sliced-ELL): FETCH 1,111,040.3 KiB x 1.99993
    # + WRITE 130,557.5 KiB x 0.99997 per full dispatch
    # (profiles/pmc_traffic_cg_spmv_cube256_modes64.md)
    0: 2409016550,
}


def traffic_bytes(kernel: int):
    return MEASURED_TRAFFIC.get(kernel)


# The same two counter runs for the block SpMM k_blk_spmm_pq<16, 2> at 127^3
# unknowns x 32 targets: FETCH 722,263 KiB x 1.99993 + WRITE 512,592 KiB
# x 0.99997 per full dispatch (profiles/pmc_traffic_block_spmm_cube128.md).
# Keyed by (N, k): other shapes were not measured.
MEASURED_BLOCK_TRAFFIC = {(128, 32): 2004021313}


KERNEL_NAMES = {0: "cg_spmv_pq (FP64 CSR SpMV + p.q)", 1: "vc_pre_smooth_1 (level 0)",
                2: "vc_post_smooth_final_rz (level 0)", 3: "vc_restrict (level 0)",
                4: "vc_prolong (level 0)", 5: "vc_pre_smooth_2 (level 0)", 6: "vc_post_residual (level 0)"}
MATRIX_KERNELS = (0, 1, 2, 5, 6)


def block_bench(P, capi, reps: int = 3, N: int = 128, k: int = 32):
    """Many targets on one mesh: 127^3 unknowns, rho = h^2, k sine-mode
    targets (seeds 2000..2000+k-1) solved as one block PCG (FP32 hierarchy,
    FP64 CG) against k sequential single-vector solves with an FP64
    hierarchy, and k sequential mixed-precision solves, all to 1e-8.
    Assembly and setup are outside the timed solves (one matrix and one
    hierarchy serve all targets)."""
    import torch
    import ocp_inputs as I
    mesh = I.kuhn_mesh(N)
    targets = [I.random_sine_modes(2000 + j) for j in range(k)]
    dm = P.upload_mesh(mesh)
    del mesh
    ctx = P.Context()
    s = P.fe_assemble(ctx, dm, 1.0 / N ** 2, targets[0])
    hm = P.amg_setup(ctx, s, precision=capi.PREC_MIXED)
    hd = P.amg_setup(ctx, s, precision=capi.PREC_FP64)
    F = s.load_multi(targets)
    cols = [F[:, j].contiguous() for j in range(k)]
    n, nnz = s.n, s.nnz
    P.pcg_solve_multi(ctx, s, hm, F, rtol=1e-8)          # warm-up
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        U, infos, rc = P.pcg_solve_multi(ctx, s, hm, F, rtol=1e-8)
        if rc != 0:
            raise RuntimeError(f"block solve status {rc}")
    torch.cuda.synchronize()
    t_block = (time.perf_counter() - t0) / reps
    launches, tot_ms = ctx.kernel_timing(capi.KERNEL_BLK_SPMM)
    ctx.profile(False)

    def seq(h):
        P.pcg_solve(ctx, s, h, f=cols[0], rtol=1e-8)     # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        its = []
        for j in range(k):
            _, info, rc = P.pcg_solve(ctx, s, h, f=cols[j], rtol=1e-8)
            if rc != 0:
                raise RuntimeError(f"sequential solve status {rc}")
            its.append(info.iterations)
        torch.cuda.synchronize()
        return time.perf_counter() - t, its

    t_seq64, its64 = seq(hd)
    t_seqm, itsm = seq(hm)
    avg_ms = tot_ms / max(launches, 1)
    alg = 12.0 * nnz + 4.0 * (n + 1) + 16.0 * k * n
    out = {"workload": f"cube{N}_block{k}", "unknowns": n, "nnz": nnz, "k": k,
           "block_mixed_ms": 1e3 * t_block, "block_dof_per_s": k * n / t_block,
           "block_iterations": [int(i.iterations) for i in infos],
           "max_true_rel_res": max(i.true_rel_res for i in infos),
           "sequential_fp64_ms": 1e3 * t_seq64, "sequential_fp64_dof_per_s": k * n / t_seq64,
           "sequential_fp64_iterations": its64,
           "sequential_mixed_ms": 1e3 * t_seqm, "sequential_mixed_dof_per_s": k * n / t_seqm,
           "speedup_vs_sequential_fp64": t_seq64 / t_block,
           "spmm_roofline": {"bound": "hbm", "kernel": "blk_spmm_pq (FP64 CSR SpMM + per-column p.q)",
                             "achieved": alg / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": alg / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if avg_ms > 0 else None,
                             "alg_bytes": alg, "launches": launches, "avg_us": 1e3 * avg_ms,
                             "traffic": MEASURED_BLOCK_TRAFFIC.get((N, k))}}
    hm.close()
    hd.close()
    s.close()
    ctx.close()
    return out


def packed_bench(P, capi, m: int = 32, N: int = 32, reps: int = 3):
    """m small solves on the N^3 mesh (the smallest serving size): each its
    own rho = 10^U(-8,-2) (seed 5000), target (seeds 5001..) and FP32
    hierarchy, solved to 1e-8 once as one packed batch (one graph launch per
    iteration for all) and once as m pcg_solve calls in a row.  Systems and
    hierarchies are built before the timing."""
    import numpy as np
    import torch
    import ocp_inputs as I
    ctx = P.Context(stream=torch.cuda.Stream())
    mesh = I.kuhn_mesh(N)
    dm = P.upload_mesh(mesh)
    base = P.fe_assemble(ctx, dm, 1.0 / N ** 2, I.single_sine(), capi.KEEP_KM)
    rng = np.random.default_rng(5000)
    rhos = [float(10.0 ** rng.uniform(-8.0, -2.0)) for _ in range(m)]
    systems = [P.fe_derive(ctx, base, r) for r in rhos]
    hs = [P.amg_setup(ctx, s, precision=capi.PREC_MIXED) for s in systems]
    fs = [s.load(I.random_sine_modes(5001 + j)) for j, s in enumerate(systems)]
    us = [torch.empty(s.view().n_vertices, dtype=torch.float64, device="cuda") for s in systems]
    P.pcg_solve_batch(ctx, systems, hs, fs, us, rtol=1e-8)          # warm-up
    for s, h, f, u in zip(systems, hs, fs, us):
        P.pcg_solve(ctx, s, h, f=f, u=u, rtol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, infos, rc = P.pcg_solve_batch(ctx, systems, hs, fs, us, rtol=1e-8)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        for s, h, f, u in zip(systems, hs, fs, us):
            P.pcg_solve(ctx, s, h, f=f, u=u, rtol=1e-8)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    n = systems[0].n
    out = {"workload": f"packed{m}_cube{N}", "solves": m, "unknowns_each": n,
           "batch_ms": 1e3 * t_batch, "sequential_ms": 1e3 * t_seq, "speedup": t_seq / t_batch,
           "batch_dof_per_s": m * n / t_batch, "sequential_dof_per_s": m * n / t_seq,
           "iterations": [min(i.iterations for i in infos), max(i.iterations for i in infos)],
           "max_true_rel_res": max(i.true_rel_res for i in infos)}
    for h in hs:
        h.close()
    for s in systems:
        s.close()
    base.close()
    ctx.close()
    return out


def serve_bench(P, capi, n_requests: int = 10000, rate: float = 200.0, slots: int = 16, rho_bucket: float = 0.5):
    """Poisson stream of solve requests (mean `rate` per second, seed 3000):
    N uniform in {32, 48, 64, 96, 128, 160}, rho = h^2 with probability 1/2
    else 10^U(-8,-2), a sine-mode target per request; each solved to 1e-8.
    The meshes and K/M systems of the six sizes are built before the stream
    starts (server start-up); hierarchies are built on demand and cached per
    (N, rho, precision).  Latency = completion time - arrival time."""
    import ocp_inputs as I
    from paper_2102_03515_amd import serve
    reqs = I.serving_requests(n_requests, rate=rate, seed=3000)
    srv = serve.Server(slots=slots, precision=capi.PREC_MIXED, rho_bucket=rho_bucket)
    t0 = time.perf_counter()
    srv.warm(I.SERVE_SIZES)
    warm_s = time.perf_counter() - t0
    out = {"workload": f"serve_poisson{int(rate)}", "requests": n_requests, "rate_per_s": rate, "slots": slots,
           "rho_bucket_decades": rho_bucket,
           "sizes": list(I.SERVE_SIZES), "startup_s": warm_s}
    for name, prec in (("mixed", capi.PREC_MIXED), ("fp64", capi.PREC_FP64)):
        srv.precision = prec
        before = dict(srv.stats)
        res, makespan = srv.run(reqs, realtime=True)
        out[name] = serve.summarize(res, makespan)
        out[name]["hierarchy_builds"] = srv.stats["misses"] - before["misses"]
        print(f"[bench] serve {name}: {json.dumps(out[name])}", file=sys.stderr, flush=True)
    srv.close()
    return out


def cpu_baseline(target_seed: int, N_sample: int = 64, N_single: int = 32):
    """The oracle (own assembly + Jacobi-PCG to 1e-8) on smaller meshes of
    the same family: N_sample^3 cubes on all host threads and N_single^3
    cubes on one thread, rho = h^2, the same 64 modes."""
    import ocp_inputs as I
    import oracle as O

    def run(N):
        mesh = I.kuhn_mesh(N)
        tgt = I.random_sine_modes(target_seed)
        t0 = time.perf_counter()
        s = O.assemble(mesh, 1.0 / N ** 2, tgt)
        x, it, rr = O.pcg(s, rtol=1e-8, maxit=100000)
        return s.n, it, time.perf_counter() - t0

    n, it, dt = run(N_sample)
    cores = O.num_threads()
    O.set_threads(1)
    n1, it1, dt1 = run(N_single)
    O.set_threads(cores)
    return {"value": n / dt, "unit": "DOF/s", "cores": cores, "kind": "oracle",
            "sample": f"Kuhn mesh {N_sample}^3 cubes ({n} unknowns), rho=h^2, the same 64 sine modes; "
                      f"oracle assembly + Jacobi-PCG to 1e-8 ({it} iterations) in {dt:.2f} s on {cores} threads",
            "single_thread": {"value": n1 / dt1, "unit": "DOF/s", "cores": 1,
                              "sample": f"Kuhn mesh {N_single}^3 cubes ({n1} unknowns), {it1} iterations, "
                                        f"{dt1:.2f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube256_modes64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-hierarchy comparison step")
    ap.add_argument("--no-block", action="store_true", help="skip the 32-target block solve at 127^3")
    ap.add_argument("--no-serve", action="store_true", help="skip the served request stream")
    ap.add_argument("--no-packed", action="store_true", help="skip the packed batch of small solves")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the served Poisson stream per precision (200/s: 10,000 take 50 s)")
    ap.add_argument("--no-error-bound", action="store_true",
                    help="skip the condition-number bound of the headline solve (profiling one step alone)")
    ap.add_argument("--skip-main", action="store_true",
                    help="skip the headline steps (profiling one of the other sections)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain elementwise copy of 1 GiB (reads 1 GiB, writes 1 GiB): the "
                         "reference dispatch for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this solver is measured per GPU "
              "(multi-GPU sharding is not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    import ocp_inputs as I
    import paper_2102_03515_amd as P
    from paper_2102_03515_amd import capi

    if args.calibrate_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
        print("[bench] calibration copy of 1 GiB done", file=sys.stderr, flush=True)

    def headline():
        wl = WORKLOADS[args.workload]
        N, rho = wl["N"], wl["rho"]
        print(f"[bench] workload={args.workload} N={N} rho={rho:.3e} steps={args.steps} warmup={args.warmup}",
              file=sys.stderr, flush=True)
        mesh = I.kuhn_mesh(N, jitter=wl["jitter"], seed=wl["seed"])
        tspec = wl["target"]
        target = I.make_target(tspec) if tspec != "modes" else None
        if isinstance(tspec, tuple):
            target = I.random_sine_modes(tspec[1])
        dmesh = P.upload_mesh(mesh)
        del mesh
        torch.cuda.synchronize()
        ctx = P.Context()

        def step(precision):
            t0 = time.perf_counter()
            s = P.fe_assemble(ctx, dmesh, rho, target)
            t1 = time.perf_counter()
            h = P.amg_setup(ctx, s, precision=precision)
            t2 = time.perf_counter()
            u, info, rc = P.pcg_solve(ctx, s, h, rtol=1e-8, maxit=500)
            t3 = time.perf_counter()
            if rc != 0:
                raise RuntimeError(f"solve did not converge: status {rc} {info.as_dict()}")
            meta = {"n": s.n, "nnz": s.nnz, "sell_entries": s.sell_entries, "sell_coded": s.sell_coded,
                    "levels": h.n_levels, "nnz_P0": int(h.level(0).nnz_P),
                    "iterations": info.iterations, "true_rel_res": info.true_rel_res,
                    "assemble_ms": 1e3 * (t1 - t0), "setup_ms": 1e3 * (t2 - t1), "solve_ms": 1e3 * (t3 - t2),
                    "solve_gpu_ms": info.solve_ms}
            h.close()
            s.close()
            del u
            return meta

        for w in range(args.warmup):
            m = step(capi.PREC_MIXED)
            print(f"[bench] warmup {w}: {json.dumps(m)}", file=sys.stderr, flush=True)

        ctx.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        metas = []
        for k in range(args.steps):
            metas.append(step(capi.PREC_MIXED))
            print(f"[bench] step {k}: {json.dumps(metas[-1])}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n, nnz = metas[0]["n"], metas[0]["nnz"]
        entries, coded = metas[0]["sell_entries"], metas[0]["sell_coded"]
        ms_per_step = 1e3 * (t1 - t0) / args.steps
        value = n * args.steps / (t1 - t0)

        # dominant kernel of the timed region, live event timings
        timings = {k: ctx.kernel_timing(k) for k in range(7)}
        dom = max(MATRIX_KERNELS, key=lambda k: timings[k][1])
        launches, tot_ms = timings[dom]
        avg_ms = tot_ms / max(launches, 1)
        stored = kernel_bytes(dom, n, entries, coded, mixed=(dom != 0))
        alg = csr_bytes(dom, n, nnz, mixed=(dom != 0))
        achieved = alg / (avg_ms * 1e-3) / 1e9
        achieved_stored = stored / (avg_ms * 1e-3) / 1e9
        kernels = {KERNEL_NAMES[k]: {"launches": timings[k][0],
                                     "avg_us": 1e3 * timings[k][1] / max(timings[k][0], 1)}
                   for k in range(7)}
        for k in MATRIX_KERNELS:
            b = csr_bytes(k, n, nnz, mixed=(k != 0))
            bs = kernel_bytes(k, n, entries, coded, mixed=(k != 0))
            t = timings[k][1] / max(timings[k][0], 1)
            kernels[KERNEL_NAMES[k]]["alg_bytes"] = b
            kernels[KERNEL_NAMES[k]]["alg_GBps"] = b / (t * 1e-3) / 1e9 if t > 0 else None
            kernels[KERNEL_NAMES[k]]["stored_bytes"] = bs
            kernels[KERNEL_NAMES[k]]["stored_GBps"] = bs / (t * 1e-3) / 1e9 if t > 0 else None

        # error against the exact discrete solution (the FP64 oracle's to its
        # 1e-14 stop): ||u - A^-1 f|| / ||A^-1 f|| <= kappa(A) ||f - A u|| / ||f||
        kap = float("nan")
        if not args.no_error_bound:
            s_b = P.fe_assemble(ctx, dmesh, rho, target)
            kap = kappa_bound(s_b, dmesh)
            s_b.close()
            torch.cuda.empty_cache()

        fp64 = None
        if not args.no_fp64:
            ctx.profile(False)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            m64 = step(capi.PREC_FP64)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            fp64 = {"dof_per_s": n / (tb - ta), "iterations": m64["iterations"], "solve_ms": m64["solve_ms"],
                    "setup_ms": m64["setup_ms"], "true_rel_res": m64["true_rel_res"],
                    "error_bound": kap * m64["true_rel_res"]}
            print(f"[bench] fp64 step: {json.dumps(m64)}", file=sys.stderr, flush=True)
        solve_ms = sum(m["solve_ms"] for m in metas) / len(metas)
        return {
            "value": value, "ms_per_step": ms_per_step,
            "config": {"workload": args.workload, "cubes_per_edge": N, "unknowns": n, "nnz": nnz,
                       "sell_entries": entries, "sell_column_codes": coded,
                       "rho": rho, "rtol": 1e-8, "stop": "||r||2/||f||2", "precision": "mixed",
                       "parallelism": "single GPU"},
            "iterations": metas[-1]["iterations"],
            "true_rel_res": metas[-1]["true_rel_res"],
            "levels": metas[-1]["levels"],
            "phase_ms": {"assemble": sum(m["assemble_ms"] for m in metas) / len(metas),
                         "setup": sum(m["setup_ms"] for m in metas) / len(metas),
                         "solve": solve_ms},
            "solve_only_dof_per_s": n / (solve_ms * 1e-3),
            "error_vs_fp64_oracle": {
                "bound": kap * metas[-1]["true_rel_res"] + kap * 1e-14, "kappa_bound": kap,
                "kind": "rigorous bound, not a measurement: ||u - u_oracle||/||u_oracle|| <= kappa(A) "
                        "(true_rel_res + 1e-14) with kappa(A) <= max row sum of |A| / (min vertex-patch volume / 20)"},
            "fp64": fp64,
            "kernels": kernels,
            "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": traffic_bytes(dom), "launches": launches, "avg_us": 1e3 * avg_ms,
                         "alg_bytes": alg, "alg_bytes_def": "12 nnz + 4(n+1) + 16 n (CSR, FP64)",
                         "stored_bytes": stored, "achieved_stored": achieved_stored,
                         "frac_stored": achieved_stored / HBM_PEAK_GBS},
        }

    head = {"value": None, "ms_per_step": None, "config": {"workload": args.workload}} if args.skip_main \
        else headline()
    wl = WORKLOADS[args.workload]
    tspec = wl["target"]

    block = None
    if not args.no_block:
        print("[bench] block solve (32 targets, 127^3) ...", file=sys.stderr, flush=True)
        block = block_bench(P, capi)
        print(f"[bench] block: {json.dumps(block)}", file=sys.stderr, flush=True)

    packed = None
    if not args.no_packed:
        print("[bench] packed batch of 32 small solves ...", file=sys.stderr, flush=True)
        packed = [packed_bench(P, capi, m=m) for m in (32, 256)]
        print(f"[bench] packed: {json.dumps(packed)}", file=sys.stderr, flush=True)

    served = None
    if not args.no_serve:
        print(f"[bench] serving stream ({args.serve_requests} requests per precision, 200/s) ...", file=sys.stderr,
              flush=True)
        served = serve_bench(P, capi, n_requests=args.serve_requests)

    cpu = None
    if not args.no_cpu_baseline and isinstance(tspec, tuple):
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(tspec[1])

    out = {
        "metric": "AMG-PCG DOF/s to 1e-8 rel. residual (assemble + AMG setup + PCG solve)",
        "value": head["value"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 CG / f32 V-cycle",
        "data": "synthetic (seeded Kuhn mesh and sine-mode target)",
    }
    out.update({k: v for k, v in head.items() if k not in ("value", "ms_per_step")})
    out.update({"block32": block, "packed_small": packed, "serve": served, "cpu_baseline": cpu})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
