"""Serving loop: a stream of solve requests on unit-cube meshes of several
sizes and values of rho, with continuous batching on one GPU.

Each request (N, rho, target) asks for the discrete solution of
(rho K + M) u = f on the N^3-cube Kuhn mesh, f the load vector of its target.
The server keeps on the device, per mesh size N, the mesh and one system
assembled with its K and M values, from which every request's system is
derived (A = rho K + M, no re-assembly).  AMG hierarchies are cached in an
LRU per (N, rho key, precision).  The rho key is rho itself for rho = h^2
(the paper's choice, shared by many requests) and, with `rho_bucket`, the
centre 10^(b w) of the bucket of width w decades that holds log10(rho)
otherwise: the hierarchy is built once at that centre and preconditions
every request of the bucket (CG and the stop test use the request's exact
system; the preconditioner is a fixed SPD operator either way).  Because the
key does not depend on which request came first, a result does not depend
on the mix it was served in.  rho_bucket=None keys hierarchies by exact rho.  Requests are admitted as solve slots free up and as the estimated
HBM footprint of what they need fits the budget (idle cache entries are
evicted first); every slot runs its solves on its own stream, so the work of
requests that arrived while others were on the GPU overlaps on the device.

All arithmetic runs in the library (fe_assemble, fe_derive, fe_load,
amg_setup, pcg_solve); this module only schedules.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import ocp_inputs as I

from . import capi


def interior_nnz(N: int) -> int:
    """Nonzeros of A on the (N-1)^3 interior unknowns of the Kuhn mesh."""
    return (N - 1) ** 3 + 2 * (3 * (N - 2) * (N - 1) ** 2 + 3 * (N - 2) ** 2 * (N - 1) + (N - 2) ** 3)


def footprint(N: int, precision: int) -> Dict[str, int]:
    """Estimated device bytes of what a request on the N^3 mesh needs.

    mesh: coordinates and tets; base: the K/M system (CSR with three value
    arrays, its sliced-ELL copy, incidence and maps); entry: a derived system
    plus its hierarchy; solve: the CG and V-cycle vectors of one solve."""
    n = (N - 1) ** 3
    nv = (N + 1) ** 3
    nt = 6 * N ** 3
    nnz = interior_nnz(N)
    vs = 4 if precision == capi.PREC_MIXED else 8
    mesh = 24 * nv + 16 * nt + nv
    pattern = 4 * (n + 1) + 4 * nnz + 8 * n + 4 * nv + 4 * n + 4 * (nv + 1) + 16 * nt
    sell = 13 * nnz + 8 * n                      # values, columns, 4-bit codes and offset tables
    base = pattern + 3 * 8 * nnz + sell
    hier = 8 * n + (vs + 4) * nnz + 40 * n * (1 + vs // 4) + 2 * (12 * nnz) // 10
    if n // 27 >= 1 << 16:                       # level 1 gets a sliced-ELL copy (~nnz/4 entries)
        hier += (12 + vs) * nnz // 4
    entry = pattern + 8 * nnz + sell + hier
    solve = 5 * 8 * n + 8 * nv + 8 * n + 6 * vs * n
    return {"mesh": mesh, "base": base, "entry": entry, "hier": hier, "solve": solve}


@dataclass
class Result:
    rid: int
    N: int
    rho: float
    n: int
    t_arrival: float
    t_start: float
    t_done: float
    iterations: int
    true_rel_res: float
    status: int
    cache_hit: bool
    slot: int
    u: Optional[object] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class _Entry:
    system: object
    hierarchy: object
    bytes: int
    users: int = 0
    ready: threading.Event = field(default_factory=threading.Event)
    error: Optional[BaseException] = None


class Server:
    """Continuous-batching solve server on the current GPU."""

    def __init__(self, slots: int = 16, precision: int = capi.PREC_MIXED, rtol: float = 1e-8, maxit: int = 500,
                 hbm_budget: Optional[int] = None, keep_solutions: bool = False, amg_kw: Optional[dict] = None,
                 rho_bucket: Optional[float] = 0.5):
        import torch
        self.torch = torch
        self.slots = slots
        self.precision = precision
        self.rtol, self.maxit = rtol, maxit
        self.keep = keep_solutions
        self.rho_bucket = rho_bucket
        self.amg_kw = dict(amg_kw or {})
        if hbm_budget is None:
            # free device memory plus what torch's caching allocator holds
            # without using it (the library allocates through that cache)
            free, _total = torch.cuda.mem_get_info()
            cached = torch.cuda.memory_reserved() - torch.cuda.memory_allocated()
            hbm_budget = int(0.8 * (free + cached))
        self.budget = hbm_budget
        self.lock = threading.Condition()
        self.meshes: Dict[int, Tuple[object, object]] = {}        # N -> (host mesh, device mesh)
        self.bases: Dict[int, object] = {}                          # N -> K/M system
        self.base_events: Dict[int, threading.Event] = {}           # N -> set once its base is built
        self.base_reserved = set()                                  # sizes whose base bytes are reserved
        self.entries: "collections.OrderedDict[tuple, _Entry]" = collections.OrderedDict()
        self.reserved = 0          # bytes of entries, bases, meshes and running solves
        self.running = 0           # admitted requests not yet released
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.ctxs = [capi.Context(stream=s) for s in self.streams]
        self.stats = {"hits": 0, "misses": 0, "evictions": 0, "admission_waits": 0}

    # ------------------------------------------------------------ caching
    def _mesh_and_base(self, N: int, ctx) -> object:
        """Device mesh and K/M system of size N, built once by the first
        request that needs them (the others wait for it)."""
        with self.lock:
            ev = self.base_events.get(N)
            builder = ev is None
            if builder:
                ev = threading.Event()
                self.base_events[N] = ev
        if builder:
            try:
                mesh = I.kuhn_mesh(N)
                dm = capi.upload_mesh(mesh)
                base = capi.fe_assemble(ctx, dm, 1.0 / (N * N), I.single_sine(), capi.KEEP_KM)
                with self.lock:
                    self.meshes[N] = (mesh, dm)
                    self.bases[N] = base
            finally:
                ev.set()
        else:
            ev.wait()
        if N not in self.bases:
            raise RuntimeError(f"building the N={N} mesh and K/M system failed")
        return self.bases[N]

    def _evict_idle(self, need: int, protect) -> bool:
        """Drop idle cache entries other than `protect`, oldest first, until
        `need` more bytes fit (called with the lock held)."""
        for key in list(self.entries.keys()):
            if self.reserved + need <= self.budget:
                break
            if key == protect:
                continue
            e = self.entries[key]
            if e.users == 0 and e.ready.is_set():
                del self.entries[key]
                self.reserved -= e.bytes
                self.stats["evictions"] += 1
                if e.hierarchy is not None:
                    e.hierarchy.close()
                if e.system is not None:
                    e.system.close()
        return self.reserved + need <= self.budget

    def rho_key(self, N: int, rho: float) -> float:
        """rho at which the hierarchy serving (N, rho) is built."""
        if self.rho_bucket is None or rho == 1.0 / (N * N):
            return rho
        import math
        b = round(math.log10(rho) / self.rho_bucket)
        return 10.0 ** (b * self.rho_bucket)

    def _admit(self, req) -> Tuple[_Entry, bool, int]:
        """Reserve what the request needs (blocking until it fits); returns
        the cache entry (possibly still being built), whether it was a hit,
        and the bytes reserved for the solve itself (its vectors, and its own
        derived system when the hierarchy was built at another rho)."""
        fp = footprint(req.N, self.precision)
        rk = self.rho_key(req.N, req.rho)
        key = (req.N, rk, self.precision)
        own = rk != req.rho
        solve_need = fp["solve"] + (fp["entry"] - fp["hier"] if own else 0)
        with self.lock:
            while True:
                e = self.entries.get(key)
                need = solve_need
                if e is None:
                    need += fp["entry"]
                if req.N not in self.base_reserved:
                    need += fp["base"] + fp["mesh"]
                # the entry this request uses is never the one evicted for it
                if self.reserved + need <= self.budget or self._evict_idle(need, key):
                    break
                if self.running == 0:
                    raise MemoryError(f"request N={req.N} needs {need} bytes, budget {self.budget}")
                self.stats["admission_waits"] += 1
                self.lock.wait()
            hit = e is not None
            if hit:
                self.entries.move_to_end(key)
                self.stats["hits"] += 1
            else:
                e = _Entry(system=None, hierarchy=None, bytes=fp["entry"])
                self.entries[key] = e
                self.stats["misses"] += 1
            if req.N not in self.base_reserved:
                self.base_reserved.add(req.N)
                self.reserved += fp["base"] + fp["mesh"]   # kept for the server's lifetime
            self.reserved += e.bytes if not hit else 0
            self.reserved += solve_need
            self.running += 1
            e.users += 1
            return e, hit, solve_need

    def _release(self, e: _Entry, solve_bytes: int):
        with self.lock:
            e.users -= 1
            self.running -= 1
            self.reserved -= solve_bytes
            if e.error is not None and e.users == 0:   # a failed build is not kept
                for key, v in list(self.entries.items()):
                    if v is e:
                        del self.entries[key]
                        self.reserved -= e.bytes
            self.lock.notify_all()

    def warm(self, sizes):
        """Build the meshes and K/M systems of the given sizes up front."""
        for N in sizes:
            fp = footprint(N, self.precision)
            with self.lock:
                if N not in self.base_reserved:
                    self.base_reserved.add(N)
                    self.reserved += fp["base"] + fp["mesh"]
            self._mesh_and_base(N, self.ctxs[0])

    def _build(self, e: _Entry, req, ctx):
        try:
            base = self._mesh_and_base(req.N, ctx)
            s = capi.fe_derive(ctx, base, self.rho_key(req.N, req.rho))
            h = capi.amg_setup(ctx, s, precision=self.precision, **self.amg_kw)
            e.system, e.hierarchy = s, h
        except BaseException as exc:   # recorded for the waiting requests
            e.error = exc
        finally:
            e.ready.set()

    # ------------------------------------------------------------ solving
    def _solve_one(self, req, slot: int) -> Result:
        ctx = self.ctxs[slot]
        torch = self.torch
        e, hit, solve_bytes = self._admit(req)
        t_start = time.perf_counter()
        try:
            if not hit:
                with torch.cuda.stream(self.streams[slot]):
                    self._build(e, req, ctx)
            e.ready.wait()
            if e.error is not None:
                raise e.error
            own = None
            with torch.cuda.stream(self.streams[slot]):
                if self.rho_key(req.N, req.rho) != req.rho:
                    own = capi.fe_derive(ctx, self.bases[req.N], req.rho)
                system = own if own is not None else e.system
                n_sys = system.n
                f = system.load(I.random_sine_modes(req.target_seed), ctx=ctx)
                u, info, rc = capi.pcg_solve(ctx, system, e.hierarchy, f=f, rtol=self.rtol, maxit=self.maxit)
                if own is not None:
                    own.close()
            res = Result(rid=req.rid, N=req.N, rho=req.rho, n=n_sys, t_arrival=req.t_arrival,
                         t_start=t_start, t_done=time.perf_counter(), iterations=info.iterations,
                         true_rel_res=info.true_rel_res, status=rc, cache_hit=hit, slot=slot,
                         u=u if self.keep else None)
        finally:
            self._release(e, solve_bytes)
        return res

    def run(self, requests: List, realtime: bool = True) -> Tuple[List[Result], float]:
        """Serve the requests (arrival offsets in seconds from the start).
        With realtime, a request is released at its arrival time; otherwise
        all are queued at once.  Returns (results by request id, makespan)."""
        queue = collections.deque()
        cv = threading.Condition()
        results: Dict[int, Result] = {}
        errors: List[BaseException] = []
        done_feeding = [False]
        t0 = time.perf_counter()

        def worker(slot):
            while True:
                with cv:
                    while not queue and not done_feeding[0]:
                        cv.wait()
                    if not queue:
                        return
                    req = queue.popleft()
                try:
                    r = self._solve_one(req, slot)
                    # latencies relative to the stream start
                    r.t_arrival, r.t_start, r.t_done = req.t_arrival, r.t_start - t0, r.t_done - t0
                    results[req.rid] = r
                except BaseException as exc:
                    errors.append(exc)

        threads = [threading.Thread(target=worker, args=(i,), daemon=True) for i in range(self.slots)]
        for th in threads:
            th.start()
        for req in sorted(requests, key=lambda q: q.t_arrival):
            if realtime:
                wait = req.t_arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
            with cv:
                queue.append(req)
                cv.notify()
        with cv:
            done_feeding[0] = True
            cv.notify_all()
        for th in threads:
            th.join()
        makespan = time.perf_counter() - t0
        if errors:
            raise errors[0]
        return [results[q.rid] for q in sorted(requests, key=lambda q: q.rid)], makespan

    def close(self):
        with self.lock:
            for e in self.entries.values():
                if e.hierarchy is not None:
                    e.hierarchy.close()
                if e.system is not None:
                    e.system.close()
            self.entries.clear()
            for b in self.bases.values():
                b.close()
            self.bases.clear()
            self.meshes.clear()
        for c in self.ctxs:
            c.close()


def summarize(results: List[Result], makespan: float) -> dict:
    """Throughput and latency percentiles of a served stream."""
    import numpy as np
    lat = np.array([r.latency for r in results])
    dofs = sum(r.n for r in results)
    return {"requests": len(results), "makespan_s": makespan, "solves_per_s": len(results) / makespan,
            "dof_per_s": dofs / makespan, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "mean_ms": 1e3 * float(lat.mean()),
            "max_iterations": int(max(r.iterations for r in results)),
            "max_true_rel_res": float(max(r.true_rel_res for r in results)),
            "cache_hits": int(sum(r.cache_hit for r in results)),
            "mean_unknowns": float(dofs / len(results))}
