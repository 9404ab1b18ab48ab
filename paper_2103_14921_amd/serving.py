"""Continuous-batching server for many Helmholtz solves (serving form).

Requests name a problem (velocity model, grid, spacing, frequency, PML and
decomposition) and carry right-hand sides.  The server keeps the set-up of
every problem it has seen resident (operators, factorisations) until device
memory is needed for something else, admits a request when its device
footprint fits next to what is resident, in flight and idle in PyTorch's
cache (``helm_footprint`` for a problem not yet set up, else the Krylov
workspace ``helm_workspace_bytes``, plus the staging of B and X),
and runs admitted work on worker threads: each resident problem has its own
library handle and HIP stream, so solves of different problems overlap on the
device.  Requests for the same problem and tolerance that are waiting when
the problem's handle becomes free are merged into one batched solve (one
Krylov space per right-hand side, so each result is the same as when solved
alone, up to rounding).  Solutions come back where the right-hand sides were
(host arrays for host arrays, device tensors for device tensors), so results
held by callers take no device memory from the admission budget unless the
caller chose device inputs.  Latency = completion time - arrival time,
including the copy of the solutions back.

Only orchestration lives here; every arithmetic step runs in the HIP library.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import helm


@dataclass(frozen=True)
class ProblemSpec:
    """Everything that determines a set-up (and so the resident factorisation)."""
    name: str
    shape: tuple
    h: float
    freq: float
    pml: tuple = (10, 10, 10, 0)
    parts: tuple = (1, 1, 1)
    overlap: int = 2
    levels: int = 2
    coarse_iters: int = 10
    precision: str = "mixed"
    restart: int = 20

    @property
    def n(self):
        return int(np.prod(self.shape))


@dataclass(eq=False)  # identity: requests carry arrays, and the queue removes them one by one
class _Request:
    spec: ProblemSpec
    B: object
    tol: float
    maxit: int
    arrival: float
    future: Future
    nrhs: int


@dataclass
class _Entry:
    spec: ProblemSpec
    solver: object = None
    resident: int = 0
    busy: bool = False
    last_used: float = 0.0


@dataclass
class ServerStats:
    latencies: list = field(default_factory=list)
    rhs: int = 0
    batches: int = 0
    setups: int = 0
    evictions: int = 0
    peak_accounted: int = 0
    retries: int = 0  # batches put back in the queue after the device ran short


class Server:
    """Continuous-batching solve server on one GPU.

    velocity_of(spec) must return the complex128 velocity [nz][ny][nx] of a
    problem (host array or device tensor); it is called once per set-up.
    budget_bytes defaults to 85 % of the device less what PyTorch holds
    allocated when the server starts.
    """

    def __init__(self, velocity_of, budget_bytes=None, workers=4, max_batch_rhs=64, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if budget_bytes is None:
            # 85 % of the device, less what the caller's tensors hold already
            free, total = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(0.85 * total) - torch.cuda.memory_allocated(self.device)
        self.budget = int(budget_bytes)
        self.velocity_of = velocity_of
        self.max_batch_rhs = max_batch_rhs
        self.weights = helm.fit_weights()
        self._pool = ThreadPoolExecutor(max_workers=workers)
        self._cv = threading.Condition()
        self._queue = collections.deque()
        self._entries = collections.OrderedDict()
        self._inflight = 0
        self._hold = False  # after a batch was put back: launch nothing until another one ends
        self._closed = False
        self.stats = ServerStats()
        self._sched = threading.Thread(target=self._loop, daemon=True)
        self._sched.start()

    # ---- public -----------------------------------------------------------
    def submit(self, spec: ProblemSpec, B, tol=1e-6, maxit=400):
        """Queue a solve; returns a Future of dict(X, iters, relres_true, latency_s, batch_rhs)."""
        fut = Future()
        req = _Request(spec, B, float(tol), int(maxit), time.perf_counter(), fut, int(B.shape[0]))
        with self._cv:
            if self._closed:
                raise RuntimeError("server closed")
            self._queue.append(req)
            self._cv.notify_all()
        return fut

    def drain(self):
        """Block until every submitted request has completed."""
        with self._cv:
            while self._queue or self._inflight_count():
                self._cv.wait(0.05)

    def close(self):
        self.drain()
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        self._sched.join()
        self._pool.shutdown(wait=True)
        for e in self._entries.values():
            if e.solver is not None:
                e.solver.close()
        self._entries.clear()

    def latency_percentiles(self):
        lat = np.array(self.stats.latencies)
        if lat.size == 0:
            return {}
        return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "max_s": float(lat.max())}

    # ---- internals ---------------------------------------------------------
    def _inflight_count(self):
        return sum(1 for e in self._entries.values() if e.busy)

    def _footprint(self, spec, nrhs):
        return helm.footprint(spec.shape, spec.parts, spec.overlap, spec.levels, spec.coarse_iters, spec.precision,
                              spec.restart, nrhs)

    def _workspace(self, spec, nrhs):
        return helm.workspace_bytes(spec.shape, spec.parts, spec.overlap, spec.levels, spec.coarse_iters,
                                    spec.precision, spec.restart, nrhs)

    @staticmethod
    def _staging(spec, nrhs):
        # B and X of the batch on the device (complex128 each)
        return 2 * 16 * nrhs * int(np.prod(spec.shape))

    def _staging_room(self, nbytes):
        """Make sure PyTorch's staging of a batch leaves the library's device headroom
        (helm_device_headroom) free: the runtime allocates for itself at dispatch,
        and a failure there aborts the queue.  Trims the library's and PyTorch's
        idle caches if needed; raises HELM_ENOMEM (the batch goes back to the
        queue while others run) if the room is still not there."""
        torch = self.torch
        if self.device.type != "cuda":
            return
        need = nbytes + helm.device_headroom()
        if torch.cuda.mem_get_info(self.device)[0] >= need:
            return
        helm.trim_cache()
        torch.cuda.empty_cache()
        if torch.cuda.mem_get_info(self.device)[0] < need:
            raise helm.HelmError(helm.HELM_ENOMEM, "no room to stage the batch above the device headroom")

    def _need(self, spec, nrhs, resident, chunk=None):
        """Device bytes a batch of nrhs right-hand sides takes while in flight when
        the library solves chunk of them at a time (all by default): the whole
        Krylov workspace of a chunk (released after every batch) when the set-up
        is resident, else the full footprint (set-up transients included), plus
        the staging of B and X."""
        k = min(chunk or nrhs, nrhs)
        base = self._workspace(spec, k) if resident else self._footprint(spec, k)
        # the library's device cache may hand out blocks up to an eighth larger
        # than asked for: reserve for that
        return base + base // 8 + self._staging(spec, nrhs) + (64 << 20)

    def _largest_chunk(self, spec, nrhs, resident):
        """Most right-hand sides per library solve that keep a request of nrhs
        within the budget (0: not even one)."""
        lo, hi = 0, nrhs
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if self._need(spec, nrhs, resident, mid) <= self.budget:
                lo = mid
            else:
                hi = mid - 1
        return lo

    def _torch_idle(self):
        # blocks PyTorch's caching allocator holds without using them: device
        # memory the library cannot get while they stay cached
        t = self.torch
        return max(t.cuda.memory_reserved(self.device) - t.cuda.memory_allocated(self.device), 0)

    def _accounted(self):
        return sum(e.resident for e in self._entries.values()) + self._inflight + self._torch_idle()

    def _evict_for(self, need, keep_key):
        """Make room for need bytes (idle PyTorch cache first, then least recently
        used set-ups); returns the accounted total with need added, or None."""
        if self._accounted() + need > self.budget and self._torch_idle() > 0:
            self.torch.cuda.empty_cache()
        for key in list(self._entries.keys()):  # least recently used first
            acc = self._accounted() + need
            if acc <= self.budget:
                return acc
            e = self._entries[key]
            if key == keep_key or e.busy:
                continue
            if e.solver is not None:
                e.solver.close()
            del self._entries[key]
            self.stats.evictions += 1
        acc = self._accounted() + need
        return acc if acc <= self.budget else None

    def _loop(self):
        with self._cv:
            while True:
                if self._closed and not self._queue:
                    return
                launched = self._try_launch()
                if not launched:
                    self._cv.wait(0.05)

    def _held(self):
        # after a batch went back to the queue, nothing new starts until another
        # batch in flight has ended; with none in flight there is nothing to wait for
        return self._hold and self._inflight_count() > 0

    def _try_launch(self):
        if self._held():
            return False
        self._hold = False
        for head in list(self._queue):
            key = (head.spec, head.tol, head.maxit)
            e = self._entries.get(head.spec)
            if e is not None and e.busy:
                continue
            resident = e is not None and e.solver is not None
            batch, nr = [], 0
            for r in self._queue:
                # merge waiting requests of the same problem while the batch stays
                # within max_batch_rhs and the device budget
                if (r.spec, r.tol, r.maxit) == key and (not batch or (
                        nr + r.nrhs <= self.max_batch_rhs
                        and self._need(head.spec, nr + r.nrhs, resident) <= self.budget)):
                    batch.append(r)
                    nr += r.nrhs
            chunk = nr
            need = self._need(head.spec, nr, resident)
            if need > self.budget:
                # a single request too large to solve at once: solve it in chunks
                # of right-hand sides, one after another on its handle
                chunk = self._largest_chunk(head.spec, nr, resident)
                if chunk == 0:  # the batch is one request (merges were checked against the budget)
                    big = batch[0]
                    self._queue.remove(big)
                    big.future.set_exception(helm.HelmError(helm.HELM_ENOMEM, "request larger than the device budget"))
                    return True
                need = self._need(head.spec, nr, resident, chunk)
            acc = self._evict_for(need, head.spec)
            if acc is None:
                continue
            if e is None:
                e = _Entry(head.spec)
                self._entries[head.spec] = e
            self._entries.move_to_end(head.spec)
            e.busy = True
            self._inflight += need
            for r in batch:
                self._queue.remove(r)
            self.stats.peak_accounted = max(self.stats.peak_accounted, acc)
            self._pool.submit(self._work, e, batch, nr, need, chunk)
            return True
        return False

    def _work(self, e, batch, nr, reserved, chunk):
        torch = self.torch
        retried = False
        try:
            spec = e.spec
            if e.solver is None:
                vel = self.velocity_of(spec)
                e.solver = helm.Solver(spec.shape, spec.h, vel, spec.freq, spec.pml, weights=self.weights,
                                       parts=spec.parts, overlap=spec.overlap, levels=spec.levels,
                                       coarse_iters=spec.coarse_iters, precision=spec.precision,
                                       restart=spec.restart)
                self.stats.setups += 1
            def stage():
                parts = []
                for r in batch:
                    b = r.B if helm._is_torch(r.B) else torch.from_numpy(np.ascontiguousarray(r.B))
                    parts.append(b.reshape(r.nrhs, -1).to(self.device))
                return torch.cat(parts, 0).contiguous() if len(parts) > 1 else parts[0].contiguous()

            self._staging_room(self._staging(spec, nr))
            Bd = helm.torch_alloc(stage)
            # a request gets X where its B was: host arrays come back as host
            # arrays, so delivered results hold no device memory outside the
            # admission accounting
            if chunk >= nr:
                X, info = e.solver.solve(Bd, tol=batch[0].tol, maxit=batch[0].maxit)
                outs, i0 = [], 0
                for r in batch:
                    Xr = X[i0:i0 + r.nrhs]
                    i0 += r.nrhs
                    outs.append(Xr.clone() if helm._is_torch(r.B) else Xr.cpu().numpy())
                del X
            else:  # one request, solved chunk right-hand sides at a time
                parts, infos = [], []
                for i0 in range(0, nr, chunk):
                    Xi, inf = e.solver.solve(Bd[i0:i0 + chunk], tol=batch[0].tol, maxit=batch[0].maxit)
                    parts.append(Xi if helm._is_torch(batch[0].B) else Xi.cpu().numpy())
                    infos.append(inf)
                    del Xi
                outs = [torch.cat(parts, 0) if helm._is_torch(batch[0].B) else np.concatenate(parts, 0)]
                info = {"iters": np.concatenate([i["iters"] for i in infos]),
                        "relres_true": np.concatenate([i["relres_true"] for i in infos]),
                        "status": max((i["status"] for i in infos), key=abs)}
            e.solver.release_workspace()
            del Bd
            done = time.perf_counter()
            i0 = 0
            with self._cv:
                self.stats.batches += 1
                self.stats.rhs += nr
                for r, Xr in zip(batch, outs):
                    sl = slice(i0, i0 + r.nrhs)
                    i0 += r.nrhs
                    lat = done - r.arrival
                    self.stats.latencies.append(lat)
                    r.future.set_result({"X": Xr, "iters": info["iters"][sl], "relres_true": info["relres_true"][sl],
                                         "status": info["status"], "latency_s": lat, "batch_rhs": nr})
        except Exception as exc:
            short = (isinstance(exc, helm.HelmError) and exc.code == helm.HELM_ENOMEM) or \
                isinstance(exc, torch.OutOfMemoryError)
            if e.solver is not None:
                try:  # whatever workspace the failed solve had taken
                    e.solver.release_workspace()
                except helm.HelmError:
                    pass
            with self._cv:
                others = any(x.busy for x in self._entries.values() if x is not e)
                if short and others:
                    # the device ran short while other batches are in flight (the
                    # footprints are estimates): put the batch back at the head of
                    # the queue and hold new launches until one of the others has
                    # ended -- set here, in the same critical section that saw them
                    # busy, so that their ends (which lift the hold) come after it
                    for r in reversed(batch):
                        self._queue.appendleft(r)
                    self.stats.retries += 1
                    self._hold = True
                    retried = True
                else:  # report the failure on every request of the batch
                    for r in batch:
                        if not r.future.done():
                            r.future.set_exception(exc)
        finally:
            with self._cv:
                if not retried:  # a batch that ended lifts a hold
                    self._hold = False
                e.resident = e.solver.resident_bytes() if e.solver is not None else 0
                e.busy = False
                e.last_used = time.perf_counter()
                self._inflight -= reserved
                self._cv.notify_all()


def run_poisson(server, requests, rate_hz, seed=4, progress=None, deadline=None):
    """Submit (spec, B, tol) requests with Poisson arrivals of the given rate; wait for all.

    ``deadline`` (a time.perf_counter() value): submit no request whose arrival
    falls after it (those already submitted still complete).
    Returns dict(elapsed_s, rhs, rhs_per_s, latency percentiles, results).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=len(requests))
    t0 = time.perf_counter()
    futs = []
    t_next = t0
    done = [0]
    lock = threading.Lock()

    def report(_):  # progress as requests complete, also while later ones are still arriving
        with lock:
            done[0] += 1
            if progress:
                progress(done[0], n_sub)

    n_sub = len(requests)
    for k, ((spec, B, tol), gap) in enumerate(zip(requests, gaps)):
        t_next += gap
        if deadline is not None and t_next > deadline:
            n_sub = k
            break
        dt = t_next - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        f = server.submit(spec, B, tol)
        f.add_done_callback(report)
        futs.append(f)
    results = []
    for f in futs:
        r = dict(f.result())
        r["nrhs"] = int(r.pop("X").shape[0])  # the stream's figures need no solutions
        results.append(r)
    elapsed = time.perf_counter() - t0
    rhs = sum(r["nrhs"] for r in results)
    out = {"elapsed_s": elapsed, "rhs": rhs, "rhs_per_s": rhs / elapsed, "requests": len(results),
           "results": results}
    out.update(server.latency_percentiles())
    return out
