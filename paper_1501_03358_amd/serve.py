"""Continuous-batching request loop for sequences of pressure-Poisson systems.

Many independent matrices (uneven grid sizes) receive solve requests as their
time steps arrive.  Each matrix keeps its operator (FP64 and FP32 bands), its
Schwarz-Jacobi coefficients and its FP32 recycle space (U, C) resident in HBM
across requests, so every new time step recycles what the previous ones built
(the hybrid of Sec. 2.4: rGCROT for the first `n_switch` steps of a matrix,
rBiCGStab afterwards; each solve is FP32 inside FP64 refinement).

Scheduling (`Scheduler`, host logic only, no GPU):
  * requests of one matrix run one at a time and in arrival order (a time
    step needs the recycle space left by the previous one);
  * a request is admitted when a slot is free and its matrix is resident or
    can be made resident within the memory budget; idle resident matrices are
    evicted least recently used first to make room;
  * among admissible requests the oldest runs first.
Execution (`Server`): `n_slots` worker threads, each with its own HIP stream
and krs context, so the kernels of concurrently admitted solves overlap on the
device; requests arriving meanwhile are admitted as slots and memory free up.
With `batch_max` > 1 a batch worker takes up to `batch_max` admissible
requests of small resident matrices past their rGCROT steps at once and
solves them with krs_ir_solve_batched: every rBiCGStab pass of all of them
runs as one launch per step (launch latency, not bandwidth, bounds such
small solves), and each result is bitwise the one its solve alone gives.

Stream ordering: a matrix's resident state is built on the stream of the
worker that admits it and that stream is synchronised before the state is
published; every solve returns only after its stream has drained, so the
next request of the matrix, on whichever stream, sees all of its updates.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Optional

import numpy as np

# status of a request whose matrix needs more device memory than the whole budget
REJECTED = -101


@dataclasses.dataclass
class Request:
    rid: int
    mid: int                 # matrix id
    step: int                # time-step index within the matrix's sequence
    b: np.ndarray            # right-hand side (FP64, host)
    t_arrival: float
    t_start: float = 0.0
    t_done: float = 0.0
    x: Optional[np.ndarray] = None
    status: int = -99
    stats: Optional[dict] = None
    done: threading.Event = dataclasses.field(default_factory=threading.Event)


class Scheduler:
    """Admission and ordering (thread-safe; no device work)."""

    def __init__(self, n_slots: int, mem_budget: float, state_bytes: Callable[[int], float],
                 classify: Optional[Callable[[int], str]] = None):
        self.n_slots = n_slots
        self.classify = classify          # mid -> "single" | "batch" (None: all single)
        self.budget = float(mem_budget)
        self.state_bytes = state_bytes
        self.lock = threading.Condition()
        self.queues = collections.defaultdict(collections.deque)   # mid -> pending requests
        self.busy = set()                 # matrices with a request running
        self.resident = collections.OrderedDict()   # mid -> bytes (LRU order)
        self.used = 0.0
        self.free_slots = n_slots
        self.closed = False
        self.evicted = []                 # log of evictions (mid)
        self.rejected = []                # requests refused at submission (too large)

    def submit(self, req: Request) -> bool:
        """Queues `req`; a request whose matrix cannot fit the whole memory
        budget is completed at once with status REJECTED (its done event is
        set) and False is returned, so it never blocks the queue."""
        need = self.state_bytes(req.mid)
        with self.lock:
            if need > self.budget:
                req.status = REJECTED
                req.t_start = req.t_done = time.perf_counter()
                self.rejected.append(req)
                req.done.set()
                return False
            self.queues[req.mid].append(req)
            self.lock.notify_all()
            return True

    def _admissible(self, mid):
        if mid in self.resident:
            return True, []
        need = self.state_bytes(mid)
        if need > self.budget:   # never queued (submit rejects it)
            return False, []
        free = self.budget - self.used
        victims = []
        for vid, vb in self.resident.items():     # least recently used first
            if free >= need:
                break
            if vid in self.busy or self.queues.get(vid):
                continue
            victims.append(vid)
            free += vb
        return free >= need, victims

    def _kind(self, mid):
        return "single" if self.classify is None else self.classify(mid)

    def _take(self, mid):
        """Admits the first request of `mid` if memory allows (lock held):
        (request, evict_list, make_resident) or None."""
        ok, victims = self._admissible(mid)
        if not ok:
            return None
        for v in victims:
            self.used -= self.resident.pop(v)
            self.evicted.append(v)
        new = mid not in self.resident
        if new:
            self.resident[mid] = self.state_bytes(mid)
            self.used += self.resident[mid]
        self.resident.move_to_end(mid)
        req = self.queues[mid].popleft()
        self.busy.add(mid)
        return req, victims, new

    def _cands(self, kind):
        return sorted((q[0].t_arrival, mid) for mid, q in self.queues.items()
                      if q and mid not in self.busy and self._kind(mid) == kind)

    def _drained(self):
        return self.closed and not any(self.queues.values()) and not self.busy

    def next(self, timeout=None):
        """Blocks until a request of kind "single" can run; returns
        (request, evict_list, make_resident) or None once closed and drained."""
        with self.lock:
            while True:
                if self.free_slots > 0:
                    for _, mid in self._cands("single"):
                        got = self._take(mid)
                        if got is not None:
                            self.free_slots -= 1
                            return got
                if self._drained():
                    return None
                if not self.lock.wait(timeout):
                    return "timeout"

    def next_batch(self, max_n, timeout=None):
        """Blocks until at least one request of kind "batch" can run; returns
        a list of up to max_n (request, evict_list, make_resident) of
        distinct matrices, oldest first, or None once closed and drained.
        The batch runs in a slot of its own (not one of n_slots)."""
        with self.lock:
            while True:
                out = []
                for _, mid in self._cands("batch"):
                    if len(out) == max_n:
                        break
                    got = self._take(mid)
                    if got is not None:
                        out.append(got)
                if out:
                    return out
                if self._drained():
                    return None
                if not self.lock.wait(timeout):
                    return "timeout"

    def finish_batch(self, reqs):
        with self.lock:
            for r in reqs:
                self.busy.discard(r.mid)
            self.lock.notify_all()

    def finish(self, req: Request):
        with self.lock:
            self.busy.discard(req.mid)
            self.free_slots += 1
            self.lock.notify_all()

    def close(self):
        with self.lock:
            self.closed = True
            self.lock.notify_all()


# ---------------------------------------------------------------------------
# GPU execution
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class MatrixSpec:
    mid: int
    shape: tuple
    periodic: tuple
    bands: np.ndarray        # [7, N] or [19, N] FP64 host
    k: Optional[int] = None  # recycle dimension (None: the server's default)
    n_switch: Optional[int] = None  # rGCROT steps before rBiCGStab (None: the server's)


class _State:
    """Resident device state of one matrix, built on the current stream of
    the admitting worker; that stream is drained before the state is used
    anywhere else."""

    def __init__(self, krs, torch, ctx, spec: MatrixSpec, k, pc):
        dev = ctx.device
        self.spec = spec
        self.b64 = torch.from_numpy(spec.bands).to(dev)
        self.b32 = self.b64.float()
        self.A64 = krs.Matrix(ctx, spec.shape, spec.periodic, self.b64)
        self.A32 = krs.Matrix(ctx, spec.shape, spec.periodic, self.b32)
        self.M32 = krs.Precond(ctx, self.A32, "schwarz", **pc)
        self.k = k
        self.rec = krs.Recycle(ctx, self.A32.n, k, torch.float32)
        self.steps_done = 0
        torch.cuda.current_stream(dev).synchronize()


def state_bytes(shape, k, tile=8, npts=7):
    """Device bytes of a resident matrix: FP64 + FP32 bands (7 or 19), the
    preconditioner (one FP32 vector, plus packed coefficients for 7-point
    bands: at most 7 values per extended-tile cell) and the FP32 recycle space."""
    n = shape[0] * shape[1] * shape[2]
    e = tile + 2
    ntile = (shape[0] // tile) * (shape[1] // tile) * (shape[2] // tile)
    pack = 4 * 7 * e ** 3 * ntile if npts == 7 else 0
    ld = (n + 63) // 64 * 64 + 1088     # leading dimension of U and C
    return npts * n * 12 + 4 * n + pack + 2 * k * 4 * ld


class Server:
    """Request loop over resident matrices with `n_slots` concurrent solves."""

    def __init__(self, specs, device="cuda:0", n_slots=4, mem_budget=64e9, m=30, k=20,
                 n_switch=3, tol=1e-8, inner_tol=1e-5, pc=None, batch_max=0,
                 batch_cells=1 << 18):
        import torch
        from paper_1501_03358_amd import krs
        self.torch, self.krs = torch, krs
        self.device = torch.device(device)
        self.specs = {s.mid: s for s in specs}
        self.m, self.k, self.n_switch, self.tol, self.inner_tol = m, k, n_switch, tol, inner_tol
        self.pc = pc or dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7,
                             global_sweeps=1, omega_global=6 / 7)
        self.k_of = {s.mid: (s.k or k) for s in specs}
        nmax = max(int(np.prod(s.shape)) for s in specs)
        self.ws_bytes = krs.workspace_size(krs.SOLVER_IR, nmax, m, max(self.k_of.values()),
                                           torch.float32)
        slot_bytes = self.ws_bytes + 3 * 8 * nmax
        budget = mem_budget - n_slots * slot_bytes
        # batch worker: small matrices past their rGCROT steps, solved together
        self.batch_max = batch_max if batch_max > 1 else 0
        self.batch_cells = min(batch_cells, nmax)
        if self.batch_max:
            self.batch_ws_bytes = krs.workspace_size(krs.SOLVER_IR, self.batch_cells, m,
                                                     max(self.k_of.values()), torch.float32)
            budget -= self.batch_max * (self.batch_ws_bytes + 3 * 8 * self.batch_cells)
        self.sched = Scheduler(n_slots, budget,
                               lambda mid: state_bytes(self.specs[mid].shape, self.k_of[mid],
                                                       self.pc["tile"],
                                                       len(self.specs[mid].bands)),
                               classify=self._classify if self.batch_max else None)
        self.states = {}
        self.states_lock = threading.Lock()
        self.completed = []
        self.errors = []
        self.threads = [threading.Thread(target=self._worker, args=(i,), daemon=True)
                        for i in range(n_slots)]
        if self.batch_max:
            self.threads.append(threading.Thread(target=self._batch_worker, daemon=True))
        self.batches = []                 # sizes of the batches run
        for th in self.threads:
            th.start()

    def submit(self, req: Request) -> bool:
        """False (and req.status == REJECTED, req.done set) when the
        request's matrix cannot fit the memory budget."""
        return self.sched.submit(req)

    def _n_switch(self, mid):
        ns = self.specs[mid].n_switch
        return self.n_switch if ns is None else ns

    def _classify(self, mid):
        """"batch": a resident 7-band matrix of at most batch_cells cells past
        its rGCROT steps (the next solve is an rBiCGStab one); else "single"."""
        spec = self.specs[mid]
        if int(np.prod(spec.shape)) > self.batch_cells or len(spec.bands) != 7:
            return "single"
        with self.states_lock:
            st = self.states.get(mid)
            return "batch" if st is not None and st.steps_done >= self._n_switch(mid) else "single"

    def close(self, wait=True):
        self.sched.close()
        if wait:
            for th in self.threads:
                th.join()

    def _worker(self, slot):
        torch, krs = self.torch, self.krs
        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            ctx = krs.Context(self.device, stream)
            ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            while True:
                item = self.sched.next(timeout=0.5)
                if item is None:
                    break
                if item == "timeout":
                    continue
                req, victims, new = item
                try:
                    with self.states_lock:
                        for v in victims:
                            self.states.pop(v, None)
                    req.t_start = time.perf_counter()
                    if new:
                        st = _State(krs, torch, ctx, self.specs[req.mid], self.k_of[req.mid],
                                    self.pc)
                        with self.states_lock:
                            self.states[req.mid] = st
                    else:
                        with self.states_lock:
                            st = self.states[req.mid]
                    n = st.A32.n
                    b = torch.from_numpy(req.b).to(self.device, non_blocking=False)
                    x = torch.empty(n, dtype=torch.float64, device=self.device)
                    inner = (krs.SOLVER_RGCROT if st.steps_done < self._n_switch(req.mid)
                             else krs.SOLVER_RBICGSTAB)
                    o = krs.make_opts(m=self.m, k=st.k, tol=self.tol, inner_solver=inner,
                                      inner_tol=self.inner_tol, max_matvecs=4000)
                    rc, sts = krs.ir_solve(ctx, st.A64, st.A32, st.M32, st.rec, b, x, o,
                                           ws[: self.ws_bytes])
                    req.x = x.cpu().numpy()
                    req.status = rc
                    req.stats = sts.as_dict()
                    st.steps_done += 1
                except Exception as exc:  # surfaced to the caller via self.errors
                    req.status = -100
                    self.errors.append((req.rid, repr(exc)))
                finally:
                    req.t_done = time.perf_counter()
                    self.completed.append(req)
                    self.sched.finish(req)
                    req.done.set()
            stream.synchronize()


    def _batch_worker(self):
        torch, krs = self.torch, self.krs
        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            ctx = krs.Context(self.device, stream)
            wss = [torch.empty(self.batch_ws_bytes, dtype=torch.uint8, device=self.device)
                   for _ in range(self.batch_max)]
            tws = torch.empty(krs.BATCH_WORKSPACE_BYTES, dtype=torch.uint8, device=self.device)
            while True:
                items = self.sched.next_batch(self.batch_max, timeout=0.5)
                if items is None:
                    break
                if items == "timeout":
                    continue
                reqs = [it[0] for it in items]
                try:
                    t0 = time.perf_counter()
                    systems, sts = [], []
                    for (req, victims, new), ws in zip(items, wss):
                        req.t_start = t0
                        with self.states_lock:
                            for v in victims:
                                self.states.pop(v, None)
                            st = self.states[req.mid]   # batch requests are resident
                        b = torch.from_numpy(req.b).to(self.device)
                        x = torch.empty(st.A32.n, dtype=torch.float64, device=self.device)
                        systems.append((st.A64, st.A32, st.M32, st.rec, b, x, ws))
                        sts.append(st)
                    o = krs.make_opts(m=self.m, k=min(st.k for st in sts), tol=self.tol,
                                      inner_solver=krs.SOLVER_RBICGSTAB,
                                      inner_tol=self.inner_tol, max_matvecs=4000)
                    rc, stats = krs.ir_solve_batched(ctx, systems, o, tws)
                    self.batches.append(len(reqs))
                    for req, sysd, sst, st in zip(reqs, systems, stats, sts):
                        req.x = sysd[5].cpu().numpy()
                        req.status = sst.status
                        req.stats = sst.as_dict()
                        st.steps_done += 1
                except Exception as exc:  # surfaced to the caller via self.errors
                    for req in reqs:
                        req.status = -100
                    self.errors.append((reqs[0].rid, repr(exc)))
                finally:
                    t1 = time.perf_counter()
                    for req in reqs:
                        req.t_done = t1
                        self.completed.append(req)
                    self.sched.finish_batch(reqs)
                    for req in reqs:
                        req.done.set()
            stream.synchronize()


def poisson_arrivals(rate, duration, n_matrices, seed):
    """(time, matrix id) pairs of a Poisson stream with uniformly chosen matrices."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            return out
        out.append((t, int(rng.integers(n_matrices))))


def latency_summary(reqs):
    lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in reqs])
    if lat.size == 0:
        return {"p50": None, "p99": None, "mean": None}
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "mean": float(lat.mean())}
