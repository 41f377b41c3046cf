"""Host logic of the serving loop (no GPU): per-matrix order and exclusivity,
admission by memory with least-recently-used eviction, continuous admission
of requests that arrive while others run."""
import threading
import time

import numpy as np
import pytest

from paper_1501_03358_amd.serve import Request, Scheduler, latency_summary, poisson_arrivals


def _run_fake(sched, n_workers, service, log, lock):
    def worker():
        while True:
            item = sched.next(timeout=0.05)
            if item is None:
                return
            if item == "timeout":
                continue
            req, victims, new = item
            t0 = time.perf_counter()
            with lock:
                log.append(("start", req.mid, req.step, t0, tuple(victims), new))
            time.sleep(service(req))
            req.t_done = time.perf_counter()
            with lock:
                log.append(("end", req.mid, req.step, req.t_done, (), False))
            sched.finish(req)
            req.done.set()

    ths = [threading.Thread(target=worker) for _ in range(n_workers)]
    for t in ths:
        t.start()
    return ths


def test_order_and_exclusivity_per_matrix():
    sched = Scheduler(3, 1e12, lambda mid: 1.0)
    log, lock = [], threading.Lock()
    ths = _run_fake(sched, 3, lambda r: 0.002 * (1 + r.mid % 3), log, lock)
    rid = 0
    for step in range(6):
        for mid in range(5):
            sched.submit(Request(rid, mid, step, np.zeros(1), time.perf_counter()))
            rid += 1
    sched.close()
    for t in ths:
        t.join()
    starts = [e for e in log if e[0] == "start"]
    assert len(starts) == 30
    for mid in range(5):
        steps = [e[2] for e in starts if e[1] == mid]
        assert steps == sorted(steps) == list(range(6))
    # never two requests of one matrix at the same time
    running = set()
    for kind, mid, *_ in sorted(log, key=lambda e: e[3]):
        if kind == "start":
            assert mid not in running
            running.add(mid)
        else:
            running.discard(mid)


def test_admission_by_memory_evicts_least_recently_used():
    sizes = {0: 4.0, 1: 4.0, 2: 4.0}
    sched = Scheduler(1, 9.0, lambda mid: sizes[mid])
    for i, mid in enumerate([0, 1, 2, 0]):
        sched.submit(Request(i, mid, i, np.zeros(1), float(i)))
    order = []
    while True:
        item = sched.next(timeout=0.01)
        if item is None or item == "timeout":
            break
        req, victims, new = item
        order.append((req.mid, tuple(victims), new))
        sched.finish(req)
        if len(order) == 4:
            break
    # 0 and 1 fit (8 <= 9); for 2 the least recently used idle matrix without
    # pending requests (1; 0 still has a queued request) is evicted; 0 then
    # runs with its state still resident
    assert order == [(0, (), True), (1, (), True), (2, (1,), True), (0, (), False)]
    assert sched.used <= 9.0


def test_lru_eviction_order():
    sizes = {m: 3.0 for m in range(4)}
    sched = Scheduler(1, 9.0, lambda mid: sizes[mid])
    for i, mid in enumerate([0, 1, 2]):
        sched.submit(Request(i, mid, 0, np.zeros(1), float(i)))
    for _ in range(3):
        req, victims, new = sched.next(timeout=0.01)
        sched.finish(req)
    sched.submit(Request(3, 1, 1, np.zeros(1), 3.0))       # touch 1 again
    req, victims, new = sched.next(timeout=0.01)
    sched.finish(req)
    sched.submit(Request(4, 3, 0, np.zeros(1), 4.0))       # needs one slot of memory
    req, victims, new = sched.next(timeout=0.01)
    assert req.mid == 3 and victims == [0] and new
    assert list(sched.resident) == [2, 1, 3]


def test_busy_matrix_is_never_evicted():
    sizes = {0: 5.0, 1: 5.0}
    sched = Scheduler(2, 6.0, lambda mid: sizes[mid])
    sched.submit(Request(0, 0, 0, np.zeros(1), 0.0))
    sched.submit(Request(1, 1, 0, np.zeros(1), 1.0))
    req0, victims, new = sched.next(timeout=0.01)
    assert req0.mid == 0
    # matrix 1 does not fit while 0 runs: no admission
    assert sched.next(timeout=0.01) == "timeout"
    sched.finish(req0)
    req1, victims, new = sched.next(timeout=0.01)
    assert req1.mid == 1 and victims == [0]


def test_oversized_matrix_rejected():
    from paper_1501_03358_amd.serve import REJECTED
    sched = Scheduler(1, 1.0, lambda mid: 2.0)
    r = Request(0, 0, 0, np.zeros(1), 0.0)
    assert sched.submit(r) is False
    assert r.done.is_set() and r.status == REJECTED
    assert sched.next(timeout=0.01) == "timeout"


def test_continuous_admission_while_running():
    """Requests submitted while the slots are busy start as soon as a slot
    frees, without waiting for a batch boundary."""
    sched = Scheduler(2, 1e12, lambda mid: 1.0)
    log, lock = [], threading.Lock()
    ths = _run_fake(sched, 2, lambda r: 0.05 if r.mid == 0 else 0.005, log, lock)
    sched.submit(Request(0, 0, 0, np.zeros(1), time.perf_counter()))
    time.sleep(0.005)
    for i in range(1, 5):
        sched.submit(Request(i, i, 0, np.zeros(1), time.perf_counter()))
    sched.close()
    for t in ths:
        t.join()
    end0 = [e[3] for e in log if e[0] == "end" and e[1] == 0][0]
    # the short requests all ran on the second slot while matrix 0 was running
    starts_short = [e[3] for e in log if e[0] == "start" and e[1] != 0]
    assert max(starts_short) < end0


def test_poisson_arrivals_and_latency_summary():
    arr = poisson_arrivals(200.0, 5.0, 64, seed=1)
    assert 800 < len(arr) < 1200
    gaps = np.diff([0.0] + [t for t, _ in arr])
    assert abs(gaps.mean() - 1 / 200) < 0.1 / 200 * 5
    assert set(m for _, m in arr) <= set(range(64))
    reqs = [Request(i, 0, i, np.zeros(1), 0.0, t_done=(i + 1) * 1e-3) for i in range(100)]
    s = latency_summary(reqs)
    assert s["p50"] == pytest.approx(50.5, rel=1e-6)
    assert s["p99"] == pytest.approx(99.01, rel=1e-3)


def test_state_bytes_counts_bands_and_pack():
    from paper_1501_03358_amd.serve import state_bytes
    n = 32 ** 3
    b7 = state_bytes((32, 32, 32), 10)
    b19 = state_bytes((32, 32, 32), 10, npts=19)
    pack7 = 4 * 7 * 10 ** 3 * 64
    rec = 2 * 10 * 4 * (n + 1088)                     # U and C, padded columns
    assert b7 == 7 * 12 * n + 4 * n + pack7 + rec
    assert b19 == 19 * 12 * n + 4 * n + rec          # no coefficient pack for 19 bands


def test_oversized_matrix_is_rejected_and_others_complete():
    """A request whose matrix needs more than the whole memory budget is
    completed at submission with status REJECTED; it does not stop the
    workers, and every other request is still served."""
    from paper_1501_03358_amd.serve import REJECTED
    sizes = {0: 4.0, 1: 100.0, 2: 4.0}
    sched = Scheduler(2, 10.0, lambda mid: sizes[mid])
    log, lock = [], threading.Lock()
    ths = _run_fake(sched, 2, lambda r: 0.001, log, lock)
    reqs = []
    for rid, (mid, step) in enumerate([(1, 0), (0, 0), (2, 0), (1, 1), (0, 1), (2, 1)]):
        r = Request(rid, mid, step, np.zeros(1), time.perf_counter())
        accepted = sched.submit(r)
        assert accepted == (mid != 1)
        reqs.append(r)
    sched.close()
    for t in ths:
        t.join(timeout=10)
        assert not t.is_alive()
    for r in reqs:
        assert r.done.wait(timeout=1)
        if r.mid == 1:
            assert r.status == REJECTED
    served = [(e[1], e[2]) for e in log if e[0] == "start"]
    assert sorted(served) == [(0, 0), (0, 1), (2, 0), (2, 1)]
    assert [r.rid for r in sched.rejected] == [0, 3]
