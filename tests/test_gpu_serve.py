"""Serving loop on the GPU: results are bitwise the same when a matrix's
sequence runs alone and when it runs interleaved with other matrices on
concurrent streams; a memory budget that holds two matrices still serves
every request to the tolerance."""
import time

import numpy as np
import pytest

import workloads as W
from oracle import stencil

pytestmark = pytest.mark.gpu


def _specs():
    from paper_1501_03358_amd.serve import MatrixSpec
    probs = [W.grf_problem(16, extra=31), W.channel_problem(24), W.porous_problem(32, extra=32),
             W.porous_problem(16, extra=33)]
    specs = [MatrixSpec(i, p.shape, p.periodic, p.bands) for i, p in enumerate(probs)]
    rhs = {i: list(W.rhs_ar1(p, 4, seed_cfg=5, extra=40 + i)) for i, p in enumerate(probs)}
    return probs, specs, rhs


def _run(server_kw, specs, rhs, order):
    from paper_1501_03358_amd.serve import Request, Server
    srv = Server(specs, **server_kw)
    reqs = []
    for rid, (mid, step) in enumerate(order):
        r = Request(rid, mid, step, rhs[mid][step], time.perf_counter())
        reqs.append(r)
        srv.submit(r)
    srv.close()
    assert not srv.errors, srv.errors
    return reqs, srv


def test_alone_equals_mixed(gpu_lib):
    probs, specs, rhs = _specs()
    kw = dict(m=20, k=10, n_switch=2, mem_budget=8e9)
    mixed_order = [(mid, step) for step in range(4) for mid in range(4)]
    mixed, srv = _run(dict(kw, n_slots=3), specs, rhs, mixed_order)
    for mid in range(4):
        alone, _ = _run(dict(kw, n_slots=1), specs, rhs, [(mid, s) for s in range(4)])
        for step in range(4):
            a = alone[step]
            b = next(r for r in mixed if r.mid == mid and r.step == step)
            assert a.status == 0 and b.status == 0
            assert np.array_equal(a.x, b.x), (mid, step)
    # every result meets the FP64 tolerance
    for r in mixed:
        p = probs[r.mid]
        res = rhs[r.mid][r.step] - stencil.apply(p.bands, p.shape, p.periodic, r.x)
        assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(rhs[r.mid][r.step])


def test_memory_budget_evicts_and_still_serves(gpu_lib):
    from paper_1501_03358_amd.serve import state_bytes
    probs, specs, rhs = _specs()
    from paper_1501_03358_amd import krs
    import torch
    nmax = max(p.n for p in probs)
    slot = krs.workspace_size(krs.SOLVER_IR, nmax, 20, 10, torch.float32) + 3 * 8 * nmax
    two = sorted(state_bytes(p.shape, 10) for p in probs)[-2:]
    budget = slot * 2 + sum(two) * 1.01
    order = [(mid, step) for step in range(3) for mid in range(4)]
    reqs, srv = _run(dict(m=20, k=10, n_switch=2, mem_budget=budget, n_slots=2), specs, rhs,
                     order)
    assert len(srv.sched.evicted) > 0
    for r in reqs:
        assert r.status == 0
        p = probs[r.mid]
        res = rhs[r.mid][r.step] - stencil.apply(p.bands, p.shape, p.periodic, r.x)
        assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(rhs[r.mid][r.step])


def test_serving_mixes_7_and_19_point_matrices(gpu_lib):
    """A 19-band (sheared-grid) matrix served next to 7-band ones: every
    request meets the tolerance, and the 19-band state is admitted with its
    own size."""
    from paper_1501_03358_amd.serve import MatrixSpec, state_bytes
    probs = [W.skewed_problem(16, extra=35), W.grf_problem(16, extra=36)]
    specs = [MatrixSpec(i, p.shape, p.periodic, p.bands) for i, p in enumerate(probs)]
    rhs = {i: list(W.rhs_ar1(p, 3, seed_cfg=5, extra=50 + i)) for i, p in enumerate(probs)}
    order = [(mid, step) for step in range(3) for mid in range(2)]
    reqs, srv = _run(dict(m=20, k=10, n_switch=2, mem_budget=8e9, n_slots=2), specs, rhs, order)
    for r in reqs:
        assert r.status == 0
        p = probs[r.mid]
        res = rhs[r.mid][r.step] - stencil.apply(p.bands, p.shape, p.periodic, r.x)
        assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(rhs[r.mid][r.step])
    assert srv.sched.resident[0] == state_bytes((16, 16, 16), 10, 8, 19)
    assert srv.sched.resident[1] == state_bytes((16, 16, 16), 10, 8, 7)
