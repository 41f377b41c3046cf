"""rBiCGStab with the stopping tests on the device (batches of iterations
between host reads, enqueued kernel by kernel or replayed as a captured HIP
graph of one iteration) against the host-tested loop: bitwise the same
iterate, history, status and counts, including exits at the half step
(the test on s), iteration caps and the FP32 path.  Graph replays are checked on
every solve, with eager solves of the other modes in between."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import Dev

pytestmark = pytest.mark.gpu


def _solve(krs, d, rec, b, tol, maxmv, flags):
    h = np.zeros(4000)
    x = d.empty()
    rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec, d.vec(b), x,
                                 krs.make_opts(tol=tol, max_matvecs=maxmv, history=h,
                                               flags=flags), d.ws)
    return rc, st, h[:st.history_len].copy(), x


def _same(a, c):
    assert a[0] == c[0]
    for f in ("iterations", "matvecs", "history_len"):
        assert getattr(a[1], f) == getattr(c[1], f), f
    for f in ("rel_res_est", "rel_res_true"):
        assert np.array_equal(getattr(a[1], f), getattr(c[1], f), equal_nan=True), f
    assert np.array_equal(a[2], c[2])
    assert torch.equal(a[3], c[3])
    assert c[1].bytes_model >= a[1].bytes_model


def _compare(krs, d, rec, b, tol, maxmv):
    a = _solve(krs, d, rec, b, tol, maxmv, krs.FLAG_HOST_LOOP)
    for flags in (0, krs.FLAG_GRAPH):
        _same(a, _solve(krs, d, rec, b, tol, maxmv, flags))
    return a[0], a[1]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("pc", ["jacobi", "schwarz"])
def test_device_loop_equals_host_loop(gpu_lib, pc, dtype):
    krs = gpu_lib
    prob = W.grf_problem(24, extra=41)
    params = dict(tile=8) if pc == "schwarz" else None
    d = Dev(krs, prob, pc, params, dtype=dtype, m=20, k=10)
    bs = W.rhs_perturbed(prob, 3, extra=41)
    # a recycle space from two rGCROT solves
    rec = krs.Recycle(d.ctx, prob.n, 10, dtype)
    for b in bs[:2]:
        x = d.empty()
        krs.rgcrot_solve(d.ctx, d.A, d.M, rec, d.vec(b), x, krs.make_opts(m=20, k=10, tol=1e-6),
                         d.ws)
    half_exits = 0
    tols = np.logspace(-2, -10 if dtype == torch.float64 else -6, 9)
    for use_rec in (None, rec):
        for tol in tols:
            rc, st = _compare(krs, d, use_rec, bs[2], float(tol), 4000)
            half_exits += st.matvecs % 2 == 1 and rc == krs.OK
    assert half_exits > 0          # the line-10 exit was exercised
    # iteration caps, odd and even: not converged, same counts
    for maxmv in (7, 8):
        rc, st = _compare(krs, d, None, bs[2], 1e-14, maxmv)
        assert rc == krs.NOT_CONVERGED and st.matvecs == maxmv + (maxmv % 2)


def test_device_loop_zero_rhs_and_converged_start(gpu_lib):
    krs = gpu_lib
    prob = W.grf_problem(8, extra=42)
    d = Dev(krs, prob, "jacobi", m=10, k=4)
    for b in (np.zeros(prob.n), np.ones(prob.n)):
        rc, st = _compare(krs, d, None, b, 1.0 if b.any() else 1e-8, 100)
        assert rc == krs.OK and st.iterations == 0


def test_graph_cache_eviction_and_reuse(gpu_lib):
    """Ten systems on one context (more than the context keeps graphs for),
    solved round-robin three times: every graph replay, new or reused after
    evictions, equals the solve without graphs."""
    krs = gpu_lib
    ctx = krs.Context(torch.device("cuda:0"))
    devs, bs = [], []
    for i in range(10):
        prob = W.grf_problem(8 if i % 2 else 16, extra=50 + i)
        devs.append(Dev(krs, prob, "schwarz" if i % 3 else "jacobi",
                        dict(tile=8) if i % 3 else None, ctx=ctx, m=10, k=4))
        bs.append(W.rhs_perturbed(prob, 1, extra=50 + i)[0])
    ref = [_solve(krs, d, None, b, 1e-8, 2000, 0) for d, b in zip(devs, bs)]
    for _ in range(3):
        for d, b, r in zip(devs, bs, ref):
            _same(r, _solve(krs, d, None, b, 1e-8, 2000, krs.FLAG_GRAPH))
            torch.cuda.synchronize()


def test_breakdown_site_reported_alike(gpu_lib):
    """A skew-symmetric operator (periodic central difference in x, zero
    diagonal) gives r~^T A r~ = 0, so BiCGStab breaks down at alpha
    in the first pass: both loops report the breakdown and its site, like the
    oracle."""
    from oracle import krylov as K
    from oracle import stencil as S
    krs = gpu_lib
    nx, ny, nz = 16, 4, 4
    n = nx * ny * nz
    bands = np.zeros((7, n))
    bands[1] = -1.0     # west
    bands[2] = 1.0      # east
    prob = W.Problem("skew", (nx, ny, nz), (True, False, False), bands, np.ones(n), False)
    d = Dev(krs, prob, "none", m=4, k=2)
    # b lives on even x positions and A b on odd ones: r~^T v = b^T A b = 0 exactly
    b = np.random.default_rng(3).standard_normal(n)
    b[np.arange(n) % 2 == 1] = 0.0
    op = lambda v: S.apply(bands, prob.shape, prob.periodic, v)
    ref = K.rbicgstab(op, lambda v: v.copy(), b, 1e-8, None)
    assert ref.status == K.BREAKDOWN
    for flags in (krs.FLAG_HOST_LOOP, 0):
        x = d.empty()
        rc, st = krs.rbicgstab_solve(d.ctx, d.A, None, None, d.vec(b), x,
                                     krs.make_opts(tol=1e-8, flags=flags), d.ws)
        assert rc == krs.BREAKDOWN and st.breakdown_site == 1, (flags, rc, st.breakdown_site)
        assert st.matvecs == ref.matvecs == 1
