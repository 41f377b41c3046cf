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
    assert half_exits > 0          # the exit after the first half-step was exercised
    # iteration caps, odd and even: not converged, same counts
    for maxmv in (7, 8):
        rc, st = _compare(krs, d, None, bs[2], 1e-14, maxmv)
        assert rc == krs.NOT_CONVERGED and st.matvecs == maxmv + (maxmv % 2)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(13, 11, 7), (5, 3, 1)])
def test_device_loop_equals_host_loop_on_ragged_grids(gpu_lib, shape, dtype):
    """Grids of 1001 and 15 cells, no multiple of a 16-byte pack: the last
    rows of every pack-wide pass (the yr pass with the half-step exit in
    front in the device loop, the separate exit launch in the host loop, the
    full step with the p update) go to the last block.  Both loops agree
    bitwise, with and without a recycle space, over tolerances that end at
    the half and at the full step, and the true residual of the tightest
    solve meets its tolerance."""
    from oracle import stencil as S
    krs = gpu_lib
    prob = W.porous_problem(shape[0], extra=60, shape=shape)
    d = Dev(krs, prob, "jacobi", dtype=dtype, m=10, k=4)
    rec = krs.Recycle(d.ctx, prob.n, 4, dtype)
    rec.U[:4, :prob.n] = torch.from_numpy(
        np.random.default_rng(4).standard_normal((4, prob.n))).to(d.dev, dtype)
    rec.set_dim(4)
    krs.recycle_update(d.ctx, d.A, d.M, rec, d.ws)
    b = W.random_vector(prob.n, 61)
    f64 = dtype == torch.float64
    tols = np.logspace(-2, -10 if f64 else -5, 9)
    half_exits = 0
    for use_rec in (None, rec):
        for tol in tols:
            rc, st = _compare(krs, d, use_rec, b, float(tol), 4000)
            assert rc == krs.OK, (use_rec is not None, tol, rc)
            half_exits += st.matvecs % 2 == 1
        x = _solve(krs, d, use_rec, b, float(tols[-1]), 4000, 0)[3]
        xh = x.double().cpu().numpy()
        res = b - S.apply(prob.bands, prob.shape, prob.periodic, xh)
        # the true residual (FP64 stencil on the FP64 bands) may exceed the
        # updated one the loop stops on by about u * cond(A D^-1) (2.5e3 on
        # the 1001-cell grid): FP64 2 tol; FP32, which also solved with
        # bands rounded to FP32, 1e-3 (the bound u32 * cond is 1.5e-4)
        bar = 2.0 * float(tols[-1]) if f64 else 1e-3
        assert np.linalg.norm(res) <= bar * np.linalg.norm(b), np.linalg.norm(res) / np.linalg.norm(b)
    assert half_exits > 0


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


# ---------------------------------------------------------------------------
# GMRES / rGCROT: the Arnoldi step ends (Givens rotations, residual estimate,
# stopping tests) on the device, read once per batch of steps, against the
# host loop that reads every step and rotates on the host
# ---------------------------------------------------------------------------

def _arnoldi_seq(krs, d, prob, bs, m, k, tol, flags, gmres=False, maxmv=4000):
    rec = krs.Recycle(d.ctx, prob.n, k, d.dtype)
    out = []
    for b in bs:
        h = np.zeros(4000)
        x = d.empty()
        o = krs.make_opts(m=m, k=k, tol=tol, history=h, flags=flags, max_matvecs=maxmv)
        if gmres:
            rc, st = krs.gmres(d.ctx, d.A, d.M, d.vec(b), x, o, d.ws)
        else:
            rc, st = krs.rgcrot_solve(d.ctx, d.A, d.M, rec, d.vec(b), x, o, d.ws)
        U, C = rec.views()
        out.append((rc, st, h[:st.history_len].copy(), x.clone(), U.clone(), C.clone()))
    return out


def _same_arnoldi(a, c):
    assert a[0] == c[0]
    for f in ("iterations", "matvecs", "cycles", "history_len", "second_passes", "eig_ties"):
        assert getattr(a[1], f) == getattr(c[1], f), (f, getattr(a[1], f), getattr(c[1], f))
    for f in ("rel_res_est", "rel_res_true"):
        assert np.array_equal(getattr(a[1], f), getattr(c[1], f), equal_nan=True), f
    assert np.array_equal(a[2], c[2])
    for i in (3, 4, 5):
        assert torch.equal(a[i], c[i])


@pytest.mark.parametrize("case", ["grf24_jacobi_f64", "porous32_schwarz_f64",
                                  "porous32_schwarz_f32", "channel32_schwarz_f64"])
def test_arnoldi_device_loop_equals_host_loop(gpu_lib, case):
    """rGCROT(m,k) sequences with recycle updates, GMRES(m), a step cap in
    the middle of a cycle, and a tolerance met inside a batch: x, U, C, the
    history, counts and statuses bitwise equal in both modes."""
    krs = gpu_lib
    name, pc, dt = case.split("_")
    dtype = torch.float64 if dt == "f64" else torch.float32
    if name == "grf24":
        prob = W.grf_problem(24, extra=61)
        bs = W.rhs_perturbed(prob, 3, extra=61)
        params = None
    else:
        prob = (W.porous_problem(32, extra=62) if name.startswith("porous")
                else W.channel_problem(32))
        bs = list(W.rhs_ar1(prob, 3, extra=62))
        params = dict(W.SCHWARZ_DEFAULT)
    d = Dev(krs, prob, pc, params, dtype=dtype, m=20, k=10)
    tol = 1e-8 if dtype == torch.float64 else 1e-5
    for gm in (False, True):
        a = _arnoldi_seq(krs, d, prob, bs, 20, 10, tol, krs.FLAG_HOST_LOOP, gmres=gm)
        c = _arnoldi_seq(krs, d, prob, bs, 20, 10, tol, 0, gmres=gm)
        for x, y in zip(a, c):
            _same_arnoldi(x, y)
        assert all(r[0] == krs.OK for r in a)
    # step caps (inside the first and the second cycle): not converged, alike
    for maxmv in (13, 27):
        a = _arnoldi_seq(krs, d, prob, bs[:1], 20, 10, 1e-14, krs.FLAG_HOST_LOOP, maxmv=maxmv)
        c = _arnoldi_seq(krs, d, prob, bs[:1], 20, 10, 1e-14, 0, maxmv=maxmv)
        _same_arnoldi(a[0], c[0])
        assert a[0][0] == krs.NOT_CONVERGED and a[0][1].iterations == maxmv


def test_arnoldi_device_loop_zero_rhs(gpu_lib):
    krs = gpu_lib
    prob = W.grf_problem(8, extra=63)
    d = Dev(krs, prob, "jacobi", m=10, k=4)
    for flags in (krs.FLAG_HOST_LOOP, 0):
        x = d.empty()
        rc, st = krs.rgcrot_solve(d.ctx, d.A, d.M, krs.Recycle(d.ctx, prob.n, 4, torch.float64),
                                  d.vec(np.zeros(prob.n)), x, krs.make_opts(m=10, k=4,
                                                                            flags=flags), d.ws)
        assert rc == krs.OK and st.iterations == 0 and float(x.abs().max()) == 0.0
