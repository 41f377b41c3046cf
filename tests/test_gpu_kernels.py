"""GPU parity of the stencil and preconditioner kernels against the oracle."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import precond, stencil
from tests.gpu_util import Dev, SMALL_SCHWARZ, rel

pytestmark = pytest.mark.gpu

DT = [torch.float64, torch.float32]
TOL = {torch.float64: 1e-13, torch.float32: 2e-6}


def _ragged(shape, periodic, seed):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    kcell = np.exp(rng.standard_normal((nz, ny, nx)))
    vol = rng.uniform(0.5, 1.5, (nz, ny, nx))
    names = 'xyz'
    bc = {names[a]: ('periodic' if periodic[a] else ('dirichlet', 'neumann')) for a in range(3)}
    bands = W.assemble(kcell, vol, (np.ones(nx), np.ones(ny), np.ones(nz)), bc)
    return W.Problem("ragged", shape, periodic, bands, vol.reshape(-1), False)


def _ragged19(shape, periodic, seed):
    """A ragged 7-point problem plus random edge couplings (19 bands)."""
    p7 = _ragged(shape, periodic, seed)
    rng = np.random.default_rng(seed + 50)
    bands = np.zeros((19, p7.n))
    bands[:7] = p7.bands
    bands[7:] = 0.05 * rng.standard_normal((12, p7.n)) * np.abs(p7.bands[0])[None]
    return W.Problem("ragged19", shape, periodic, np.ascontiguousarray(bands), p7.vol, False)


STENCIL_CASES = [
    lambda: W.grf_problem(24),
    lambda: W.channel_problem(16),
    lambda: _ragged((13, 7, 5), (False, True, False), 1),
    lambda: _ragged((1, 1, 1), (False, False, False), 2),
    lambda: _ragged((67, 3, 9), (True, True, True), 3),
    lambda: _ragged((5, 300, 2), (False, False, False), 4),
    # 19-point operators (non-orthogonal grids)
    lambda: W.skewed_problem(16),
    lambda: _ragged19((13, 7, 5), (False, True, False), 11),
    lambda: _ragged19((3, 3, 3), (True, True, True), 12),
    lambda: _ragged19((67, 3, 9), (True, False, True), 13),
]


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("case", range(len(STENCIL_CASES)))
def test_stencil_matches_oracle(gpu_lib, dtype, case):
    krs = gpu_lib
    prob = STENCIL_CASES[case]()
    d = Dev(krs, prob, "none", dtype=dtype)
    rng = np.random.default_rng(case)
    u = rng.standard_normal(prob.n)
    b = rng.standard_normal(prob.n)
    ref_bands = d.bands.double().cpu().numpy()   # FP32 bands as rounded on the device
    y = d.empty()
    krs.stencil_apply(d.ctx, d.A, d.vec(u), y)
    ref = stencil.apply(ref_bands, prob.shape, prob.periodic, d.vec(u).double().cpu().numpy())
    torch.cuda.synchronize()
    scale = np.abs(ref_bands).sum(0) * np.abs(u).max()
    err = np.abs(y.double().cpu().numpy() - ref) / np.maximum(scale, 1e-300)
    assert err.max() <= TOL[dtype] * 10
    # y = -A u + b  (residual form) and y = 2 A u + 0.5 y
    y2 = d.empty()
    krs.stencil_apply(d.ctx, d.A, d.vec(u), y2, -1.0, 1.0, d.vec(b))
    bb = d.vec(b).double().cpu().numpy()
    ref2 = bb - ref
    err2 = np.abs(y2.double().cpu().numpy() - ref2) / np.maximum(scale + np.abs(bb), 1e-300)
    assert err2.max() <= TOL[dtype] * 10
    y3 = y.clone()
    krs.stencil_apply(d.ctx, d.A, d.vec(u), y3, 2.0, 0.5, None)
    ref3 = 2 * ref + 0.5 * y.double().cpu().numpy()
    err3 = np.abs(y3.double().cpu().numpy() - ref3) / np.maximum(scale, 1e-300)
    assert err3.max() <= TOL[dtype] * 10


PC_CASES = [
    ("grf16_t8", lambda: W.grf_problem(16, extra=3), dict(tile=8)),
    ("grf16_t4", lambda: W.grf_problem(16, extra=3), SMALL_SCHWARZ),
    ("channel24_t8", lambda: W.channel_problem(24), dict(tile=8)),
    ("porous32_t8", lambda: W.porous_problem(32, extra=5), dict(tile=8)),
    # even tile counts on every axis: FP32 runs the two-tiles-per-block form
    ("pairs32x16x48_periodic", lambda: _ragged((32, 16, 48), (True, False, True), 16),
     dict(tile=8)),
    ("grf8_t4_nosweep", lambda: W.grf_problem(8, extra=4), dict(tile=4, global_sweeps=0)),
    ("grf8_t4_2global", lambda: W.grf_problem(8, extra=4), dict(tile=4, global_sweeps=2)),
    # SSOR local smoother (colour-ordered forward and backward sweeps)
    ("grf16_t8_ssor", lambda: W.grf_problem(16, extra=3),
     dict(tile=8, local_solver="ssor", omega_local=1.0)),
    ("channel24_t8_ssor13", lambda: W.channel_problem(24),
     dict(tile=8, local_solver="ssor", omega_local=1.3)),
    ("porous32_t4_ssor", lambda: W.porous_problem(32, extra=5),
     dict(tile=4, local_solver="ssor", omega_local=1.0, local_sweeps=3)),
    # 19-point operators: local solves over the 18 neighbours (bands read directly)
    ("skewed16_t8", lambda: W.skewed_problem(16), dict(tile=8)),
    ("skewed16_t4", lambda: W.skewed_problem(16), SMALL_SCHWARZ),
    ("ragged19_24x16x16_t8", lambda: _ragged19((24, 16, 16), (True, False, True), 14),
     dict(tile=8, global_sweeps=2)),
]


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("case", range(len(PC_CASES)))
def test_schwarz_jacobi_matches_oracle(gpu_lib, dtype, case):
    krs = gpu_lib
    name, mk, params = PC_CASES[case]
    prob = mk()
    p = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
             omega_global=6 / 7)
    p.update(params)
    d = Dev(krs, prob, "schwarz", p, dtype=dtype)
    r = np.random.default_rng(case).standard_normal(prob.n)
    z = d.empty()
    krs.precond_apply(d.ctx, d.M, d.vec(r), z)
    ref_bands = d.bands.double().cpu().numpy()
    ref = precond.schwarz_jacobi(ref_bands, prob.shape, prob.periodic,
                                 d.vec(r).double().cpu().numpy(), **p)
    torch.cuda.synchronize()
    assert rel(z.double().cpu().numpy(), ref) <= (1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("dtype", DT)
def test_point_jacobi_matches_oracle(gpu_lib, dtype):
    krs = gpu_lib
    prob = W.grf_problem(24)
    d = Dev(krs, prob, "jacobi", dtype=dtype)
    r = np.random.default_rng(3).standard_normal(prob.n)
    z = d.empty()
    krs.precond_apply(d.ctx, d.M, d.vec(r), z)
    ref = precond.jacobi(d.bands.double().cpu().numpy(), d.vec(r).double().cpu().numpy())
    assert rel(z.double().cpu().numpy(), ref) <= TOL[dtype]


def test_full_size_channel128_stencil_and_schwarz(gpu_lib):
    """Full 128^3 channel operator, the launch configuration of the solver runs."""
    krs = gpu_lib
    prob = W.channel_problem(128)
    d = Dev(krs, prob, "schwarz", dict(tile=8))
    u = np.random.default_rng(9).standard_normal(prob.n)
    y = d.empty()
    krs.stencil_apply(d.ctx, d.A, d.vec(u), y)
    ref = stencil.apply(prob.bands, prob.shape, prob.periodic, u)
    assert rel(y.cpu().numpy(), ref) <= 1e-13
    z = d.empty()
    krs.precond_apply(d.ctx, d.M, d.vec(u), z)
    # sampled: all cells of 24 random tiles (oracle restricted to those tiles'
    # owners would need the full sweep; compare the whole vector instead)
    zr = precond.schwarz_jacobi(prob.bands, prob.shape, prob.periodic, u, tile=8)
    assert rel(z.cpu().numpy(), zr) <= 1e-12


def test_stencil_rejects_aliasing(gpu_lib):
    krs = gpu_lib
    d = Dev(krs, W.grf_problem(8), "none")
    x = d.vec(np.ones(d.prob.n))
    with pytest.raises(krs.KrsError):
        krs.stencil_apply(d.ctx, d.A, x, x)


def test_schwarz_refresh_after_band_change(gpu_lib):
    """The preconditioner stores its local-solve coefficients; after the
    bands change, refresh() makes it follow the new operator."""
    krs = gpu_lib
    prob = W.grf_problem(16, extra=21)
    p = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
             omega_global=6 / 7)
    d = Dev(krs, prob, "schwarz", p)
    r = np.random.default_rng(5).standard_normal(prob.n)
    d.bands.mul_(2.0)
    d.M.refresh()
    z = d.empty()
    krs.precond_apply(d.ctx, d.M, d.vec(r), z)
    ref = precond.schwarz_jacobi(2.0 * prob.bands, prob.shape, prob.periodic, r, **p)
    assert rel(z.cpu().numpy(), ref) <= 1e-12


OP_CASES = PC_CASES + [
    ("grf40x16x8_t8", lambda: _ragged((40, 16, 8), (False, True, False), 7), dict(tile=8)),
    # from 2^22 cells the sweep and the matvec run fused: ragged 64 x 8 and
    # 32 x 16 column tiles, periodic and bounded axes
    ("fused72x24x2432_periodic", lambda: _ragged((72, 24, 2432), (True, True, True), 8),
     dict(tile=8)),
    ("fused40x40x2624", lambda: _ragged((40, 40, 2624), (False, True, False), 9), dict(tile=8)),
    ("fused24x24x7296_px", lambda: _ragged((24, 24, 7296), (True, False, False), 10),
     dict(tile=8)),
    ("fused_pairs64x32x2048", lambda: _ragged((64, 32, 2048), (True, True, False), 17),
     dict(tile=8)),
    # rows of at least 128 cells: 128 x 8 columns (FP32), a ragged second one
    ("fused136x16x1928_px", lambda: _ragged((136, 16, 1928), (True, False, True), 18),
     dict(tile=8)),
    # a 19-point operator of that size runs the sweep and the matvec separately
    ("ragged19_72x24x2432_periodic", lambda: _ragged19((72, 24, 2432), (True, True, True), 15),
     dict(tile=8)),
]


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("case", range(len(OP_CASES)))
def test_operator_apply_matches_oracle(gpu_lib, dtype, case):
    """w = A M^-1 v against the oracle's Schwarz-Jacobi followed by its
    stencil, for the separate kernels (small grids, other sweep counts) and
    the fused sweep + matvec (large grids)."""
    krs = gpu_lib
    name, mk, params = OP_CASES[case]
    prob = mk()
    p = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
             omega_global=6 / 7)
    p.update(params)
    d = Dev(krs, prob, "schwarz", p, dtype=dtype)
    v = np.random.default_rng(100 + case).standard_normal(prob.n)
    w, tmp = d.empty(), d.empty()
    krs.operator_apply(d.ctx, d.A, d.M, d.vec(v), w, tmp)
    ref_bands = d.bands.double().cpu().numpy()
    vv = d.vec(v).double().cpu().numpy()
    z = precond.schwarz_jacobi(ref_bands, prob.shape, prob.periodic, vv, **p)
    ref = stencil.apply(ref_bands, prob.shape, prob.periodic, z)
    assert rel(w.double().cpu().numpy(), ref) <= (1e-12 if dtype == torch.float64 else 1e-5)
    # no preconditioner: the matvec
    krs.operator_apply(d.ctx, d.A, None, d.vec(v), w, tmp)
    ref0 = stencil.apply(ref_bands, prob.shape, prob.periodic, vv)
    assert rel(w.double().cpu().numpy(), ref0) <= (1e-13 if dtype == torch.float64 else 1e-6)


def test_operator_apply_full_size_porous256_fp32(gpu_lib):
    """The 256^3 FP32 operator of the benchmark, in the launch configuration
    the solvers use, on sampled rows: w_i from the oracle's local solves of
    the tiles around cell i (the Schwarz result is exact per tile)."""
    krs = gpu_lib
    prob = W.porous_problem(256, seed_cfg=4)
    p = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
             omega_global=6 / 7)
    d = Dev(krs, prob, "schwarz", p, dtype=torch.float32, m=2, k=1)
    v = np.random.default_rng(7).standard_normal(prob.n)
    w, tmp = d.empty(), d.empty()
    krs.operator_apply(d.ctx, d.A, d.M, d.vec(v), w, tmp)
    # the same operator from the separate kernels: M^-1 v then A (M^-1 v)
    z, w2 = d.empty(), d.empty()
    krs.precond_apply(d.ctx, d.M, d.vec(v), z)
    krs.stencil_apply(d.ctx, d.A, z, w2)
    a, b = w.double().cpu().numpy(), w2.double().cpu().numpy()
    assert rel(a, b) <= 1e-6
    # sampled 8^3 tiles against the oracle on a 40^3 window centred on each:
    # the tile's w needs the swept values one cell out and the local-solve
    # values two cells out, which the window's tiles next to the centre
    # compute exactly as on the full grid (their extended tiles lie inside)
    rng = np.random.default_rng(8)
    bands = d.bands.double().cpu().numpy().reshape(7, 256, 256, 256)
    vv = d.vec(v).double().cpu().numpy().reshape(256, 256, 256)
    for _ in range(6):
        c = rng.integers(2, 30, size=3) * 8       # centre tile origin (x, y, z)
        sl = tuple(slice(int(o) - 16, int(o) + 24) for o in c[::-1])
        sub_b = np.ascontiguousarray(bands[(slice(None),) + sl]).reshape(7, -1)
        sub_v = vv[sl].reshape(-1)
        zs = precond.schwarz_jacobi(sub_b, (40, 40, 40), (False,) * 3, sub_v, **p)
        ws = stencil.apply(sub_b, (40, 40, 40), (False,) * 3, zs).reshape(40, 40, 40)
        got = a.reshape(256, 256, 256)[sl][16:24, 16:24, 16:24]
        refw = ws[16:24, 16:24, 16:24]
        assert np.abs(got - refw).max() <= 1e-4 * np.abs(refw).max()


def test_19pt_ssor_local_solver_rejected(gpu_lib):
    krs = gpu_lib
    prob = W.skewed_problem(8)
    with pytest.raises(krs.KrsError, match="SSOR"):
        Dev(krs, prob, "schwarz", dict(tile=4, local_solver="ssor", omega_local=1.0))


def test_timing_restricted_to_classes(gpu_lib):
    """Kernel timing of selected classes only: launches of other classes get
    no events and no counts; None restores every class."""
    krs = gpu_lib
    prob = W.porous_problem(32, extra=5)
    d = Dev(krs, prob, "schwarz", dict(W.SCHWARZ_DEFAULT), dtype=torch.float32)
    v = d.vec(np.random.default_rng(3).standard_normal(prob.n))
    w, tmp = d.empty(), d.empty()
    krs.timing_reset(d.ctx)
    krs.timing_classes(d.ctx, ["schwarz_local"])
    krs.timing_enable(d.ctx, True)
    krs.operator_apply(d.ctx, d.A, d.M, v, w, tmp)
    krs.timing_enable(d.ctx, False)
    kt = krs.timing_read(d.ctx)
    assert kt["schwarz_local"][0] == 1 and kt["schwarz_local"][1] > 0
    assert all(n == 0 for c, (n, ms, by) in kt.items() if c != "schwarz_local")
    krs.timing_reset(d.ctx)
    krs.timing_classes(d.ctx, None)
    krs.timing_enable(d.ctx, True)
    krs.operator_apply(d.ctx, d.A, d.M, v, w, tmp)
    krs.timing_enable(d.ctx, False)
    kt = krs.timing_read(d.ctx)
    assert kt["schwarz_local"][0] == 1 and sum(n for n, _, _ in kt.values()) >= 3
