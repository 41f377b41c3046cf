"""GPU FP64 solver parity with the oracle: residual history within 1e-10
(relative) over the first 20 iterations, iteration counts within 2, final x
within 1e-8 (relative; modulo the constant for singular systems); recycle
space invariants; FP32 + FP64 iterative refinement to a 1e-8 true residual."""
import numpy as np
import pytest
import scipy.linalg
import torch

import workloads as W
from oracle import krylov as K
from oracle import precond, stencil
from tests.gpu_util import Dev, SMALL_SCHWARZ, mod_const, oracle_ops, recycle_to_oracle, rel

pytestmark = pytest.mark.gpu

HIST_TOL = 1e-10
X_TOL = 1e-8


def _hist(n=4000):
    return np.zeros(n)


def _check_history(h_gpu, h_ref, nfirst=20, tol=HIST_TOL):
    n = min(nfirst, len(h_ref), len(h_gpu))
    assert n > 0
    a = np.asarray(h_gpu[:n])
    b = np.asarray(h_ref[:n])
    assert np.all(np.abs(a - b) <= tol * np.abs(b)), (a, b)


def test_gmres_matches_oracle_grf24(gpu_lib):
    krs = gpu_lib
    prob = W.grf_problem(24)
    d = Dev(krs, prob, "jacobi", m=20, k=10)
    _, Mi, op = oracle_ops(prob, "jacobi")
    b = W.rhs_perturbed(prob, 1)[0]
    h = _hist()
    x = d.empty()
    rc, st = krs.gmres(d.ctx, d.A, d.M, d.vec(b), x, krs.make_opts(m=20, tol=1e-8, history=h),
                       d.ws)
    ref = K.gmres(op, Mi, b, 20, 1e-8)
    assert rc == krs.OK and ref.status == K.CONVERGED
    _check_history(h[:st.history_len], ref.history)
    assert abs(st.iterations - ref.iterations) <= 2
    assert rel(x.cpu().numpy(), ref.x) <= X_TOL
    assert st.rel_res_true <= 1e-8


def _rgcrot_sequence(krs, prob, pc, params, m, k, steps, bs, tol=1e-8, stepwise=True,
                     gcrot=None):
    """Runs the GPU rGCROT over a sequence of right-hand sides next to the
    oracle.  stepwise: before every system the oracle receives a copy of the
    GPU's recycle space, so that both sides solve the same problem and only
    the step's own rounding differs; otherwise each side keeps its own space
    (recycle updates then amplify rounding through the eigenvector step).
    gcrot: oracle GcrotParams; both sides then update by the GCROT rule."""
    d = Dev(krs, prob, pc, params, m=m, k=k,
            solver=krs.SOLVER_RGCROT_T if gcrot is not None else None)
    extra = {} if gcrot is None else dict(recycle_rule=krs.RECYCLE_GCROT, gcrot_kt=gcrot.kt,
                                          gcrot_s=gcrot.s, gcrot_p=gcrot.p)
    _, Mi, op = oracle_ops(prob, pc, params)
    rec = krs.Recycle(d.ctx, prob.n, k, torch.float64)
    orec = K.Recycle.empty(prob.n)
    out = []
    for t in range(steps):
        b = bs[t]
        if stepwise:
            orec = recycle_to_oracle(rec)
        h = _hist()
        x = d.empty()
        rc, st = krs.rgcrot_solve(d.ctx, d.A, d.M, rec, d.vec(b), x,
                                  krs.make_opts(m=m, k=k, tol=tol, history=h, **extra), d.ws)
        ref = K.rgcrot(op, Mi, b, m, k, tol, orec, gcrot=gcrot)
        out.append((rc, st, h[:st.history_len].copy(), x.cpu().numpy(), ref))
    return d, rec, orec, op, out


def _check_solution(prob, x, xr):
    if prob.singular:
        assert rel(mod_const(x, prob.vol), mod_const(xr, prob.vol)) <= X_TOL
    else:
        assert rel(x, xr) <= X_TOL


def test_rgcrot_stepwise_matches_oracle_grf24(gpu_lib):
    """24^3 GRF workload, point Jacobi, rGCROT(20,10), 5 right-hand sides;
    every system compared from the same recycle space."""
    krs = gpu_lib
    prob = W.grf_problem(24)
    bs = W.rhs_perturbed(prob, 5)
    d, rec, orec, op, out = _rgcrot_sequence(krs, prob, "jacobi", None, 20, 10, 5, bs)
    for t, (rc, st, h, x, ref) in enumerate(out):
        assert rc == krs.OK and ref.status == K.CONVERGED, t
        assert st.eig_ties == 0 and ref.eig_ties == 0
        _check_history(h, ref.history)
        assert abs(st.iterations - ref.iterations) <= 2, (t, st.iterations, ref.iterations)
        _check_solution(prob, x, ref.x)
    # recycle spaces after the last system: same range, A~ U = C, C^T C = I
    g = recycle_to_oracle(rec)
    assert g.dim == orec.dim == 10
    assert scipy.linalg.subspace_angles(g.C, orec.C).max() < 1e-6
    AU = np.column_stack([op(g.U[:, i]) for i in range(g.dim)])
    assert np.linalg.norm(AU - g.C) / np.linalg.norm(g.C) <= 1e-11
    assert np.linalg.norm(g.C.T @ g.C - np.eye(g.dim)) <= 1e-12
    # recycling pays: later systems need fewer iterations than the first
    assert out[-1][1].iterations < out[0][1].iterations


def test_rgcrot_independent_sequence_grf24(gpu_lib):
    """Each side keeps its own recycle space over the 5 systems: iteration
    counts within 2 and solutions within 1e-8; the first system's history
    (no recycle space yet) within 1e-10."""
    krs = gpu_lib
    prob = W.grf_problem(24)
    bs = W.rhs_perturbed(prob, 5)
    d, rec, orec, op, out = _rgcrot_sequence(krs, prob, "jacobi", None, 20, 10, 5, bs,
                                             stepwise=False)
    _check_history(out[0][2], out[0][4].history)
    for t, (rc, st, h, x, ref) in enumerate(out):
        assert rc == krs.OK and ref.status == K.CONVERGED, t
        assert abs(st.iterations - ref.iterations) <= 2, (t, st.iterations, ref.iterations)
        _check_solution(prob, x, ref.x)


@pytest.mark.parametrize("kind", ["channel", "porous"])
def test_rgcrot_schwarz_matches_oracle(gpu_lib, kind):
    krs = gpu_lib
    prob = W.channel_problem(24) if kind == "channel" else W.porous_problem(24, extra=7)
    bs = list(W.rhs_ar1(prob, 3, extra=7))
    params = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
                  omega_global=6 / 7)
    d, rec, orec, op, out = _rgcrot_sequence(krs, prob, "schwarz", params, 30, 20, 3, bs)
    for t, (rc, st, h, x, ref) in enumerate(out):
        assert rc == krs.OK and ref.status == K.CONVERGED
        _check_history(h, ref.history)
        assert abs(st.iterations - ref.iterations) <= 2
        _check_solution(prob, x, ref.x)


# Rounding-level perturbations: relative changes of b of at most 1e-15, and
# operators whose every output element is scaled by (1 + d), |d| <= u = 2^-53
# (seeded): one unit of rounding per operation, as two correct
# implementations with different summation orders differ.  The oracle's own
# spread of exit steps and solutions under them is what a GPU result may
# differ by where the exit step is not determined by the method (BiCGStab's
# irregular residual near the tolerance).
ROUNDING_EPS = (1.1e-16, -1.1e-16, 4.4e-16, -4.4e-16, 1e-15, -1e-15)
UNIT_ROUNDOFF = 2.0 ** -53
ROUNDING_SEEDS = 16


def _rounded(op, seed):
    rng = np.random.default_rng(seed)

    def opr(v):
        w = op(v)
        return w * (1.0 + UNIT_ROUNDOFF * rng.uniform(-1.0, 1.0, w.size))
    return opr


def _oracle_spread(solve, op, b, ref):
    """Exit steps and x-spread of the oracle under rounding-level
    perturbations (of b, and of every operator application):
    (min its, max its, max relative x distance to ref).  solve(b, op)."""
    its, dx = [ref.iterations], 0.0
    runs = [solve(b * (1 + eps), op) for eps in ROUNDING_EPS]
    runs += [solve(b, _rounded(op, seed)) for seed in range(ROUNDING_SEEDS)]
    for r in runs:
        its.append(r.iterations)
        dx = max(dx, rel(r.x, ref.x))
    return min(its), max(its), dx


@pytest.mark.parametrize("pc", ["schwarz", "jacobi"])
def test_rbicgstab_plain_and_recycled_match_oracle(gpu_lib, pc):
    """Schwarz preconditioning: smooth convergence in a few dozen
    iterations.  Point Jacobi: 130+ iterations with the irregular residual
    of BiCGStab.  History within 1e-10 over 20 iterations; the count within
    2 of the range of exits the oracle itself takes under rounding-level
    perturbations (b by at most 1e-15 relative, every operator output by at
    most one unit roundoff); x at tol 1e-8 within the oracle's own x-spread
    under those perturbations (times 3, at least 1e-8), and at tol 1e-12
    within 1e-8."""
    krs = gpu_lib
    prob = W.grf_problem(24)
    bs = W.rhs_perturbed(prob, 5)
    params = dict(tile=8) if pc == "schwarz" else None
    d, rec, orec, op, out = _rgcrot_sequence(krs, prob, pc, params, 20, 10, 3, bs)
    _, Mi, _ = oracle_ops(prob, pc, params)
    g = recycle_to_oracle(rec)             # oracle runs with the GPU's recycle space
    st_plain = None
    for use_rec in (False, True):
        b = bs[4]
        h = _hist()
        x = d.empty()
        rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec if use_rec else None, d.vec(b), x,
                                     krs.make_opts(tol=1e-8, history=h), d.ws)
        solve = lambda bb, opx: K.rbicgstab(opx, Mi, bb, 1e-8, g if use_rec else None)
        ref = solve(b, op)
        assert rc == krs.OK and ref.status == K.CONVERGED
        _check_history(h[:st.history_len], ref.history)
        lo, hi, spread = _oracle_spread(solve, op, b, ref)
        assert lo - 2 <= st.iterations <= hi + 2, (st.iterations, ref.iterations, lo, hi)
        assert rel(x.cpu().numpy(), ref.x) <= max(X_TOL, 3 * spread), spread
        assert st.rel_res_true <= 2e-8
        if use_rec:
            assert st.iterations < st_plain.iterations
        else:
            st_plain = st
        x2 = d.empty()
        rc2, st2 = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec if use_rec else None, d.vec(b), x2,
                                       krs.make_opts(tol=1e-12), d.ws)
        ref2 = K.rbicgstab(op, Mi, b, 1e-12, g if use_rec else None)
        assert rc2 == krs.OK and ref2.status == K.CONVERGED
        assert rel(x2.cpu().numpy(), ref2.x) <= X_TOL


def test_rbicgstab_history_on_a_512_block_grid(gpu_lib):
    """Above 2^19 cells the BiCGStab passes run on 512 blocks and the alpha and
    omega steps in front of the update passes sum 512 partials per column
    (the path the benchmark's grids take): FP64 plain and recycled BiCGStab
    with point Jacobi on a 96^3 random-field medium, the residual history
    against the oracle's over the first 20 iterations (1e-10)."""
    krs = gpu_lib
    prob = W.grf_problem(96, extra=11)
    d = Dev(krs, prob, "jacobi", m=1, k=6)
    _, Mi, op = oracle_ops(prob, "jacobi")
    b = next(W.rhs_ar1(prob, 1, extra=11))
    rec = krs.Recycle(d.ctx, prob.n, 6, torch.float64)
    U0 = np.random.default_rng(6).standard_normal((prob.n, 6))
    rec.U[:6, :prob.n] = torch.from_numpy(U0.T.copy()).to(d.dev)
    rec.set_dim(6)
    krs.recycle_update(d.ctx, d.A, d.M, rec, d.ws)
    g = recycle_to_oracle(rec)
    for use_rec in (False, True):
        h = _hist()
        x = d.empty()
        rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec if use_rec else None, d.vec(b), x,
                                     krs.make_opts(tol=1e-8, max_matvecs=80, history=h), d.ws)
        ref = K.rbicgstab(op, Mi, b, 1e-8, g if use_rec else None, max_matvecs=80)
        assert st.history_len >= 20 and len(ref.history) >= 20
        _check_history(h[:st.history_len], ref.history)


@pytest.mark.parametrize("n", [96, 128])
def test_rbicgstab_true_residual_on_large_grids(gpu_lib, n):
    """On grids above 2^19 cells the residual kernel runs on more blocks
    than the BiCGStab passes (1024 against 512): the reported true residual
    must sum all of its partials.  FP64 porous medium with Schwarz-Jacobi,
    plain and with a recycle space (random U set up on the device);
    stats.rel_res_true against ||b - A x|| / ||b|| from the oracle's stencil."""
    krs = gpu_lib
    prob = W.porous_problem(n, extra=7)
    params = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
                  omega_global=6 / 7)
    d = Dev(krs, prob, "schwarz", params, m=1, k=8)
    rec = krs.Recycle(d.ctx, prob.n, 8, torch.float64)
    U0 = np.random.default_rng(5).standard_normal((prob.n, 8))
    rec.U[:8, :prob.n] = torch.from_numpy(U0.T.copy()).to(d.dev)
    rec.set_dim(8)
    krs.recycle_update(d.ctx, d.A, d.M, rec, d.ws)
    b = next(W.rhs_ar1(prob, 1, extra=7))
    for r in (None, rec):
        x = d.empty()
        rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, r, d.vec(b), x,
                                     krs.make_opts(tol=1e-8, max_matvecs=4000), d.ws)
        assert rc == krs.OK
        res = b - stencil.apply(prob.bands, prob.shape, prob.periodic, x.cpu().numpy())
        host = np.linalg.norm(res) / np.linalg.norm(b)
        assert abs(st.rel_res_true - host) <= 1e-4 * host, (n, st.rel_res_true, host)
        assert host <= 1.5e-8


@pytest.mark.parametrize("kd", [6, 62])
def test_recycle_update_cholqr(gpu_lib, kd):
    """Recycle-space setup: C = qr(A~ U).Q, U <- U R^-1: invariants and the oracle's range.
    kd = 62, the largest space: a 62 x 62 Gram matrix (256 4 x 4 tiles, one per
    thread, 32-row LDS staging in FP64).  Random U: the errors grow with the
    condition of A~ U, hence the looser bounds for the wide space."""
    krs = gpu_lib
    prob = W.grf_problem(16, extra=9)
    d = Dev(krs, prob, "jacobi", m=10, k=kd)
    _, Mi, op = oracle_ops(prob, "jacobi")
    U0 = np.random.default_rng(4).standard_normal((prob.n, kd))
    rec = krs.Recycle(d.ctx, prob.n, kd, torch.float64)
    rec.U[:kd, :prob.n] = torch.from_numpy(U0.T.copy()).to(d.dev)
    rec.set_dim(kd)
    krs.recycle_update(d.ctx, d.A, d.M, rec, d.ws)
    g = recycle_to_oracle(rec)
    o = K.Recycle(U0.copy(), np.zeros_like(U0))
    K.recycle_setup(op, o)
    AU = np.column_stack([op(g.U[:, i]) for i in range(kd)])
    wide = kd > 32
    assert np.linalg.norm(AU - g.C) / np.linalg.norm(g.C) <= (1e-11 if wide else 1e-12)
    assert np.linalg.norm(g.C.T @ g.C - np.eye(kd)) <= 1e-13
    assert scipy.linalg.subspace_angles(g.C, o.C).max() < (1e-9 if wide else 1e-10)
    assert scipy.linalg.subspace_angles(g.U, o.U).max() < (1e-9 if wide else 1e-10)


def test_hybrid_sequence(gpu_lib):
    """Hybrid: rGCROT for the first n_switch systems, rBiCGStab with the
    frozen space afterwards; each solve to the tolerance, and the recycled
    rBiCGStab systems need fewer matvecs than plain BiCGStab."""
    krs = gpu_lib
    prob = W.porous_problem(32, extra=11)
    params = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
                  omega_global=6 / 7)
    d = Dev(krs, prob, "schwarz", params, m=30, k=20)
    rec = krs.Recycle(d.ctx, prob.n, 20, torch.float64)
    bs = list(W.rhs_ar1(prob, 5, extra=11))
    A, Mi, op = oracle_ops(prob, "schwarz", params)
    orec = K.Recycle.empty(prob.n)
    for t, b in enumerate(bs):
        x = d.empty()
        rc, st = krs.hybrid_solve(d.ctx, d.A, d.M, rec, t, 3, d.vec(b), x,
                                  krs.make_opts(m=30, k=20, tol=1e-8), d.ws)
        ref = K.hybrid_step(t, 3, op, Mi, b, 30, 20, 1e-8, orec)
        assert rc == krs.OK
        assert (st.cycles > 0) == (t < 3)
        r = b - A(x.cpu().numpy())
        assert np.linalg.norm(r) <= 1.5e-8 * np.linalg.norm(b)
        assert abs(st.iterations - ref.iterations) <= 2
        assert rel(x.cpu().numpy(), ref.x) <= X_TOL
        if t == 4:
            xp = d.empty()
            rcp, stp = krs.rbicgstab_solve(d.ctx, d.A, d.M, None, d.vec(b), xp,
                                           krs.make_opts(tol=1e-8), d.ws)
            assert st.matvecs < stp.matvecs


def test_ir_fp32_inner_reaches_fp64_tolerance(gpu_lib):
    """FP32 stencil/preconditioner/projections inside FP64 refinement reach a
    1e-8 true residual; error against the FP64 oracle solution reported."""
    krs = gpu_lib
    prob = W.porous_problem(32, extra=12)
    params = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
                  omega_global=6 / 7)
    dev = torch.device("cuda:0")
    ctx = krs.Context(dev)
    b64 = torch.from_numpy(prob.bands).to(dev)
    b32 = b64.float()
    A64 = krs.Matrix(ctx, prob.shape, prob.periodic, b64)
    A32 = krs.Matrix(ctx, prob.shape, prob.periodic, b32)
    M32 = krs.Precond(ctx, A32, "schwarz", **params)
    rec = krs.Recycle(ctx, prob.n, 20, torch.float32)
    ws = torch.empty(krs.workspace_size(krs.SOLVER_IR, prob.n, 30, 20, torch.float32),
                     dtype=torch.uint8, device=dev)
    A, Mi, op = oracle_ops(prob, "schwarz", params)
    orec = K.Recycle.empty(prob.n)
    for t, b in enumerate(W.rhs_ar1(prob, 4, extra=12)):
        x = torch.empty(prob.n, dtype=torch.float64, device=dev)
        inner = krs.SOLVER_RGCROT if t < 2 else krs.SOLVER_RBICGSTAB
        rc, st = krs.ir_solve(ctx, A64, A32, M32, rec, torch.from_numpy(b).to(dev), x,
                              krs.make_opts(m=30, k=20, tol=1e-8, inner_solver=inner,
                                            inner_tol=1e-5), ws)
        assert rc == krs.OK, (t, rc, st.as_dict())
        xc = x.cpu().numpy()
        assert np.linalg.norm(b - A(xc)) <= 1e-8 * np.linalg.norm(b)
        ref = K.hybrid_step(t, 2, op, Mi, b, 30, 20, 1e-10, orec)
        err = rel(xc, ref.x)
        print(f"IR step {t}: outer {st.outer} inner its {st.iterations} |x-x64|/|x64| {err:.2e}")
        assert err <= 1e-4


def test_edge_cases(gpu_lib):
    krs = gpu_lib
    prob = W.grf_problem(8, extra=13)
    d = Dev(krs, prob, "jacobi", m=10, k=4)
    x = d.empty()
    rc, st = krs.gmres(d.ctx, d.A, d.M, d.vec(np.zeros(prob.n)), x, krs.make_opts(m=10), d.ws)
    assert rc == krs.OK and float(x.abs().max()) == 0.0
    b = W.random_vector(prob.n, 3)
    rc, st = krs.gmres(d.ctx, d.A, d.M, d.vec(b), x, krs.make_opts(m=10, tol=1e-14,
                                                                   max_matvecs=5), d.ws)
    assert rc == krs.NOT_CONVERGED and st.iterations == 5
    rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, None, d.vec(b), x,
                                 krs.make_opts(tol=1e-14, max_matvecs=4), d.ws)
    assert rc == krs.NOT_CONVERGED and st.iterations == 2
    rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, None, d.vec(np.full(prob.n, np.nan)), x,
                                 krs.make_opts(tol=1e-8), d.ws)
    assert rc == krs.DIVERGED
    with pytest.raises(krs.KrsError):
        krs.gmres(d.ctx, d.A, d.M, d.vec(b), x, krs.make_opts(m=0), d.ws)
    small = torch.empty(16, dtype=torch.uint8, device=d.dev)
    with pytest.raises(krs.KrsError):
        krs.gmres(d.ctx, d.A, d.M, d.vec(b), x, krs.make_opts(m=10), small)
    # b in range(C): rBiCGStab needs no iteration
    rec = krs.Recycle(d.ctx, prob.n, 4, torch.float64)
    rec.U[:4, :prob.n] = torch.from_numpy(np.random.default_rng(1).standard_normal((4, prob.n))).to(d.dev)
    rec.set_dim(4)
    krs.recycle_update(d.ctx, d.A, d.M, rec, d.ws)
    _, C = rec.views()
    bc = (C @ torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device=d.dev)).contiguous()
    rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec, bc, x, krs.make_opts(tol=1e-10), d.ws)
    assert rc == krs.OK and st.iterations == 0
    # arguments the kernels would read out of bounds are refused before any launch
    x0 = x.clone()
    with pytest.raises(ValueError, match="dtype"):
        krs.rbicgstab_solve(d.ctx, d.A, d.M, None, d.vec(b).float(), x, krs.make_opts(), d.ws)
    with pytest.raises(ValueError, match="values"):
        krs.gmres(d.ctx, d.A, d.M, d.vec(b), x[:-1], krs.make_opts(m=10), d.ws)
    with pytest.raises(ValueError, match="contiguous"):
        krs.rgcrot_solve(d.ctx, d.A, d.M, rec, d.vec(b), torch.zeros(2 * prob.n,
                         dtype=torch.float64, device=d.dev)[::2], krs.make_opts(m=10, k=4), d.ws)
    with pytest.raises(ValueError, match="is on"):
        krs.hybrid_solve(d.ctx, d.A, d.M, rec, 5, 2, torch.from_numpy(b), x,
                         krs.make_opts(m=10, k=4), d.ws)
    with pytest.raises(ValueError, match="dtype"):
        krs.ir_solve(d.ctx, d.A, d.A, None, None, d.vec(b).float(), x, krs.make_opts(), d.ws)
    assert torch.equal(x, x0)
    # rGCROT without updates still needs dim + m + 1 <= 64 columns per block pass
    wide = krs.Recycle(d.ctx, prob.n, 40, torch.float64)
    wide.U[:40, :prob.n] = torch.from_numpy(
        np.random.default_rng(2).standard_normal((40, prob.n))).to(d.dev)
    wide.set_dim(40)
    krs.recycle_update(d.ctx, d.A, d.M, wide, d.ws)
    with pytest.raises(krs.KrsError, match="64"):
        krs.rgcrot_solve(d.ctx, d.A, d.M, wide, d.vec(b), x,
                         krs.make_opts(m=30, k=4, update_recycle=False), d.ws)
    assert torch.equal(x, x0)


def test_hybrid_changing_matrix_and_switch_back(gpu_lib):
    """Sequence on two different 32^3 porous media (the matrix changes at
    system 5): the space is marked stale and re-formed from U before the
    next solve, the poor convergence that follows makes the next system run
    rGCROT (switch back, Sec. 2.4).  The solver chosen at every step, the
    re-forming, the iteration counts and x match the oracle."""
    krs = gpu_lib
    params = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
                  omega_global=6 / 7)
    p1 = W.porous_problem(32, extra=11)
    p2 = W.porous_problem(32, extra=12)
    d = Dev(krs, p1, "schwarz", params, m=30, k=20)
    rec = krs.Recycle(d.ctx, p1.n, 20, torch.float64)
    bs = list(W.rhs_ar1(p1, 9, extra=11))
    o1, o2 = oracle_ops(p1, "schwarz", params), oracle_ops(p2, "schwarz", params)
    orec, ost = K.Recycle.empty(p1.n), K.HybridState()
    names = {krs.SOLVER_RGCROT: "rgcrot", krs.SOLVER_RBICGSTAB: "rbicgstab"}
    seq = []
    for t, b in enumerate(bs):
        A, Mi, op = o1 if t < 5 else o2
        if t == 5:
            d.bands.copy_(torch.from_numpy(p2.bands).to(d.dev))
            d.M.refresh()
            rec.mark_stale()
            ost.stale = True
        x = d.empty()
        rc, st = krs.hybrid_solve(d.ctx, d.A, d.M, rec, t, 2, d.vec(b), x,
                                  krs.make_opts(m=30, k=20, tol=1e-8, switch_back=1.3), d.ws)
        ref = K.hybrid_step(t, 2, op, Mi, b, 30, 20, 1e-8, orec, switch_back=1.3, state=ost)
        assert rc == krs.OK and ref.status == K.CONVERGED
        assert names[st.solver] == ref.solver, (t, names[st.solver], ref.solver)
        assert bool(st.refreshed) == ref.refreshed
        r = b - A(x.cpu().numpy())
        assert np.linalg.norm(r) <= 1.5e-8 * np.linalg.norm(b)
        if ref.solver == "rgcrot":
            assert abs(st.iterations - ref.iterations) <= 2, (t, st.iterations, ref.iterations)
            assert rel(x.cpu().numpy(), ref.x) <= X_TOL
        else:
            # with the poorly matched space after the change BiCGStab converges
            # irregularly: the count must lie within 2 of the range of exits
            # the oracle takes under rounding-level perturbations, and x
            # within 3 times the oracle's own x-spread under them
            solve = lambda bb, opx: K.rbicgstab(opx, Mi, bb, 1e-8, orec)
            lo, hi, spread = _oracle_spread(solve, op, b, ref)
            assert lo - 2 <= st.iterations <= hi + 2, (t, st.iterations, ref.iterations, lo, hi)
            assert rel(x.cpu().numpy(), ref.x) <= max(X_TOL, 3 * spread), (t, spread)
        seq.append(ref.solver)
        # the oracle continues from the GPU's recycle space (step-wise parity)
        orec = recycle_to_oracle(rec)
    assert seq[:2] == ["rgcrot"] * 2 and seq[5] == "rbicgstab" and seq[6] == "rgcrot", seq


def test_hybrid_with_ssor_local_smoother(gpu_lib):
    """Hybrid sequence with the SSOR local smoother (Sec. 2.1 alternative):
    parity with the oracle using the same smoother, and fewer matvecs per
    recycled system than with damped Jacobi on the same sequence."""
    krs = gpu_lib
    prob = W.porous_problem(32, extra=11)
    bs = list(W.rhs_ar1(prob, 5, extra=11))
    counts = {}
    for smoother, w in (("jacobi", 6 / 7), ("ssor", 1.0)):
        params = dict(tile=8, overlap=1, local_sweeps=5, omega_local=w, global_sweeps=1,
                      omega_global=6 / 7, local_solver=smoother)
        d = Dev(krs, prob, "schwarz", params, m=30, k=20)
        rec = krs.Recycle(d.ctx, prob.n, 20, torch.float64)
        A, Mi, op = oracle_ops(prob, "schwarz", params)
        orec = K.Recycle.empty(prob.n)
        mv = 0
        for t, b in enumerate(bs):
            x = d.empty()
            rc, st = krs.hybrid_solve(d.ctx, d.A, d.M, rec, t, 2, d.vec(b), x,
                                      krs.make_opts(m=30, k=20, tol=1e-8), d.ws)
            ref = K.hybrid_step(t, 2, op, Mi, b, 30, 20, 1e-8, orec)
            assert rc == krs.OK and ref.status == K.CONVERGED
            r = b - A(x.cpu().numpy())
            assert np.linalg.norm(r) <= 1.5e-8 * np.linalg.norm(b)
            assert abs(st.iterations - ref.iterations) <= 2, (smoother, t)
            assert rel(x.cpu().numpy(), ref.x) <= X_TOL
            orec = recycle_to_oracle(rec)
            if t >= 2:
                mv += st.matvecs
        counts[smoother] = mv
    assert counts["ssor"] < counts["jacobi"], counts


def test_full_size_porous256_fp32_ir_properties(gpu_lib):
    """The benchmark's 256^3 system in its launch configuration (FP32 inner
    solves in FP64 refinement, rGCROT(30,20) then rBiCGStab): the FP64 true
    residual recomputed by the oracle's stencil meets 1e-8, the recycle space
    is orthonormal to FP32 accuracy, and A~ U = C holds column by column to
    the accuracy FP32 arithmetic allows.  The columns of U have norms up to
    ~4e4 (A~ u_c = c_c with ||c_c|| = 1 for the harmonic Ritz vectors of the
    smallest eigenvalues), so every FP32 evaluation involving u_c carries an
    error of order u32 ||u_c|| ||A~||: the bar is 16 u32 ||u_c|| per column
    (||A~|| <= 2 for this preconditioned operator; the products that form U
    at each recycle update accumulate in FP64 and are rounded once).
    A~ is applied in FP64 on the device to the FP32-rounded bands; one column
    of it is checked against the oracle's stencil and preconditioner."""
    krs = gpu_lib
    prob = W.porous_problem(256, seed_cfg=4)
    params = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
                  omega_global=6 / 7)
    dev = torch.device("cuda:0")
    ctx = krs.Context(dev)
    b64 = torch.from_numpy(prob.bands).to(dev)
    b32 = b64.float()
    A64 = krs.Matrix(ctx, prob.shape, prob.periodic, b64)
    A32 = krs.Matrix(ctx, prob.shape, prob.periodic, b32)
    M32 = krs.Precond(ctx, A32, "schwarz", **params)
    rec = krs.Recycle(ctx, prob.n, 20, torch.float32)
    ws = torch.empty(krs.workspace_size(krs.SOLVER_IR, prob.n, 30, 20, torch.float32),
                     dtype=torch.uint8, device=dev)
    gen = W.rhs_ar1(prob, 2, seed_cfg=4)
    for t in range(2):
        b = next(gen)
        x = torch.zeros(prob.n, dtype=torch.float64, device=dev)
        o = krs.make_opts(m=30, k=20, tol=1e-8, max_matvecs=4000,
                          inner_solver=krs.SOLVER_RGCROT if t == 0 else krs.SOLVER_RBICGSTAB)
        rc, st = krs.ir_solve(ctx, A64, A32, M32, rec, torch.from_numpy(b).to(dev), x, o, ws)
        assert rc == krs.OK
        r = b - stencil.apply(prob.bands, prob.shape, prob.periodic, x.cpu().numpy())
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)
    del ws
    U, C = rec.views()
    Cd = C.double()
    G = Cd.T @ Cd
    assert float((G - torch.eye(G.shape[0], device=dev, dtype=torch.float64)).abs().max()) <= 1e-5
    # FP64 operator on the FP32-rounded bands (the operator the FP32 path represents)
    b32d = b32.double()
    A64r = krs.Matrix(ctx, prob.shape, prob.periodic, b32d)
    M64r = krs.Precond(ctx, A64r, "schwarz", **params)
    w64 = torch.empty(prob.n, dtype=torch.float64, device=dev)
    t64 = torch.empty_like(w64)
    u32 = 2.0 ** -24
    worst = 0.0
    for c in range(rec.dim):
        u = U[:, c].double().contiguous()
        krs.operator_apply(ctx, A64r, M64r, u, w64, t64)
        cc = C[:, c].double()
        err = float((w64 - cc).norm() / cc.norm())
        un = float(u.norm())
        worst = max(worst, err / (u32 * un))
        assert err <= 16 * u32 * un, (c, err, un)
        if c == 3:
            # the device FP64 operator against the oracle's on this column:
            # both round at u64 relative to |A~| |u|, while ||A~ u|| = 1 and
            # ||u|| is large, so they agree to about u64 ||u|| ||A~||
            uh = u.cpu().numpy()
            z = precond.schwarz_jacobi(b32d.cpu().numpy(), prob.shape, prob.periodic, uh,
                                       **params)
            au = stencil.apply(b32d.cpu().numpy(), prob.shape, prob.periodic, z)
            assert rel(w64.cpu().numpy(), au) <= 64 * 2.0 ** -53 * un, (un,)
    print(f"[A~U=C] worst column: ||A~u - c|| = {worst:.2f} u32 ||u||")


@pytest.mark.parametrize("pc", ["jacobi", "schwarz"])
def test_left_preconditioned_gmres_and_rgcrot(gpu_lib, pc):
    """Paper-literal left preconditioning (Sec. 2.1) for GMRES(m) and
    rGCROT(m,k): the oracle's solvers on M^-1 A x = M^-1 b (no final M^-1);
    history, counts and x match, the stop is on the preconditioned residual,
    and the reported true residual is the unpreconditioned one."""
    krs = gpu_lib
    prob = W.grf_problem(24, extra=71)
    params = dict(tile=8) if pc == "schwarz" else None
    d = Dev(krs, prob, pc, params, m=20, k=10)
    A, Mi, _ = oracle_ops(prob, pc, params)
    opL = lambda v: Mi(A(v))
    ident = lambda v: np.array(v, copy=True)
    bs = W.rhs_perturbed(prob, 3, extra=71)
    left = krs.FLAG_LEFT_PRECOND
    # GMRES(20)
    b = bs[0]
    h = _hist()
    x = d.empty()
    rc, st = krs.gmres(d.ctx, d.A, d.M, d.vec(b), x,
                       krs.make_opts(m=20, tol=1e-8, history=h, flags=left), d.ws)
    ref = K.gmres(opL, ident, Mi(b), 20, 1e-8)
    assert rc == krs.OK and ref.status == K.CONVERGED
    _check_history(h[:st.history_len], ref.history)
    assert abs(st.iterations - ref.iterations) <= 2
    xg = x.cpu().numpy()
    assert rel(xg, ref.x) <= X_TOL
    assert st.rel_res_true == pytest.approx(np.linalg.norm(b - A(xg)) / np.linalg.norm(b),
                                            rel=1e-6)
    assert np.linalg.norm(Mi(b - A(xg))) <= 1.5e-8 * np.linalg.norm(Mi(b))
    # rGCROT(20,10) over three systems, the oracle stepping from the GPU's space
    rec = krs.Recycle(d.ctx, prob.n, 10, torch.float64)
    for t in range(3):
        b = bs[t]
        orec = recycle_to_oracle(rec)
        h = _hist()
        x = d.empty()
        rc, st = krs.rgcrot_solve(d.ctx, d.A, d.M, rec, d.vec(b), x,
                                  krs.make_opts(m=20, k=10, tol=1e-8, history=h, flags=left),
                                  d.ws)
        ref = K.rgcrot(opL, ident, Mi(b), 20, 10, 1e-8, orec)
        assert rc == krs.OK and ref.status == K.CONVERGED, t
        _check_history(h[:st.history_len], ref.history)
        assert abs(st.iterations - ref.iterations) <= 2, (t, st.iterations, ref.iterations)
        assert rel(x.cpu().numpy(), ref.x) <= X_TOL
    # the space belongs to M^-1 A
    g = recycle_to_oracle(rec)
    AU = np.column_stack([opL(g.U[:, i]) for i in range(g.dim)])
    assert np.linalg.norm(AU - g.C) <= 1e-10 * np.linalg.norm(g.C)
    # drivers that are right-preconditioned refuse the flag
    with pytest.raises(krs.KrsError):
        krs.rbicgstab_solve(d.ctx, d.A, d.M, None, d.vec(b), x,
                            krs.make_opts(tol=1e-8, flags=left), d.ws)


def test_rgcrot_large_recycle_space(gpu_lib):
    """rGCROT(10,40), the porous-media parameters of Sec. 3, stepwise against
    the oracle; rBiCGStab with the resulting 40-dimensional space; the limit
    k + m + 1 = 64 (one block pass over [C, V]) and the rejected sizes."""
    krs = gpu_lib
    prob = W.porous_problem(24, extra=71)
    bs = list(W.rhs_ar1(prob, 4, extra=71))
    params = dict(SMALL_SCHWARZ)
    d, rec, orec, op, out = _rgcrot_sequence(krs, prob, "schwarz", params, 10, 40, 3, bs)
    for t, (rc, st, h, x, ref) in enumerate(out):
        assert rc == krs.OK and ref.status == K.CONVERGED, t
        _check_history(h, ref.history)
        assert abs(st.iterations - ref.iterations) <= 2, (t, st.iterations, ref.iterations)
        _check_solution(prob, x, ref.x)
    assert rec.dim == 40
    g = recycle_to_oracle(rec)
    AU = np.column_stack([op(g.U[:, i]) for i in range(g.dim)])
    assert np.linalg.norm(AU - g.C) / np.linalg.norm(g.C) <= 1e-10
    assert np.linalg.norm(g.C.T @ g.C - np.eye(g.dim)) <= 1e-12
    _, Mi, _ = oracle_ops(prob, "schwarz", params)
    h = _hist()
    x = d.empty()
    rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec, d.vec(bs[3]), x,
                                 krs.make_opts(tol=1e-8, history=h), d.ws)
    ref = K.rbicgstab(op, Mi, bs[3], 1e-8, g)
    assert rc == krs.OK and ref.status == K.CONVERGED
    _check_history(h[:st.history_len], ref.history)
    assert abs(st.iterations - ref.iterations) <= 2
    _check_solution(prob, x.cpu().numpy(), ref.x)
    # k + m + 1 = 64: the widest block pass
    d2, rec2, _, _, out2 = _rgcrot_sequence(krs, prob, "schwarz", params, 10, 53, 2, bs)
    for rc, st, h, x, ref in out2:
        assert rc == krs.OK and ref.status == K.CONVERGED
        _check_history(h, ref.history)
        assert abs(st.iterations - ref.iterations) <= 2
        _check_solution(prob, x, ref.x)
    with pytest.raises(krs.KrsError):
        krs.rgcrot_solve(d2.ctx, d2.A, d2.M, rec2, d2.vec(bs[0]), d2.empty(),
                         krs.make_opts(m=11, k=53, tol=1e-8), d2.ws)
    with pytest.raises(krs.KrsError):
        krs.Recycle(d2.ctx, prob.n, 63, torch.float64)


@pytest.mark.parametrize("kind,m,k,par", [
    ("grf", 20, 10, (5, 10, 1)),       # Jacobi: cuts and one selected vector per cycle
    ("porous", 30, 20, (10, 15, 2)),   # Schwarz, the channel parameters of Sec. 3 with p = 2
    ("channel", 10, 40, (30, 5, 2)),   # the porous-media parameters rGCROT(10,40) of Sec. 3
    ("grf", 8, 2, (1, 4, 2)),          # k = 2 < 1 + p: the selection is capped at k - 1
])
def test_rgcrot_gcrot_rule_matches_oracle(gpu_lib, kind, m, k, par):
    """The GCROT recycle-space rule, stepwise against the oracle: history
    within 1e-10 over 20 steps, counts within 2, x within 1e-8; after the
    last system the same outer space (subspace angles), A~ U = C, C^T C = I."""
    krs = gpu_lib
    gp = K.GcrotParams(*par)
    if kind == "grf":
        prob, pc, params = W.grf_problem(16, extra=81), "jacobi", None
        bs = W.rhs_perturbed(prob, 4, extra=81)
    else:
        prob = W.porous_problem(24, extra=82) if kind == "porous" else W.channel_problem(24)
        pc, params = "schwarz", dict(SMALL_SCHWARZ)
        bs = list(W.rhs_ar1(prob, 4, extra=82))
    d, rec, orec, op, out = _rgcrot_sequence(krs, prob, pc, params, m, k, 4, bs, gcrot=gp)
    for t, (rc, st, h, x, ref) in enumerate(out):
        assert rc == krs.OK and ref.status == K.CONVERGED, t
        assert st.eig_ties == 0 and ref.eig_ties == 0
        _check_history(h, ref.history)
        assert abs(st.iterations - ref.iterations) <= 2, (t, st.iterations, ref.iterations)
        _check_solution(prob, x, ref.x)
    g = recycle_to_oracle(rec)
    assert g.dim == orec.dim >= 1
    assert scipy.linalg.subspace_angles(g.C, orec.C).max() < 1e-6
    AU = np.column_stack([op(g.U[:, i]) for i in range(g.dim)])
    assert np.linalg.norm(AU - g.C) / np.linalg.norm(g.C) <= 1e-10
    assert np.linalg.norm(g.C.T @ g.C - np.eye(g.dim)) <= 1e-12


def test_rgcrot_gcrot_rule_rejected_where_unsupported(gpu_lib):
    krs = gpu_lib
    prob = W.grf_problem(8, extra=83)
    d = Dev(krs, prob, "jacobi", m=10, k=6)
    dt = Dev(krs, prob, "jacobi", m=10, k=6, solver=krs.SOLVER_RGCROT_T, ctx=d.ctx)
    assert dt.wsb > d.wsb
    rec = krs.Recycle(d.ctx, prob.n, 6, torch.float64)
    b = d.vec(W.random_vector(prob.n, 2))
    o = krs.make_opts(m=10, k=6, recycle_rule=krs.RECYCLE_GCROT)
    with pytest.raises(krs.KrsError, match="workspace"):   # no room for the selection space
        krs.rgcrot_solve(d.ctx, d.A, d.M, rec, b, d.empty(), o, d.ws)
    with pytest.raises(krs.KrsError, match="harmonic"):
        krs.hybrid_solve(dt.ctx, dt.A, dt.M, rec, 0, 2, b, dt.empty(), o, dt.ws)
    for bad in (dict(gcrot_p=5), dict(gcrot_s=11), dict(gcrot_kt=6)):
        with pytest.raises(krs.KrsError, match="gcrot"):
            krs.rgcrot_solve(dt.ctx, dt.A, dt.M, rec, b, dt.empty(),
                             krs.make_opts(m=10, k=6, recycle_rule=krs.RECYCLE_GCROT, **bad),
                             dt.ws)
    rc, st = krs.rgcrot_solve(dt.ctx, dt.A, dt.M, rec, b, dt.empty(),
                              krs.make_opts(m=10, k=6, recycle_rule=krs.RECYCLE_GCROT), dt.ws)
    assert rc == krs.OK and 1 <= rec.dim <= 6


def test_19pt_operator_solvers_match_oracle(gpu_lib):
    """Sheared-grid 19-point operator (Schwarz local solves over the 18
    neighbours): rGCROT stepwise against the oracle, rBiCGStab with the
    resulting space, and FP32 inner solves in FP64 refinement to a 1e-8 true
    residual."""
    krs = gpu_lib
    prob = W.skewed_problem(24, extra=91)
    params = dict(SMALL_SCHWARZ)
    bs = list(W.rhs_ar1(prob, 4, extra=91))
    d, rec, orec, op, out = _rgcrot_sequence(krs, prob, "schwarz", params, 20, 10, 3, bs)
    for t, (rc, st, h, x, ref) in enumerate(out):
        assert rc == krs.OK and ref.status == K.CONVERGED, t
        _check_history(h, ref.history)
        assert abs(st.iterations - ref.iterations) <= 2, (t, st.iterations, ref.iterations)
        _check_solution(prob, x, ref.x)
    _, Mi, _ = oracle_ops(prob, "schwarz", params)
    g = recycle_to_oracle(rec)
    h = _hist()
    x = d.empty()
    rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec, d.vec(bs[3]), x,
                                 krs.make_opts(tol=1e-8, history=h), d.ws)
    ref = K.rbicgstab(op, Mi, bs[3], 1e-8, g)
    assert rc == krs.OK and ref.status == K.CONVERGED
    _check_history(h[:st.history_len], ref.history)
    assert abs(st.iterations - ref.iterations) <= 2
    _check_solution(prob, x.cpu().numpy(), ref.x)
    # FP32 inner solves in FP64 refinement
    dev = torch.device("cuda:0")
    ctx = d.ctx
    b64 = torch.from_numpy(prob.bands).to(dev)
    b32 = b64.float()
    A64 = krs.Matrix(ctx, prob.shape, prob.periodic, b64)
    A32 = krs.Matrix(ctx, prob.shape, prob.periodic, b32)
    M32 = krs.Precond(ctx, A32, "schwarz", **params)
    rec32 = krs.Recycle(ctx, prob.n, 10, torch.float32)
    ws = torch.empty(krs.workspace_size(krs.SOLVER_IR, prob.n, 20, 10, torch.float32),
                     dtype=torch.uint8, device=dev)
    A = lambda v: stencil.apply(prob.bands, prob.shape, prob.periodic, v)
    for t, b in enumerate(bs):
        x = torch.empty(prob.n, dtype=torch.float64, device=dev)
        inner = krs.SOLVER_RGCROT if t < 2 else krs.SOLVER_RBICGSTAB
        rc, st = krs.ir_solve(ctx, A64, A32, M32, rec32, torch.from_numpy(b).to(dev), x,
                              krs.make_opts(m=20, k=10, tol=1e-8, inner_solver=inner,
                                            inner_tol=1e-5), ws)
        assert rc == krs.OK, (t, rc)
        assert np.linalg.norm(b - A(x.cpu().numpy())) <= 1e-8 * np.linalg.norm(b)


def _shifted_grf(n):
    """GRF operator with its diagonal scaled by 1.3 (nonsingular, strongly
    diagonally dominant): BiCGStab converges in under 20 iterations, so the
    oracle finishes in seconds at sizes with hundreds of per-block partials."""
    import dataclasses
    p0 = W.grf_problem(n, extra=5)
    bands = p0.bands.copy()
    bands[0] = 1.3 * bands[0]
    return dataclasses.replace(p0, bands=bands, singular=False)


@pytest.mark.parametrize("n,kd,dtype", [(66, 40, torch.float64), (66, 62, torch.float64),
                                        (20, 62, torch.float64), (66, 40, torch.float32)])
def test_rbicgstab_wide_space_finishing_paths(gpu_lib, n, kd, dtype):
    """rBiCGStab with a wide recycle space (random U, set up on the device):
    at 66^3 the passes leave 281 per-block partials, so the finishing
    reductions of the alpha and omega steps take the all-threads path over
    three or four 16-column groups (kd + 1, kd + 2 columns); at 20^3 (8
    partials) the one-group path with up to 64 columns.  FP64: history and
    iteration count against the oracle run with the device's space; FP32:
    count within 2 and the FP64 true residual at the FP32 tolerance."""
    krs = gpu_lib
    prob = _shifted_grf(n)
    d = Dev(krs, prob, "jacobi", m=1, k=kd, dtype=dtype)
    _, Mi, op = oracle_ops(prob, "jacobi")
    U0 = np.random.default_rng(4).standard_normal((prob.n, kd))
    rec = krs.Recycle(d.ctx, prob.n, kd, dtype)
    rec.U[:kd, :prob.n] = torch.from_numpy(U0.T.copy()).to(d.dev, dtype)
    rec.set_dim(kd)
    krs.recycle_update(d.ctx, d.A, d.M, rec, d.ws)
    g = recycle_to_oracle(rec)
    b = W.rhs_perturbed(prob, 1)[0]
    tol = 1e-8 if dtype == torch.float64 else 1e-5
    h = _hist()
    x = d.empty()
    rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec, d.vec(b), x,
                                 krs.make_opts(tol=tol, history=h), d.ws)
    ref = K.rbicgstab(op, Mi, b, tol, g)
    assert rc == krs.OK and ref.status == K.CONVERGED
    assert abs(st.iterations - ref.iterations) <= 2, (st.iterations, ref.iterations)
    xs = x.double().cpu().numpy()
    res = b - stencil.apply(prob.bands, prob.shape, prob.periodic, xs)
    assert np.linalg.norm(res) <= 2 * tol * np.linalg.norm(b)
    if dtype == torch.float64:
        _check_history(h[:st.history_len], ref.history)
        assert rel(xs, ref.x) <= 1e-6
