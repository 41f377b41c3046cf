"""Pins of the oracle Krylov solvers against dense linear algebra, closed
forms, brute-force least squares and invariants of the method."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg

import workloads as W
from oracle import krylov as K
from oracle import precond, stencil
from tests import _fvm


def _ops(prob, pc="jacobi", params=None):
    A = lambda v: stencil.apply(prob.bands, prob.shape, prob.periodic, v)
    Mi = precond.make(prob.bands, prob.shape, prob.periodic, pc, params)
    return A, Mi, (lambda v: A(Mi(v)))


def _dense(op, n):
    return np.column_stack([op(e) for e in np.eye(n)])


SMALL = dict(tile=4, overlap=1)


# ---------------------------------------------------------------------------
# dense LU
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("pc", ["jacobi", "schwarz"])
def test_solvers_match_dense_lu(pc):
    prob = W.grf_problem(8, extra=1)
    A, Mi, op = _ops(prob, pc, SMALL if pc == "schwarz" else None)
    Ad = _dense(A, prob.n)
    b = W.rhs_perturbed(prob, 2, extra=1)[1]
    xs = np.linalg.solve(Ad, b)
    cond = np.linalg.cond(Ad)
    tol = 1e-11
    rec = K.Recycle.empty(prob.n)
    for res in (K.gmres(op, Mi, b, 20, tol),
                K.rgcrot(op, Mi, b, 20, 8, tol, rec),
                K.rgcrot(op, Mi, b, 20, 8, tol, rec),       # with a recycle space
                K.rbicgstab(op, Mi, b, tol, None),
                K.rbicgstab(op, Mi, b, tol, rec)):
        assert res.status == K.CONVERGED
        err = np.linalg.norm(res.x - xs) / np.linalg.norm(xs)
        assert err <= 10 * cond * tol
        assert np.linalg.norm(b - Ad @ res.x) <= 1.5 * tol * np.linalg.norm(b)


# ---------------------------------------------------------------------------
# GMRES
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [4, 8])
def test_unrestarted_gmres_converges_within_n_steps(n):
    prob = W.grf_problem(n, extra=2)
    _, Mi, op = _ops(prob)
    b = W.random_vector(prob.n, 1)
    res = K.gmres(op, Mi, b, prob.n, 1e-10)
    assert res.status == K.CONVERGED
    assert res.iterations <= prob.n
    h = np.array(res.history)
    assert np.all(np.diff(h) <= 1e-14)                       # monotone


def _krylov_lstsq_residuals(op, r0, jmax, C=None):
    """min over c of ||r0 - op(K c)|| for K = explicitly orthonormalised
    Krylov basis of op_C = (I - C C^T) op; built from operator powers."""
    proj = (lambda v: v - C @ (C.T @ v)) if C is not None else (lambda v: v)
    cols = [r0 / np.linalg.norm(r0)]
    out = []
    for j in range(1, jmax + 1):
        Q, _ = np.linalg.qr(np.column_stack(cols))
        AQ = np.column_stack([proj(op(Q[:, i])) for i in range(j)])
        c = np.linalg.lstsq(AQ, r0, rcond=None)[0]
        out.append(np.linalg.norm(r0 - AQ @ c))
        w = proj(op(cols[-1]))
        cols.append(w / np.linalg.norm(w))
    return np.array(out)


def test_gmres_iterates_are_krylov_least_squares():
    prob = W.grf_problem(8, extra=3)
    _, Mi, op = _ops(prob)
    b = W.random_vector(prob.n, 2)
    res = K.gmres(op, Mi, b, 30, 1e-12, max_its=10)
    ref = _krylov_lstsq_residuals(op, b, 10) / np.linalg.norm(b)
    assert np.allclose(res.history[:10], ref, rtol=1e-9, atol=0)


def test_mgs_and_cgs2_agree_early():
    prob = W.grf_problem(8, extra=3)
    _, Mi, op = _ops(prob)
    b = W.random_vector(prob.n, 3)
    a = K.gmres(op, Mi, b, 20, 1e-12, max_its=20, orth="mgs")
    c = K.gmres(op, Mi, b, 20, 1e-12, max_its=20, orth="cgs2")
    assert np.allclose(a.history, c.history, rtol=1e-10, atol=0)


# ---------------------------------------------------------------------------
# rGCROT
# ---------------------------------------------------------------------------

def test_rgcrot_without_recycling_is_gmres():
    prob = W.grf_problem(8, extra=4)
    _, Mi, op = _ops(prob)
    b = W.random_vector(prob.n, 4)
    g = K.gmres(op, Mi, b, 10, 1e-10)
    r = K.rgcrot(op, Mi, b, 10, 5, 1e-10, K.Recycle.empty(prob.n), update=False)
    assert g.iterations == r.iterations
    assert np.allclose(g.history, r.history, rtol=1e-12, atol=0)
    assert np.allclose(g.x, r.x, rtol=0, atol=1e-12 * np.abs(g.x).max())


def _some_recycle_space(op, n, k, seed):
    U = np.random.default_rng(seed).standard_normal((n, k))
    rec = K.Recycle(U, np.zeros((n, k)))
    K.recycle_setup(op, rec)
    return rec


def test_rgcrot_cycle_minimises_over_recycle_plus_krylov():
    """One cycle of j steps gives the minimum residual over
    range(U) + K_j((I - C C^T) A~, (I - C C^T) b): checks z = -B y and the
    sign of the U-term in the solution update."""
    prob = W.grf_problem(8, extra=5)
    _, Mi, op = _ops(prob)
    b = W.random_vector(prob.n, 5)
    rec = _some_recycle_space(op, prob.n, 6, 1)
    for j in (1, 4, 9):
        traces = []
        res = K.rgcrot(op, Mi, b, j, 6, 1e-14, K.Recycle(rec.U.copy(), rec.C.copy()),
                       update=False, max_its=j, trace=traces.append)
        # brute force: min ||b - A~ [U, Kr] c||
        r0 = b - rec.C @ (rec.C.T @ b)
        cols = [r0 / np.linalg.norm(r0)]
        for _ in range(j - 1):
            w = op(cols[-1])
            w = w - rec.C @ (rec.C.T @ w)
            cols.append(w / np.linalg.norm(w))
        S = np.column_stack([rec.U] + [np.linalg.qr(np.column_stack(cols))[0]])
        AS = np.column_stack([op(S[:, i]) for i in range(S.shape[1])])
        c = np.linalg.lstsq(AS, b, rcond=None)[0]
        best = np.linalg.norm(b - AS @ c)
        true = np.linalg.norm(b - op(res.y))
        assert abs(true - best) <= 1e-9 * best
        assert res.history[-1] * np.linalg.norm(b) == pytest.approx(best, rel=1e-8)
        # the sign printed in the algorithm's U-term (x - U z = x + U B y) does worse
        tr = traces[0]
        rho0 = np.linalg.norm(r0)
        e1 = np.zeros(j + 1)
        e1[0] = rho0
        y = np.linalg.lstsq(tr["H"], e1, rcond=None)[0]
        wrong = tr["y_acc"] + 2.0 * rec.U @ (tr["B"] @ y)
        assert np.linalg.norm(b - op(wrong)) > 1.01 * best


def test_rgcrot_invariants_and_augmented_arnoldi():
    prob = W.grf_problem(8, extra=6)
    _, Mi, op = _ops(prob)
    rec = K.Recycle.empty(prob.n)
    traces = []
    for t, b in enumerate(W.rhs_perturbed(prob, 3, extra=6)):
        K.rgcrot(op, Mi, b, 12, 6, 1e-10, rec, trace=traces.append)
        AU = np.column_stack([op(rec.U[:, i]) for i in range(rec.dim)])
        assert np.linalg.norm(AU - rec.C) <= 1e-12 * np.linalg.norm(rec.C) * 10
        assert np.linalg.norm(rec.C.T @ rec.C - np.eye(rec.dim)) <= 1e-12
    for tr in traces:
        V, H, B, C = tr["V"], tr["H"], tr["B"], tr["C"]
        j = H.shape[1]
        AV = np.column_stack([op(V[:, i]) for i in range(j)])
        rel = np.linalg.norm(AV - C @ B - V @ H) / np.linalg.norm(AV)
        assert rel <= 1e-12
        assert np.linalg.norm(C.T @ V) <= 1e-12
        assert np.linalg.norm(V.T @ V - np.eye(j + 1)) <= 1e-12


def test_residual_orthogonal_to_recycle_space():
    prob = W.grf_problem(8, extra=7)
    _, Mi, op = _ops(prob)
    rec = K.Recycle.empty(prob.n)
    bs = W.rhs_perturbed(prob, 3, extra=7)
    for b in bs:
        traces = []
        K.rgcrot(op, Mi, b, 10, 6, 1e-10, rec, trace=traces.append)
        for tr in traces:
            if tr["C"].shape[1]:
                # r_true after the cycle is orthogonal to the old C (LS optimality)
                r = tr["r"]
                assert np.linalg.norm(tr["C"].T @ r) <= 1e-9 * np.linalg.norm(r) + 1e-14 * np.linalg.norm(b)


def test_exact_deflation_keeps_invariant_subspace():
    """U = eigenvectors of the k smallest eigenvalues of a symmetric operator
    (closed form): the harmonic Ritz update keeps exactly that space."""
    shape = (12, 7, 5)
    bc = {'x': ('dirichlet', 'dirichlet'), 'y': ('neumann', 'neumann'),
          'z': ('neumann', 'neumann')}
    prob = W.unit_laplacian(shape, bc)
    A, _, _ = _ops(prob, "none")
    Mi = lambda v: v.copy()
    modes = []
    for px in _fvm.mode_range(bc['x'], 12):
        for py in _fvm.mode_range(bc['y'], 7):
            for pz in _fvm.mode_range(bc['z'], 5):
                u, lam = _fvm.mode_3d(bc, shape, (px, py, pz))
                modes.append((lam, u / np.linalg.norm(u)))
    modes.sort(key=lambda t: t[0])
    k = 6
    lams = np.array([m[0] for m in modes])
    assert lams[k] - lams[k - 1] > 1e-3                         # gap at the cut
    Uex = np.column_stack([m[1] for m in modes[:k]])
    rec = K.Recycle(Uex.copy(), np.zeros_like(Uex))
    K.recycle_setup(A, rec)
    b = W.random_vector(prob.n, 8)
    K.rgcrot(A, Mi, b, 15, k, 1e-14, rec, update=True, max_its=15)
    ang = scipy.linalg.subspace_angles(rec.U, Uex)
    assert ang.max() < 1e-8
    # deflation helps: fewer steps than GMRES to reach 1e-8
    g = K.gmres(A, Mi, b, 200, 1e-8)
    d = K.rgcrot(A, Mi, b, 200, k, 1e-8, rec, update=False)
    assert d.iterations < g.iterations


def test_harmonic_ritz_standard_form_when_no_recycle_space():
    """kc = 0: G^T G z = theta G^T F z reduces to
    (H + h^2 H^-T e_j e_j^T) z = theta z (the GMRES-DR form)."""
    prob = W.grf_problem(8, extra=8)
    _, Mi, op = _ops(prob)
    traces = []
    K.rgcrot(op, Mi, W.random_vector(prob.n, 9), 10, 4, 1e-14, K.Recycle.empty(prob.n),
             update=False, max_its=10, trace=traces.append)
    V, Hb = traces[0]["V"], traces[0]["H"]
    j = Hb.shape[1]
    F = V.T @ V[:, :j]
    theta, Z = K.harmonic_ritz_pairs(Hb, F)
    H = Hb[:j, :]
    e = np.zeros(j)
    e[-1] = 1
    Mstd = H + Hb[j, j - 1] ** 2 * np.linalg.solve(H.T, np.outer(e, e))
    ref = np.linalg.eigvals(Mstd)
    assert np.allclose(np.sort_complex(theta), np.sort_complex(ref), rtol=1e-9)
    # generalized eigen residual
    Ga, Gb = Hb.T @ Hb, Hb.T @ F
    for i in range(j):
        res = Ga @ Z[:, i] - theta[i] * (Gb @ Z[:, i])
        assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(Ga) * np.linalg.norm(Z[:, i])


def _pair_at_cut_case(seed):
    """A synthetic cycle with kc = 0 (random orthonormal V_{j+1}, random
    upper Hessenberg Hbar) whose GMRES-DR matrix H + h^2 H^-T e_j e_j^T has
    a complex-conjugate pair, well separated in |theta| from its neighbours,
    at sorted positions i, i+1 with i >= 2.  Eigen-decomposition by
    numpy.linalg.eig of that standard matrix (the oracle solves the
    generalized pencil with QZ).  Returns (V, Hbar, eigenvalues and
    eigenvectors sorted by |theta|, i) or None."""
    rng = np.random.default_rng(seed)
    j, n = 9, 60
    Hb = np.triu(rng.standard_normal((j + 1, j)), -1)
    V = np.linalg.qr(rng.standard_normal((n, j + 1)))[0]
    H = Hb[:j, :]
    e = np.zeros(j)
    e[-1] = 1.0
    T = H + Hb[j, j - 1] ** 2 * np.linalg.solve(H.T, np.outer(e, e))
    ev, EV = np.linalg.eig(T)
    order = np.argsort(np.abs(ev))
    ev, EV = ev[order], EV[:, order]
    mag = np.abs(ev)
    if np.min(np.diff(mag)[np.abs(np.diff(mag)) > 1e-12] / mag[1:][np.abs(np.diff(mag)) > 1e-12],
              initial=1.0) < 1e-3:
        return None                               # near-ties other than a pair
    for i in range(2, j - 1):
        if abs(ev[i].imag) > 1e-3 * mag[i] and np.isclose(ev[i + 1], np.conj(ev[i])):
            pairs_before = sum(1 for q in range(i) if abs(ev[q].imag) > 0)
            if pairs_before % 2 == 0:            # no pair split before position i
                return V, Hb, ev, EV, i
    return None


def _real_basis(ev, EV, count):
    """Real basis of the eigenvectors of the first `count` sorted values
    (a complex pair as the real and imaginary part of one member)."""
    cols, q = [], 0
    while q < count:
        if abs(ev[q].imag) > 0:
            cols += [EV[:, q].real, EV[:, q].imag]
            q += 2
        else:
            cols.append(EV[:, q].real)
            q += 1
    return np.column_stack(cols)


def _pair_cut_cases():
    out = []
    for seed in range(200):
        c = _pair_at_cut_case(seed)
        if c is not None:
            out.append(c)
        if len(out) == 3:
            return out
    raise AssertionError("no synthetic cycle with a well separated pair at the cut")


def _check_pair_cut(cases):
    """For each case: k = i + 1 puts the cut between the pair's members,
    k = i + 2 keeps the pair.  The oracle's update must keep exactly k - 1
    (resp. k) columns spanning V_j times the real invariant subspace of the
    GMRES-DR matrix for the values before the cut (principal angles
    < 1e-8).  Returns a list of failure descriptions (empty: pinned)."""
    fails = []
    for V, Hb, ev, EV, i in cases:
        j = Hb.shape[1]
        for k, want in ((i + 1, i), (i + 2, i + 2)):
            rec = K.Recycle.empty(V.shape[0])
            K.harmonic_ritz_update(rec, V, Hb, np.zeros((0, j)), k)
            if rec.dim != want:
                fails.append(("columns", k, rec.dim, want))
                continue
            expect = V[:, :j] @ _real_basis(ev, EV, want)
            ang = scipy.linalg.subspace_angles(rec.U, expect).max()
            if not ang < 1e-8:
                fails.append(("angle", k, ang))
    return fails


def test_harmonic_ritz_cut_never_splits_a_conjugate_pair():
    """The harmonic Ritz selection at a cycle end of Alg. 3 (GCRODR rule):
    a complex-conjugate pair straddling the k-th smallest |theta| is left
    out (k - 1 columns), a pair inside the first k is kept as the real and
    imaginary parts of its eigenvector; checked against the eigenvectors of
    the standard GMRES-DR matrix from numpy.linalg.eig."""
    assert _check_pair_cut(_pair_cut_cases()) == []


def _mistake_keep_real_part(theta, Z, k):
    # a split pair keeps the real part of its member inside the cut
    order = np.argsort(np.abs(theta), kind="stable")[:k]
    cols, done = [], set()
    for q in order:
        if q in done:
            continue
        partner = [p for p in order if p != q and np.isclose(theta[p], np.conj(theta[q]))]
        if abs(theta[q].imag) > 0 and partner:
            cols += [Z[:, q].real, Z[:, q].imag]
            done.add(partner[0])
        else:
            cols.append(Z[:, q].real)
        done.add(q)
    return np.array(cols).T, 0


_SELECT = K.harmonic_ritz_select


def _mistake_take_next(theta, Z, k):
    # a split pair is replaced by the next value after it (k columns)
    P, t = _SELECT(theta, Z, k)
    if P.shape[1] == k - 1:
        order = np.argsort(np.abs(theta), kind="stable")
        P = np.column_stack([P, Z[:, order[k + 1]].real])
    return P, t


def _mistake_wrong_split(theta, Z, k):
    # a kept pair contributes its real part and its modulus, not Re and Im
    P, t = _SELECT(theta, Z, k)
    order = np.argsort(np.abs(theta), kind="stable")
    cols, done = [], set()
    for a in order[:k]:
        if a in done:
            continue
        partner = [p for p in order[:k] if p != a and np.isclose(theta[p], np.conj(theta[a]))]
        if abs(theta[a].imag) > 0:
            if not partner:
                continue
            cols += [Z[:, a].real, np.abs(Z[:, a])]
            done.add(partner[0])
        else:
            cols.append(Z[:, a].real)
        done.add(a)
    return np.array(cols).T, t


@pytest.mark.parametrize("mistake", [_mistake_keep_real_part, _mistake_take_next,
                                     _mistake_wrong_split])
def test_conjugate_pair_pin_detects_planted_mistakes(monkeypatch, mistake):
    """The pin above fails for plausible mistakes in the selection (planted
    in the oracle on the CPU): keeping the real part of a split pair's
    member, replacing a split pair by the next value, and a wrong real basis
    of a kept pair."""
    cases = _pair_cut_cases()
    monkeypatch.setattr(K, "harmonic_ritz_select", mistake)
    assert _check_pair_cut(cases) != []


def test_harmonic_ritz_values_real_for_symmetric_operator():
    shape = (8, 8, 8)
    bc = {'x': ('dirichlet', 'dirichlet'), 'y': ('neumann', 'neumann'),
          'z': ('neumann', 'neumann')}
    prob = W.unit_laplacian(shape, bc)
    A, _, _ = _ops(prob, "none")
    traces = []
    K.rgcrot(A, lambda v: v, W.random_vector(prob.n, 10), 10, 4, 1e-14, K.Recycle.empty(prob.n),
             update=False, max_its=10, trace=traces.append)
    V, Hb = traces[0]["V"], traces[0]["H"]
    theta, _ = K.harmonic_ritz_pairs(Hb, V.T @ V[:, :Hb.shape[1]])
    assert np.abs(theta.imag).max() <= 1e-8 * np.abs(theta).max()


def test_recycle_setup_gives_orthonormal_c():
    prob = W.grf_problem(8, extra=9)
    _, _, op = _ops(prob)
    rec = _some_recycle_space(op, prob.n, 5, 2)
    AU = np.column_stack([op(rec.U[:, i]) for i in range(5)])
    assert np.linalg.norm(AU - rec.C) <= 1e-12 * np.linalg.norm(rec.C)
    assert np.linalg.norm(rec.C.T @ rec.C - np.eye(5)) <= 1e-13


# ---------------------------------------------------------------------------
# (r)BiCGStab
# ---------------------------------------------------------------------------

def test_bicgstab_matches_scipy_iterates():
    """Without a recycle space, Alg. 4 is Alg. 2; compared with SciPy's
    BiCGStab (x0 = 0, shadow residual r0, preconditioner applied on the
    right) after the same number of iterations."""
    prob = W.grf_problem(8, extra=10)
    A, Mi, op = _ops(prob)
    Aop = scipy.sparse.linalg.LinearOperator((prob.n, prob.n), matvec=A)
    Mop = scipy.sparse.linalg.LinearOperator((prob.n, prob.n), matvec=Mi)
    b = W.random_vector(prob.n, 11)
    for its in (1, 3, 7):
        xs, _ = scipy.sparse.linalg.bicgstab(Aop, b, rtol=1e-300, atol=0.0, maxiter=its, M=Mop)
        ours = K.rbicgstab(op, Mi, b, 0.0, None, max_matvecs=2 * its)
        assert np.linalg.norm(ours.x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_rbicgstab_residual_stays_orthogonal_to_c():
    prob = W.grf_problem(8, extra=11)
    _, Mi, op = _ops(prob)
    rec = K.Recycle.empty(prob.n)
    bs = W.rhs_perturbed(prob, 3, extra=11)
    for b in bs[:2]:
        K.rgcrot(op, Mi, b, 12, 6, 1e-10, rec)
    traces = []
    res = K.rbicgstab(op, Mi, bs[2], 1e-10, rec, trace=traces.append)
    assert res.status == K.CONVERGED
    for tr in traces:
        rn = np.linalg.norm(tr["r"])
        assert np.linalg.norm(rec.C.T @ tr["r"]) <= 1e-9 * rn + 1e-14 * np.linalg.norm(bs[2])
    # updated vs true residual after the postponed U-update
    assert res.rel_res_true <= 10 * 1e-10


def test_rbicgstab_rhs_in_range_of_c_needs_no_iteration():
    prob = W.grf_problem(8, extra=12)
    _, Mi, op = _ops(prob)
    rec = _some_recycle_space(op, prob.n, 4, 3)
    b = rec.C @ np.array([1.0, -2.0, 0.5, 3.0])
    res = K.rbicgstab(op, Mi, b, 1e-10, rec)
    assert res.iterations == 0 and res.status == K.CONVERGED
    assert np.linalg.norm(b - op(res.y)) <= 1e-12 * np.linalg.norm(b)


def test_rbicgstab_breakdown_on_zero_shadow_product():
    """rho = r~^T r = 0 forced by a zero right-hand side component pattern is
    not reachable with r~ = r_0 != 0, so check the status path with b = 0 ->
    converged immediately and with max_matvecs reached -> not converged."""
    prob = W.grf_problem(8, extra=13)
    _, Mi, op = _ops(prob)
    b = W.random_vector(prob.n, 12)
    res = K.rbicgstab(op, Mi, b, 1e-14, None, max_matvecs=4)
    assert res.status == K.NOT_CONVERGED and res.matvecs == 4


def test_hybrid_switches_and_falls_back():
    prob = W.grf_problem(8, extra=14)
    _, Mi, op = _ops(prob)
    rec = K.Recycle.empty(prob.n)
    bs = W.rhs_perturbed(prob, 4, extra=14)
    r0 = K.hybrid_step(0, 2, op, Mi, bs[0], 12, 6, 1e-10, rec)
    assert r0.cycles >= 1 and rec.dim == 6
    r2 = K.hybrid_step(2, 2, op, Mi, bs[2], 12, 6, 1e-10, rec)
    assert r2.cycles == 0 and r2.status == K.CONVERGED and not r2.fallback
    # forced failure of rBiCGStab (tiny matvec budget) -> rGCROT re-solve
    r3 = K.hybrid_step(3, 2, op, Mi, bs[3], 12, 6, 1e-10, rec, max_its=3)
    assert r3.fallback


def _two_porous(n=16):
    params = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
                  omega_global=6 / 7)
    p1 = W.porous_problem(n, extra=61)
    p2 = W.porous_problem(n, extra=62)
    ops = []
    for p in (p1, p2):
        Mi = lambda v, p=p: precond.schwarz_jacobi(p.bands, p.shape, p.periodic, v, **params)
        op = lambda v, p=p, Mi=Mi: stencil.apply(p.bands, p.shape, p.periodic, Mi(v))
        ops.append((p, Mi, op))
    return ops


def test_hybrid_stale_space_is_reformed_for_the_new_matrix():
    """The recycle-space setup of Alg. 3 when the matrix changed: after the hybrid step on the
    new operator, A~_new U = C and C^T C = I hold, and the system converges."""
    (p1, Mi1, op1), (p2, Mi2, op2) = _two_porous()
    bs = list(W.rhs_ar1(p1, 4, extra=61))
    rec, st = K.Recycle.empty(p1.n), K.HybridState()
    for t in range(3):
        K.hybrid_step(t, 2, op1, Mi1, bs[t], 20, 8, 1e-10, rec, state=st)
    st.stale = True
    res = K.hybrid_step(3, 2, op2, Mi2, bs[3], 20, 8, 1e-10, rec, state=st)
    assert res.refreshed and res.solver == "rbicgstab" and res.status == K.CONVERGED
    AU = np.column_stack([op2(rec.U[:, i]) for i in range(rec.dim)])
    assert np.linalg.norm(AU - rec.C) <= 1e-10 * np.linalg.norm(rec.C)
    assert np.linalg.norm(rec.C.T @ rec.C - np.eye(rec.dim)) <= 1e-12
    A2 = lambda v: stencil.apply(p2.bands, p2.shape, p2.periodic, v)
    assert np.linalg.norm(bs[3] - A2(res.x)) <= 2e-10 * np.linalg.norm(bs[3])


def test_hybrid_switches_back_after_poor_convergence():
    """Sec. 2.4 switch back: a converged rBiCGStab system needing more than
    switch_back times the matvecs of the first one since rGCROT makes the next
    system run rGCROT; the reference restarts after it."""
    (p1, Mi1, op1), (p2, Mi2, op2) = _two_porous()
    bs = list(W.rhs_ar1(p1, 8, extra=63))
    rec, st = K.Recycle.empty(p1.n), K.HybridState()
    seq, mvs, ref = [], [], 0
    expect_rg = False
    for t, b in enumerate(bs):
        op, Mi = (op1, Mi1) if t < 4 else (op2, Mi2)
        if t == 4:
            st.stale = True
        res = K.hybrid_step(t, 2, op, Mi, b, 20, 8, 1e-10, rec, switch_back=1.3, state=st)
        seq.append(res.solver)
        assert res.status == K.CONVERGED
        want = "rgcrot" if (t < 2 or expect_rg) else "rbicgstab"
        assert res.solver == want, (t, seq)
        if want == "rgcrot":
            ref, expect_rg = 0, False
        elif ref == 0:
            ref = res.matvecs
        else:
            expect_rg = res.matvecs > 1.3 * ref
        mvs.append(res.matvecs)
    # the new matrix with the old (re-formed) space converged poorly, and the
    # policy reacted within the sequence
    assert "rgcrot" in seq[5:], (seq, mvs)


def test_hybrid_switch_back_policy_on_scripted_counts(monkeypatch):
    """The switch-back reading of Sec. 2.4 on scripted solver outcomes (the
    two solvers replaced by stubs): the expected sequence below is written
    out by hand from the reading (n_switch = 2, factor 1.3: the first
    rBiCGStab system after rGCROT sets the reference; a converged system
    above 1.3 times it sends the next one to rGCROT; a failed rBiCGStab solve
    is repeated by rGCROT and also resets the reference)."""
    script = iter([(100, K.CONVERGED), (120, K.CONVERGED), (140, K.CONVERGED),
                   (200, K.CONVERGED), (250, K.CONVERGED), (300, K.NOT_CONVERGED),
                   (90, K.CONVERGED), (118, K.CONVERGED)])

    def fake_bicg(op, minv, b, tol, rec, max_its=2000, div_factor=1e2):
        mv, status = next(script)
        return K.Result(b, b, status, [], mv // 2, mv)

    def fake_rgcrot(op, minv, b, m, k, tol, rec, update=True, max_its=2000, orth="cgs2"):
        return K.Result(b, b, K.CONVERGED, [], 30, 31)

    monkeypatch.setattr(K, "rbicgstab", fake_bicg)
    monkeypatch.setattr(K, "rgcrot", fake_rgcrot)
    st, rec, b = K.HybridState(), K.Recycle.empty(4), np.ones(4)
    seq = [K.hybrid_step(t, 2, None, None, b, 30, 20, 1e-8, rec, switch_back=1.3,
                         state=st) for t in range(11)]
    got = [(r.solver, r.fallback) for r in seq]
    assert got == [("rgcrot", False), ("rgcrot", False),
                   ("rbicgstab", False),   # 100: reference
                   ("rbicgstab", False),   # 120 <= 130
                   ("rbicgstab", False),   # 140 > 130: next runs rGCROT
                   ("rgcrot", False),      # forced; reference reset
                   ("rbicgstab", False),   # 200: new reference
                   ("rbicgstab", False),   # 250 <= 260
                   ("rgcrot", True),       # 300, not converged: solved again by rGCROT
                   ("rbicgstab", False),   # 90: reference after the fallback
                   ("rbicgstab", False)]   # 118 > 117 = 1.3 * 90: next would run rGCROT
    assert st.force_rgcrot and st.ref_mv == 90


# ---------------------------------------------------------------------------
# GCROT rule of the cycle-end update (selection by angles between successive search
# spaces, truncation of the outer space).  Every check below rebuilds the
# spaces with applications of A~, not from the Hessenberg relation the
# update itself uses.
# ---------------------------------------------------------------------------

def _gcrot_run(m=10, k=8, par=K.GcrotParams(kt=5, s=5, p=1), n_sys=3, extra=21):
    prob = W.grf_problem(10, extra=extra)
    _, Mi, op = _ops(prob)
    rec = K.Recycle.empty(prob.n)
    runs = []
    for b in W.rhs_perturbed(prob, n_sys, extra=extra):
        traces = []
        res = K.rgcrot(op, Mi, b, m, k, 1e-10, rec, trace=traces.append, gcrot=par)
        # rec after each cycle: the next trace's (U, C), or the final rec
        afters = [(t["U"], t["C"]) for t in traces[1:]] + [(rec.U.copy(), rec.C.copy())]
        runs.append((b, res, traces, afters))
    return prob, op, rec, runs


def _in_range(C, v):
    return np.linalg.norm(v - C @ (C.T @ v)) / np.linalg.norm(v)


def test_gcrot_rule_invariants_and_cycle_correction():
    """After every update: A~ U = C, C^T C = I, dim <= k; the cycle's
    residual decrease A~ (V_j y - U B y) lies in the new range(C)."""
    prob, op, rec, runs = _gcrot_run()
    ncycles = 0
    for b, res, traces, afters in runs:
        assert res.status == K.CONVERGED and res.eig_ties == 0
        for tr, (U, C) in zip(traces, afters):
            ncycles += 1
            assert C.shape[1] <= 8
            AU = np.column_stack([op(U[:, i]) for i in range(U.shape[1])])
            assert np.linalg.norm(AU - C) <= 1e-11 * np.linalg.norm(C)
            assert np.linalg.norm(C.T @ C - np.eye(C.shape[1])) <= 1e-13
            j = tr["H"].shape[1]
            corr = tr["V"][:, :j] @ tr["y"] - tr["U"] @ (tr["B"] @ tr["y"])
            dec = op(corr)
            assert _in_range(C, dec) <= 1e-9
    assert ncycles >= 6


def test_gcrot_rule_selects_smallest_angle_with_previous_cycle():
    """p = 1: the principal vector of this cycle's selection space (images of
    the last s inner vectors) closest to the previous cycle's selection space
    lies in the new range(C); both spaces rebuilt from A~ applications."""
    prob, op, rec, runs = _gcrot_run(par=K.GcrotParams(kt=5, s=5, p=1))
    checked = 0
    for b, res, traces, afters in runs:
        for tr, (U, C) in zip(traces, afters):
            if tr["prev"] is None:
                continue
            V, B, Uo = tr["V"], tr["B"], tr["U"]
            j = tr["H"].shape[1]
            sj = min(5, j)
            # images of the last sj inner vectors: A~ (v_i - U B e_i)
            S = np.column_stack([op(V[:, i] - Uo @ B[:, i]) for i in range(j - sj, j)])
            Qs, _ = np.linalg.qr(S)
            Ql, _ = np.linalg.qr(tr["prev"])
            _, sig, Vt = np.linalg.svd(Ql.T @ Qs)
            w = Qs @ Vt[0]
            assert _in_range(C, w) <= 1e-8
            checked += 1
    assert checked >= 3


def test_gcrot_rule_truncation_keeps_smallest_angles():
    """When the outer space is cut, the kept old columns are those making the
    smallest angles with A~ range(V_j) (cosines from A~ applications); the
    dropped ones leave the space."""
    prob, op, rec, runs = _gcrot_run(m=6, k=6, par=K.GcrotParams(kt=3, s=3, p=1), n_sys=3)
    cuts = 0
    for b, res, traces, afters in runs:
        for tr, (U, C) in zip(traces, afters):
            Co = tr["C"]
            kc = Co.shape[1]
            j = tr["H"].shape[1]
            if kc == 0:
                continue
            AV = np.column_stack([op(tr["V"][:, i]) for i in range(j)])
            Qa, _ = np.linalg.qr(AV)
            cos = np.linalg.norm(Qa.T @ Co, axis=0)
            q = 1 + (tr["prev"] is not None)      # the cycle's correction (+ one selected)
            if kc + q <= 6:
                continue                  # no cut in this update
            ktp = min(3, 6 - q)
            assert C.shape[1] == ktp + q
            order = sorted(range(kc), key=lambda i: (-cos[i], -i))
            for i in order[:ktp]:
                assert _in_range(C, Co[:, i]) <= 1e-9
            for i in order[ktp:]:
                assert _in_range(C, Co[:, i]) > 1e-3
            cuts += 1
    assert cuts >= 2


def test_gcrot_rule_without_selection_is_gcro():
    """p = 0 and k above the number of cycles: no selection and no cut, so
    range(C) is spanned by the residual decreases of all cycles (GCRO with
    the full outer space), rebuilt from true residuals."""
    prob = W.grf_problem(10, extra=23)
    _, Mi, op = _ops(prob)
    b = W.rhs_perturbed(prob, 1, extra=23)[0]
    rec = K.Recycle.empty(prob.n)
    traces = []
    res = K.rgcrot(op, Mi, b, 5, 60, 1e-10, rec, trace=traces.append,
                   gcrot=K.GcrotParams(kt=50, s=3, p=0))
    assert res.status == K.CONVERGED
    decs = []
    for tr in traces:
        j = tr["H"].shape[1]
        decs.append(op(tr["V"][:, :j] @ tr["y"] - tr["U"] @ (tr["B"] @ tr["y"])))
    D = np.column_stack(decs)
    assert rec.dim == D.shape[1] == len(traces) >= 5
    assert scipy.linalg.subspace_angles(rec.C, D).max() <= 1e-7


def test_gcrot_rule_small_k_never_exceeds_k():
    """k = 2 with p = 2: the cycle's correction plus at most k - 1 selected
    vectors, so the outer space never holds more than k columns."""
    prob, op, rec, runs = _gcrot_run(m=8, k=2, par=K.GcrotParams(kt=1, s=4, p=2), n_sys=2)
    for b, res, traces, afters in runs:
        assert res.status == K.CONVERGED
        for U, C in afters:
            assert 1 <= C.shape[1] <= 2
            assert np.linalg.norm(C.T @ C - np.eye(C.shape[1])) <= 1e-13
