"""Krylov solvers with and without subspace recycling (oracle; test infrastructure).

All solvers are right-preconditioned: they work with the operator
A~ = A M^-1 (`op`) on the iterate y and return x = M^-1 y (`minv`).  This is
the reading under which the recycle space built by rGCROT is valid for
rBiCGStab (Sec. 2.4 reuses range(U), range(C) of rGCROT in rBiCGStab, so both
must see the same operator); Sec. 2.2 notes that the operator and right-hand
side of Alg. 1 may be taken as the preconditioned ones.

The initial guess is always zero, so r_0 = b (Sec. 2.2).  The stopping test
is ||r|| <= tol * ||b|| (the loop test of Alg. 1-4).

Recycle space convention: U, C with A~ U = C and C^T C = I, i.e. the factor R
of the recycle-space setup of Alg. 3 is absorbed into U (U R^-1 is stored as U).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

CONVERGED, NOT_CONVERGED, BREAKDOWN, DIVERGED = 0, 1, 2, 3


@dataclasses.dataclass
class Recycle:
    """Recycle space: columns of U (N x kc) and C (N x kc) with A~ U = C."""
    U: np.ndarray
    C: np.ndarray

    @classmethod
    def empty(cls, n):
        return cls(np.zeros((n, 0)), np.zeros((n, 0)))

    @property
    def dim(self):
        return self.U.shape[1]


@dataclasses.dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    status: int
    history: list
    iterations: int          # Arnoldi steps (GMRES type) or while-loop passes
    matvecs: int             # applications of A~ inside the iteration
    cycles: int = 0
    rel_res_true: float = float("nan")
    eig_ties: int = 0
    fallback: bool = False
    events: list = dataclasses.field(default_factory=list)
    solver: str = ""         # hybrid: "rgcrot" or "rbicgstab" (the one that produced x)
    refreshed: bool = False  # hybrid: C was re-formed from U first


@dataclasses.dataclass
class HybridState:
    """State of the hybrid policy across a sequence of systems.

    stale: A or M changed since C = A~ U was formed (the recycle-space setup of Alg. 3: form C
    again when the matrix has changed); force_rgcrot: the next system runs
    rGCROT; ref_mv: matvecs of the first rBiCGStab system since the last
    rGCROT one (the reference for switching back, Sec. 2.4)."""
    stale: bool = False
    force_rgcrot: bool = False
    ref_mv: int = 0


def _norm(v):
    return float(np.sqrt(np.dot(v, v)))


def _ls(Hbar, rho):
    """The least-squares step of Alg. 1/3: y = argmin || e1 rho - Hbar y ||, and that minimum."""
    rhs = np.zeros(Hbar.shape[0])
    rhs[0] = rho
    y = np.linalg.lstsq(Hbar, rhs, rcond=None)[0]
    return y, _norm(rhs - Hbar @ y)


def _orthogonalize(w, blocks, orth):
    """Orthogonalise w against the columns of each matrix in `blocks` (in order).

    'mgs': one column at a time, as in the orthogonalisation loops of Alg. 1
    and Alg. 3.  'cgs2': classical Gram-Schmidt against all columns at
    once, applied twice, coefficients summed.  Both give the same coefficients
    in exact arithmetic.  Returns (w, list of coefficient vectors per block)."""
    coefs = [np.zeros(Q.shape[1]) for Q in blocks]
    if orth == "mgs":
        for Q, c in zip(blocks, coefs):
            for l in range(Q.shape[1]):
                c[l] = Q[:, l] @ w
                w = w - Q[:, l] * c[l]
        return w, coefs
    if orth != "cgs2":
        raise ValueError(orth)
    Qall = np.hstack(blocks)
    tot = np.zeros(Qall.shape[1])
    for _ in range(2):
        c = Qall.T @ w
        w = w - Qall @ c
        tot += c
    off = 0
    for Q, c in zip(blocks, coefs):
        c[:] = tot[off:off + Q.shape[1]]
        off += Q.shape[1]
    return w, coefs


# ---------------------------------------------------------------------------
# Alg. 1: GMRES(m)
# ---------------------------------------------------------------------------

def gmres(op, minv, b, m, tol, max_its=2000, orth="cgs2"):
    """Restarted GMRES, Alg. 1, right-preconditioned, x_0 = 0.

    Convergence is tested inside the cycle on the least-squares residual
    (the estimate mentioned in the note to Alg. 1) and confirmed at the end of
    the cycle with the true residual b - A~ y; if the confirmation
    fails the next cycle starts."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    nb = _norm(b)
    y_acc = np.zeros(n)
    r = b.copy()
    rho = _norm(r)
    hist, its, mv, cycles = [], 0, 0, 0
    status = NOT_CONVERGED
    while rho > tol * nb and its < max_its:
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        V[:, 0] = r / rho
        jj = 0
        for j in range(m):
            w = op(V[:, j])
            its += 1
            mv += 1
            w, (h,) = _orthogonalize(w, [V[:, :j + 1]], orth)
            H[:j + 1, j] = h
            H[j + 1, j] = _norm(w)
            jj = j + 1
            _, est = _ls(H[:j + 2, :j + 1], rho)
            hist.append(est / nb)
            if H[j + 1, j] != 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            if est <= tol * nb or H[j + 1, j] == 0.0 or its >= max_its:
                break
        y, _ = _ls(H[:jj + 1, :jj], rho)
        y_acc = y_acc + V[:, :jj] @ y                     # solution update of the cycle
        r = b - op(y_acc)                                 # true residual
        mv += 1
        rho = _norm(r)
        cycles += 1
        if not np.isfinite(rho):
            status = DIVERGED
            break
    if rho <= tol * nb:
        status = CONVERGED
    return Result(minv(y_acc), y_acc, status, hist, its, mv, cycles, rho / nb)


# ---------------------------------------------------------------------------
# Alg. 3: rGCROT(m,k) / GCRODR(m,k) with the harmonic-Ritz update at cycle ends
# ---------------------------------------------------------------------------

def harmonic_ritz_pairs(G, F):
    """Harmonic Ritz pairs of the GCRODR rule: G^T G z = theta G^T F z, with
    F = W^T V^ (QZ via scipy.linalg.eig)."""
    return scipy.linalg.eig(G.T @ G, G.T @ F)


def harmonic_ritz_select(theta, Z, k):
    """Selection step of the GCRODR rule: a real basis P of the eigenvectors
    belonging to the k harmonic Ritz values of smallest |theta| (non-finite
    values last).  A complex-conjugate pair contributes the real and the
    imaginary part of one of its eigenvectors; when the cut at k falls
    between the two members of a pair, both are left out (k - 1 columns).
    Returns (P, number of near-ties at the cut)."""
    ties = 0
    mag = np.where(np.isfinite(theta), np.abs(theta), np.inf)
    order = np.argsort(mag, kind="stable")
    sel = list(order[:k])
    if k < len(order) and np.isfinite(mag[order[k]]) and mag[order[k - 1]] > 0:
        if (mag[order[k]] - mag[order[k - 1]]) / mag[order[k - 1]] < 1e-8:
            ties += 1
    # do not split a complex-conjugate pair
    chosen = []
    for i in sel:
        if abs(theta[i].imag) > 0:
            partner = [q for q in sel if q != i and np.isclose(theta[q], np.conj(theta[i]),
                                                             rtol=1e-10, atol=0)]
            if not partner:
                continue
        chosen.append(i)
    cols = []
    done = set()
    for i in chosen:
        if i in done:
            continue
        z = Z[:, i]
        if abs(theta[i].imag) > 0:
            cols.append(z.real)
            cols.append(z.imag)
            for q in chosen:
                if q != i and np.isclose(theta[q], np.conj(theta[i]), rtol=1e-10, atol=0):
                    done.add(q)
        else:
            cols.append(z.real)
        done.add(i)
    return np.array(cols).T, ties


def harmonic_ritz_update(rec: Recycle, V, Hbar, B, k):
    """The recycle-space update at the end of a cycle of Alg. 3, by the GCRODR rule (the recycle space is spanned
    by harmonic Ritz vectors of the search space range(U) + range(V_j)).

    V: N x (j+1) Arnoldi basis, Hbar: (j+1) x j, B = C^T A~ V_j: kc x j.
    With D = diag(1/||u_i||), W^ = [C, V_{j+1}], V^ = [U D, V_j] and
    G = [[D, B], [0, Hbar]] one has A~ V^ = W^ G (augmented Arnoldi
    relation).  If kc + j <= k the whole search space is kept; otherwise the
    harmonic Ritz problem G^T G z = theta G^T W^T V^ z is solved and the k
    vectors with the smallest |theta| are kept (a complex pair is never
    split).  With G P = Q R: C <- W^ Q, U <- V^ P R^-1, so A~ U = C and
    C^T C = I.  Returns the number of near-ties at the cut."""
    kc = rec.dim
    j = Hbar.shape[1]
    if j == 0:
        return 0
    d = 1.0 / np.sqrt(np.sum(rec.U * rec.U, axis=0)) if kc else np.zeros(0)
    D = np.diag(d)
    G = np.zeros((kc + j + 1, kc + j))
    G[:kc, :kc] = D
    G[:kc, kc:] = B
    G[kc:, kc:] = Hbar
    What = np.hstack([rec.C, V[:, :j + 1]])
    Vhat = np.hstack([rec.U * d[None, :], V[:, :j]])
    ties = 0
    if kc + j <= k:
        P = np.eye(kc + j)
    else:
        theta, Z = harmonic_ritz_pairs(G, What.T @ Vhat)
        P, ties = harmonic_ritz_select(theta, Z, k)
    Q, R = np.linalg.qr(G @ P)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    Q = Q * s[None, :]
    R = R * s[:, None]
    rec.C = What @ Q
    rec.U = scipy.linalg.solve_triangular(R, (Vhat @ P).T, trans="T", lower=False).T
    return ties


@dataclasses.dataclass
class GcrotParams:
    """Parameters of the GCROT rule for the cycle-end recycle update (Sec. 3 lists them with
    their values): kt outer vectors kept at a truncation (k - 10 there), s
    latest inner vectors to select from (m / 2), p inner vectors selected per
    cycle (1 or 2).  The fourth parameter, latest inner vectors kept, is 0
    in every run of the paper and is not modelled."""
    kt: int
    s: int
    p: int


def _small_gs(H, G, drop=1e-10):
    """Orthonormalise the columns of H G ((j+1) x q) in order, classical
    Gram-Schmidt applied twice, dropping a column whose remainder is at most
    `drop` times its norm.  Returns (Q, Gc) with H Gc = Q, Q^T Q = I."""
    Q, Gc = [], []
    for i in range(G.shape[1]):
        g = G[:, i].copy()
        h = H @ g
        h0 = _norm(h)
        if h0 == 0.0:
            continue
        for _ in range(2):
            for q, gc in zip(Q, Gc):
                t = q @ h
                h = h - t * q
                g = g - t * gc
        nrm = _norm(h)
        if nrm <= drop * h0:
            continue
        Q.append(h / nrm)
        Gc.append(g / nrm)
    if not Q:
        return np.zeros((H.shape[0], 0)), np.zeros((G.shape[0], 0))
    return np.column_stack(Q), np.column_stack(Gc)


def gcrot_update(rec: Recycle, V, Hbar, B, y, k, par: GcrotParams, prev):
    """The cycle-end recycle update of Alg. 3 by the GCROT rule, which takes the recycle space
    from angles between successive search spaces (Sec. 2.3; the details are
    in the GCROT references, so this is a reading).

    The cycle's search space is range(V_j) + range(U) with images
    A~ (V_j g - U B g) = V_{j+1} Hbar g, orthogonal to C.
      1. The cycle's own correction g = y (its image is r_old - r_new) joins
         the outer space.
      2. Selection space of this cycle: the images of the last s inner
         vectors, S = V_{j+1} Hbar[:, j-s:j] with orthonormal basis V Qs.
         With `prev` the previous cycle's selection space (orthonormal
         columns), the p principal vectors of S making the smallest angles
         with `prev` (largest singular values of prev^T V Qs, each vector's
         largest component made positive; at most dim(prev) and k - 1 of
         them, and none with a zero cosine) join the outer space too.
      3. The new images are orthonormalised in order (Gram-Schmidt twice,
         dropping dependent ones): q new pairs u = (V_j - U B) g,
         c = V_{j+1} Hbar g.
      4. If kc + q > k, the outer space is first cut to kt' = min(kt, k - q)
         of its columns: those making the smallest angles with the cycle's
         search space A~ range(V_j) (largest ||Q_K[i, :]||, Q_K an
         orthonormal basis of [B; Hbar], the coefficients of A~ V_j in
         [C, V_{j+1}]); on equal cosines the newer column wins.
      5. The new C is orthogonal to the kept one only as far as the Arnoldi
         basis is; two Cholesky-QR passes (C <- C R^-1, U <- U R^-1) keep
         C^T C = I over many cycles.
    Returns (new prev, ties), ties counting near-equal singular values or
    cosines at a cut."""
    kc = rec.dim
    j = Hbar.shape[1]
    if j == 0:
        return prev, 0
    ties = 0
    sj = min(par.s, j)
    # 2. selection space of this cycle
    Qs, Rs = np.linalg.qr(Hbar[:, j - sj:])
    sg = np.sign(np.diag(Rs))
    sg[sg == 0] = 1.0
    Qs = Qs * sg[None, :]
    Rs = Rs * sg[:, None]
    cand = [y.copy()]
    if prev is not None and prev.shape[1] and par.p > 0:
        M = (prev.T @ V) @ Qs                         # cosines: singular values
        _, sig, Vt = np.linalg.svd(M)
        # only directions with a nonzero cosine are defined
        npick = min(par.p, sj, prev.shape[1], k - 1)      # with y, at most k new columns
        while npick > 0 and sig[npick - 1] <= 1e-12:
            npick -= 1
        if 0 < npick < len(sig) and (sig[npick - 1] - sig[npick]) / sig[npick - 1] < 1e-8:
            ties += 1
        for i in range(npick):
            r = Vt[i].copy()
            if r[np.argmax(np.abs(r))] < 0:
                r = -r
            g = np.zeros(j)
            g[j - sj:] = scipy.linalg.solve_triangular(Rs, r, lower=False)
            cand.append(g)
    Qn, Gc = _small_gs(Hbar, np.column_stack(cand))
    q = Qn.shape[1]
    new_prev = V @ Qs
    # 4. truncation of the outer space
    keep = list(range(kc))
    if kc + q > k:
        ktp = max(0, min(par.kt, k - q))
        Qk, _ = np.linalg.qr(np.vstack([B, Hbar]))
        cos = np.sqrt(np.sum(Qk[:kc] ** 2, axis=1))
        order = sorted(range(kc), key=lambda i: (-cos[i], -i))
        if 0 < ktp < kc and cos[order[ktp - 1]] > 0 and \
                (cos[order[ktp - 1]] - cos[order[ktp]]) / cos[order[ktp - 1]] < 1e-8:
            ties += 1
        keep = sorted(order[:ktp])
    # 3. new pairs, appended after the kept columns
    Unew = V[:, :j] @ Gc - rec.U @ (B @ Gc)
    Cnew = V @ Qn
    rec.U = np.hstack([rec.U[:, keep], Unew])
    rec.C = np.hstack([rec.C[:, keep], Cnew])
    for _ in range(2):
        R = np.linalg.cholesky(rec.C.T @ rec.C).T
        rec.C = scipy.linalg.solve_triangular(R, rec.C.T, trans="T", lower=False).T
        rec.U = scipy.linalg.solve_triangular(R, rec.U.T, trans="T", lower=False).T
    return new_prev, ties


def recycle_setup(op, rec: Recycle):
    """Recycle-space setup of Alg. 3: C~ = A~ U, thin QR C~ = C R, U <- U R^-1."""
    if rec.dim == 0:
        return
    Ct = np.column_stack([op(rec.U[:, i]) for i in range(rec.dim)])
    Q, R = np.linalg.qr(Ct)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    Q = Q * s[None, :]
    R = R * s[:, None]
    rec.C = Q
    rec.U = scipy.linalg.solve_triangular(R, rec.U.T, trans="T", lower=False).T


def rgcrot(op, minv, b, m, k, tol, rec: Recycle, update=True, max_its=2000, orth="cgs2",
           trace=None, gcrot: GcrotParams | None = None):
    """rGCROT(m,k), Alg. 3, right-preconditioned, x^ = 0, R absorbed in U.

    b is first projected against C; each new Arnoldi vector is
    orthogonalised against C before V; the U-coefficients are z = -B y, and
    the update of the solution uses V y + U z = V y - U B y (the form that
    minimises the residual over range(U) + range(V_m), eq. for x_m and its
    argmin; the sign printed in the U-term of the algorithm's solution update
    would add +U B y instead).  Each cycle ends with the true residual, the
    update of (U, C) when `update`, and the residual is then
    re-projected against the new C so that the next cycle starts with
    r, v_1 orthogonal to C.  `rec` is updated in place.  gcrot: the update
    follows the GCROT rule (gcrot_update) instead of the harmonic-Ritz one;
    the previous cycle's selection space is kept within one solve."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    nb = _norm(b)
    hist, its, mv, cycles, ties = [], 0, 0, 0, 0
    status = NOT_CONVERGED
    if rec.dim:
        xi = rec.C.T @ b                                  # project b against C
        r = b - rec.C @ xi
        y_acc = rec.U @ xi
    else:
        r = b.copy()
        y_acc = np.zeros(n)
    rho = _norm(r)
    prev = None
    while rho > tol * nb and its < max_its:
        kc = rec.dim
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        Bm = np.zeros((kc, m))
        V[:, 0] = r / rho
        jj = 0
        for j in range(m):
            w = op(V[:, j])
            its += 1
            mv += 1
            w, (bcol, h) = _orthogonalize(w, [rec.C, V[:, :j + 1]], orth)  # against C, then V
            Bm[:, j] = bcol
            H[:j + 1, j] = h
            H[j + 1, j] = _norm(w)
            jj = j + 1
            _, est = _ls(H[:j + 2, :j + 1], rho)
            hist.append(est / nb)
            if H[j + 1, j] != 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            if est <= tol * nb or H[j + 1, j] == 0.0 or its >= max_its:
                break
        y, _ = _ls(H[:jj + 1, :jj], rho)
        z = -Bm[:, :jj] @ y                               # U-coefficients
        y_acc = y_acc + V[:, :jj] @ y + rec.U @ z
        r = b - op(y_acc)                                 # true residual
        mv += 1
        cycles += 1
        if trace is not None:
            trace(dict(V=V[:, :jj + 1].copy(), H=H[:jj + 1, :jj].copy(), B=Bm[:, :jj].copy(),
                       U=rec.U.copy(), C=rec.C.copy(), y_acc=y_acc.copy(), r=r.copy(),
                       y=y.copy(), prev=None if prev is None else prev.copy()))
        if update and gcrot is not None:                 # cycle-end recycle update
            prev, t = gcrot_update(rec, V[:, :jj + 1], H[:jj + 1, :jj], Bm[:, :jj], y, k,
                                   gcrot, prev)
            ties += t
        elif update:
            ties += harmonic_ritz_update(rec, V[:, :jj + 1], H[:jj + 1, :jj], Bm[:, :jj], k)
        if rec.dim:
            xi = rec.C.T @ r
            r = r - rec.C @ xi
            y_acc = y_acc + rec.U @ xi
        rho = _norm(r)
        if not np.isfinite(rho):
            status = DIVERGED
            break
    if rho <= tol * nb:
        status = CONVERGED
    res = Result(minv(y_acc), y_acc, status, hist, its, mv, cycles, rho / nb)
    res.eig_ties = ties
    return res


# ---------------------------------------------------------------------------
# Alg. 2 / Alg. 4: BiCGStab and rBiCGStab with one recycle space
# ---------------------------------------------------------------------------

def rbicgstab(op, minv, b, tol, rec: Recycle | None = None, max_matvecs=2000,
              div_factor=1e2, trace=None):
    """rBiCGStab with one recycle space, Alg. 4 (Alg. 2 when the space is empty).

    Runs BiCGStab on A~_C = (I - C C^T) A~ from r_0 = (I - C C^T) b
    (projecting b, v and t against C) with r~ = r_0; the U-parts of the
    solution updates are accumulated in xi (at the start, the half step and
    the full step) and applied once at the end (y <- y - U xi).  The loop test
    and the half-step test on s use the updated residual.  Breakdown (rho = 0, r~^T v = 0 or t^T t = 0) ends the
    iteration; so does a non-finite residual or one above div_factor*||b||
    (divergence guard for the hybrid solver)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    nb = _norm(b)
    if rec is None:
        rec = Recycle.empty(n)
    C, U = rec.C, rec.U
    eta1 = C.T @ b                                        # project b against C
    r = b - C @ eta1
    xi = -eta1
    rt = r.copy()                                         # r~ = r_0
    y = np.zeros(n)
    p = np.zeros(n)
    v = np.zeros(n)
    hist, its, mv = [], 0, 0
    status = NOT_CONVERGED
    rho_old = alpha = omega = 0.0
    rnorm = _norm(r)
    while rnorm > tol * nb and mv < max_matvecs:
        rho = rt @ r
        if rho == 0.0:
            status = BREAKDOWN
            break
        if its == 0:
            p = r.copy()
        else:
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
        v = op(p)
        mv += 1
        eta1 = C.T @ v                                    # project v against C
        v = v - C @ eta1
        rtv = rt @ v
        if rtv == 0.0:
            status = BREAKDOWN
            break
        alpha = rho / rtv
        s = r - alpha * v
        snorm = _norm(s)
        hist.append(snorm / nb)
        its += 1
        if snorm <= tol * nb:                             # half-step exit
            y = y + alpha * p
            r = s
            xi = xi + alpha * eta1
            rnorm = snorm
            break
        t = op(s)
        mv += 1
        eta2 = C.T @ t                                    # project t against C
        t = t - C @ eta2
        tt = t @ t
        if tt == 0.0:
            status = BREAKDOWN
            y = y + alpha * p
            xi = xi + alpha * eta1
            r = s
            rnorm = snorm
            break
        omega = (t @ s) / tt
        xi = xi + alpha * eta1 + omega * eta2             # U-part of the update
        y = y + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        rnorm = _norm(r)
        hist.append(rnorm / nb)
        if trace is not None:
            trace(dict(r=r.copy(), s=s.copy(), t=t.copy(), v=v.copy(), xi=xi.copy(), y=y.copy()))
        if not np.isfinite(rnorm) or rnorm > div_factor * nb:
            status = DIVERGED
            break
    y = y - U @ xi                                        # postponed U-update
    if status == NOT_CONVERGED and rnorm <= tol * nb:
        status = CONVERGED
    true = _norm(b - op(y)) / nb
    return Result(minv(y), y, status, hist, its, mv, 0, true)


# ---------------------------------------------------------------------------
# Sec. 2.4: hybrid rGCROT -> rBiCGStab over a sequence of systems
# ---------------------------------------------------------------------------

def hybrid_step(step, n_switch, op, minv, b, m, k, tol, rec: Recycle,
                max_its=2000, orth="cgs2", div_factor=1e2, switch_back=0.0,
                state: HybridState = None):
    """One system of the hybrid sequence (Sec. 2.4): the first n_switch systems
    are solved by rGCROT(m,k), which builds (U, C); later systems by
    rBiCGStab with that space held fixed.  If rBiCGStab diverges, breaks down
    or fails to converge, the system is solved again by rGCROT.

    Readings for the two options Sec. 2.4 names without fixing them:
    * a changing matrix (state.stale): C is formed again from U (the recycle-space setup)
      before the system is solved;
    * switching back when convergence becomes poor (switch_back > 0): if a
      converged rBiCGStab system needed more than switch_back times the
      matvecs of the first rBiCGStab system since the last rGCROT one, the
      next system runs rGCROT (which also refreshes the space)."""
    state = state if state is not None else HybridState()
    refreshed = False
    if state.stale:
        if rec.dim > 0:
            recycle_setup(op, rec)
            refreshed = True
        state.stale = False
    if step < n_switch or state.force_rgcrot:
        state.force_rgcrot = False
        state.ref_mv = 0
        res = rgcrot(op, minv, b, m, k, tol, rec, True, max_its, orth)
        res.solver, res.refreshed = "rgcrot", refreshed
        return res
    res = rbicgstab(op, minv, b, tol, rec, max_its, div_factor)
    if res.status == CONVERGED:
        if switch_back > 0:
            if state.ref_mv == 0:
                state.ref_mv = res.matvecs
            elif res.matvecs > switch_back * state.ref_mv:
                state.force_rgcrot = True
        res.solver, res.refreshed = "rbicgstab", refreshed
        return res
    state.ref_mv = 0
    again = rgcrot(op, minv, b, m, k, tol, rec, True, max_its, orth)
    again.fallback = True
    again.events = [("rbicgstab_status", res.status)]
    again.solver, again.refreshed = "rgcrot", refreshed
    return again
