"""The host dense linear algebra of the solvers (csrc/dense.cpp: thin QR,
Cholesky, triangular inverse and solve, the symmetric Jacobi eigensolver, the
Hessenberg/double-shift QR eigenvalues, the harmonic-Ritz selection) against
NumPy/SciPy's LAPACK routines, run through a small driver built with the
address and undefined-behaviour sanitizers (any invalid access or undefined
operation aborts the driver and fails the test)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("dense") / "dense_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "dense_driver.cpp"),
           os.path.join(ROOT, "paper_1501_03358_amd", "csrc", "dense.cpp"), "-o", out]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr
    return out


def _fmt(a):
    return " ".join(repr(float(x)) for x in np.asarray(a, dtype=np.float64).ravel(order="F"))


def _run(driver, cases):
    """cases: list of (header, [arrays]); returns one token list per case."""
    text = "\n".join(h + " " + " ".join(_fmt(a) for a in arrs) for h, arrs in cases) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([driver], input=text, capture_output=True, text=True, env=env,
                       timeout=120)
    assert p.returncode == 0, p.stderr[-4000:]
    lines = p.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    return [ln.split() for ln in lines]


def _vals(tok, start, n, shape=None):
    v = np.array([float(x) for x in tok[start:start + n]])
    return v.reshape(shape, order="F") if shape else v


def test_thin_qr(driver):
    rng = np.random.default_rng(11)
    shapes = [(1, 1), (5, 3), (7, 7), (31, 30), (64, 20), (51, 50)]
    mats = [rng.standard_normal(s) for s in shapes]
    out = _run(driver, [(f"qr {m} {n}", [A]) for (m, n), A in zip(shapes, mats)])
    for (m, n), A, tok in zip(shapes, mats, out):
        assert tok[0] == "qr"
        Q = _vals(tok, 1, m * n, (m, n))
        R = _vals(tok, 1 + m * n, n * n, (n, n))
        assert np.allclose(np.tril(R, -1), 0)
        assert np.all(np.diag(R) >= 0)
        assert np.linalg.norm(Q @ R - A) <= 1e-13 * np.linalg.norm(A)
        assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13 * n
        # unique with diag(R) >= 0: LAPACK's factor with its signs flipped
        Qn, Rn = np.linalg.qr(A)
        s = np.sign(np.diag(Rn))
        s[s == 0] = 1
        assert np.linalg.norm(R - s[:, None] * Rn) <= 1e-12 * np.linalg.norm(A)


def test_cholesky_inverse_and_solve(driver):
    rng = np.random.default_rng(12)
    cases, spd = [], []
    for n in (1, 5, 30, 62):
        B = rng.standard_normal((n, n))
        A = B @ B.T + n * np.eye(n)
        spd.append(A)
        cases.append((f"chol {n}", [A]))
    indef = np.diag([2.0, -1.0, 3.0])
    cases.append(("chol 3", [indef]))
    ups = []
    for n in (1, 4, 40):
        R = np.triu(rng.standard_normal((n, n))) + 3 * np.eye(n)
        ups.append(R)
        cases.append((f"uinv {n}", [R]))
    sing = np.triu(np.ones((3, 3)))
    sing[1, 1] = 0.0
    cases.append(("uinv 3", [sing]))
    g = rng.standard_normal(40)
    cases.append(("usolve 40", [ups[-1], g]))
    out = _run(driver, cases)
    for A, tok in zip(spd, out[:4]):
        n = A.shape[0]
        assert tok[:2] == ["chol", "ok"]
        R = _vals(tok, 2, n * n, (n, n))
        assert np.linalg.norm(R - np.linalg.cholesky(A).T) <= 1e-12 * np.linalg.norm(R)
    assert out[4][:2] == ["chol", "fail"]
    for R, tok in zip(ups, out[5:8]):
        n = R.shape[0]
        assert tok[:2] == ["uinv", "ok"]
        Ri = _vals(tok, 2, n * n, (n, n))
        assert np.allclose(np.tril(Ri, -1), 0)
        assert np.linalg.norm(R @ Ri - np.eye(n)) <= 1e-12 * n
    assert out[8][:2] == ["uinv", "fail"]
    y = _vals(out[9], 1, 40)
    assert np.linalg.norm(ups[-1] @ y - g) <= 1e-12 * np.linalg.norm(g)
    assert np.linalg.norm(y - scipy.linalg.solve_triangular(ups[-1], g)) <= 1e-12 * np.linalg.norm(y)


def test_symmetric_jacobi_eigensolver(driver):
    rng = np.random.default_rng(13)
    mats = []
    for n in (1, 2, 10, 32, 62):
        B = rng.standard_normal((n, n))
        mats.append(B + B.T)
    # repeated eigenvalues: the eigenvectors are only fixed up to a rotation
    Q, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    mats.append(Q @ np.diag([3.0, 3.0, 3.0, 1.0, 1.0, -2.0, 0.0, 0.0]) @ Q.T)
    mats.append(np.zeros((4, 4)))
    out = _run(driver, [(f"symeig {A.shape[0]}", [A]) for A in mats])
    for A, tok in zip(mats, out):
        n = A.shape[0]
        assert tok[:2] == ["symeig", "ok"]
        w = _vals(tok, 2, n)
        Z = _vals(tok, 2 + n, n * n, (n, n))
        scale = max(np.linalg.norm(A), 1.0)
        assert np.all(np.diff(w) <= 0)                             # descending
        assert np.linalg.norm(w - np.linalg.eigvalsh(A)[::-1]) <= 1e-12 * scale * n
        assert np.linalg.norm(A @ Z - Z * w) <= 1e-12 * scale * n
        assert np.linalg.norm(Z.T @ Z - np.eye(n)) <= 1e-12 * n


def _match(a, b):
    """Largest distance of a greedy one-to-one matching of two multisets."""
    b = list(b)
    worst = 0.0
    for x in a:
        j = int(np.argmin([abs(x - y) for y in b]))
        worst = max(worst, abs(x - b[j]))
        b.pop(j)
    return worst


def test_real_eigenvalues_double_shift_qr(driver):
    rng = np.random.default_rng(14)
    mats = [rng.standard_normal((n, n)) for n in (1, 2, 5, 20, 51)]
    # known spectrum with complex pairs: block diagonal rotations, similarity
    blk = scipy.linalg.block_diag([[1.0, -2.0], [2.0, 1.0]], [[0.5, 3.0], [-3.0, 0.5]], [[4.0]])
    T = rng.standard_normal((5, 5)) + 5 * np.eye(5)
    mats.append(T @ blk @ np.linalg.inv(T))
    mats.append(np.triu(rng.standard_normal((6, 6))))            # already triangular
    out = _run(driver, [(f"eig {A.shape[0]}", [A]) for A in mats])
    for A, tok in zip(mats, out):
        n = A.shape[0]
        assert tok[:2] == ["eig", "ok"]
        v = _vals(tok, 2, 2 * n)
        lam = v[0::2] + 1j * v[1::2]
        ref = np.linalg.eigvals(A)
        assert _match(lam, ref) <= 1e-9 * max(np.linalg.norm(A), 1.0)
    lam6 = _vals(out[5], 2, 10)
    assert _match(lam6[0::2] + 1j * lam6[1::2], [1 + 2j, 1 - 2j, 0.5 + 3j, 0.5 - 3j, 4.0]) <= 1e-9


def _expected_span(G, F, k):
    """SciPy's generalized eigenproblem G^T G z = theta G^T F z: the k values
    of smallest |theta| (a complex value whose conjugate falls outside the k
    is left out) and a real orthonormal basis of their eigenvectors' span."""
    th, Z = scipy.linalg.eig(G.T @ G, G.T @ F)
    order = np.argsort(np.abs(th), kind="stable")
    sel = list(order[:k])

    def conj_of(i, j):
        return abs(th[i] - np.conj(th[j])) <= 1e-9 * abs(th[i]) and th[i].imag != 0

    keep = [i for i in sel
            if th[i].imag == 0 or any(j != i and conj_of(i, j) for j in sel)]
    E = np.column_stack([np.real(Z[:, i]) for i in keep] + [np.imag(Z[:, i]) for i in keep])
    U, s, _ = np.linalg.svd(E, full_matrices=False)
    r = int(np.sum(s > 1e-10 * s[0]))
    m = np.abs(th[order])

    def rgap(i):            # relative gap between positions i - 1 and i of the order
        return m[i] / m[i - 1] - 1 if 0 < i < len(m) else 1.0

    cut_pair = k < len(th) and conj_of(order[k - 1], order[k])
    # a clear cut: between k - 1 and k, or around the pair the cut falls in
    gap = min(rgap(k - 1), rgap(k + 1)) if cut_pair else rgap(k)
    return U[:, :r], len(keep), gap, cut_pair


def test_harmonic_ritz_selection_matches_scipy(driver):
    """Random pencils of the recycle-space update's shape (G: (ng+1) x ng),
    kept away from near ties at the cut; one case per size where the cut
    falls inside a complex-conjugate pair (the pair is left out whole)."""
    rng = np.random.default_rng(15)
    cases, refs = [], []
    for ng, k in ((6, 3), (12, 5), (30, 10), (50, 20), (51, 20), (20, 20)):
        want_pair_cut = ng in (12, 30)
        for _ in range(200):
            G = rng.standard_normal((ng + 1, ng))
            F = rng.standard_normal((ng + 1, ng))
            E, kk, gap, cut_pair = _expected_span(G, F, k)
            if gap > 1e-3 and cut_pair == want_pair_cut:
                break
        else:
            pytest.fail(f"no suitable pencil for ng={ng}")
        cases.append((f"hr {ng + 1} {ng} {k}", [G, F]))
        refs.append((ng, E, kk, cut_pair))
    out = _run(driver, cases)
    for (ng, E, kk, cut_pair), tok in zip(refs, out):
        assert tok[:2] == ["hr", "ok"]
        got_kk, ties = int(tok[2]), int(tok[3])
        assert got_kk == kk and ties == 0
        P = _vals(tok, 4, ng * got_kk, (ng, got_kk))
        assert np.linalg.matrix_rank(P) == kk
        assert scipy.linalg.subspace_angles(P, E).max() < 1e-8
