"""Pins of the oracle stencil y = A u (and of the band assembly feeding it)."""
import numpy as np
import pytest

import workloads as W
from oracle import stencil
from tests import _fvm

BCS = [
    {'x': ('dirichlet', 'dirichlet'), 'y': ('neumann', 'neumann'), 'z': 'periodic'},
    {'x': 'periodic', 'y': ('dirichlet', 'dirichlet'), 'z': ('neumann', 'neumann')},
    {'x': ('neumann', 'neumann'), 'y': 'periodic', 'z': ('dirichlet', 'dirichlet')},
]


@pytest.mark.parametrize("n", [8, 24])
@pytest.mark.parametrize("bci", range(len(BCS)))
def test_closed_form_eigenpairs(n, bci):
    """Unit coefficients, unit spacing, uniform volume v: tensor products of
    the 1-D cell-centred modes are eigenvectors with eigenvalue sum(lambda_d)/v."""
    bc = BCS[bci]
    shape = (n, n - 2 if n > 8 else n, n + 2 if n > 8 else n)
    v = 2.5
    prob = W.unit_laplacian(shape, bc, vol=v)
    rng = np.random.default_rng(5)
    for _ in range(12):
        ps = [int(rng.choice(list(_fvm.mode_range(bc[a], shape[i]))))
              for i, a in enumerate('xyz')]
        u, lam = _fvm.mode_3d(bc, shape, ps)
        y = stencil.apply(prob.bands, prob.shape, prob.periodic, u)
        assert np.linalg.norm(y - lam / v * u) <= 1e-13 * max(lam / v, 1.0) * np.linalg.norm(u) * 10


def test_constant_null_vector_of_singular_operator():
    prob = W.channel_problem(8)
    y = stencil.apply(prob.bands, prob.shape, prob.periodic, np.ones(prob.n))
    assert np.abs(y).max() <= 1e-12 * np.abs(prob.bands[0]).max()


@pytest.mark.parametrize("shape", [(5, 6, 7), (7, 3, 4)])
def test_matches_face_by_face_sparse_assembly(shape):
    """Random conductivities, volumes and non-uniform widths with mixed
    boundary rules; the banded oracle product equals the CSR product of an
    operator assembled face by face."""
    nx, ny, nz = shape
    rng = np.random.default_rng(11)
    kcell = np.exp(rng.standard_normal((nz, ny, nx)))
    vol = rng.uniform(0.5, 1.5, (nz, ny, nx))
    widths = (rng.uniform(0.5, 2, nx), rng.uniform(0.5, 2, ny), rng.uniform(0.5, 2, nz))
    bc = {'x': 'periodic', 'y': ('dirichlet', 'neumann'), 'z': ('neumann', 'dirichlet')}
    bands = W.assemble(kcell, vol, widths, bc)
    A = _fvm.csr_assemble(kcell, vol, widths, bc)
    u = rng.standard_normal(nx * ny * nz)
    y = stencil.apply(bands, shape, (True, False, False), u)
    ref = A @ u
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)


def test_volume_scaling_makes_operator_nonsymmetric():
    prob = W.grf_problem(8)
    rng = np.random.default_rng(1)
    u, w = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    Au = stencil.apply(prob.bands, prob.shape, prob.periodic, u)
    Aw = stencil.apply(prob.bands, prob.shape, prob.periodic, w)
    assert abs(w @ Au - u @ Aw) > 1e-3 * abs(w @ Au)
    # but vol * A is symmetric
    assert abs(w @ (prob.vol * Au) - u @ (prob.vol * Aw)) <= 1e-12 * abs(w @ (prob.vol * Au))


# ---------------------------------------------------------------------------
# 19-point operators (non-orthogonal grids)
# ---------------------------------------------------------------------------

def _dense19_by_loops(bands, shape, periodic):
    """Dense matrix of a 19-band operator from explicit per-cell loops over
    the neighbour offsets, with wrap or drop per axis."""
    nx, ny, nz = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    offs = [(0, 0, 0)] + list(stencil.OFFSETS19)
    dims = (nx, ny, nz)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = x + nx * (y + ny * z)
                for band, d in enumerate(offs):
                    c = [x + d[0], y + d[1], z + d[2]]
                    ok = True
                    for a in range(3):
                        if not 0 <= c[a] < dims[a]:
                            if periodic[a]:
                                c[a] %= dims[a]
                            else:
                                ok = False
                    if ok:
                        A[i, c[0] + nx * (c[1] + ny * c[2])] += bands[band, i]
    return A


@pytest.mark.parametrize("shape,periodic", [((5, 6, 7), (False, False, False)),
                                            ((4, 3, 5), (True, False, True)),
                                            ((3, 4, 3), (True, True, True))])
def test_19pt_matches_loop_assembly(shape, periodic):
    rng = np.random.default_rng(11)
    n = shape[0] * shape[1] * shape[2]
    bands = rng.standard_normal((19, n))
    A = _dense19_by_loops(bands, shape, periodic)
    u = rng.standard_normal(n)
    y = stencil.apply(bands, shape, periodic, u)
    assert np.linalg.norm(y - A @ u) <= 1e-13 * np.linalg.norm(A @ u)


def test_19pt_with_zero_edges_equals_7pt():
    prob = W.grf_problem(8, extra=3)
    b19 = np.zeros((19, prob.n))
    b19[:7] = prob.bands
    u = np.random.default_rng(4).standard_normal(prob.n)
    assert np.array_equal(stencil.apply(b19, prob.shape, prob.periodic, u),
                          stencil.apply(prob.bands, prob.shape, prob.periodic, u))


def test_19pt_cross_term_closed_form():
    """Edge bands only, c * dx * dy on the four xy edges: applied to u = x y
    every interior cell gets c * sum (a b)(x + a)(y + b) = 4 c."""
    shape = (6, 5, 4)
    n = 120
    b19 = np.zeros((19, n))
    c = 0.37
    for band, (dx, dy, dz) in enumerate(stencil.OFFSETS19[6:10], start=7):
        b19[band] = c * dx * dy
    z, y, x = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    u = (x * y).astype(float).reshape(-1)
    out = stencil.apply(b19, shape, (False, False, False), u).reshape(4, 5, 6)
    assert np.allclose(out[:, 1:-1, 1:-1], 4 * c, rtol=0, atol=1e-14)


def test_skewed_problem_is_symmetric_positive_definite_19pt():
    """The sheared-grid workload: 19 coupled neighbours per interior cell,
    symmetric (edge couplings use the pair's harmonic mean), positive definite."""
    prob = W.skewed_problem(6)
    A = _dense19_by_loops(prob.bands, prob.shape, prob.periodic)
    assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
    assert (np.abs(A) > 0).sum(axis=1).max() == 19
    assert np.linalg.eigvalsh(A).min() > 0


def test_19pt_offset_layout():
    """Bands 1-6 are the faces in the 7-point order; bands 7-18 are the 12
    offsets with two nonzero +-1 components, grouped by plane (xy, xz, yz),
    the first axis of the plane varying fastest."""
    offs = stencil.OFFSETS19
    assert offs[:6] == ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))
    for g, (p, q) in enumerate(((0, 1), (0, 2), (1, 2))):
        grp = offs[6 + 4 * g:10 + 4 * g]
        for j, o in enumerate(grp):
            assert sum(1 for c in o if c) == 2 and o[p] and o[q]
            assert o[p] == (-1 if j % 2 == 0 else 1) and o[q] == (-1 if j < 2 else 1)
