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
