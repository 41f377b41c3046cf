"""Pins of the oracle Schwarz-Jacobi preconditioner: an explicit dense
construction (restriction matrices, local operators, loops), linearity, and
the exact-solve limit."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import precond
from tests import _fvm


def _random_problem(shape, bc, seed):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    kcell = np.exp(rng.standard_normal((nz, ny, nx)))
    vol = rng.uniform(0.5, 1.5, (nz, ny, nx))
    widths = (np.ones(nx), np.ones(ny), np.ones(nz))
    bands = W.assemble(kcell, vol, widths, bc)
    A = _fvm.csr_assemble(kcell, vol, widths, bc).toarray()
    periodic = tuple(bc[a] == 'periodic' for a in 'xyz')
    return bands, A, periodic


def _dense_schwarz(A, shape, periodic, r, tile, overlap, sweeps, wl, gsweeps, wg):
    """Restricted additive Schwarz with damped-Jacobi local solves, built from
    dense restriction matrices R_s (extended tile) and owner sets, then
    global damped Jacobi, all with explicit loops."""
    nx, ny, nz = shape
    dims = (nx, ny, nz)
    z = np.zeros(A.shape[0])
    tiles = [range(d // tile) for d in dims]
    for t in itertools.product(*tiles):
        ext = []
        for e in itertools.product(*[range(-overlap, tile + overlap)] * 3):
            c = [t[a] * tile + e[a] for a in range(3)]
            ok = True
            for a in range(3):
                if periodic[a]:
                    c[a] %= dims[a]
                elif not 0 <= c[a] < dims[a]:
                    ok = False
            if ok:
                owned = all(0 <= e[a] < tile for a in range(3))
                ext.append((c[0] + nx * (c[1] + ny * c[2]), owned))
        idx = [g for g, _ in ext]
        R = np.zeros((len(idx), A.shape[0]))
        R[np.arange(len(idx)), idx] = 1.0
        As = R @ A @ R.T
        Ds = np.diag(As)
        rs = R @ r
        zs = np.zeros(len(idx))
        for _ in range(sweeps):
            zs = zs + wl * (rs - As @ zs) / Ds
        for (g, owned), val in zip(ext, zs):
            if owned:
                z[g] = val
    D = np.diag(A)
    for _ in range(gsweeps):
        z = z + wg * (r - A @ z) / D
    return z


CASES = [
    ((8, 8, 8), {'x': ('dirichlet', 'dirichlet'), 'y': ('neumann', 'neumann'),
                 'z': ('neumann', 'neumann')}, 4, 1),
    ((8, 12, 8), {'x': 'periodic', 'y': ('neumann', 'neumann'), 'z': 'periodic'}, 4, 1),
    ((12, 12, 8), {'x': ('neumann', 'dirichlet'), 'y': 'periodic',
                   'z': ('neumann', 'neumann')}, 4, 2),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_matches_dense_construction(case):
    shape, bc, tile, overlap = CASES[case]
    bands, A, periodic = _random_problem(shape, bc, 100 + case)
    r = np.random.default_rng(7).standard_normal(A.shape[0])
    params = dict(tile=tile, overlap=overlap, local_sweeps=5, omega_local=6 / 7,
                  global_sweeps=1, omega_global=6 / 7)
    z = precond.schwarz_jacobi(bands, shape, periodic, r, **params)
    ref = _dense_schwarz(A, shape, periodic, r, tile, overlap, 5, 6 / 7, 1, 6 / 7)
    assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref)


def test_linearity():
    shape, bc, tile, overlap = CASES[1]
    bands, _, periodic = _random_problem(shape, bc, 3)
    rng = np.random.default_rng(8)
    r1, r2 = rng.standard_normal((2, bands.shape[1]))
    M = lambda r: precond.schwarz_jacobi(bands, shape, periodic, r, tile=tile, overlap=overlap)
    lhs = M(2.0 * r1 - 3.0 * r2)
    rhs = 2.0 * M(r1) - 3.0 * M(r2)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


def test_single_tile_many_sweeps_is_exact_inverse():
    """One tile covering the grid, no overlap, Jacobi run to convergence and no
    global sweep: M^-1 = A^-1 (A nonsingular)."""
    shape = (8, 8, 8)
    bc = {'x': ('dirichlet', 'dirichlet'), 'y': ('dirichlet', 'dirichlet'),
          'z': ('dirichlet', 'dirichlet')}
    bands, A, periodic = _random_problem(shape, bc, 4)
    r = np.random.default_rng(9).standard_normal(A.shape[0])
    z = precond.schwarz_jacobi(bands, shape, periodic, r, tile=8, overlap=0,
                               local_sweeps=3000, omega_local=1.0, global_sweeps=0)
    ref = np.linalg.solve(A, r)
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


def test_point_jacobi_is_inverse_diagonal():
    shape, bc, _, _ = CASES[0]
    bands, A, _ = _random_problem(shape, bc, 5)
    r = np.random.default_rng(10).standard_normal(A.shape[0])
    assert np.allclose(precond.jacobi(bands, r) * np.diag(A), r, rtol=1e-15, atol=0)


def test_periodic_axis_must_exceed_extended_tile():
    shape = (8, 8, 8)
    bc = {'x': 'periodic', 'y': ('neumann', 'neumann'), 'z': ('neumann', 'neumann')}
    bands, _, periodic = _random_problem(shape, bc, 6)
    with pytest.raises(ValueError):
        precond.schwarz_jacobi(bands, shape, periodic, np.ones(512), tile=4, overlap=2)


def _dense_schwarz_ssor(A, shape, periodic, r, tile, overlap, sweeps, w, gsweeps, wg):
    """Restricted additive Schwarz with SSOR local solves written out cell by
    cell: Gauss-Seidel with relaxation w over the cells of each extended tile
    in the order even colour then odd colour (forward), odd then even
    (backward), colour = parity of the extended-tile position."""
    nx, ny, nz = shape
    dims = (nx, ny, nz)
    z = np.zeros(A.shape[0])
    tiles = [range(d // tile) for d in dims]
    for t in itertools.product(*tiles):
        ext = []
        for e in itertools.product(*[range(-overlap, tile + overlap)] * 3):
            c = [t[a] * tile + e[a] for a in range(3)]
            ok = True
            for a in range(3):
                if periodic[a]:
                    c[a] %= dims[a]
                elif not 0 <= c[a] < dims[a]:
                    ok = False
            if ok:
                owned = all(0 <= e[a] < tile for a in range(3))
                colour = (e[0] + e[1] + e[2] + 3 * overlap) % 2
                ext.append((c[0] + nx * (c[1] + ny * c[2]), owned, colour))
        idx = [g for g, _, _ in ext]
        R = np.zeros((len(idx), A.shape[0]))
        R[np.arange(len(idx)), idx] = 1.0
        As = R @ A @ R.T
        rs = R @ r
        zs = np.zeros(len(idx))
        even = [i for i, (_, _, c) in enumerate(ext) if c == 0]
        odd = [i for i, (_, _, c) in enumerate(ext) if c == 1]
        for _ in range(sweeps):
            for i in even + odd + odd[::-1] + even[::-1]:
                zs[i] += w * (rs[i] - As[i] @ zs) / As[i, i]
        for (g, owned, _), val in zip(ext, zs):
            if owned:
                z[g] = val
    D = np.diag(A)
    for _ in range(gsweeps):
        z = z + wg * (r - A @ z) / D
    return z


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("w", [1.0, 1.3])
def test_ssor_local_solver_matches_cellwise_gauss_seidel(case, w):
    shape, bc, tile, overlap = CASES[case]
    bands, A, periodic = _random_problem(shape, bc, 200 + case)
    r = np.random.default_rng(17).standard_normal(A.shape[0])
    z = precond.schwarz_jacobi(bands, shape, periodic, r, tile=tile, overlap=overlap,
                               local_sweeps=3, omega_local=w, global_sweeps=1,
                               omega_global=6 / 7, local_solver="ssor")
    ref = _dense_schwarz_ssor(A, shape, periodic, r, tile, overlap, 3, w, 1, 6 / 7)
    assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref)


def test_ssor_single_tile_converges_to_inverse():
    """Symmetric Gauss-Seidel on one tile covering the grid converges to A^-1 r
    (and faster than damped Jacobi)."""
    shape = (8, 8, 8)
    bc = {'x': ('dirichlet', 'dirichlet'), 'y': ('dirichlet', 'dirichlet'),
          'z': ('dirichlet', 'dirichlet')}
    bands, A, periodic = _random_problem(shape, bc, 24)
    r = np.random.default_rng(25).standard_normal(A.shape[0])
    ref = np.linalg.solve(A, r)
    z = precond.schwarz_jacobi(bands, shape, periodic, r, tile=8, overlap=0,
                               local_sweeps=400, omega_local=1.0, global_sweeps=0,
                               local_solver="ssor")
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    zs = precond.schwarz_jacobi(bands, shape, periodic, r, tile=8, overlap=0, local_sweeps=5,
                                omega_local=1.0, global_sweeps=0, local_solver="ssor")
    zj = precond.schwarz_jacobi(bands, shape, periodic, r, tile=8, overlap=0, local_sweeps=10,
                                omega_local=1.0, global_sweeps=0)
    assert np.linalg.norm(zs - ref) < np.linalg.norm(zj - ref)


def _random_19pt(shape, periodic, seed):
    """A 7-point random operator plus small random edge couplings (19 bands),
    and its dense matrix built by explicit loops."""
    from oracle import stencil
    from tests.test_oracle_stencil import _dense19_by_loops
    bc = {a: ('periodic' if periodic[i] else ('dirichlet', 'neumann')) for i, a in enumerate('xyz')}
    b7, _, _ = _random_problem(shape, bc, seed)
    rng = np.random.default_rng(seed + 1)
    bands = np.zeros((19, b7.shape[1]))
    bands[:7] = b7
    bands[7:] = 0.05 * rng.standard_normal((12, b7.shape[1])) * np.abs(b7[0])[None]
    return bands, _dense19_by_loops(bands, shape, periodic), stencil


@pytest.mark.parametrize("case", [((8, 8, 8), (False, False, False), 4, 1),
                                  ((8, 12, 8), (True, False, True), 4, 1)])
def test_19pt_schwarz_matches_dense_construction(case):
    shape, periodic, tile, overlap = case
    bands, A, _ = _random_19pt(shape, periodic, 31)
    r = np.random.default_rng(12).standard_normal(A.shape[0])
    z = precond.schwarz_jacobi(bands, shape, periodic, r, tile=tile, overlap=overlap,
                               local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
                               omega_global=6 / 7)
    ref = _dense_schwarz(A, shape, periodic, r, tile, overlap, 5, 6 / 7, 1, 6 / 7)
    assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref)


def test_19pt_ssor_local_solver_rejected():
    bands, _, _ = _random_19pt((8, 8, 8), (False, False, False), 5)
    with pytest.raises(ValueError):
        precond.schwarz_jacobi(bands, (8, 8, 8), (False, False, False), np.ones(512),
                               tile=4, local_solver="ssor")
