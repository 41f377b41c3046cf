"""Seeded synthetic inputs for the pressure-Poisson system sequences.

This module produces *inputs only*: the 7-band matrix of a finite-volume
Poisson operator on a structured grid (Sec. 2.1, "Data Layout": banded
storage of the 7 coefficients per cell of an orthogonal grid), the right-hand
side sequences b_t, and the solver/preconditioner parameter sets of the
workloads.  It contains none of the solvers' arithmetic, and both the CPU
oracle and the GPU path draw their inputs from it.

Conventions shared by every consumer:

* grid ``(nx, ny, nz)``, unknown ``i = x + nx*(y + ny*z)`` (x fastest);
* bands ``[7, N]`` in the order C, W(x-1), E(x+1), S(y-1), N(y+1), B(z-1),
  T(z+1): ``(A u)_i = C_i u_i + W_i u_{i-1} + E_i u_{i+1} + ...``;
* a periodic axis wraps; across a non-periodic boundary the band is 0
  (Neumann) or the face is folded into C (Dirichlet, half-cell distance);
* ``A = diag(1/vol) L`` with L the symmetric flux-sum operator, so A is
  nonsymmetric whenever the volumes vary.

Synthetic stand-ins (the paper's channel-flow and porous-medium pressure
systems of Sec. 3 are not available): a Gaussian-random-field conductivity
case, a stretched channel grid periodic in x and z, and a sphere-pack porous
medium with a 1000:1 conductivity contrast.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator

import numpy as np

SEED_BASE = 150103358

BAND_NAMES = ("C", "W", "E", "S", "N", "B", "T")

# Schwarz-Jacobi preconditioner parameters (Sec. 2.1, "Preconditioners in
# GenIDLEST": overlapping subdomains, five under-relaxed Jacobi sweeps per
# subdomain, then one global point-Jacobi sweep).  Subdomain size, overlap and
# relaxation factors are not given in the paper; these are the values used
# by every workload.
SCHWARZ_DEFAULT = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6.0 / 7.0,
                       global_sweeps=1, omega_global=6.0 / 7.0)


@dataclasses.dataclass
class Problem:
    name: str
    shape: tuple            # (nx, ny, nz)
    periodic: tuple         # (px, py, pz) booleans
    bands: np.ndarray       # [7, N] float64
    vol: np.ndarray         # [N] float64 row-scaling volumes
    singular: bool          # True when A has the constant null vector

    @property
    def n(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


# --------------------------------------------------------------------------
# random fields and geometry
# --------------------------------------------------------------------------

def gaussian_random_field(shape_zyx, ell, rng):
    """White noise N(0,1) filtered by exp(-ell^2 |kappa|^2 / 4) on a periodic
    box (covariance exp(-d^2 / (2 ell^2))), then normalised to mean 0, std 1."""
    noise = rng.standard_normal(shape_zyx)
    f = np.fft.fftn(noise)
    k2 = np.zeros(shape_zyx)
    for ax, n in enumerate(shape_zyx):
        kk = 2.0 * np.pi * np.fft.fftfreq(n)
        sh = [1, 1, 1]
        sh[ax] = n
        k2 = k2 + (kk ** 2).reshape(sh)
    g = np.real(np.fft.ifftn(f * np.exp(-(ell ** 2) * k2 / 4.0)))
    g = g - g.mean()
    return g / g.std()


def sphere_pack(shape_zyx, rmin, rmax, solid_fraction, rng):
    """Solid mask: spheres with centres uniform in the box and radius uniform in
    [rmin, rmax] cells are added until the solid fraction reaches the target.
    A cell is solid when its centre lies within r of a sphere centre."""
    nz, ny, nx = shape_zyx
    solid = np.zeros(shape_zyx, dtype=bool)
    target = solid_fraction * solid.size
    count = 0
    while count < target:
        c = rng.uniform(0.0, 1.0, 3) * np.array([nx, ny, nz], dtype=float)
        r = rng.uniform(rmin, rmax)
        lo = np.maximum(np.floor(c - r).astype(int), 0)
        hi = np.minimum(np.ceil(c + r).astype(int) + 1, [nx, ny, nz])
        xs = np.arange(lo[0], hi[0]) + 0.5
        ys = np.arange(lo[1], hi[1]) + 0.5
        zs = np.arange(lo[2], hi[2]) + 0.5
        d2 = ((zs[:, None, None] - c[2]) ** 2 + (ys[None, :, None] - c[1]) ** 2
              + (xs[None, None, :] - c[0]) ** 2)
        inside = d2 <= r * r
        sub = solid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        count += int(np.count_nonzero(inside & ~sub))
        sub |= inside
    return solid


def tanh_faces_widths(n, length, g):
    """Cell widths for faces y_j = (L/2) tanh(g (2j/n - 1)) / tanh(g)."""
    s = np.tanh(g * (2.0 * np.arange(n + 1) / n - 1.0)) / np.tanh(g)
    return np.diff(s) * (length / 2.0)


def tanh_widths(n, length, ratio):
    """Cell widths of a wall-clustered grid with faces
    y_j = (L/2) tanh(g (2j/n - 1)) / tanh(g), g chosen by bisection so that the
    largest ratio of adjacent widths equals `ratio`."""
    def widths(g):
        return tanh_faces_widths(n, length, g)

    def max_ratio(g):
        w = widths(g)
        q = w[1:] / w[:-1]
        return max(q.max(), (1.0 / q).max())

    lo, hi = 1e-6, 20.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if max_ratio(mid) > ratio:
            hi = mid
        else:
            lo = mid
    return widths(lo)


# --------------------------------------------------------------------------
# finite-volume assembly into 7 bands
# --------------------------------------------------------------------------

def assemble(kcell, vol, widths, bc):
    """Two-point flux finite-volume Poisson operator in banded storage.

    kcell : (nz, ny, nx) cell conductivity; face conductivity is the harmonic
            mean of the two adjacent cells.
    vol   : (nz, ny, nx) row-scaling volumes (A = diag(1/vol) L).
    widths: (dx[nx], dy[ny], dz[nz]) cell widths.
    bc    : per axis ('x', 'y', 'z') either 'periodic' or a (low, high) pair of
            'dirichlet' / 'neumann'.
    Face transmissibility T = k_f * area / distance between cell centres; a
    Dirichlet face uses the half-cell distance and only adds to C.
    """
    nz, ny, nx = kcell.shape
    dx, dy, dz = (np.asarray(w, dtype=float) for w in widths)
    L = np.zeros((7, nz, ny, nx))
    # (array axis, widths along it, face area, band index toward -, toward +)
    area = {
        2: dy[None, :, None] * dz[:, None, None] * np.ones((1, 1, nx)),
        1: dx[None, None, :] * dz[:, None, None] * np.ones((1, ny, 1)),
        0: dx[None, None, :] * dy[None, :, None] * np.ones((nz, 1, 1)),
    }
    spec = [(2, dx, 'x', 1, 2), (1, dy, 'y', 3, 4), (0, dz, 'z', 5, 6)]
    for ax, w, name, bm, bp in spec:
        n = kcell.shape[ax]
        a = np.broadcast_to(area[ax], kcell.shape)
        kk = np.moveaxis(kcell, ax, 0)
        aa = np.moveaxis(a, ax, 0)
        # faces between cell c and c+1 (interior)
        kf = 2.0 * kk[:-1] * kk[1:] / (kk[:-1] + kk[1:])
        d = 0.5 * (w[:-1] + w[1:]).reshape((-1,) + (1,) * 2)
        af = 0.5 * (aa[:-1] + aa[1:])
        T = kf * af / d
        Lp = np.moveaxis(L, ax + 1, 1)       # view with the axis first (after band)
        Lp[bp, :-1] -= T
        Lp[bm, 1:] -= T
        Lp[0, :-1] += T
        Lp[0, 1:] += T
        rule = bc[name]
        if rule == 'periodic':
            if n < 3:
                raise ValueError("periodic axis needs at least 3 cells")
            kf = 2.0 * kk[-1] * kk[0] / (kk[-1] + kk[0])
            d = 0.5 * (w[-1] + w[0])
            T = kf * 0.5 * (aa[-1] + aa[0]) / d
            Lp[bp, -1] -= T
            Lp[bm, 0] -= T
            Lp[0, -1] += T
            Lp[0, 0] += T
        else:
            low, high = rule
            if low == 'dirichlet':
                Lp[0, 0] += kk[0] * aa[0] / (0.5 * w[0])
            if high == 'dirichlet':
                Lp[0, -1] += kk[-1] * aa[-1] / (0.5 * w[-1])
    bands = (L / vol[None]).reshape(7, -1)
    return np.ascontiguousarray(bands)


# --------------------------------------------------------------------------
# workload families
# --------------------------------------------------------------------------

def _seeds(cfg_id, extra=0):
    ss = np.random.SeedSequence(SEED_BASE + cfg_id + 1000 * extra)
    coef, vol, b0, seq = ss.spawn(4)
    return coef, vol, b0, seq


def grf_problem(n=24, seed_cfg=1, extra=0, ell=4.0):
    """Uniform n^3 grid, k = exp(g) with g a Gaussian random field, random
    volumes in [0.5, 1.5], Dirichlet on both x faces, Neumann elsewhere."""
    s_coef, s_vol, _, _ = _seeds(seed_cfg, extra)
    g = gaussian_random_field((n, n, n), ell, np.random.default_rng(s_coef))
    kcell = np.exp(g)
    vol = np.random.default_rng(s_vol).uniform(0.5, 1.5, (n, n, n))
    bc = {'x': ('dirichlet', 'dirichlet'), 'y': ('neumann', 'neumann'),
          'z': ('neumann', 'neumann')}
    ones = np.ones(n)
    bands = assemble(kcell, vol, (ones, ones, ones), bc)
    return Problem(f"grf{n}", (n, n, n), (False, False, False), bands,
                   vol.reshape(-1), False)


def skewed_problem(n=32, seed_cfg=5, extra=0, shear=(0.2, 0.15, 0.1), ell=4.0):
    """19-point operator of a non-orthogonal (sheared) grid: k = exp(g) on a
    uniform n^3 grid with unit volumes, Dirichlet on both x faces, Neumann
    elsewhere, plus the cross-derivative terms of a constant metric whose
    off-diagonal entries are `shear` = (xy, xz, yz).  The term
    -d_p(s k d_q u) - d_q(s k d_p u) by central differences couples a cell to
    its four edge neighbours (c + a e_p + b e_q, a, b = +-1) with -s a b k_e / 2,
    k_e the harmonic mean of the two cells' k (symmetric); beyond a boundary
    the edge neighbour is dropped.  Bands in the 19-point layout."""
    s_coef, _, _, _ = _seeds(seed_cfg, extra)
    g = gaussian_random_field((n, n, n), ell, np.random.default_rng(s_coef))
    kcell = np.exp(g)
    vol = np.ones((n, n, n))
    bc = {'x': ('dirichlet', 'dirichlet'), 'y': ('neumann', 'neumann'),
          'z': ('neumann', 'neumann')}
    ones = np.ones(n)
    b7 = assemble(kcell, vol, (ones, ones, ones), bc)
    bands = np.zeros((19, n ** 3))
    bands[:7] = b7
    # edge bands 7..18: (dx, dy, dz) as in the 19-point layout
    edges = ((-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 1, 0),
             (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (1, 0, 1),
             (0, -1, -1), (0, 1, -1), (0, -1, 1), (0, 1, 1))
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for e, (dx, dy, dz) in enumerate(edges):
        gam = shear[0] if dz == 0 else (shear[1] if dy == 0 else shear[2])
        sign = (dx or 1) * (dy or 1) * (dz or 1)      # product of the two nonzero offsets
        xn, yn, zn = x + dx, y + dy, z + dz
        ok = (xn >= 0) & (xn < n) & (yn >= 0) & (yn < n) & (zn >= 0) & (zn < n)
        kn = kcell[np.clip(zn, 0, n - 1), np.clip(yn, 0, n - 1), np.clip(xn, 0, n - 1)]
        ke = 2.0 * kcell * kn / (kcell + kn)
        bands[7 + e] = np.where(ok, -gam * sign * ke / 2.0, 0.0).reshape(-1)
    return Problem(f"skewed{n}", (n, n, n), (False, False, False), np.ascontiguousarray(bands),
                   vol.reshape(-1), False)


# tanh clustering strength of the 128^3 channel grid with adjacent width
# ratio 1.1; the same wall clustering at other resolutions (largest/smallest
# width ~ 94..112 for 32^3..192^3)
CHANNEL_G128 = 3.0646


def channel_problem(n=128, ratio=1.1, g=None):
    """Channel-like grid: Lx = 2 pi, Ly = 2, Lz = pi, periodic in x and z,
    Neumann walls in y with tanh clustering (largest adjacent width ratio
    `ratio`, or the clustering strength `g` when given); k = 1; volumes are
    the cell volumes, so the row scaling makes A nonsymmetric.  Singular
    (constant null vector)."""
    dx = np.full(n, 2.0 * np.pi / n)
    dz = np.full(n, np.pi / n)
    dy = tanh_widths(n, 2.0, ratio) if g is None else tanh_faces_widths(n, 2.0, g)
    vol = dz[:, None, None] * dy[None, :, None] * dx[None, None, :]
    kcell = np.ones((n, n, n))
    bc = {'x': 'periodic', 'y': ('neumann', 'neumann'), 'z': 'periodic'}
    bands = assemble(kcell, vol, (dx, dy, dz), bc)
    return Problem(f"channel{n}", (n, n, n), (True, False, True), bands,
                   vol.reshape(-1).copy(), True)


def porous_problem(n=128, seed_cfg=3, extra=0, solid_fraction=0.4,
                   k_solid=1e-3, rmin=3.0, rmax=6.0, shape=None):
    """Sphere-pack porous medium on a uniform n^3 grid, or on an
    nx x ny x nz grid when `shape` = (nx, ny, nz) is given (unit volumes):
    k = 1 in fluid and k_solid in solid cells; Dirichlet p = 0 on the x-max
    face, Neumann elsewhere (nonsingular)."""
    nx, ny, nz = (n, n, n) if shape is None else tuple(int(v) for v in shape)
    s_coef, _, _, _ = _seeds(seed_cfg, extra)
    solid = sphere_pack((nz, ny, nx), rmin, rmax, solid_fraction,
                        np.random.default_rng(s_coef))
    kcell = np.where(solid, k_solid, 1.0)
    vol = np.ones((nz, ny, nx))
    bc = {'x': ('neumann', 'dirichlet'), 'y': ('neumann', 'neumann'),
          'z': ('neumann', 'neumann')}
    bands = assemble(kcell, vol, (np.ones(nx), np.ones(ny), np.ones(nz)), bc)
    name = f"porous{n}" if shape is None else f"porous{nx}x{ny}x{nz}"
    return Problem(name, (nx, ny, nz), (False, False, False), bands,
                   vol.reshape(-1), False)


def make_compatible(b, prob: Problem):
    """Remove the mean (volume-weighted when A is singular, so that b lies in
    the range of A = diag(1/vol) L; plain mean otherwise)."""
    if prob.singular:
        return b - (prob.vol @ b) / prob.vol.sum()
    return b - b.mean()


def rhs_perturbed(prob: Problem, nsteps=5, seed_cfg=1, extra=0) -> list:
    """b_t = b_0 + 0.05 t eta_t with b_0, eta_t uniform in [-1, 1], mean-free."""
    _, _, s_b0, s_seq = _seeds(seed_cfg, extra)
    b0 = make_compatible(np.random.default_rng(s_b0).uniform(-1, 1, prob.n), prob)
    out = [b0]
    for t, s in zip(range(1, nsteps), s_seq.spawn(nsteps - 1)):
        eta = make_compatible(np.random.default_rng(s).uniform(-1, 1, prob.n), prob)
        out.append(b0 + 0.05 * t * eta)
    return out


def rhs_ar1(prob: Problem, nsteps, seed_cfg=2, extra=0, dtype=np.float64) -> Iterator:
    """AR(1) walk b_0 = xi_0, b_t = 0.98 b_{t-1} + 0.02 xi_t, xi_t ~ N(0, 1)
    made compatible with A.  Yields the b_t one at a time."""
    _, _, s_b0, s_seq = _seeds(seed_cfg, extra)
    b = make_compatible(np.random.default_rng(s_b0).standard_normal(prob.n), prob)
    yield b.astype(dtype, copy=True)
    for s in s_seq.spawn(max(nsteps - 1, 0)):
        xi = make_compatible(np.random.default_rng(s).standard_normal(prob.n), prob)
        b = 0.98 * b + 0.02 * xi
        yield b.astype(dtype, copy=True)


def random_vector(n, seed, kind="normal"):
    rng = np.random.default_rng(np.random.SeedSequence(SEED_BASE + 7 * 10 ** 6 + seed))
    if kind == "normal":
        return rng.standard_normal(n)
    return rng.uniform(-1.0, 1.0, n)


def unit_laplacian(shape, bc, vol=1.0):
    """Unit-conductivity, unit-spacing operator (for closed-form checks)."""
    nx, ny, nz = shape
    kcell = np.ones((nz, ny, nx))
    v = np.full((nz, ny, nx), float(vol))
    bands = assemble(kcell, v, (np.ones(nx), np.ones(ny), np.ones(nz)), bc)
    periodic = tuple(bc[a] == 'periodic' for a in 'xyz')
    singular = all(bc[a] == 'periodic' or bc[a] == ('neumann', 'neumann') for a in 'xyz')
    return Problem("unit", (nx, ny, nz), periodic, bands, v.reshape(-1), singular)


# The five named workloads (grid, operator family, solvers, tolerance).
WORKLOADS = {
    "grf24": dict(kind="grf", n=24, precond="jacobi", m=20, k=10, tol=1e-8, steps=5),
    "channel128": dict(kind="channel", n=128, precond="schwarz", m=30, k=20, tol=1e-8, steps=50),
    "porous128_hybrid": dict(kind="porous", n=128, precond="schwarz", m=30, k=20, tol=1e-8,
                             steps=100, n_switch=3),
    "porous256_ir": dict(kind="porous", n=256, precond="schwarz", m=30, k=20, tol=1e-8,
                         steps=20, n_switch=3),
}


def build_problem(kind, n, extra=0):
    if kind == "grf":
        return grf_problem(n, extra=extra)
    if kind == "channel":
        return channel_problem(n)
    if kind == "porous":
        return porous_problem(n, extra=extra)
    if kind == "skewed":
        return skewed_problem(n, extra=extra)
    raise ValueError(kind)
