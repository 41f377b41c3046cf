"""Preconditioners z = M^-1 r (oracle; test infrastructure).

Sec. 2.1 ("Preconditioners in GenIDLEST"): the grid is split into many
overlapping subdomains; each subdomain problem is solved inexactly by five
under-relaxed Jacobi sweeps (additive Schwarz), and a sweep of point Jacobi on
the whole grid then couples distant subdomains.  M^-1 is a fixed linear
operator.

Readings where the paper is silent (parity unpinned against the paper):
subdomains are the T^3 tiles of the grid extended by `overlap` cells on every
side (wrapped on periodic axes, clipped at non-periodic ones); the local
problem is A restricted to the extended tile with zero values outside it; the
local sweeps start from zero; each cell takes the value computed by the tile
that owns it (restricted additive Schwarz); the global sweep is damped Jacobi
on the full operator started from that value.

The paper's alternative local smoother is SSOR (Sec. 2.1, and the porous
medium tables of Sec. 3 comparing the two).  Reading: one SSOR iteration is a
forward SOR sweep followed by a backward one over the extended tile, with
the cells ordered by colour (x + y + z of the extended-tile position even,
then odd; backward: odd, then even) so that each colour is updated at once;
relaxation omega_local (1 = symmetric Gauss-Seidel).
"""
import numpy as np

from . import stencil


def jacobi(bands, r):
    """Point Jacobi, M = diag(A)."""
    return r / bands[0]


def _axis_windows(n, tile, overlap, periodic):
    """For every tile along one axis: global index and validity of each of the
    tile + 2*overlap extended positions."""
    if n % tile:
        raise ValueError("grid size must be a multiple of the tile size")
    if periodic and n <= tile + 2 * overlap:
        # the two ends of an extended tile would be neighbours of each other
        raise ValueError("periodic axis must be longer than an extended tile")
    nt = n // tile
    e = np.arange(-overlap, tile + overlap)
    idx = np.arange(nt)[:, None] * tile + e[None, :]
    if periodic:
        return idx % n, np.ones_like(idx, dtype=bool)
    valid = (idx >= 0) & (idx < n)
    return np.clip(idx, 0, n - 1), valid


def schwarz_jacobi(bands, shape, periodic, r, tile=8, overlap=1, local_sweeps=5,
                   omega_local=6.0 / 7.0, global_sweeps=1, omega_global=6.0 / 7.0,
                   local_solver="jacobi"):
    """Two-level Schwarz preconditioner applied to r: `local_sweeps` damped
    Jacobi sweeps (local_solver="jacobi") or SSOR iterations ("ssor") on every
    extended tile, restricted write-back, then global damped Jacobi sweeps."""
    if local_solver not in ("jacobi", "ssor"):
        raise ValueError(local_solver)
    if local_solver == "ssor" and bands.shape[0] != 7:
        raise ValueError("the two-colour SSOR ordering decouples 7-point bands only")
    nx, ny, nz = shape
    ix, vx = _axis_windows(nx, tile, overlap, periodic[0])
    iy, vy = _axis_windows(ny, tile, overlap, periodic[1])
    iz, vz = _axis_windows(nz, tile, overlap, periodic[2])
    ntx, nty, ntz = ix.shape[0], iy.shape[0], iz.shape[0]
    E = tile + 2 * overlap
    # gathered index of every extended cell: [tz, ty, tx, ez, ey, ex]
    g = (ix[None, None, :, None, None, :]
         + nx * (iy[None, :, None, None, :, None]
                 + ny * iz[:, None, None, :, None, None]))
    valid = (vx[None, None, :, None, None, :] & vy[None, :, None, None, :, None]
             & vz[:, None, None, :, None, None])
    g = np.broadcast_to(g, (ntz, nty, ntx, E, E, E))
    valid = np.broadcast_to(valid, g.shape)
    rs = np.where(valid, r[g], 0.0)
    bs = np.where(valid[None], bands[:, g], 0.0)
    diag = np.where(valid, bs[0], 1.0)

    # local sweeps on every extended tile, starting from zero; neighbours
    # outside the extended tile count as zero
    z = np.zeros_like(rs)

    def a_times(z):
        az = bs[0] * z
        for band in range(1, bands.shape[0]):
            # neighbour at offset (dx, dy, dz) inside the extended tile
            # (axes 5, 4, 3 of z), zero beyond it
            nb = np.zeros_like(z)
            src = [slice(None)] * 6
            dst = [slice(None)] * 6
            for ax, off in zip((5, 4, 3), stencil.OFFSETS19[band - 1]):
                if off > 0:
                    dst[ax] = slice(0, E - 1)
                    src[ax] = slice(1, E)
                elif off < 0:
                    dst[ax] = slice(1, E)
                    src[ax] = slice(0, E - 1)
            nb[tuple(dst)] = z[tuple(src)]
            az = az + bs[band] * nb
        return az

    if local_solver == "jacobi":
        for _ in range(local_sweeps):
            z = z + omega_local * (rs - a_times(z)) / diag
    else:
        e = np.arange(E)
        colour = (e[:, None, None] + e[None, :, None] + e[None, None, :]) % 2   # [ez, ey, ex]
        for _ in range(local_sweeps):
            for c in (0, 1, 1, 0):            # forward sweep, then backward sweep
                upd = z + omega_local * (rs - a_times(z)) / diag
                z = np.where(colour == c, upd, z)
    # restricted write-back: each tile provides its owned cells
    own = slice(overlap, overlap + tile)
    zo = z[:, :, :, own, own, own]                    # [tz, ty, tx, T, T, T]
    zg = zo.transpose(0, 3, 1, 4, 2, 5).reshape(-1)   # (z, y, x) order
    # global point-Jacobi sweeps
    for _ in range(global_sweeps):
        zg = zg + omega_global * stencil.residual(bands, shape, periodic, r, zg) / bands[0]
    return zg


def make(bands, shape, periodic, kind, params=None):
    """Return a callable r -> M^-1 r."""
    if kind == "none":
        return lambda r: np.array(r, dtype=np.float64, copy=True)
    if kind == "jacobi":
        return lambda r: jacobi(bands, r)
    if kind == "schwarz":
        p = dict(params or {})
        return lambda r: schwarz_jacobi(bands, shape, periodic, r, **p)
    raise ValueError(kind)
