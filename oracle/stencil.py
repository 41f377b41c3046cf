"""y = A u for a 7- or 19-point operator stored as bands (oracle; test infrastructure).

Follows Sec. 2.1 ("Data Layout"): each unknown stores the coefficients of its
7-point (orthogonal grids) or 19-point (non-orthogonal grids) stencil.  Band
order C, W, E, S, N, B, T couples cell (x, y, z) to itself, x-1, x+1, y-1,
y+1, z-1, z+1; a 19-point operator adds 12 bands for the edge neighbours in
the order of OFFSETS19[6:].  A periodic axis wraps; across a non-periodic
boundary the neighbour does not exist and contributes nothing.
"""
import numpy as np

# (band, array axis in (z, y, x) order, offset along that axis)
NEIGHBOURS = ((1, 2, -1), (2, 2, +1), (3, 1, -1), (4, 1, +1), (5, 0, -1), (6, 0, +1))

# (dx, dy, dz) of bands 1..18 of a 19-point operator: the six faces, then the
# edges of the xy, xz and yz planes
OFFSETS19 = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1),
             (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 1, 0),
             (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (1, 0, 1),
             (0, -1, -1), (0, 1, -1), (0, -1, 1), (0, 1, 1))


def shifted(u3, d, per_zyx):
    """Entry at cell c: u at c + d, d = (dx, dy, dz); 0 where that cell lies
    outside a non-periodic grid."""
    v = u3
    for axis, off in ((2, d[0]), (1, d[1]), (0, d[2])):
        if off:
            v = neighbour_values(v, axis, off, per_zyx[axis])
    return v


def neighbour_values(u3, axis, offset, periodic_axis):
    """Array whose entry at cell c is u at c + offset along `axis` (0 where
    that cell lies outside a non-periodic grid)."""
    v = np.roll(u3, -offset, axis=axis)
    if not periodic_axis:
        sl = [slice(None)] * 3
        sl[axis] = -1 if offset > 0 else 0
        v[tuple(sl)] = 0.0
    return v


def apply(bands, shape, periodic, u):
    """Return A u, with A given by `bands` [7, N] or [19, N] on grid
    `shape` = (nx, ny, nz)."""
    nx, ny, nz = shape
    per_zyx = (periodic[2], periodic[1], periodic[0])
    u3 = np.asarray(u, dtype=np.float64).reshape(nz, ny, nx)
    nb = bands.shape[0]
    if nb not in (7, 19):
        raise ValueError("7 or 19 bands")
    b = bands.reshape(nb, nz, ny, nx)
    y = b[0] * u3
    for band in range(1, nb):
        y = y + b[band] * shifted(u3, OFFSETS19[band - 1], per_zyx)
    return y.reshape(-1)


def residual(bands, shape, periodic, b, x):
    """b - A x."""
    return b - apply(bands, shape, periodic, x)
