"""y = A u for a 7-point operator stored as 7 bands (oracle; test infrastructure).

Follows Sec. 2.1 ("Data Layout"): each unknown stores its 7 stencil
coefficients.  Band order C, W, E, S, N, B, T couples cell (x, y, z) to
itself, x-1, x+1, y-1, y+1, z-1, z+1.  A periodic axis wraps; across a
non-periodic boundary the neighbour does not exist and contributes nothing.
"""
import numpy as np

# (band, array axis in (z, y, x) order, offset along that axis)
NEIGHBOURS = ((1, 2, -1), (2, 2, +1), (3, 1, -1), (4, 1, +1), (5, 0, -1), (6, 0, +1))


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
    """Return A u, with A given by `bands` [7, N] on grid `shape` = (nx, ny, nz)."""
    nx, ny, nz = shape
    per_zyx = (periodic[2], periodic[1], periodic[0])
    u3 = np.asarray(u, dtype=np.float64).reshape(nz, ny, nx)
    b = bands.reshape(7, nz, ny, nx)
    y = b[0] * u3
    for band, axis, off in NEIGHBOURS:
        y = y + b[band] * neighbour_values(u3, axis, off, per_zyx[axis])
    return y.reshape(-1)


def residual(bands, shape, periodic, b, x):
    """b - A x."""
    return b - apply(bands, shape, periodic, x)
