"""Independent test helpers: a face-by-face sparse assembly of the finite-volume
operator (written from the definition, not from the banded storage) and the
closed-form eigenpairs of the unit-coefficient operator."""
import itertools

import numpy as np
import scipy.sparse as sp


def csr_assemble(kcell, vol, widths, bc):
    """A = diag(1/vol) L assembled by looping over cell faces; kcell, vol have
    shape (nz, ny, nx); widths = (dx, dy, dz); bc as for workloads.assemble."""
    nz, ny, nx = kcell.shape
    dims = (nx, ny, nz)
    w = [np.asarray(a, float) for a in widths]
    N = nx * ny * nz
    rows, cols, vals = [], [], []

    def idx(c):
        return c[0] + nx * (c[1] + ny * c[2])

    def kval(c):
        return kcell[c[2], c[1], c[0]]

    def area(c, ax):
        other = [a for a in range(3) if a != ax]
        return w[other[0]][c[other[0]]] * w[other[1]][c[other[1]]]

    names = "xyz"
    for c in itertools.product(range(nx), range(ny), range(nz)):
        for ax in range(3):
            rule = bc[names[ax]]
            n = dims[ax]
            # + face of cell c
            nb = list(c)
            nb[ax] += 1
            if nb[ax] == n:
                if rule == 'periodic':
                    nb[ax] = 0
                else:
                    if rule[1] == 'dirichlet':
                        T = kval(c) * area(c, ax) / (0.5 * w[ax][c[ax]])
                        rows.append(idx(c)); cols.append(idx(c)); vals.append(T)
                    nb = None
            if nb is not None:
                kf = 2 * kval(c) * kval(nb) / (kval(c) + kval(nb))
                d = 0.5 * (w[ax][c[ax]] + w[ax][nb[ax]])
                af = 0.5 * (area(c, ax) + area(tuple(nb), ax))
                T = kf * af / d
                i, j = idx(c), idx(nb)
                rows += [i, j, i, j]
                cols += [i, j, j, i]
                vals += [T, T, -T, -T]
            # - boundary face (Dirichlet only)
            if c[ax] == 0 and rule != 'periodic' and rule[0] == 'dirichlet':
                T = kval(c) * area(c, ax) / (0.5 * w[ax][c[ax]])
                rows.append(idx(c)); cols.append(idx(c)); vals.append(T)
    L = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    v = np.array([vol[c[2], c[1], c[0]] for c in itertools.product(range(nx), range(ny), range(nz))])
    order = [idx(c) for c in itertools.product(range(nx), range(ny), range(nz))]
    vv = np.empty(N)
    vv[order] = v
    return sp.diags(1.0 / vv) @ L


def mode_1d(rule, n, p):
    """Closed-form eigenvector and eigenvalue of the 1-D unit cell-centred
    operator: Dirichlet (half-cell boundary face) sin(pi p (i+1/2)/n), Neumann
    cos(pi p (i+1/2)/n), both with lambda = 4 sin^2(pi p / 2n); periodic
    cos(2 pi p i / n) with lambda = 4 sin^2(pi p / n)."""
    i = np.arange(n)
    if rule == 'periodic':
        return np.cos(2 * np.pi * p * i / n), 4 * np.sin(np.pi * p / n) ** 2
    lam = 4 * np.sin(np.pi * p / (2 * n)) ** 2
    if rule == ('dirichlet', 'dirichlet'):
        return np.sin(np.pi * p * (i + 0.5) / n), lam
    if rule == ('neumann', 'neumann'):
        return np.cos(np.pi * p * (i + 0.5) / n), lam
    raise ValueError(rule)


def mode_range(rule, n):
    if rule == ('dirichlet', 'dirichlet'):
        return range(1, n + 1)
    return range(0, n)


def mode_3d(bc, shape, ps):
    """Tensor-product eigenvector (flattened x fastest) and its eigenvalue."""
    nx, ny, nz = shape
    ux, lx = mode_1d(bc['x'], nx, ps[0])
    uy, ly = mode_1d(bc['y'], ny, ps[1])
    uz, lz = mode_1d(bc['z'], nz, ps[2])
    u = uz[:, None, None] * uy[None, :, None] * ux[None, None, :]
    return u.reshape(-1), lx + ly + lz
