"""Shared helpers of the GPU tests (inputs and oracle handles)."""
import numpy as np
import torch

import workloads as W
from oracle import krylov as K
from oracle import precond, stencil

SMALL_SCHWARZ = dict(tile=4, overlap=1, local_sweeps=5, omega_local=6 / 7,
                     global_sweeps=1, omega_global=6 / 7)


def oracle_ops(prob, pc, params=None):
    A = lambda v: stencil.apply(prob.bands, prob.shape, prob.periodic, v)
    Mi = precond.make(prob.bands, prob.shape, prob.periodic, pc, params)
    return A, Mi, (lambda v: A(Mi(v)))


class Dev:
    """A problem's matrix, preconditioner and workspace on the GPU."""

    def __init__(self, krs, prob, pc="jacobi", params=None, dtype=torch.float64, ctx=None,
                 m=30, k=20, solver=None):
        self.krs = krs
        self.prob = prob
        self.dev = torch.device("cuda:0")
        self.ctx = ctx or krs.Context(self.dev)
        self.dtype = dtype
        self.bands = torch.from_numpy(prob.bands).to(self.dev, dtype)
        self.A = krs.Matrix(self.ctx, prob.shape, prob.periodic, self.bands)
        p = dict(params or {})
        self.M = krs.Precond(self.ctx, self.A, pc, **p) if pc != "none" else None
        self.wsb = krs.workspace_size(krs.SOLVER_RGCROT if solver is None else solver, prob.n,
                                      m, k, dtype)
        self.ws = torch.empty(self.wsb, dtype=torch.uint8, device=self.dev)

    def vec(self, a):
        return torch.from_numpy(np.asarray(a)).to(self.dev, self.dtype)

    def empty(self):
        return torch.empty(self.prob.n, dtype=self.dtype, device=self.dev)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def mod_const(x, vol):
    """Remove the volume-weighted mean (solutions of singular systems)."""
    return x - (vol @ x) / vol.sum()


def recycle_to_oracle(rec):
    U, C = rec.views()
    return K.Recycle(U.double().cpu().numpy().copy(), C.double().cpu().numpy().copy())
