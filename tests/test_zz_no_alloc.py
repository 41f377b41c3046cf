"""The entry point without allocations (krs_rbicgstab_solve_noalloc, static
per-GPU workspace) against krs_rbicgstab_solve with a caller workspace:
same kernels, same fixed reduction trees, so x, the history and the counts
must be bitwise equal.  Two calls in a row, the second on a smaller system
(the static array then holds the first call's values), and the size limit
is refused before any launch."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import Dev

pytestmark = pytest.mark.gpu


def _solve_both(krs, prob, pc, params, kd):
    d = Dev(krs, prob, pc, params, m=1, k=kd, solver=krs.SOLVER_RBICGSTAB)
    rec = None
    if kd:
        rec = krs.Recycle(d.ctx, prob.n, kd, torch.float64)
        U0 = np.random.default_rng(3).standard_normal((kd, prob.n))
        rec.U[:kd, :prob.n] = torch.from_numpy(U0).to(d.dev)
        rec.set_dim(kd)
        ws = torch.empty(krs.workspace_size(krs.SOLVER_RGCROT, prob.n, 1, kd, torch.float64),
                         dtype=torch.uint8, device=d.dev)
        krs.recycle_update(d.ctx, d.A, d.M, rec, ws)
    b = d.vec(next(W.rhs_ar1(prob, 1, extra=9)))
    out = []
    for noalloc in (False, True):
        h = np.zeros(4000)
        x = torch.full((prob.n,), float("nan"), dtype=torch.float64, device=d.dev)
        o = krs.make_opts(tol=1e-9, history=h, max_matvecs=3000)
        if noalloc:
            rc, st = krs.rbicgstab_solve_noalloc(d.ctx, d.A, d.M, rec, b, x, o)
        else:
            rc, st = krs.rbicgstab_solve(d.ctx, d.A, d.M, rec, b, x, o, d.ws)
        out.append((rc, st.iterations, st.rel_res_true, h[:st.history_len].copy(),
                    x.cpu().numpy()))
    return out


def test_noalloc_matches_workspace_entry_point(gpu_lib):
    krs = gpu_lib
    params = dict(W.SCHWARZ_DEFAULT)
    cases = [(W.porous_problem(64, extra=21), "schwarz", params, 12),
             (W.grf_problem(24, extra=22), "jacobi", None, 0)]
    for prob, pc, prm, kd in cases:
        print(f"[noalloc] {prob.name} N={prob.n} {pc} k={kd}", flush=True)
        (rc0, it0, rr0, h0, x0), (rc1, it1, rr1, h1, x1) = _solve_both(krs, prob, pc, prm, kd)
        assert rc0 == krs.OK and rc1 == krs.OK
        assert it0 == it1 and rr0 == rr1
        assert np.array_equal(h0, h1)
        assert np.array_equal(x0, x1)


def test_noalloc_refuses_oversized_and_graph(gpu_lib):
    krs = gpu_lib
    prob = W.porous_problem(96, extra=23)             # 884,736 FP64 unknowns > the static size
    d = Dev(krs, prob, "jacobi", None, m=1, k=1, solver=krs.SOLVER_RBICGSTAB)
    x = d.empty()
    b = d.vec(next(W.rhs_ar1(prob, 1, extra=23)))
    with pytest.raises(krs.KrsError, match="static workspace"):
        krs.rbicgstab_solve_noalloc(d.ctx, d.A, d.M, None, b, x, krs.make_opts())
    with pytest.raises(krs.KrsError, match="GRAPH"):
        krs.rbicgstab_solve_noalloc(d.ctx, d.A, d.M, None, b, x,
                                    krs.make_opts(flags=krs.FLAG_GRAPH))
