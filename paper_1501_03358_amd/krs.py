"""Python binding of the krs C-ABI (include/krs.h).

Argument marshalling only: every operation runs in the HIP library
``libkrs.so`` built in this directory.  PyTorch supplies device memory
(``tensor.data_ptr()``) and the HIP stream of the current device.  There is
no fallback: when the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkrs.so")

# status codes
OK, NOT_CONVERGED, BREAKDOWN, DIVERGED = 0, 1, 2, 3
ERR_ARG, ERR_HIP, ERR_WORKSPACE, ERR_STATE, ERR_EIG = -1, -2, -3, -4, -5
F64, F32 = 0, 1
SOLVER_GMRES, SOLVER_RGCROT, SOLVER_RBICGSTAB, SOLVER_IR, SOLVER_RGCROT_T = 0, 1, 2, 3, 4
RECYCLE_HARMONIC, RECYCLE_GCROT = 0, 1
PC_NONE, PC_JACOBI, PC_SCHWARZ_JACOBI = 0, 1, 2
LOCAL_JACOBI, LOCAL_SSOR = 0, 1
FLAG_TRUST_ESTIMATE = 1
FLAG_HOST_LOOP = 2
FLAG_GRAPH = 4
FLAG_LEFT_PRECOND = 8

EXPORTS = (
    "krs_create", "krs_destroy", "krs_last_error", "krs_set_stream", "krs_matrix_create",
    "krs_matrix_create_19pt",
    "krs_matrix_destroy", "krs_precond_create", "krs_precond_workspace_size",
    "krs_precond_refresh", "krs_precond_destroy", "krs_recycle_create", "krs_recycle_destroy", "krs_recycle_dim",
    "krs_recycle_set_dim", "krs_recycle_mark_stale", "krs_workspace_size", "krs_stencil_apply", "krs_precond_apply",
    "krs_operator_apply", "krs_gmres", "krs_rgcrot_solve", "krs_rbicgstab_solve",
    "krs_rbicgstab_solve_noalloc", "krs_recycle_update",
    "krs_hybrid_solve", "krs_ir_solve", "krs_ir_solve_batched", "krs_version", "krs_timing_enable", "krs_timing_classes", "krs_timing_reset",
    "krs_timing_read",
)


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("periodic", ctypes.c_int32 * 3)]


class PrecondDesc(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("tile", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("local_sweeps", ctypes.c_int32), ("global_sweeps", ctypes.c_int32),
                ("local_solver", ctypes.c_int32), ("omega_local", ctypes.c_double),
                ("omega_global", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("k", ctypes.c_int32), ("update_recycle", ctypes.c_int32),
                ("inner_solver", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_matvecs", ctypes.c_int64), ("div_factor", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("history", ctypes.POINTER(ctypes.c_double)),
                ("history_cap", ctypes.c_int64), ("switch_back", ctypes.c_double),
                ("recycle_rule", ctypes.c_int32), ("gcrot_kt", ctypes.c_int32),
                ("gcrot_s", ctypes.c_int32), ("gcrot_p", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("eig_ties", ctypes.c_int32),
                ("matvecs", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("cycles", ctypes.c_int64), ("outer", ctypes.c_int64),
                ("history_len", ctypes.c_int64), ("rel_res_true", ctypes.c_double),
                ("rel_res_est", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("host_eig_ms", ctypes.c_double), ("bytes_model", ctypes.c_double),
                ("second_passes", ctypes.c_int64), ("solver", ctypes.c_int64),
                ("refreshed", ctypes.c_int64), ("breakdown_site", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_LIB = None
P = ctypes.c_void_p


class IrSystem(ctypes.Structure):
    _fields_ = [("A64", ctypes.c_void_p), ("A32", ctypes.c_void_p), ("M32", ctypes.c_void_p),
                ("rec32", ctypes.c_void_p), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
                ("stats", ctypes.POINTER(Stats))]


BATCH_WORKSPACE_BYTES = 64 << 10


def _declare(L):
    i32, i64, dbl, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "krs_create": (i32, [ctypes.POINTER(P), P]),
        "krs_destroy": (None, [P]),
        "krs_last_error": (ctypes.c_char_p, [P]),
        "krs_set_stream": (i32, [P, P]),
        "krs_matrix_create": (i32, [P, ctypes.POINTER(Grid), i32, P, ctypes.POINTER(P)]),
        "krs_matrix_create_19pt": (i32, [P, ctypes.POINTER(Grid), i32, P, ctypes.POINTER(P)]),
        "krs_matrix_destroy": (None, [P]),
        "krs_precond_create": (i32, [P, P, ctypes.POINTER(PrecondDesc), P, sz, ctypes.POINTER(P)]),
        "krs_precond_workspace_size": (sz, [P, ctypes.POINTER(PrecondDesc)]),
        "krs_precond_refresh": (i32, [P, P]),
        "krs_precond_destroy": (None, [P]),
        "krs_recycle_create": (i32, [P, i64, i32, i32, P, P, i64, ctypes.POINTER(P)]),
        "krs_recycle_destroy": (None, [P]),
        "krs_recycle_dim": (i32, [P]),
        "krs_recycle_set_dim": (i32, [P, i32]),
        "krs_recycle_mark_stale": (i32, [P]),
        "krs_workspace_size": (i32, [i32, i64, i32, i32, i32, ctypes.POINTER(sz)]),
        "krs_stencil_apply": (i32, [P, P, P, P, dbl, dbl, P]),
        "krs_precond_apply": (i32, [P, P, P, P]),
        "krs_operator_apply": (i32, [P, P, P, P, P, P]),
        "krs_gmres": (i32, [P, P, P, P, P, ctypes.POINTER(Opts), P, sz, ctypes.POINTER(Stats)]),
        "krs_rgcrot_solve": (i32, [P, P, P, P, P, P, ctypes.POINTER(Opts), P, sz,
                                   ctypes.POINTER(Stats)]),
        "krs_rbicgstab_solve": (i32, [P, P, P, P, P, P, ctypes.POINTER(Opts), P, sz,
                                      ctypes.POINTER(Stats)]),
        "krs_rbicgstab_solve_noalloc": (i32, [P, P, P, P, P, P, ctypes.POINTER(Opts),
                                              ctypes.POINTER(Stats)]),
        "krs_recycle_update": (i32, [P, P, P, P, P, sz]),
        "krs_hybrid_solve": (i32, [P, P, P, P, i32, i32, P, P, ctypes.POINTER(Opts), P, sz,
                                   ctypes.POINTER(Stats)]),
        "krs_ir_solve": (i32, [P, P, P, P, P, P, P, ctypes.POINTER(Opts), P, sz,
                               ctypes.POINTER(Stats)]),
        "krs_ir_solve_batched": (i32, [P, i32, ctypes.POINTER(IrSystem), ctypes.POINTER(Opts), P,
                                       sz]),
        "krs_version": (ctypes.c_char_p, []),
        "krs_timing_enable": (i32, [P, i32]),
        "krs_timing_classes": (i32, [P, ctypes.c_uint]),
        "krs_timing_reset": (i32, [P]),
        "krs_timing_read": (i32, [P, i32, ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                  ctypes.POINTER(dbl)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


def lib():
    """Load libkrs.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkrs.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _LIB = L
    return _LIB


class KrsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"krs error {code}: {msg}")
        self.code = code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dt(t):
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("tensors must be float64 or float32")


LD_PAD = 1088


def vec_ld(n):
    """Leading dimension of U and C (the library's rule for its own
    multi-vectors): N rounded up to 64 values plus a pad, so that the columns
    do not all start at the same offset modulo a large power of two."""
    return (n + 63) // 64 * 64 + LD_PAD


class Context:
    def __init__(self, device=None, stream=None):
        self.device = torch.device(device or "cuda:0")
        if self.device.type != "cuda":
            raise RuntimeError("krs needs a GPU device")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        torch.cuda.set_device(self.device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        h = P()
        rc = lib().krs_create(ctypes.byref(h), ctypes.c_void_p(s.cuda_stream))
        if rc != OK:
            raise KrsError(rc, "krs_create failed")
        self.h = h

    def check(self, rc, allow_outcome=False):
        if rc < 0 or (rc > 0 and not allow_outcome):
            raise KrsError(rc, lib().krs_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().krs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """7- or 19-band operator on an (nx, ny, nz) grid; `bands` is a [7, N] or
    [19, N] device tensor (krs_matrix_create / krs_matrix_create_19pt)."""

    def __init__(self, ctx, shape, periodic, bands):
        if not bands.is_cuda or not bands.is_contiguous() or bands.shape[0] not in (7, 19):
            raise ValueError("bands must be a contiguous [7, N] or [19, N] device tensor")
        self.ctx, self.bands = ctx, bands
        self.shape = tuple(int(s) for s in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.dtype = bands.dtype
        g = Grid(self.shape[0], self.shape[1], self.shape[2],
                 (ctypes.c_int32 * 3)(*[1 if p else 0 for p in periodic]))
        h = P()
        create = lib().krs_matrix_create if bands.shape[0] == 7 else lib().krs_matrix_create_19pt
        ctx.check(create(ctx.h, ctypes.byref(g), _dt(bands), _ptr(bands), ctypes.byref(h)))
        self.h = h

    def __del__(self):
        try:
            lib().krs_matrix_destroy(self.h)
        except Exception:
            pass


class Precond:
    def __init__(self, ctx, A, kind="schwarz", tile=8, overlap=1, local_sweeps=5,
                 omega_local=6.0 / 7.0, global_sweeps=1, omega_global=6.0 / 7.0,
                 local_solver="jacobi"):
        t = {"none": PC_NONE, "jacobi": PC_JACOBI, "schwarz": PC_SCHWARZ_JACOBI}[kind]
        ls = {"jacobi": LOCAL_JACOBI, "ssor": LOCAL_SSOR}[local_solver]
        self.ctx, self.A = ctx, A
        self.desc = PrecondDesc(t, tile, overlap, local_sweeps, global_sweeps, ls, omega_local,
                                omega_global)
        nbytes = lib().krs_precond_workspace_size(A.h, ctypes.byref(self.desc))
        self.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=A.bands.device)
        h = P()
        ctx.check(lib().krs_precond_create(ctx.h, A.h, ctypes.byref(self.desc), _ptr(self.ws),
                                           nbytes, ctypes.byref(h)))
        self.h = h

    def refresh(self):
        """Rebuild the stored coefficients after the matrix bands changed."""
        return self.ctx.check(lib().krs_precond_refresh(self.ctx.h, self.h))

    def __del__(self):
        try:
            lib().krs_precond_destroy(self.h)
        except Exception:
            pass


class Recycle:
    """Recycle space (U, C): kmax columns each, leading dimension vec_ld(N)."""

    def __init__(self, ctx, n, kmax, dtype, device=None):
        self.ctx, self.n, self.kmax = ctx, n, kmax
        self.ld = vec_ld(n)
        dev = device or ctx.device
        self.U = torch.zeros(kmax, self.ld, dtype=dtype, device=dev)
        self.C = torch.zeros(kmax, self.ld, dtype=dtype, device=dev)
        h = P()
        ctx.check(lib().krs_recycle_create(ctx.h, n, kmax, _dt(self.U), _ptr(self.U), _ptr(self.C),
                                           self.ld, ctypes.byref(h)))
        self.h = h

    @property
    def dim(self):
        return lib().krs_recycle_dim(self.h)

    def set_dim(self, k):
        rc = lib().krs_recycle_set_dim(self.h, k)
        if rc != OK:
            raise KrsError(rc, "bad recycle dimension")

    def mark_stale(self):
        """A or M changed: the next hybrid solve re-forms C = qr(A~ U).Q first."""
        rc = lib().krs_recycle_mark_stale(self.h)
        if rc != OK:
            raise KrsError(rc, "krs_recycle_mark_stale")

    def views(self):
        k = self.dim
        return self.U[:k, :self.n].T, self.C[:k, :self.n].T

    def __del__(self):
        try:
            lib().krs_recycle_destroy(self.h)
        except Exception:
            pass


def workspace_size(solver, n, m, k, dtype):
    out = ctypes.c_size_t()
    dt = F64 if dtype == torch.float64 else F32
    rc = lib().krs_workspace_size(solver, n, m, k, dt, ctypes.byref(out))
    if rc != OK:
        raise KrsError(rc, "krs_workspace_size")
    return out.value


class Workspace:
    """Device scratch buffer, grown on demand."""

    def __init__(self, device):
        self.device = device
        self.buf = torch.empty(0, dtype=torch.uint8, device=device)

    def get(self, nbytes):
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


def make_opts(m=30, k=20, tol=1e-8, max_matvecs=2000, update_recycle=True, inner_solver=None,
              div_factor=1e2, inner_tol=1e-5, max_outer=20, history=None, flags=0,
              switch_back=0.0, recycle_rule=RECYCLE_HARMONIC, gcrot_kt=0, gcrot_s=0, gcrot_p=1):
    o = Opts()
    o.switch_back = switch_back
    o.recycle_rule, o.gcrot_kt, o.gcrot_s, o.gcrot_p = recycle_rule, gcrot_kt, gcrot_s, gcrot_p
    o.flags = flags
    o.m, o.k, o.update_recycle = m, k, 1 if update_recycle else 0
    o.inner_solver = SOLVER_RGCROT if inner_solver is None else inner_solver
    o.tol, o.max_matvecs, o.div_factor = tol, max_matvecs, div_factor
    o.inner_tol, o.max_outer = inner_tol, max_outer
    if history is not None:
        o.history = history.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.history_cap = history.size
    return o


# --------------------------------------------------------------------------
# entry points (same names as the C-ABI)
# --------------------------------------------------------------------------

def stencil_apply(ctx, A, x, y, alpha=1.0, beta=0.0, b=None):
    check_vec(x, A.n, A.dtype, ctx.device, "x")
    check_vec(y, A.n, A.dtype, ctx.device, "y")
    if b is not None:
        check_vec(b, A.n, A.dtype, ctx.device, "b")
    return ctx.check(lib().krs_stencil_apply(ctx.h, A.h, _ptr(x), _ptr(y), alpha, beta, _ptr(b)))


def precond_apply(ctx, M, r, z):
    check_vec(r, M.A.n, M.A.dtype, ctx.device, "r")
    check_vec(z, M.A.n, M.A.dtype, ctx.device, "z")
    return ctx.check(lib().krs_precond_apply(ctx.h, M.h, _ptr(r), _ptr(z)))


def operator_apply(ctx, A, M, v, w, tmp):
    for t, name in ((v, "v"), (w, "w"), (tmp, "tmp")):
        check_vec(t, A.n, A.dtype, ctx.device, name)
    return ctx.check(lib().krs_operator_apply(ctx.h, A.h, _h(M), _ptr(v), _ptr(w), _ptr(tmp)))


def _h(obj):
    return None if obj is None else obj.h


def check_vec(t, n, dtype, device, name):
    """Raises ValueError unless `t` is a contiguous tensor of `n` values of
    `dtype` on `device` (the library reads and writes exactly n values
    through the raw pointer, so anything else would be out of bounds)."""
    if t is None:
        raise ValueError(f"{name} is None")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, the matrix needs {dtype}")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} values, the matrix has {n} unknowns")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != torch.device(device):
        raise ValueError(f"{name} is on {t.device}, the context on {device}")


def check_ws(ws, nbytes, device):
    """Raises ValueError unless `ws` is a contiguous uint8 buffer of at least
    `nbytes` bytes on `device`."""
    if ws is None or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 tensor")
    if ws.numel() < nbytes:
        raise ValueError(f"workspace has {ws.numel()} bytes, {nbytes} needed")
    if ws.device != torch.device(device):
        raise ValueError(f"workspace is on {ws.device}, the context on {device}")


def _check_solve(ctx, A, b, x, ws, dtype=None):
    dt = A.dtype if dtype is None else dtype
    check_vec(b, A.n, dt, ctx.device, "b")
    check_vec(x, A.n, dt, ctx.device, "x")
    check_ws(ws, 1, ctx.device)


def gmres(ctx, A, M, b, x, opts, ws, stats=None):
    _check_solve(ctx, A, b, x, ws)
    st = stats or Stats()
    rc = lib().krs_gmres(ctx.h, A.h, _h(M), _ptr(b), _ptr(x), ctypes.byref(opts), _ptr(ws),
                         ws.numel(), ctypes.byref(st))
    ctx.check(rc, allow_outcome=True)
    return rc, st


def rgcrot_solve(ctx, A, M, rec, b, x, opts, ws, stats=None):
    _check_solve(ctx, A, b, x, ws)
    st = stats or Stats()
    rc = lib().krs_rgcrot_solve(ctx.h, A.h, _h(M), _h(rec), _ptr(b), _ptr(x), ctypes.byref(opts),
                                _ptr(ws), ws.numel(), ctypes.byref(st))
    ctx.check(rc, allow_outcome=True)
    return rc, st


def rbicgstab_solve(ctx, A, M, rec, b, x, opts, ws, stats=None):
    _check_solve(ctx, A, b, x, ws)
    st = stats or Stats()
    rc = lib().krs_rbicgstab_solve(ctx.h, A.h, _h(M), _h(rec), _ptr(b), _ptr(x),
                                   ctypes.byref(opts), _ptr(ws), ws.numel(), ctypes.byref(st))
    ctx.check(rc, allow_outcome=True)
    return rc, st


def rbicgstab_solve_noalloc(ctx, A, M, rec, b, x, opts, stats=None):
    """krs_rbicgstab_solve with the library's static per-GPU workspace
    (no workspace argument, no allocation)."""
    check_vec(b, A.n, A.dtype, ctx.device, "b")
    check_vec(x, A.n, A.dtype, ctx.device, "x")
    st = stats or Stats()
    rc = lib().krs_rbicgstab_solve_noalloc(ctx.h, A.h, _h(M), _h(rec), _ptr(b), _ptr(x),
                                           ctypes.byref(opts), ctypes.byref(st))
    ctx.check(rc, allow_outcome=True)
    return rc, st


def recycle_update(ctx, A, M, rec, ws):
    check_ws(ws, 1, ctx.device)
    return ctx.check(lib().krs_recycle_update(ctx.h, A.h, _h(M), rec.h, _ptr(ws), ws.numel()))


def hybrid_solve(ctx, A, M, rec, step, n_switch, b, x, opts, ws, stats=None):
    _check_solve(ctx, A, b, x, ws)
    st = stats or Stats()
    rc = lib().krs_hybrid_solve(ctx.h, A.h, _h(M), rec.h, step, n_switch, _ptr(b), _ptr(x),
                                ctypes.byref(opts), _ptr(ws), ws.numel(), ctypes.byref(st))
    ctx.check(rc, allow_outcome=True)
    return rc, st


def ir_solve(ctx, A64, A32, M32, rec32, b, x, opts, ws, stats=None):
    _check_solve(ctx, A64, b, x, ws, torch.float64)
    st = stats or Stats()
    rc = lib().krs_ir_solve(ctx.h, A64.h, A32.h, _h(M32), _h(rec32), _ptr(b), _ptr(x),
                            ctypes.byref(opts), _ptr(ws), ws.numel(), ctypes.byref(st))
    ctx.check(rc, allow_outcome=True)
    return rc, st


def ir_solve_batched(ctx, systems, opts, ws):
    """krs_ir_solve_batched.  systems: list of (A64, A32, M32, rec32, b, x, ws)
    tuples (the arguments of ir_solve for each system); ws: a device buffer of
    BATCH_WORKSPACE_BYTES.  Returns (rc, [Stats per system])."""
    check_ws(ws, BATCH_WORKSPACE_BYTES, ctx.device)
    arr = (IrSystem * max(1, len(systems)))()
    stats = [Stats() for _ in systems]
    for i, (A64, A32, M32, rec32, b, x, wsi) in enumerate(systems):
        _check_solve(ctx, A64, b, x, wsi, torch.float64)
        arr[i] = IrSystem(A64.h, A32.h, _h(M32), _h(rec32), b.data_ptr(), x.data_ptr(),
                          wsi.data_ptr(), wsi.numel(), ctypes.pointer(stats[i]))
    rc = lib().krs_ir_solve_batched(ctx.h, len(systems), arr, ctypes.byref(opts), _ptr(ws),
                                    ws.numel())
    ctx.check(rc, allow_outcome=True)
    return rc, stats


KERNEL_CLASSES = ("stencil", "residual", "schwarz_local", "jacobi_sweep", "block_dot",
                  "block_dot2", "block_update", "bicg_p", "bicg_sv", "bicg_yr", "gram",
                  "row_transform", "other", "sweep_stencil")


def timing_enable(ctx, on=True):
    return ctx.check(lib().krs_timing_enable(ctx.h, 1 if on else 0))


def timing_classes(ctx, names=None):
    """Time only the named kernel classes (None: every class)."""
    mask = 0xFFFFFFFF if names is None else sum(1 << KERNEL_CLASSES.index(n) for n in names)
    return ctx.check(lib().krs_timing_classes(ctx.h, mask))


def timing_reset(ctx):
    return ctx.check(lib().krs_timing_reset(ctx.h))


def timing_read(ctx):
    """{class: (launches, ms, bytes)} accumulated since the last reset."""
    out = {}
    for i, name in enumerate(KERNEL_CLASSES):
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        ctx.check(lib().krs_timing_read(ctx.h, i, ctypes.byref(n), ctypes.byref(ms),
                                        ctypes.byref(by)))
        out[name] = (n.value, ms.value, by.value)
    return out


def version():
    return lib().krs_version().decode()
