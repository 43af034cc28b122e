"""fab: restarted, sketched, window-truncated Krylov approximation of f(A) b on MI355X.

Thin Python binding of libfab (include/fab.h): argument marshalling over torch device
tensors, nothing else.  Every step of the method runs in the HIP kernels of the library;
if ``libfab.so`` is not built, importing the binding's entry points raises.

    ctx = fab.Context()
    A = fab.CSROperator.from_arrays(ctx, rowptr, colind, vals)     # torch/numpy, copied to the GPU
    x, info = fab.solve(A, b, "exp", t=1e-3, m=20, k=2, d=80, zeta=8, tol=1e-10)
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import FabError, fab_info, fab_params

FUN = {"exp": 0, "invsqrt": 1, "phi1": 2, "cos_sqrt": 3}
SKETCH_APPLY_WORK_PER_ROW = 16384  # fab_sketch_apply's workspace: 2048 block partials per sketch row
METHOD = {"sketched": 0, "plain": 1, "growing": 2}
DTYPE = {torch.float64: 0, torch.float32: 1}

__all__ = ["Context", "CSROperator", "Params", "solve", "solve_batched", "solve_ragged", "workspace_size", "spmv", "sketch_apply",
           "sketch_table", "cycle_debug", "dot", "batch_group", "divergence_limit", "ExpAction", "exp_action", "timing_enable", "timing_read",
           "FabError", "lib_path"]


def lib_path() -> str:
    return _lib.LIB_PATH


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A libfab context bound to one GPU and to the current torch stream of that GPU."""

    def __init__(self, device=None, stream: torch.cuda.Stream | None = None):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("fab needs a ROCm GPU; torch.cuda.is_available() is False")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _lib.check(self.lib.fab_create(ctypes.byref(h), ctypes.c_void_p(s.cuda_stream)), "fab_create", ok=(0,))
        self.handle = h
        self._ws = {}

    def workspace(self, nbytes: int) -> torch.Tensor:
        """A cached device byte buffer of at least nbytes (256-byte aligned)."""
        buf = self._ws.get("main")
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            assert buf.data_ptr() % 256 == 0
            self._ws["main"] = buf
        return buf

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fab_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CSROperator:
    """A CSR matrix on the device (int32 indices, FP64 or FP32 values); libfab borrows the arrays."""

    def __init__(self, ctx: Context, rowptr: torch.Tensor, colind: torch.Tensor, vals: torch.Tensor):
        assert rowptr.dtype == torch.int32 and colind.dtype == torch.int32 and vals.dtype in DTYPE
        assert rowptr.is_cuda and colind.is_cuda and vals.is_cuda
        self.ctx, self.rowptr, self.colind, self.vals = ctx, rowptr.contiguous(), colind.contiguous(), vals.contiguous()
        self.n = rowptr.numel() - 1
        self.nnz = colind.numel()
        self.dtype = vals.dtype
        h = ctypes.c_void_p()
        _lib.check(ctx.lib.fab_csr_create(ctx.handle, self.n, self.nnz, _ptr(self.rowptr), _ptr(self.colind),
                                          _ptr(self.vals), DTYPE[self.dtype], ctypes.byref(h)),
                   "fab_csr_create", ok=(0,))
        self.handle = h

    def transpose(self) -> "CSROperator":
        """A^T on the device (fab_op_transpose); the library owns its arrays."""
        h = ctypes.c_void_p()
        _lib.check(self.ctx.lib.fab_op_transpose(self.ctx.handle, self.handle, ctypes.byref(h)),
                   "fab_op_transpose", ok=(0,))
        op = CSROperator.__new__(CSROperator)
        op.ctx, op.rowptr, op.colind, op.vals = self.ctx, None, None, None
        op.n, op.nnz, op.dtype, op.handle = self.n, self.nnz, self.dtype, h
        return op

    def index_bytes(self) -> int:
        """Bytes per column index the products read (2 with the 16-bit tile offsets, else 4)."""
        v = ctypes.c_int32()
        _lib.check(self.ctx.lib.fab_op_index_bytes(self.handle, ctypes.byref(v)), "fab_op_index_bytes", ok=(0,))
        return v.value

    def store_policy(self, policy: str = "size") -> bool:
        """Cache policy of a single solve's step stores: "size" (non-temporal when the CSR arrays
        exceed the 256 MB memory-side cache), "default" or "streaming".  Returns True when the
        stores are non-temporal.  Timing only: results do not change."""
        code = {"size": 0, "default": 1, "streaming": 2}[policy]
        v = ctypes.c_int32()
        _lib.check(self.ctx.lib.fab_op_store_policy(self.handle, code, ctypes.byref(v)), "fab_op_store_policy",
                   ok=(0,))
        return bool(v.value)

    def arrays(self):
        """Copies of the operator's (rowptr, colind, vals) as device tensors."""
        dev = self.ctx.device
        rp = torch.empty(self.n + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        va = torch.empty(max(self.nnz, 1), dtype=self.dtype, device=dev)
        _lib.check(self.ctx.lib.fab_op_copy_arrays(self.ctx.handle, self.handle, _ptr(rp), _ptr(ci), _ptr(va)),
                   "fab_op_copy_arrays", ok=(0,))
        return rp, ci[:self.nnz], va[:self.nnz]

    @classmethod
    def from_arrays(cls, ctx: Context, rowptr, colind, vals, dtype=None):
        dev = ctx.device
        rp = torch.as_tensor(np.asarray(rowptr, dtype=np.int32)).to(dev)
        ci = torch.as_tensor(np.asarray(colind, dtype=np.int32)).to(dev)
        v = torch.as_tensor(np.asarray(vals))
        if dtype is not None:
            v = v.to(dtype)
        return cls(ctx, rp, ci, v.to(dev))

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.fab_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def Params(m=20, k=2, d=80, zeta=8, seed=1, tol=1e-10, max_cycles=100, method="sketched", n_quad=0,
           spec=None) -> fab_params:
    lo, hi = (0.0, 0.0) if spec is None else (float(spec[0]), float(spec[1]))
    return fab_params(int(m), int(k), int(d), int(zeta), int(seed) & (2 ** 64 - 1), float(tol), int(max_cycles),
                      METHOD[method] if isinstance(method, str) else int(method), int(n_quad), lo, hi)


def workspace_size(op: CSROperator, p: fab_params, nt: int = 1) -> int:
    nb = ctypes.c_size_t()
    _lib.check(op.ctx.lib.fab_workspace_size(op.handle, ctypes.byref(p), int(nt), ctypes.byref(nb)),
               "fab_workspace_size", ok=(0,))
    return int(nb.value)


def solve(op: CSROperator, b: torch.Tensor, fun: str = "exp", t=1e-3, x: torch.Tensor | None = None,
          work: torch.Tensor | None = None, check: bool = True, **kw):
    """x[:, i] = f_i(A) b.  Returns (x, info) with x of shape (n, nt) (FP64) and info a dict.

    ``t`` is a float or a sequence of time points (exp only).  Extra keywords go to ``Params``.
    Negative statuses raise FabError when ``check`` is true.
    """
    ctx = op.ctx
    p = kw.pop("params", None) or Params(**kw)
    ts = np.atleast_1d(np.asarray(t, dtype=np.float64)) if fun != "invsqrt" else np.ones(1)
    nt = len(ts)
    assert b.is_cuda and b.dtype == op.dtype and b.numel() == op.n
    b = b.contiguous()
    if x is None:
        x = torch.empty((nt, op.n), dtype=torch.float64, device=ctx.device)
    assert x.dtype == torch.float64 and x.is_contiguous() and x.numel() == nt * op.n
    nbytes = workspace_size(op, p, nt)
    if work is None:
        work = ctx.workspace(nbytes)
    info = fab_info()
    tarr = (ctypes.c_double * nt)(*ts.tolist())
    st = ctx.lib.fab_solve(ctx.handle, op.handle, FUN[fun], tarr, nt, _ptr(b), _ptr(x), ctypes.byref(p),
                           _ptr(work), work.numel(), ctypes.byref(info))
    if check:
        _lib.check(st, "fab_solve")
    out = {"status": _lib.STATUS.get(info.status, info.status), "code": int(st), "cycles": info.cycles,
           "matvecs": info.matvecs, "est_rel_update": info.est_rel_update,
           "quad_rule_error": info.quad_rule_error, "kappa_T": info.kappa_T, "err_est": info.err_est}
    return x.view(nt, op.n).t(), out


def _info_dict(info, code):
    return {"status": _lib.STATUS.get(info.status, info.status), "code": int(code), "cycles": info.cycles,
            "matvecs": info.matvecs, "est_rel_update": info.est_rel_update, "quad_rule_error": info.quad_rule_error,
            "kappa_T": info.kappa_T, "group": info.group, "err_est": info.err_est}


def solve_batched(op: CSROperator, B: torch.Tensor, fun: str = "exp", t=1e-3, work: torch.Tensor | None = None,
                  check: bool = True, **kw):
    """X[:, r, i] = f_i(A) B[:, r] for the nb columns of B (n x nb) in one batched solve.

    Returns (X, infos): X of shape (n, nb, nt) (FP64, a view of the column-major result), and one
    info dict per column.  Negative statuses raise FabError when ``check`` is true.
    """
    ctx = op.ctx
    p = kw.pop("params", None) or Params(**kw)
    ts = np.atleast_1d(np.asarray(t, dtype=np.float64)) if fun != "invsqrt" else np.ones(1)
    nt = len(ts)
    assert B.is_cuda and B.dtype == op.dtype and B.dim() == 2 and B.shape[0] == op.n
    nb = B.shape[1]
    Bc = B.t().contiguous()                      # member r at Bc[r], leading dimension n
    x = torch.empty((nb * nt, op.n), dtype=torch.float64, device=ctx.device)
    nbytes = ctypes.c_size_t()
    _lib.check(ctx.lib.fab_workspace_size_batched(op.handle, ctypes.byref(p), nt, nb, ctypes.byref(nbytes)),
               "fab_workspace_size_batched", ok=(0,))
    if work is None:
        work = ctx.workspace(nbytes.value)
    infos = (fab_info * nb)()
    tarr = (ctypes.c_double * nt)(*ts.tolist())
    st = ctx.lib.fab_solve_batched(ctx.handle, op.handle, FUN[fun], tarr, nt, nb, _ptr(Bc), op.n, _ptr(x), op.n,
                                   ctypes.byref(p), _ptr(work), work.numel(), infos)
    if check:
        _lib.check(st, "fab_solve_batched")
    return x.view(nb, nt, op.n).permute(2, 0, 1), [_info_dict(infos[r], st) for r in range(nb)]


def solve_ragged(ops, bs, fun: str = "exp", t=1e-3, work: torch.Tensor | None = None, check: bool = True,
                 xs=None, **kw):
    """[f(A_i) b_i] for operators of uneven size in one ragged solve (fab_solve_ragged).

    ``ops`` and ``bs`` are equal-length lists (b_i on the device, in A_i's dtype).  Returns
    (xs, infos): xs[i] of shape (n_i, nt) FP64, and one info dict per operator.  ``xs`` may pass in
    the outputs of an earlier call (or tensors of that shape and layout) to be written again: the
    captured ragged graph is keyed on the output addresses among other things, so a repeated call on
    the same outputs replays it without capturing it again.
    """
    ctx = ops[0].ctx
    nops = len(ops)
    assert len(bs) == nops and all(op.ctx is ctx for op in ops)
    p = kw.pop("params", None) or Params(**kw)
    ts = np.atleast_1d(np.asarray(t, dtype=np.float64)) if fun != "invsqrt" else np.ones(1)
    nt = len(ts)
    bs = [b.contiguous() for b in bs]
    for op, b in zip(ops, bs):
        assert b.is_cuda and b.dtype == op.dtype and b.numel() == op.n
    if xs is None:
        xs = [torch.empty((nt, op.n), dtype=torch.float64, device=ctx.device) for op in ops]
    else:
        assert len(xs) == nops
        xs = [v.t() for v in xs]
        for op, v in zip(ops, xs):
            assert v.is_cuda and v.dtype == torch.float64 and v.shape == (nt, op.n) and v.is_contiguous()
    handles = (ctypes.c_void_p * nops)(*[op.handle.value for op in ops])
    nbytes = ctypes.c_size_t()
    _lib.check(ctx.lib.fab_workspace_size_ragged(nops, handles, ctypes.byref(p), nt, ctypes.byref(nbytes)),
               "fab_workspace_size_ragged", ok=(0,))
    if work is None:
        work = ctx.workspace(nbytes.value)
    infos = (fab_info * nops)()
    tarr = (ctypes.c_double * nt)(*ts.tolist())
    bp = (ctypes.c_void_p * nops)(*[b.data_ptr() for b in bs])
    xp = (ctypes.c_void_p * nops)(*[x.data_ptr() for x in xs])
    st = ctx.lib.fab_solve_ragged(ctx.handle, nops, handles, FUN[fun], tarr, nt, bp, xp, ctypes.byref(p), _ptr(work),
                                  work.numel(), infos)
    if check:
        _lib.check(st, "fab_solve_ragged")
    return [x.t() for x in xs], [_info_dict(infos[i], st) for i in range(nops)]


def divergence_limit(ctx: Context, limit: float = 1e8):
    """Relative increment above which a solve is abandoned with FAB_E_DIVERGED (test hook; default 1e8)."""
    _lib.check(ctx.lib.fab_divergence_limit(ctx.handle, float(limit)), "fab_divergence_limit", ok=(0,))


def batch_group(ctx: Context, G: int = 0):
    """Pin the members per block of the batched kernel (1, 4, 8 or 16); 0 = autotune (default)."""
    _lib.check(ctx.lib.fab_batch_group(ctx.handle, int(G)), "fab_batch_group", ok=(0,))


def timing_enable(ctx: Context, on=True):
    """HIP-event timing: True/1 = each product, update and step loop; 2 = the step loops only; False/0 = off."""
    mode = int(on) if not isinstance(on, bool) else (1 if on else 0)
    _lib.check(ctx.lib.fab_timing_enable(ctx.handle, mode), "fab_timing_enable", ok=(0,))


def timing_read(ctx: Context) -> dict:
    """Accumulated HIP-event durations of the SpMV+sketch kernel, the window updates and the step loops (ms)."""
    a, b_, c, d = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    e, f = ctypes.c_double(), ctypes.c_int64()
    _lib.check(ctx.lib.fab_timing_read(ctx.handle, ctypes.byref(a), ctypes.byref(b_), ctypes.byref(c),
                                       ctypes.byref(d), ctypes.byref(e), ctypes.byref(f)), "fab_timing_read", ok=(0,))
    return {"spmv_ms": a.value, "spmv_launches": b_.value, "loop_ms": c.value, "loop_steps": d.value,
            "update_ms": e.value, "update_launches": f.value}


def spmv(op: CSROperator, xv: torch.Tensor) -> torch.Tensor:
    y = torch.empty_like(xv)
    _lib.check(op.ctx.lib.fab_spmv(op.ctx.handle, op.handle, _ptr(xv.contiguous()), _ptr(y), None, 0),
               "fab_spmv", ok=(0,))
    return y


def sketch_apply(ctx: Context, xv: torch.Tensor, d: int, zeta: int, seed: int) -> torch.Tensor:
    out = torch.empty(d, dtype=torch.float64, device=ctx.device)
    ws = torch.empty(SKETCH_APPLY_WORK_PER_ROW * d + 256, dtype=torch.uint8, device=ctx.device)
    _lib.check(ctx.lib.fab_sketch_apply(ctx.handle, xv.numel(), d, zeta, int(seed), DTYPE[xv.dtype],
                                        _ptr(xv.contiguous()), _ptr(out), _ptr(ws), ws.numel()),
               "fab_sketch_apply", ok=(0,))
    return out


def sketch_table(ctx: Context, col0: int, count: int, d: int, zeta: int, seed: int):
    rows = torch.empty((count, zeta), dtype=torch.int32, device=ctx.device)
    signs = torch.empty((count, zeta), dtype=torch.int8, device=ctx.device)
    _lib.check(ctx.lib.fab_sketch_table(ctx.handle, col0, count, d, zeta, int(seed), _ptr(rows), _ptr(signs)),
               "fab_sketch_table", ok=(0,))
    return rows, signs


def cycle_debug(op: CSROperator, v: torch.Tensor, **kw):
    """One cycle from v; returns the basis W, its sketch U, R, the whitening factor T, the projected
    matrix Rt = R_m + r T_m^{-1} t e_m^T in the basis W, and the scalars alpha, beta, h."""
    ctx = op.ctx
    p = Params(**kw)
    m, d = p.m, p.d
    dev = ctx.device
    W = torch.empty((m + 1, op.n), dtype=op.dtype, device=dev)
    U = torch.zeros((m + 1, d), dtype=torch.float64, device=dev)
    R = torch.empty((m, m + 1), dtype=torch.float64, device=dev)
    T = torch.empty((m + 1, m + 1), dtype=torch.float64, device=dev)
    X = torch.empty((m, m), dtype=torch.float64, device=dev)
    scal = (ctypes.c_double * 5)()
    work = ctx.workspace(workspace_size(op, p, 1))
    st = ctx.lib.fab_cycle_debug(ctx.handle, op.handle, _ptr(v.contiguous()), ctypes.byref(p), _ptr(W), _ptr(U),
                                 _ptr(R), _ptr(T), _ptr(X), scal, _ptr(work), work.numel())
    _lib.check(st, "fab_cycle_debug", ok=(0,))
    meff = int(scal[3])
    return {"W": W.t(), "U": U.t(), "R": R.t(), "T": T.t(), "Rt": X.t(), "alpha": scal[0], "beta": scal[1],
            "h": scal[2], "m": meff, "whiten": "cholesky" if scal[4] == 1.0 else "householder"}


def dot(ctx: Context, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """<x, y> of two FP64 device vectors (fab_dot), as a 0-d device tensor."""
    assert x.dtype == torch.float64 and y.dtype == torch.float64 and x.numel() == y.numel()
    out = torch.empty((), dtype=torch.float64, device=ctx.device)
    _lib.check(ctx.lib.fab_dot(ctx.handle, x.numel(), _ptr(x.contiguous()), _ptr(y.contiguous()), _ptr(out)),
               "fab_dot", ok=(0,))
    return out


class ExpAction(torch.autograd.Function):
    """x = exp(-t A) b with gradients for b and t (FP64 operators).

    Backward, for an upstream gradient c = dL/dx:
      dL/db = exp(-t A^T) c   (adjoint identity <c, f(A) b> = <f(A^T) c, b>): the same restarted
                              sketched Krylov solve, run on A^T, which recomputes its own basis;
      dL/dt = -<c, A x>       (d/dt exp(-t A) b = -A exp(-t A) b): one product with A and a dot.
    Nothing of the forward basis is stored; only x is kept.
    """

    @staticmethod
    def forward(fctx, b, t, op, op_t, params):
        tv = float(t)
        x, info = solve(op, b, "exp", t=tv, params=params)
        x = x[:, 0].contiguous()
        fctx.save_for_backward(x)
        fctx.op, fctx.op_t, fctx.params, fctx.tv = op, op_t, params, tv
        fctx.t_shape = t.shape if isinstance(t, torch.Tensor) else None
        fctx.t_device = t.device if isinstance(t, torch.Tensor) else None
        return x

    @staticmethod
    def backward(fctx, gx):
        (x,) = fctx.saved_tensors
        gb = gt = None
        gx = gx.contiguous()
        if fctx.needs_input_grad[0]:
            y, _ = solve(fctx.op_t, gx, "exp", t=fctx.tv, params=fctx.params)
            gb = y[:, 0]
        if fctx.needs_input_grad[1]:
            ax = spmv(fctx.op, x)
            g = -dot(fctx.op.ctx, gx, ax)
            gt = g.to(fctx.t_device).reshape(fctx.t_shape)
        return gb, gt, None, None, None


def exp_action(op: CSROperator, b: torch.Tensor, t, op_t: CSROperator | None = None, **kw) -> torch.Tensor:
    """Differentiable exp(-t A) b (see ExpAction); op_t defaults to op.transpose()."""
    assert op.dtype == torch.float64, "the differentiable action is provided for FP64 operators"
    if op_t is None:
        op_t = op.transpose()
    if not isinstance(t, torch.Tensor):
        t = torch.tensor(float(t), dtype=torch.float64)
    return ExpAction.apply(b, t, op, op_t, Params(**kw))
