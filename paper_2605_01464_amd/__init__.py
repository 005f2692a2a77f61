"""Python binding of libqpinv.so (quaternion Moore--Penrose pseudoinverse on MI355X / gfx950).

Argument marshalling only: every step of a solve runs in the library's HIP kernels.  PyTorch is used
for device memory and streams.  A quaternion matrix is a CUDA (HIP) tensor of shape (4, rows, cols)
holding the planes (s, x, y, z), float32 or float64, with unit stride along columns.

The functions named ``qpinv_*`` mirror the C ABI in include/qpinv.h one to one and return its status
codes; ``solve``, ``step``, ``residuals``, ``qgemm`` and ``features`` are thin conveniences that
raise ``QpinvError`` on failure.  If the shared library has not been built the import of this
module fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from collections.abc import Sequence
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpinv.so")

# ------------------------------------------------------------------------------------------ constants
OK, EINVAL, ENONFINITE, EDIVERGED, ENOTCONVERGED, EHIP, ENOMEM, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
METHOD = {"ns": 0, "hpi": 1, "qsai": 2, "qhpi19": 3, "qrapid": 4}
SCALING = {"power": 0, "frob": 1, "given": 2, "learned": 3, "x0": 4}
STOP = {"dx_abs": 0, "dx_rel": 1, "e1_rel": 2, "guarded": 3}
PRECISION = {"f64": 0, "f32": 1, "f32_f64finish": 2, "mixed": 3}
GEMM_PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}
SIDE = {"auto": 0, "left": 1, "right": 2}
REASON = {0: "tol", 1: "rise", 2: "max_iter", 3: "diverged"}
DEFAULT_ORDER = {"ns": 2, "hpi": None, "qsai": 10, "qhpi19": 19, "qrapid": 5}


class QMat(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("plane_stride", ctypes.c_int64), ("dtype", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("iters_bf16", ctypes.c_int32), ("iters_f32", ctypes.c_int32),
                ("iters_f64", ctypes.c_int32), ("returned", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
                ("side", ctypes.c_int32), ("alpha_clamped", ctypes.c_int32), ("fallback_used", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("alpha_used", ctypes.c_double), ("mu_used", ctypes.c_double),
                ("sigma1_sq_est", ctypes.c_double), ("final_dx_rel", ctypes.c_double),
                ("e1_rel", ctypes.c_double), ("seconds", ctypes.c_double), ("gemm_flops", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}
        d["reason"] = REASON.get(self.stop_reason, "?")
        return d


class QpinvError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {message} (status {status})")
        self.status = status


def _load() -> ctypes.CDLL:
    # PyTorch ships its own HIP runtime with the same SONAME as ROCm's; importing it first makes the
    # library bind to that one runtime instance instead of loading a second one into the process.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2605_01464_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    QP = ctypes.POINTER(QMat)
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "qpinv_init": (I, [ctypes.POINTER(P), I, ctypes.c_char_p]),
        "qpinv_set_option": (I, [P, ctypes.c_char_p, D]),
        "qpinv_finalize": (I, [P]),
        "qpinv_strerror": (ctypes.c_char_p, [I]),
        "qpinv_last_error": (ctypes.c_char_p, []),
        "qpinv_solve": (I, [P, I, I, QP, I, D, D, I, I, I, QP, ctypes.POINTER(Info), P]),
        "qpinv_solve_noalloc": (I, [P, I, I, QP, I, D, D, I, I, I, QP, ctypes.POINTER(Info), P]),
        "qpinv_step": (I, [P, I, I, I, I, QP, QP, QP, DP, P]),
        "qpinv_solve_batched": (I, [P, I, I, I, QP, QP, I, DP, D, I, I, ctypes.POINTER(Info), P]),
        "qpinv_residuals": (I, [P, QP, QP, DP, DP, P]),
        "qpinv_qgemm": (I, [P, I, QP, QP, QP, D, D, D, P]),
        "qpinv_qgemm_cfg": (I, [P, I, I, QP, QP, QP, D, D, D, P]),
        "qpinv_x0": (I, [P, QP, D, QP, P]),
        "qpinv_submatrix": (I, [P, QP, P, I, P, I, QP, P]),
        "qpinv_masked_merge": (I, [P, QP, P, I64, QP, QP, P]),
        "qpinv_gl_krylov": (I, [P, I, QP, QP, QP, QP, D, I, ctypes.POINTER(I), DP, DP, DP, I, P]),
        "qpinv_features": (I, [P, QP, I, DP, P]),
        "qpinv_autotune": (I, [P, I, I64, I64, I64, DP, P]),
        "qpinv_tune_save": (I, [P, ctypes.c_char_p]),
        "qpinv_tune_load": (I, [P, ctypes.c_char_p]),
        "qpinv_num_tile_configs": (I, [I]),
        "qpinv_tile_config_name": (ctypes.c_char_p, [I, I]),
        "qpinv_num_batched_configs": (I, []),
        "qpinv_batched_config_name": (ctypes.c_char_p, [I]),
        "qpinv_controller_replay": (I, [I, D, I, DP, DP, DP, ctypes.POINTER(ctypes.c_int)]),
        "qpinv_gemm_stats": (I, [P, DP, I]),
        "qpinv_mlp_init": (I, [P, ctypes.c_uint64]),
        "qpinv_mlp_fit_normalization": (I, [P, P, I, P]),
        "qpinv_mlp_train_step": (I, [P, P, P, P, I, D, DP, P]),
        "qpinv_mlp_gradient": (I, [P, P, P, I, P, DP, P]),
        "qpinv_mlp_predict": (I, [P, P, I, P, P]),
        "qpinv_mlp_num_params": (I, []),
        "qpinv_mlp_get_params": (I, [P, ctypes.POINTER(ctypes.c_float), I]),
        "qpinv_mlp_set_params": (I, [P, ctypes.POINTER(ctypes.c_float), I]),
        "qpinv_spectral_labels": (I, [P, I, I, P, P, I, P, D, I, I, D, D, D, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


# ------------------------------------------------------------------------------------------ marshalling
def qmat(t) -> QMat:
    """Describe a (4, rows, cols) float32/float64 device tensor with unit column stride."""
    import torch

    if t.dim() != 3 or t.shape[0] != 4:
        raise ValueError("a quaternion matrix is a tensor of shape (4, rows, cols)")
    if t.dtype not in (torch.float32, torch.float64):
        raise ValueError("quaternion planes must be float32 or float64")
    if not t.is_cuda:
        raise ValueError("quaternion matrices must live in GPU memory")
    rows, cols = int(t.shape[1]), int(t.shape[2])
    if cols > 1 and rows > 0 and t.stride(2) != 1:  # (an empty tensor's strides are arbitrary)
        raise ValueError("columns must have unit stride")
    ld = int(t.stride(1)) if rows > 1 else max(cols, 1)
    ps = int(t.stride(0))
    return QMat(t.data_ptr(), rows, cols, max(ld, cols, 1), max(ps, rows * max(ld, cols, 1)),
                F64 if t.dtype == torch.float64 else F32)


def _stream(stream):
    import torch

    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def _err(status: int, where: str) -> None:
    if status != OK:
        raise QpinvError(status, where, _lib.qpinv_last_error().decode() or _lib.qpinv_strerror(status).decode())


# ------------------------------------------------------------------------------------------ C ABI mirror
def qpinv_init(device: int = 0, config: str | None = None):
    h = ctypes.c_void_p()
    st = _lib.qpinv_init(ctypes.byref(h), device, config.encode() if config else None)
    return st, h


def qpinv_set_option(ctx, key: str, value: float) -> int:
    return _lib.qpinv_set_option(ctx, key.encode(), float(value))


def qpinv_finalize(ctx) -> int:
    return _lib.qpinv_finalize(ctx)


def qpinv_strerror(status: int) -> str:
    return _lib.qpinv_strerror(status).decode()


def qpinv_last_error() -> str:
    return _lib.qpinv_last_error().decode()


def qpinv_solve(ctx, method, order, A, scaling, alpha_or_mu, tol, max_iter, stop, precision, X, stream=None):
    info = Info()
    st = _lib.qpinv_solve(ctx, method, order, ctypes.byref(qmat(A)), scaling, float(alpha_or_mu), float(tol),
                          int(max_iter), stop, precision, ctypes.byref(qmat(X)), ctypes.byref(info), _stream(stream))
    return st, info


def qpinv_solve_noalloc(ctx, method, order, A, scaling, alpha_or_mu, tol, max_iter, stop, precision, X, stream=None):
    info = Info()
    st = _lib.qpinv_solve_noalloc(ctx, method, order, ctypes.byref(qmat(A)), scaling, float(alpha_or_mu), float(tol),
                                  int(max_iter), stop, precision, ctypes.byref(qmat(X)), ctypes.byref(info),
                                  _stream(stream))
    return st, info


def qpinv_solve_batched(ctx, method, order, As, Xs, scaling, alphas, tol, max_iter, stop, stream=None, Aq=None,
                        Xq=None):
    """Aq, Xq: descriptor arrays of As, Xs already built (BatchArgs); the raw Info array is returned."""
    n = len(As)
    if Aq is None:
        Aq = (QMat * max(n, 1))(*[qmat(a) for a in As])
    if Xq is None:
        Xq = (QMat * max(n, 1))(*[qmat(x) for x in Xs])
    al = (ctypes.c_double * max(n, 1))(*alphas) if alphas is not None else None
    infos = (Info * max(n, 1))()
    st = _lib.qpinv_solve_batched(ctx, method, order, n, Aq, Xq, scaling, al, float(tol), int(max_iter), stop, infos,
                                  _stream(stream))
    return st, infos


def qpinv_step(ctx, method, order, side, gemm_prec, A, X_in, X_out, stream=None):
    dx = (ctypes.c_double * 2)()
    st = _lib.qpinv_step(ctx, method, order, side, gemm_prec, ctypes.byref(qmat(A)), ctypes.byref(qmat(X_in)),
                         ctypes.byref(qmat(X_out)), dx, _stream(stream))
    return st, (dx[0], dx[1])


def qpinv_residuals(ctx, A, X, stream=None):
    Ea = (ctypes.c_double * 4)()
    Er = (ctypes.c_double * 4)()
    st = _lib.qpinv_residuals(ctx, ctypes.byref(qmat(A)), ctypes.byref(qmat(X)), Ea, Er, _stream(stream))
    return st, tuple(Ea), tuple(Er)


def qpinv_qgemm(ctx, gemm_prec, A, B, C, alpha=1.0, beta=0.0, gamma=0.0, stream=None) -> int:
    return _lib.qpinv_qgemm(ctx, gemm_prec, ctypes.byref(qmat(A)), ctypes.byref(qmat(B)), ctypes.byref(qmat(C)),
                            float(alpha), float(beta), float(gamma), _stream(stream))


def qpinv_qgemm_cfg(ctx, gemm_prec, cfg, A, B, C, alpha=1.0, beta=0.0, gamma=0.0, stream=None) -> int:
    return _lib.qpinv_qgemm_cfg(ctx, gemm_prec, cfg, ctypes.byref(qmat(A)), ctypes.byref(qmat(B)),
                                ctypes.byref(qmat(C)), float(alpha), float(beta), float(gamma), _stream(stream))


def qpinv_x0(ctx, A, alpha, X, stream=None) -> int:
    return _lib.qpinv_x0(ctx, ctypes.byref(qmat(A)), float(alpha), ctypes.byref(qmat(X)), _stream(stream))


def qpinv_submatrix(ctx, A, rows, nrows, cols, ncols, B, stream=None) -> int:
    return _lib.qpinv_submatrix(ctx, ctypes.byref(qmat(A)), _ptr(rows) if rows is not None else None, int(nrows),
                                _ptr(cols) if cols is not None else None, int(ncols), ctypes.byref(qmat(B)),
                                _stream(stream))


def qpinv_masked_merge(ctx, M, mask, mask_ld, X, Y, stream=None) -> int:
    return _lib.qpinv_masked_merge(ctx, ctypes.byref(qmat(M)), _ptr(mask), int(mask_ld), ctypes.byref(qmat(X)),
                                   ctypes.byref(qmat(Y)), _stream(stream))


def qpinv_gl_krylov(ctx, method, A, B, M, X, tol, max_iter, history_cap=0, stream=None):
    iters, rr, trr = ctypes.c_int(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    hist = (ctypes.c_double * max(history_cap, 1))()
    st = _lib.qpinv_gl_krylov(ctx, int(method), ctypes.byref(qmat(A)), ctypes.byref(qmat(B)),
                              ctypes.byref(qmat(M)) if M is not None else None, ctypes.byref(qmat(X)), float(tol),
                              int(max_iter), ctypes.byref(iters), ctypes.byref(rr), ctypes.byref(trr),
                              hist if history_cap > 0 else None, int(history_cap), _stream(stream))
    return st, iters.value, rr.value, trr.value, list(hist[:min(iters.value, history_cap)])


def qpinv_features(ctx, A, power_steps=0, stream=None):
    out = (ctypes.c_double * 7)()
    st = _lib.qpinv_features(ctx, ctypes.byref(qmat(A)), int(power_steps), out, _stream(stream))
    return st, tuple(out)


def qpinv_autotune(ctx, gemm_prec, M, N, K, stream=None):
    ms = ctypes.c_double(0.0)
    r = _lib.qpinv_autotune(ctx, gemm_prec, int(M), int(N), int(K), ctypes.byref(ms), _stream(stream))
    return r, ms.value


def qpinv_tune_save(ctx, path) -> int:
    return _lib.qpinv_tune_save(ctx, os.fsencode(path))


def qpinv_tune_load(ctx, path) -> int:
    return _lib.qpinv_tune_load(ctx, os.fsencode(path))


def qpinv_num_tile_configs(gemm_prec) -> int:
    return _lib.qpinv_num_tile_configs(gemm_prec)


def qpinv_tile_config_name(gemm_prec, cfg) -> str:
    return _lib.qpinv_tile_config_name(gemm_prec, cfg).decode()


def qpinv_num_batched_configs() -> int:
    return _lib.qpinv_num_batched_configs()


def qpinv_batched_config_name(cfg) -> str:
    return _lib.qpinv_batched_config_name(cfg).decode()


def qpinv_gemm_stats(ctx, max_rows=32):
    """Rows {gemm_prec, cfg, launches, flops, ms} per kernel since the last call (status < 0 on error)."""
    out = (ctypes.c_double * (5 * max_rows))()
    n = _lib.qpinv_gemm_stats(ctx, out, max_rows)
    if n < 0:
        return n, []
    rows = [dict(prec=int(out[5 * i]), cfg=int(out[5 * i + 1]), launches=int(out[5 * i + 2]),
                 flops=out[5 * i + 3], ms=out[5 * i + 4]) for i in range(n)]
    return OK, rows


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def qpinv_mlp_init(ctx, seed: int) -> int:
    return _lib.qpinv_mlp_init(ctx, ctypes.c_uint64(seed))


def qpinv_mlp_fit_normalization(ctx, raw, stream=None) -> int:
    return _lib.qpinv_mlp_fit_normalization(ctx, _ptr(raw), int(raw.shape[0]), _stream(stream))


def qpinv_mlp_train_step(ctx, raw, target, idx, batch, lr, stream=None):
    loss = ctypes.c_double(0.0)
    st = _lib.qpinv_mlp_train_step(ctx, _ptr(raw), _ptr(target), _ptr(idx), int(batch), float(lr),
                                   ctypes.byref(loss), _stream(stream))
    return st, loss.value


def qpinv_mlp_gradient(ctx, raw, target, grad, stream=None):
    loss = ctypes.c_double(0.0)
    st = _lib.qpinv_mlp_gradient(ctx, _ptr(raw), _ptr(target), int(raw.shape[0]), _ptr(grad), ctypes.byref(loss),
                                 _stream(stream))
    return st, loss.value


def qpinv_mlp_predict(ctx, raw, mu, stream=None) -> int:
    return _lib.qpinv_mlp_predict(ctx, _ptr(raw), int(raw.shape[0]), _ptr(mu), _stream(stream))


def qpinv_mlp_num_params() -> int:
    return _lib.qpinv_mlp_num_params()


def qpinv_mlp_get_params(ctx):
    n = qpinv_mlp_num_params() + 20
    buf = (ctypes.c_float * n)()
    st = _lib.qpinv_mlp_get_params(ctx, buf, n)
    return (st if st < 0 else OK), list(buf)


def qpinv_mlp_set_params(ctx, values) -> int:
    buf = (ctypes.c_float * len(values))(*values)
    return _lib.qpinv_mlp_set_params(ctx, buf, len(values))


def qpinv_spectral_labels(ctx, method, order, spectra, offsets, s1sq_est, tol, max_iter, ngrid, mu_lo, mu_hi,
                          mu_target, mu_out, j_best, j_classical, stream=None) -> int:
    return _lib.qpinv_spectral_labels(ctx, method, order, _ptr(spectra), _ptr(offsets), int(s1sq_est.shape[0]),
                                      _ptr(s1sq_est), float(tol), int(max_iter), int(ngrid), float(mu_lo),
                                      float(mu_hi), float(mu_target), _ptr(mu_out), _ptr(j_best), _ptr(j_classical),
                                      _stream(stream))


def qpinv_controller_replay(stop, tol, d_abs, x_norm, e1_rel=None):
    n = len(d_abs)
    Da = (ctypes.c_double * n)(*d_abs)
    Xn = (ctypes.c_double * n)(*x_norm)
    E1 = (ctypes.c_double * n)(*e1_rel) if e1_rel is not None else None
    dec = (ctypes.c_int * n)()
    used = _lib.qpinv_controller_replay(stop, float(tol), n, Da, Xn, E1, dec)
    return used, list(dec)


# ------------------------------------------------------------------------------------------ conveniences
class Context:
    """Owns a qpinv context on one device; usable as a context manager."""

    def __init__(self, device: int = 0, config: str | None = None):
        st, h = qpinv_init(device, config)
        _err(st, "qpinv_init")
        self.handle = h

    def close(self):
        if self.handle:
            qpinv_finalize(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, key: str, value: float):
        _err(qpinv_set_option(self.handle, key, value), f"set_option({key})")

    def save_tuning(self, path) -> int:
        """Write this context's tuned tile choices to `path`; returns the number of entries."""
        r = qpinv_tune_save(self.handle, path)
        _err(r if r < 0 else OK, "qpinv_tune_save")
        return r

    def load_tuning(self, path) -> int:
        """Merge tile choices saved by save_tuning (on the same kind of device); returns the entries applied."""
        r = qpinv_tune_load(self.handle, path)
        _err(r if r < 0 else OK, "qpinv_tune_load")
        return r


def _order(method: str, order):
    if order is not None:
        return int(order)
    d = DEFAULT_ORDER[method]
    if d is None:
        raise ValueError(f"method {method!r} needs an explicit order")
    return d


def solve(ctx: Context, A, method="qhpi19", order=None, scaling="power", alpha=0.0, tol=1e-6, max_iter=500,
          stop="guarded", precision=None, X=None, out_dtype=None, stream=None, check=True):
    """X ~= A^dagger.  Returns (X, info dict).  ENOTCONVERGED is reported in info, not raised."""
    import torch

    if precision is None:
        precision = "f64" if A.dtype == torch.float64 else "f32"
    if X is None:
        X = torch.empty((4, A.shape[2], A.shape[1]), dtype=out_dtype or A.dtype, device=A.device)
    st, info = qpinv_solve(ctx.handle, METHOD[method], _order(method, order), A, SCALING[scaling], alpha, tol,
                           max_iter, STOP[stop], PRECISION[precision], X, stream)
    d = info.as_dict()
    d["status"] = st
    if check and st not in (OK, ENOTCONVERGED):
        _err(st, "qpinv_solve")
    return X, d


def solve_noalloc(ctx: Context, A, X, method="qhpi19", order=None, scaling="power", alpha=0.0, tol=1e-6, max_iter=500,
                  stop="guarded", precision=None, stream=None, check=True):
    """solve() through the allocation-free entry point: X (n x m, caller-allocated) receives the result and the
    library allocates nothing during the call (workspace from its static per-GPU scratch).  Returns info."""
    import torch

    if X is None:
        raise ValueError("solve_noalloc: X must be allocated by the caller")
    if precision is None:
        precision = "f64" if A.dtype == torch.float64 else "f32"
    st, info = qpinv_solve_noalloc(ctx.handle, METHOD[method], _order(method, order), A, SCALING[scaling], alpha, tol,
                                   max_iter, STOP[stop], PRECISION[precision], X, stream)
    d = info.as_dict()
    d["status"] = st
    if check and st not in (OK, ENOTCONVERGED):
        _err(st, "qpinv_solve_noalloc")
    return d


class BatchArgs:
    """The marshalled arguments of a batched solve: the descriptors of the matrices As and of the outputs Xs
    (allocated here when not given), built once.  Passing it to solve_batched in place of the list skips the
    per-call marshalling of every tensor; the tensors must stay as they are (same storage, shape, strides)."""

    def __init__(self, As, Xs=None):
        import torch

        self.As = list(As)
        if Xs is None:
            Xs = [torch.empty((4, a.shape[2], a.shape[1]), dtype=torch.float32, device=a.device) for a in self.As]
        self.Xs = list(Xs)
        if len(self.Xs) != len(self.As):
            raise ValueError("one output per matrix")
        n = max(len(self.As), 1)
        self.Aq = (QMat * n)(*[qmat(a) for a in self.As])
        self.Xq = (QMat * n)(*[qmat(x) for x in self.Xs])


class BatchInfos(Sequence):
    """The per-matrix results of a batched solve, each converted to a dict (as solve returns) when read."""

    def __init__(self, raw, n):
        self._raw, self._n, self._done = raw, n, {}

    def __len__(self):
        return self._n

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[k] for k in range(*i.indices(self._n))]
        if i < 0:
            i += self._n
        if not 0 <= i < self._n:
            raise IndexError(i)
        d = self._done.get(i)
        if d is None:
            d = self._raw[i].as_dict()
            d["status"] = self._raw[i].reserved
            self._done[i] = d
        return d


def solve_batched(ctx: Context, As, method="qhpi19", order=None, scaling="power", alphas=None, tol=1e-6,
                  max_iter=100, stop="guarded", Xs=None, stream=None, check=True):
    """X_b ~= A_b^dagger for every FP32 matrix of the list (or of a BatchArgs), in one persistent launch.
    Returns (Xs, infos)."""
    import torch

    if isinstance(As, BatchArgs):
        if Xs is not None:
            raise ValueError("the outputs of a BatchArgs are its own")
        args = As
        As, Xs, Aq, Xq = args.As, args.Xs, args.Aq, args.Xq
    else:
        if Xs is None:
            Xs = [torch.empty((4, a.shape[2], a.shape[1]), dtype=torch.float32, device=a.device) for a in As]
        Aq = Xq = None
    st, raw = qpinv_solve_batched(ctx.handle, METHOD[method], _order(method, order), As, Xs, SCALING[scaling],
                                  alphas, tol, max_iter, STOP[stop], stream, Aq, Xq)
    if check and st not in (OK, ENOTCONVERGED):
        _err(st, "qpinv_solve_batched")
    return Xs, BatchInfos(raw, len(As))


def step(ctx: Context, A, X, method="qhpi19", order=None, side="auto", gemm_prec=None, out=None, stream=None):
    import torch

    if gemm_prec is None:
        gemm_prec = "f64" if A.dtype == torch.float64 else "f32"
    out = torch.empty_like(X) if out is None else out
    st, dx = qpinv_step(ctx.handle, METHOD[method], _order(method, order), SIDE[side], GEMM_PREC[gemm_prec], A, X,
                        out, stream)
    _err(st, "qpinv_step")
    return out, dx


def residuals(ctx: Context, A, X, stream=None):
    st, Ea, Er = qpinv_residuals(ctx.handle, A, X, stream)
    _err(st, "qpinv_residuals")
    return Ea, Er


def qgemm(ctx: Context, A, B, C=None, alpha=1.0, beta=0.0, gamma=0.0, gemm_prec=None, cfg=None, stream=None):
    import torch

    if gemm_prec is None:
        gemm_prec = "f64" if A.dtype == torch.float64 else "f32"
    if C is None:
        C = torch.zeros((4, A.shape[1], B.shape[2]), dtype=A.dtype, device=A.device)
    if cfg is None:
        st = qpinv_qgemm(ctx.handle, GEMM_PREC[gemm_prec], A, B, C, alpha, beta, gamma, stream)
    else:
        st = qpinv_qgemm_cfg(ctx.handle, GEMM_PREC[gemm_prec], cfg, A, B, C, alpha, beta, gamma, stream)
    _err(st, "qpinv_qgemm")
    return C


def filter_design(ctx: Context, X, s, method="qsai", order=None, tol=1e-13, max_iter=100, stop="guarded",
                  precision=None):
    """Quaternion filter design of Section 5.2: h = X^dagger s and s_hat = X h.  The pseudoinverse comes
    from the chosen iteration, both products from the quaternion GEMM.  Returns (h, s_hat, info)."""
    Xp, info = solve(ctx, X, method, order=order, tol=tol, max_iter=max_iter, stop=stop, precision=precision)
    h = qgemm(ctx, Xp, s)
    s_hat = qgemm(ctx, X, h)
    return h, s_hat, info


KRYLOV = {"fom": 0, "gmres": 1}


def gl_krylov(ctx: Context, A, B, method="gmres", M=None, X0=None, tol=1e-6, max_iter=3000, history=False,
              stream=None):
    """Global quaternion FOM / GMRES for A X = B (FP64), left-preconditioned by M when given.  Returns
    (X, info) with info = {status, iters, rr, true_rr, history}."""
    import torch

    X = torch.zeros((4, A.shape[2], B.shape[2]), dtype=torch.float64, device=A.device) if X0 is None else \
        X0.clone().contiguous()
    st, it, rr, trr, hist = qpinv_gl_krylov(ctx.handle, KRYLOV[method], A, B, M, X, tol, max_iter,
                                            max_iter if history else 0, stream)
    if st not in (OK, ENOTCONVERGED):
        _err(st, "qpinv_gl_krylov")
    return X, {"status": st, "iters": it, "rr": rr, "true_rr": trr, "history": hist}


def submatrix(ctx: Context, A, rows=None, cols=None, out=None, stream=None):
    """A[rows, cols] for device int32 index tensors (None: all rows / columns)."""
    import torch

    nr = A.shape[1] if rows is None else int(rows.numel())
    nc = A.shape[2] if cols is None else int(cols.numel())
    for t in (rows, cols):
        if t is not None and (t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous()):
            raise ValueError("index sets are contiguous int32 device tensors")
    if out is None:
        out = torch.empty((4, nr, nc), dtype=A.dtype, device=A.device)
    _err(qpinv_submatrix(ctx.handle, A, rows, nr, cols, nc, out, stream), "qpinv_submatrix")
    return out


def masked_merge(ctx: Context, M, mask, X, out=None, stream=None):
    """mask ? M : X elementwise (mask: contiguous uint8 device tensor rows x cols)."""
    import torch

    if mask.dtype != torch.uint8 or not mask.is_cuda or mask.dim() != 2 or mask.stride(1) != 1:
        raise ValueError("the mask is a row-major uint8 device tensor")
    if out is None:
        out = torch.empty_like(X)
    _err(qpinv_masked_merge(ctx.handle, M, mask, mask.stride(0), X, out, stream), "qpinv_masked_merge")
    return out


def cur_reconstruct(ctx: Context, A, rows, cols, method="qhpi19", tol=1e-10, max_iter=100, stop="guarded",
                    precision=None, stream=None):
    """CUR approximation of Section 5.1 with the Frobenius-optimal coupling U = C^dagger A R^dagger:
    C = A[:, cols], R = A[rows, :], returns (C U R, U, infos of the two pseudoinverse solves)."""
    C = submatrix(ctx, A, None, cols, stream=stream)
    R = submatrix(ctx, A, rows, None, stream=stream)
    Cp, ic = solve(ctx, C, method, tol=tol, max_iter=max_iter, stop=stop, precision=precision, stream=stream)
    Rp, ir = solve(ctx, R, method, tol=tol, max_iter=max_iter, stop=stop, precision=precision, stream=stream)
    U = qgemm(ctx, Cp, qgemm(ctx, A, Rp, stream=stream), stream=stream)
    X = qgemm(ctx, qgemm(ctx, C, U, stream=stream), R, stream=stream)
    return X, U, (ic, ir)


def cur_complete(ctx: Context, M, mask, rows, cols, iters=25, method="qhpi19", tol=1e-10, max_iter=100,
                 stop="guarded", precision=None, on_iter=None, stream=None):
    """Impute-reconstruct completion of Section 5.1: X_t = CUR(C_t), C_{t+1} = mask ? M : X_t, from
    C_0 = mask ? M : 0.  on_iter(t, X_t) is called after every reconstruction.  Returns X_{iters-1}."""
    import torch

    Ct = masked_merge(ctx, M, mask, torch.zeros_like(M), stream=stream)
    X = None
    for t in range(iters):
        X, _, _ = cur_reconstruct(ctx, Ct, rows, cols, method, tol, max_iter, stop, precision, stream)
        if on_iter is not None:
            on_iter(t, X)
        masked_merge(ctx, M, mask, X, out=Ct, stream=stream)
    return X


def features(ctx: Context, A, power_steps=0, stream=None):
    st, out = qpinv_features(ctx.handle, A, power_steps, stream)
    _err(st, "qpinv_features")
    return {"sigma1_sq": out[0], "fro": out[1], "norm1": out[2], "norminf": out[3], "m": int(out[4]),
            "n": int(out[5]), "sigma1_sq_prev": out[6]}


def raw_features(f: dict):
    """The network's raw feature row (s1sq, s1sq_prev, fro, norm1, norminf, m, n) from features()."""
    return [f["sigma1_sq"], f["sigma1_sq_prev"], f["fro"], f["norm1"], f["norminf"], float(f["m"]), float(f["n"])]


def x0(ctx: Context, A, alpha, out_dtype=None, stream=None):
    import torch

    X = torch.empty((4, A.shape[2], A.shape[1]), dtype=out_dtype or A.dtype, device=A.device)
    _err(qpinv_x0(ctx.handle, A, alpha, X, stream), "qpinv_x0")
    return X
