"""Thin Python binding of libmds (argument marshalling only).

Every computation runs in the HIP library; torch supplies device memory and
the current stream.  Names mirror the C ABI in include/mds.h.
"""

import ctypes

import numpy as np

from . import _lib

OK = 0
ERR_INVALID_ARG = 1
ERR_OOM = 2
ERR_BUDGET = 3
ERR_DEGENERATE = 4
ERR_HIP = 5
ERR_NOT_CONVERGED = 6
ERR_NOT_FOUND = 7
ERR_STATE = 8

F32 = 0
F64 = 1

PREC = {"fp64": 0, "fp32": 1, "split_bf16": 2, "split_fp16": 3}


class MDSError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libmds status {status}: {message}")
        self.status = status


def _check(status):
    if status != OK:
        raise MDSError(status, _lib.lib().mds_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("X must be float32 or float64")


def _check_matrix(X, name):
    if not X.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if X.dim() != 2 or (X.shape[0] > 1 and X.stride(1) != 1) or (X.shape[1] > 1 and X.stride(1) != 1):
        raise ValueError(f"{name} must be a 2-D row-major tensor with unit column stride")


def sample_landmarks(n, l, seed):
    """Landmark indices exactly as mds_fit_landmarks draws them (host)."""
    out = np.empty(int(l), dtype=np.int64)
    _check(_lib.lib().mds_sample_landmarks(int(n), int(l), int(seed) & (2**64 - 1),
                                           out.ctypes.data_as(_lib.P_i64)))
    return out


class Model:
    """A fitted landmark configuration resident on the device."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def _info(self):
        n_fit, p, l = _lib.c_i64(), _lib.c_i64(), _lib.c_i64()
        r, r_eff = _lib.c_i32(), _lib.c_i32()
        _check(_lib.lib().mds_model_info(self._h, ctypes.byref(n_fit), ctypes.byref(p),
                                         ctypes.byref(l), ctypes.byref(r), ctypes.byref(r_eff)))
        return n_fit.value, p.value, l.value, r.value, r_eff.value

    @property
    def n_fit(self):
        return self._info()[0]

    @property
    def p(self):
        return self._info()[1]

    @property
    def l(self):
        return self._info()[2]

    @property
    def r(self):
        return self._info()[3]

    @property
    def r_eff(self):
        return self._info()[4]

    def landmarks(self):
        out = np.empty(self.l, dtype=np.int64)
        _check(_lib.lib().mds_get_landmarks(self._h, out.ctypes.data_as(_lib.P_i64)))
        return out

    def eigenvalues(self):
        out = np.empty(self.r, dtype=np.float64)
        _check(_lib.lib().mds_get_eigenvalues(self._h, out.ctypes.data_as(_lib.P_dbl)))
        return out

    def landmark_coords(self):
        out = np.empty((self.l, self.r), dtype=np.float64)
        _check(_lib.lib().mds_get_landmark_coords(self._h, out.ctypes.data_as(_lib.P_dbl)))
        return out

    def q(self):
        out = np.empty(self.l, dtype=np.float64)
        _check(_lib.lib().mds_get_q(self._h, out.ctypes.data_as(_lib.P_dbl)))
        return out

    @property
    def nbytes(self):
        return int(_lib.lib().mds_model_bytes(self._h))

    def fit_stats(self):
        steps, restarts = _lib.c_i32(), _lib.c_i32()
        _check(_lib.lib().mds_fit_stats(self._h, ctypes.byref(steps), ctypes.byref(restarts)))
        return {"lanczos_steps": steps.value, "restarts": restarts.value}

    def free(self):
        if self._h and self._h.value:
            _lib.lib().mds_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fit_landmarks(X, l, r, seed=0, idx=None, stream=None):
    """mds_fit_landmarks: classical MDS on l landmark rows of the device
    tensor X (n x p, float32 or float64)."""
    _check_matrix(X, "X")
    n, p = X.shape
    idx_p = None
    if idx is not None:
        idx_arr = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        if idx_arr.shape != (int(l),):
            raise ValueError("idx must have l entries")
        idx_p = idx_arr.ctypes.data_as(_lib.P_i64)
    out = ctypes.c_void_p()
    ldx = X.stride(0) if n > 1 else p
    _check(_lib.lib().mds_fit_landmarks(
        ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n, p, ldx, int(l), int(r),
        int(seed) & (2**64 - 1), idx_p, _stream_ptr(stream), ctypes.byref(out)))
    return Model(out.value)


def embed(model, X, prec="fp32", Y=None, stream=None):
    """mds_embed: Gower interpolation of every row of the device tensor X.

    Returns Y (n x r): float64 for prec="fp64", float32 otherwise."""
    import torch
    _check_matrix(X, "X")
    n = X.shape[0]
    code = PREC[prec]
    ydt = torch.float64 if code == PREC["fp64"] else torch.float32
    r = model.r
    if Y is None:
        Y = torch.empty((n, r), dtype=ydt, device=X.device)
    else:
        _check_matrix(Y, "Y")
        if Y.dtype != ydt or Y.shape[0] != n or Y.shape[1] < r:
            raise ValueError("Y has the wrong dtype or shape")
    ldx = X.stride(0) if n > 1 else X.shape[1]
    ldy = Y.stride(0) if n > 1 else Y.shape[1]
    _check(_lib.lib().mds_embed(model.handle, ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n,
                                ldx, code, ctypes.c_void_p(Y.data_ptr()), ldy, _stream_ptr(stream)))
    return Y


def fit_from_sqdist(D1, r, stream=None):
    """mds_fit_from_sqdist: classical MDS of l points from their l x l
    squared dissimilarities (device float64 tensor)."""
    import torch
    _check_matrix(D1, "D1")
    if D1.dtype != torch.float64 or D1.shape[0] != D1.shape[1]:
        raise ValueError("D1 must be a square float64 device tensor")
    l = D1.shape[0]
    out = ctypes.c_void_p()
    _check(_lib.lib().mds_fit_from_sqdist(ctypes.c_void_p(D1.data_ptr()), l,
                                          D1.stride(0) if l > 1 else 1, int(r),
                                          _stream_ptr(stream), ctypes.byref(out)))
    return Model(out.value)


def embed_from_sqdist(model, A2, prec="fp32", Y=None, stream=None):
    """mds_embed_from_sqdist: eq. (2) for rows of squared dissimilarities
    A2 (n x l device tensor) to the model's landmarks."""
    import torch
    _check_matrix(A2, "A2")
    n = A2.shape[0]
    code = PREC[prec]
    ydt = torch.float64 if code == PREC["fp64"] else torch.float32
    if Y is None:
        Y = torch.empty((n, model.r), dtype=ydt, device=A2.device)
    lda = A2.stride(0) if n > 1 else A2.shape[1]
    ldy = Y.stride(0) if n > 1 else Y.shape[1]
    _check(_lib.lib().mds_embed_from_sqdist(model.handle, ctypes.c_void_p(A2.data_ptr()),
                                            _dtype_code(A2), n, lda, code,
                                            ctypes.c_void_p(Y.data_ptr()), ldy, _stream_ptr(stream)))
    return Y


def maxmin_landmarks(X, l, first=0, stream=None):
    """mds_maxmin_landmarks: l row indices of X chosen by MaxMin from row
    `first`, in selection order (numpy int64)."""
    _check_matrix(X, "X")
    n, p = X.shape
    out = np.empty(l, dtype=np.int64)
    ldx = X.stride(0) if n > 1 else p
    _check(_lib.lib().mds_maxmin_landmarks(ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n, p, ldx, l,
                                           first, out.ctypes.data_as(_lib.P_i64), _stream_ptr(stream)))
    return out


def maxmin_landmarks_noalloc(X, l, first=0, stream=None):
    """mds_maxmin_landmarks_noalloc: as maxmin_landmarks, on the library's
    static scratch array (no device allocation; n <= 2^20, l <= 16384;
    calls on one GPU must not overlap)."""
    _check_matrix(X, "X")
    n, p = X.shape
    out = np.empty(l, dtype=np.int64)
    ldx = X.stride(0) if n > 1 else p
    _check(_lib.lib().mds_maxmin_landmarks_noalloc(ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n, p, ldx,
                                                   l, first, out.ctypes.data_as(_lib.P_i64),
                                                   _stream_ptr(stream)))
    return out


def pivot_mds(X, l, r, seed=0, idx=None, Y=None, stream=None):
    """mds_pivot_mds: pivot MDS of the rows of X; returns (Y, lam, r_eff)."""
    import torch
    _check_matrix(X, "X")
    n, p = X.shape
    if Y is None:
        Y = torch.empty((n, r), dtype=torch.float64, device=X.device)
    ldx = X.stride(0) if n > 1 else p
    ldy = Y.stride(0) if n > 1 else r
    lam = (ctypes.c_double * r)()
    r_eff = ctypes.c_int32(0)
    idx_arr = None
    if idx is not None:
        idx_arr = np.ascontiguousarray(idx, dtype=np.int64)
    _check(_lib.lib().mds_pivot_mds(
        ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n, p, ldx, l, r, seed,
        idx_arr.ctypes.data_as(_lib.P_i64) if idx_arr is not None else None,
        ctypes.c_void_p(Y.data_ptr()), ldy, lam, ctypes.byref(r_eff), _stream_ptr(stream)))
    return Y, np.array(lam[:], dtype=np.float64), int(r_eff.value)


def embed_affine(model, X, prec="fp32", Y=None, stream=None):
    """mds_embed_affine: eq. (2) in its affine form y = A x + b (squared
    Euclidean distances only; a separate mode, not the distance path)."""
    import torch
    _check_matrix(X, "X")
    n = X.shape[0]
    code = PREC[prec]
    ydt = torch.float64 if code == PREC["fp64"] else torch.float32
    if Y is None:
        Y = torch.empty((n, model.r), dtype=ydt, device=X.device)
    ldx = X.stride(0) if n > 1 else X.shape[1]
    ldy = Y.stride(0) if n > 1 else Y.shape[1]
    _check(_lib.lib().mds_embed_affine(model.handle, ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n,
                                       ldx, code, ctypes.c_void_p(Y.data_ptr()), ldy,
                                       _stream_ptr(stream)))
    return Y


def divide_conquer(X, l, c, r, seed=0, Y=None, return_order=False, stream=None):
    """mds_divide_conquer (Section 3.2): divide-and-conquer MDS of the rows
    of X (n x p device tensor, float32 or float64).  Returns (Y, lam_bar,
    r_eff), plus the row order defining the parts if return_order."""
    import torch
    _check_matrix(X, "X")
    n, p = X.shape
    if Y is None:
        Y = torch.empty((n, r), dtype=torch.float64, device=X.device)
    order = torch.empty(n, dtype=torch.int64, device=X.device) if return_order else None
    ldx = X.stride(0) if n > 1 else p
    ldy = Y.stride(0) if n > 1 else r
    lam_bar = (ctypes.c_double * r)()
    r_eff = ctypes.c_int32(0)
    _check(_lib.lib().mds_divide_conquer(
        ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n, p, ldx, l, c, r, seed,
        ctypes.c_void_p(Y.data_ptr()), ldy, lam_bar, ctypes.byref(r_eff),
        ctypes.c_void_p(order.data_ptr()) if order is not None else None, _stream_ptr(stream)))
    out = (Y, np.array(lam_bar[:], dtype=np.float64), int(r_eff.value))
    return out + (order,) if return_order else out


def free(model):
    """mds_free."""
    model.free()
