"""Thin binding of the continuous-batching server (mds_serve_* in mds.h)."""

import ctypes

from . import _lib
from .api import F32, PREC, _check, _check_matrix


class Server:
    """Resident models + admission by bytes/slots + persistent graph steps."""

    def __init__(self, budget_bytes, max_slots=64, tiles_per_step=0):
        import torch
        self._device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        _check(_lib.lib().mds_serve_create(int(budget_bytes), int(max_slots), int(tiles_per_step),
                                           ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def add_model(self, model):
        mid = _lib.c_i32()
        _check(_lib.lib().mds_serve_add_model(self._h, model.handle, ctypes.byref(mid)))
        self._keep[mid.value] = model
        return mid.value

    def submit(self, model_id, X, prec, Y):
        """Queue rows X (device, float32, n x p) for model_id; results go to
        Y (device, float32, n x >= r), both on the server's device."""
        import torch
        _check_matrix(X, "X")
        _check_matrix(Y, "Y")
        model = self._keep.get(int(model_id))
        if model is None:
            raise ValueError(f"unknown model id {model_id}")
        if X.dtype != torch.float32 or Y.dtype != torch.float32:
            raise ValueError("serving takes float32 X and Y")
        n = X.shape[0]
        if X.shape[1] != model.p:
            raise ValueError(f"X has {X.shape[1]} columns, the model has p = {model.p}")
        if Y.shape[0] != n or Y.shape[1] < model.r:
            raise ValueError(f"Y must be {n} x (>= {model.r})")
        if X.device != Y.device or X.device.index != self._device:
            raise ValueError("X and Y must sit on the server's device")
        ldx = X.stride(0) if n > 1 else X.shape[1]
        ldy = Y.stride(0) if n > 1 else Y.shape[1]
        t = _lib.c_i64()
        _check(_lib.lib().mds_serve_submit(self._h, int(model_id), ctypes.c_void_p(X.data_ptr()),
                                           F32, n, ldx, PREC[prec], ctypes.c_void_p(Y.data_ptr()),
                                           ldy, ctypes.byref(t)))
        return t.value

    def poll(self, ticket):
        st = _lib.c_i32()
        ts, ta, td = _lib.c_dbl(), _lib.c_dbl(), _lib.c_dbl()
        _check(_lib.lib().mds_serve_poll(self._h, int(ticket), ctypes.byref(st), ctypes.byref(ts),
                                         ctypes.byref(ta), ctypes.byref(td)))
        return {"state": st.value, "t_submit": ts.value, "t_admit": ta.value, "t_done": td.value}

    def wait(self, ticket, timeout=-1.0):
        _check(_lib.lib().mds_serve_wait(self._h, int(ticket), float(timeout)))

    def stats(self):
        s = _lib.ServeStats()
        _check(_lib.lib().mds_serve_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in _lib.ServeStats._fields_}

    def now(self):
        return float(_lib.lib().mds_serve_now(self._h))

    def close(self):
        if self._h and self._h.value:
            _lib.lib().mds_serve_destroy(self._h)
            self._h = ctypes.c_void_p(0)
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
