"""Thin Python binding of the surrogate C ABI (include/sur.h).

Argument marshalling only; every computation runs in libens.  Device arrays
are torch CUDA tensors (memory and stream only).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import ens

N_PARAMS = 148800
N_IN, N_HIDDEN, N_OUT = 2, 256, 64


class sur_screen_opts(C.Structure):
    _fields_ = [("margin", C.c_double), ("spread", C.c_double), ("flag_margin", C.c_double),
                ("label_margin", C.c_double)]


_bound = False


def _lib():
    global _bound
    L = ens.load()
    if not _bound:
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        dp = C.POINTER(C.c_double)
        L.sur_create.argtypes = [i32, vp, i64, C.POINTER(vp)]
        L.sur_destroy.argtypes = [vp]
        L.sur_last_error.argtypes = [vp]
        L.sur_last_error.restype = C.c_char_p
        L.sur_set_params.argtypes = [vp, dp]
        L.sur_get_params.argtypes = [vp, dp]
        L.sur_set_norm.argtypes = [vp, dp, dp, dp, dp]
        L.sur_build_dataset.argtypes = [vp, vp, vp, i64, vp, vp]
        L.sur_set_adam.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
        L.sur_train_step.argtypes = [vp, vp, vp, i64, vp, i32]
        L.sur_gradients.argtypes = [vp, vp, vp, i64, vp, vp, i32]
        L.sur_forward.argtypes = [vp, vp, i64, vp, i32]
        L.sur_reserve.argtypes = [vp, i64]
        L.sur_screen.argtypes = [vp, vp, i64, C.POINTER(sur_screen_opts), vp, vp, vp, vp,
                                 C.POINTER(i64)]
        L.sur_fit_label_map.argtypes = [vp, vp, i32, vp]
        L.sur_fit_norm.argtypes = [vp, dp, dp, vp, i64, dp, dp]
        L.sur_train_epoch.argtypes = [vp, vp, vp, i64, vp, i64, C.POINTER(C.c_float)]
        L.sur_train_epochs.argtypes = [vp, vp, vp, vp, i64, i64, i64, dp, C.c_uint64,
                                       C.POINTER(C.c_float)]
        L.sur_exact_labels.argtypes = [vp, vp, i64, vp, vp]
        _bound = True
    return L


def _check(rc, h=None):
    if rc != ens.ENS_OK:
        msg = _lib().sur_last_error(h)
        raise ens.EnsError(rc, msg.decode() if msg else "")


def _dptr(a):
    return C.cast(C.c_void_p(a.ctypes.data), C.POINTER(C.c_double))


def _ptr(x):
    """(pointer, where, keepalive) for a host numpy array or a CUDA tensor."""
    if x is None:
        return None, ens.ENS_HOST, None
    if ens._is_torch(x) and x.is_cuda:
        return C.c_void_p(x.data_ptr()), ens.ENS_DEVICE, x
    a = np.ascontiguousarray(x, dtype=np.float32)
    return C.c_void_p(a.ctypes.data), ens.ENS_HOST, a


class Surrogate:
    """The 2-256-256-256-64 GELU network, trained and evaluated on one device."""

    def __init__(self, device: int = 0, stream=None, max_batch: int = 4096):
        L = _lib()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        sp = int(getattr(stream, "cuda_stream", stream) or 0)
        h = C.c_void_p()
        _check(L.sur_create(int(device), sp, int(max_batch), C.byref(h)))
        self.h = h
        self.device = int(device)
        self.max_batch = int(max_batch)

    def close(self):
        if getattr(self, "h", None):
            _check(_lib().sur_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float64)
        if a.size != N_PARAMS:
            raise ValueError("expected 148800 parameters")
        _check(_lib().sur_set_params(self.h, _dptr(a)), self.h)

    def get_params(self):
        a = np.empty(N_PARAMS, dtype=np.float64)
        _check(_lib().sur_get_params(self.h, _dptr(a)), self.h)
        return a

    def set_norm(self, in_lo, in_hi, out_mean, out_std):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (in_lo, in_hi, out_mean, out_std)]
        _check(_lib().sur_set_norm(self.h, *[_dptr(a) for a in arrs]), self.h)

    def set_adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(_lib().sur_set_adam(self.h, lr, beta1, beta2, eps), self.h)

    def build_dataset(self, params_dev, records_dev, n):
        """Device float tensors x [n][2], y [n][64] from device params [2][n]
        and the last 64 cycle maxima [64][n] (both float64)."""
        import torch
        x = torch.empty((n, N_IN), dtype=torch.float32, device=f"cuda:{self.device}")
        y = torch.empty((n, N_OUT), dtype=torch.float32, device=f"cuda:{self.device}")
        _check(_lib().sur_build_dataset(self.h, C.c_void_p(params_dev.data_ptr()),
                                        C.c_void_p(records_dev.data_ptr()), int(n),
                                        C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())),
               self.h)
        return x, y

    def train_step(self, x, target, m=None, loss=None):
        px, w, kx = _ptr(x)
        pt, w2, kt = _ptr(target)
        if w != w2:
            raise ValueError("x and target must both be host or both device")
        m = int(m if m is not None else x.shape[0])
        pl = None
        if loss is not None:
            pl = C.c_void_p(loss.data_ptr()) if w == ens.ENS_DEVICE else C.c_void_p(loss.ctypes.data)
        _check(_lib().sur_train_step(self.h, px, pt, m, pl, w), self.h)

    def gradients(self, x, target):
        px, w, kx = _ptr(x)
        pt, _, kt = _ptr(target)
        m = int(x.shape[0])
        g = np.empty(N_PARAMS, dtype=np.float32)
        loss = np.empty(1, dtype=np.float32)
        if w != ens.ENS_HOST:
            raise ValueError("gradients() takes host arrays")
        _check(_lib().sur_gradients(self.h, px, pt, m, C.c_void_p(g.ctypes.data),
                                    C.c_void_p(loss.ctypes.data), w), self.h)
        return g, float(loss[0])

    def train_epochs(self, x_dev, y_dev, rows_dev, batch, lrs, seed):
        """Epochs over device dataset rows (see sur_train_epochs); returns the
        per-epoch mean losses."""
        lr = np.ascontiguousarray(lrs, dtype=np.float64)
        out = np.empty(lr.size, dtype=np.float32)
        _check(_lib().sur_train_epochs(self.h, C.c_void_p(x_dev.data_ptr()),
                                       C.c_void_p(y_dev.data_ptr()),
                                       C.c_void_p(rows_dev.data_ptr()), int(rows_dev.numel()),
                                       int(batch), int(lr.size), _dptr(lr), int(seed),
                                       out.ctypes.data_as(C.POINTER(C.c_float))), self.h)
        return out

    def forward(self, x):
        px, w, kx = _ptr(x)
        m = int(x.shape[0])
        if w == ens.ENS_DEVICE:
            import torch
            out = torch.empty((m, N_OUT), dtype=torch.float32, device=x.device)
            _check(_lib().sur_forward(self.h, px, m, C.c_void_p(out.data_ptr()), w), self.h)
            return out
        out = np.empty((m, N_OUT), dtype=np.float32)
        _check(_lib().sur_forward(self.h, px, m, C.c_void_p(out.ctypes.data), w), self.h)
        return out

    def fit_label_map(self, records_dev, G):
        """Exact labels of a G x G training grid (device int8 [G*G])."""
        import torch
        out = torch.empty(G * G, dtype=torch.int8, device=records_dev.device)
        _check(_lib().sur_fit_label_map(self.h, C.c_void_p(records_dev.data_ptr()), int(G),
                                        C.c_void_p(out.data_ptr())), self.h)
        return out

    def reserve(self, n_screen):
        """Size the compaction scratch for screens of up to n_screen points."""
        _check(_lib().sur_reserve(self.h, int(n_screen)), self.h)

    @staticmethod
    def screen_outputs(n, device):
        """Output tensors for screen(..., out=): label, resolve, pred_max, idx."""
        import torch
        return (torch.empty(n, dtype=torch.int8, device=device),
                torch.empty(n, dtype=torch.uint8, device=device),
                torch.empty(n, dtype=torch.float32, device=device),
                torch.empty(max(n, 1), dtype=torch.int64, device=device))

    def screen(self, params_dev, margin, spread, flag_margin, label_margin=-1.0, out=None):
        """Screen device params [2][n] (float64).  Returns device tensors
        (label int8, resolve uint8, pred_max float32, resolve_idx int64[:k]);
        `out` (from screen_outputs) receives them instead of new tensors."""
        n = int(params_dev.shape[1])
        label, resolve, pmax, idx = out if out is not None else \
            self.screen_outputs(n, params_dev.device)
        k = C.c_int64()
        o = sur_screen_opts(float(margin), float(spread), float(flag_margin),
                            float(label_margin))
        _check(_lib().sur_screen(self.h, C.c_void_p(params_dev.data_ptr()), n, C.byref(o),
                                 C.c_void_p(label.data_ptr()), C.c_void_p(resolve.data_ptr()),
                                 C.c_void_p(pmax.data_ptr()), C.c_void_p(idx.data_ptr()),
                                 C.byref(k)), self.h)
        return label, resolve, pmax, idx[:k.value]
