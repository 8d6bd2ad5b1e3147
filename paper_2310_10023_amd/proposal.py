"""Binding of the learned proposal network (argument marshalling only).

The network, its training step and the bird's-eye polar image all run in
libbbs (BF16 MFMA kernels); this module passes arrays in and out.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import BbsError, _check, _points, lib

YAW_BINS = 64
XY_CELLS = 32
N_OUT = YAW_BINS + XY_CELLS * XY_CELLS


def _bind():
    L = lib()
    if getattr(L, "_net_bound", False):
        return L
    P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    L.bbs_net_param_count.restype = I64
    L.bbs_net_create.argtypes = [I32, C.POINTER(P)]
    L.bbs_net_create.restype = C.c_int
    L.bbs_net_free.argtypes = [P]
    L.bbs_net_set_params.argtypes = [P, P, I64]
    L.bbs_net_set_params.restype = C.c_int
    L.bbs_net_get_params.argtypes = [P, P, I64]
    L.bbs_net_get_params.restype = C.c_int
    L.bbs_net_forward.argtypes = [P, P, I32, I32, P]
    L.bbs_net_forward.restype = C.c_int
    L.bbs_net_train_step.argtypes = [P, P, I32, P, P, I32, F, F, P, P]
    L.bbs_net_train_step.restype = C.c_int
    L.bbs_bev_image.argtypes = [P, I64, I32, P]
    L.bbs_bev_image.restype = C.c_int
    L.bbs_net_prior.argtypes = [P, P, I64, I32, P]
    L.bbs_net_prior.restype = C.c_int
    L._net_bound = True
    return L


def param_count() -> int:
    return int(_bind().bbs_net_param_count())


def bev_image(scan) -> np.ndarray:
    """[64, 64] uint8 bird's-eye polar counts of a scan (device kernel)."""
    L = _bind()
    ptr, k, dev, keep = _points(scan, "scan")
    out = np.zeros((64, 64), np.uint8)
    _check(L.bbs_bev_image(ptr, k, dev, out.ctypes.data))
    del keep
    return out


class Net:
    def __init__(self, max_batch: int = 256, params: np.ndarray | None = None):
        L = _bind()
        h = C.c_void_p()
        _check(L.bbs_net_create(int(max_batch), C.byref(h)))
        self._h = h
        self.max_batch = int(max_batch)
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().bbs_net_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32).ravel()
        _check(_bind().bbs_net_set_params(self._h, p.ctypes.data, p.size))

    def get_params(self) -> np.ndarray:
        p = np.zeros(param_count(), np.float32)
        _check(_bind().bbs_net_get_params(self._h, p.ctypes.data, p.size))
        return p

    def forward(self, images) -> np.ndarray:
        img = np.ascontiguousarray(images, np.uint8).reshape(-1, 64, 64)
        out = np.zeros((len(img), N_OUT), np.float32)
        _check(_bind().bbs_net_forward(self._h, img.ctypes.data, 0, len(img), out.ctypes.data))
        return out

    def prior(self, scan) -> np.ndarray:
        """The 1088 logits of one scan (host array or device tensor): BEV image
        and forward pass on the device, no host copy of the scan."""
        ptr, k, dev, keep = _points(scan, "scan")
        out = np.zeros(N_OUT, np.float32)
        _check(_bind().bbs_net_prior(self._h, ptr, k, dev, out.ctypes.data))
        del keep
        return out

    def train_step(self, images, yaw, xy, lr: float, weight_decay: float = 0.0, want_grads: bool = False):
        """One AdamW step (lr < 0: gradients only).  Returns (loss, grads or None)."""
        img = np.ascontiguousarray(images, np.uint8).reshape(-1, 64, 64)
        y = np.ascontiguousarray(yaw, np.int32)
        c = np.ascontiguousarray(xy, np.int32)
        loss = C.c_float()
        g = np.zeros(param_count(), np.float32) if want_grads else None
        _check(_bind().bbs_net_train_step(self._h, img.ctypes.data, 0, y.ctypes.data, c.ctypes.data, len(img),
                                          float(lr), float(weight_decay), C.byref(loss),
                                          g.ctypes.data if g is not None else None))
        return float(loss.value), g


def yaw_bin(yaw: float) -> int:
    """Yaw bin of an angle: floor((yaw mod 2 pi) / (2 pi / 64))."""
    return int(math.floor((yaw % (2 * math.pi)) / (2 * math.pi / YAW_BINS))) % YAW_BINS


def xy_cell(x: float, y: float, rmin, rmax) -> int:
    """Translation cell of (x, y) on the 32 x 32 grid over the search box (x outer)."""
    cx = int(math.floor(XY_CELLS * (x - float(rmin[0])) / (float(rmax[0]) - float(rmin[0]))))
    cy = int(math.floor(XY_CELLS * (y - float(rmin[1])) / (float(rmax[1]) - float(rmin[1]))))
    return min(max(cx, 0), XY_CELLS - 1) * XY_CELLS + min(max(cy, 0), XY_CELLS - 1)
