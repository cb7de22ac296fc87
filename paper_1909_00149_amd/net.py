"""Python binding of the warm-start network ABI (include/uotnet.h).

Argument marshalling only: forward, loss, backward, Adam and the conversion
of the network output into a solver start all run in the HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .uot import UOTError, _cstate, _ptr


class NetConfig(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("ch", ctypes.c_int32 * 4), ("batch_max", ctypes.c_int32), ("seed", ctypes.c_uint64)]


_SIGS = {
    "uotnet_create": (ctypes.c_int, [ctypes.POINTER(NetConfig), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "uotnet_destroy": (None, [ctypes.c_void_p]),
    "uotnet_num_params": (ctypes.c_int64, [ctypes.c_void_p]),
    "uotnet_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "uotnet_get_grads": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "uotnet_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "uotnet_warm_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.POINTER(_lib.State)]),
    "uotnet_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.POINTER(ctypes.c_double)]),
    "uotnet_conv": (ctypes.c_int, [ctypes.c_int32] * 6 + [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_void_p,
                                                                                  ctypes.c_void_p]),
}

_bound = False


def _load():
    global _bound
    lib = _lib.load()
    if not _bound:
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return lib


def _u16ptr(t):
    if not (t.is_cuda and t.dtype == torch.int16 and t.is_contiguous()):
        raise ValueError("bf16 tensors are passed as contiguous int16 bit patterns")
    return t.data_ptr()


def bf16_bits(x: torch.Tensor) -> torch.Tensor:
    """bf16 bit patterns (int16) of a float tensor, round to nearest even."""
    return x.to(torch.bfloat16).view(torch.int16).contiguous()


def bits_to_float(b: torch.Tensor) -> torch.Tensor:
    return b.view(torch.bfloat16).float()


def conv(op, N, H, W, Cin, Cout, X=None, Wt=None, G=None, bias=None, relu=False, out=None, stream=None):
    """uotnet_conv: op 0 forward, 1 input gradient, 2 weight gradient."""
    lib = _load()
    if out is None:
        shape = {0: (N, H, W, Cout), 1: (N, H, W, Cin), 2: (Cout, 9, Cin)}[op]
        dev = next(t for t in (X, Wt, G) if t is not None).device
        out = torch.empty(shape, dtype=torch.float32, device=dev)
    s = (stream or torch.cuda.current_stream()).cuda_stream
    rc = lib.uotnet_conv(op, N, H, W, Cin, Cout,
                         _u16ptr(X) if X is not None else None, _u16ptr(Wt) if Wt is not None else None,
                         _u16ptr(G) if G is not None else None, _ptr(bias) if bias is not None else None,
                         int(relu), _ptr(out), ctypes.c_void_p(s))
    if rc != 0:
        raise UOTError(rc, "uotnet_conv")
    return out


class WarmStartNet:
    def __init__(self, height, width, ch=(32, 64, 128, 128), batch_max=16, seed=0, stream=None):
        self.lib = _load()
        cfg = NetConfig()
        cfg.height, cfg.width, cfg.levels = height, width, len(ch)
        for i, c in enumerate(ch):
            cfg.ch[i] = c
        cfg.batch_max, cfg.seed = batch_max, seed
        self.cfg = cfg
        self.ch = tuple(ch)
        self.height, self.width, self.batch_max = height, width, batch_max
        s = (stream or torch.cuda.current_stream()).cuda_stream
        h = ctypes.c_void_p()
        rc = self.lib.uotnet_create(ctypes.byref(cfg), ctypes.c_void_p(s), ctypes.byref(h))
        if rc != 0:
            raise UOTError(rc, "uotnet_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.uotnet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self):
        return int(self.lib.uotnet_num_params(self._h))

    def get_params(self):
        buf = np.zeros(self.num_params(), np.float32)
        rc = self.lib.uotnet_get_params(self._h, buf.ctypes.data, buf.size)
        if rc != 0:
            raise UOTError(rc, "uotnet_get_params")
        return buf

    def get_grads(self):
        buf = np.zeros(self.num_params(), np.float32)
        rc = self.lib.uotnet_get_grads(self._h, buf.ctypes.data, buf.size)
        if rc != 0:
            raise UOTError(rc, "uotnet_get_grads")
        return buf

    def set_params(self, flat):
        buf = np.ascontiguousarray(flat, dtype=np.float32)
        rc = self.lib.uotnet_set_params(self._h, buf.ctypes.data, buf.size)
        if rc != 0:
            raise UOTError(rc, "uotnet_set_params")

    def warm_state(self, src, dst, state, in_scale, s_flux, s_dual):
        B = src.numel() // (self.height * self.width)
        cs = _cstate(state)
        rc = self.lib.uotnet_warm_state(self._h, B, _ptr(src), _ptr(dst), float(in_scale), float(s_flux),
                                        float(s_dual), ctypes.byref(cs))
        if rc != 0:
            raise UOTError(rc, "uotnet_warm_state")
        return state

    def train_step(self, src, dst, tMx, tMy, ta, in_scale, s_flux, s_dual, lr):
        B = src.numel() // (self.height * self.width)
        loss = ctypes.c_double()
        rc = self.lib.uotnet_train_step(self._h, B, _ptr(src), _ptr(dst), float(in_scale), _ptr(tMx), _ptr(tMy),
                                        _ptr(ta), float(s_flux), float(s_dual), float(lr), ctypes.byref(loss))
        if rc != 0:
            raise UOTError(rc, "uotnet_train_step")
        return loss.value


def flat_to_layers(flat, cin, ch):
    """Host parameter vector -> {name.w, name.b} in the oracle's layout."""
    from itertools import accumulate  # noqa: F401
    out, o = {}, 0
    for name, ci, co in layer_list(cin, ch):
        nw = co * 9 * ci
        out[name + ".w"] = flat[o:o + nw].reshape(co, 3, 3, ci)
        o += nw
        out[name + ".b"] = flat[o:o + co]
        o += co
    return out


def layers_to_flat(P, cin, ch):
    parts = []
    for name, ci, co in layer_list(cin, ch):
        parts += [np.asarray(P[name + ".w"], np.float32).reshape(-1), np.asarray(P[name + ".b"], np.float32)]
    return np.concatenate(parts)


def layer_list(cin, ch):
    L = len(ch)
    out = [("enc0a", cin, ch[0]), ("enc0b", ch[0], ch[0])]
    for l in range(1, L):
        out += [(f"enc{l}a", ch[l - 1], ch[l]), (f"enc{l}b", ch[l], ch[l])]
    for l in range(L - 2, -1, -1):
        out += [(f"dec{l}a", ch[l + 1] + ch[l], ch[l]), (f"dec{l}b", ch[l], ch[l])]
    out.append(("head", ch[0], 3))
    return out
