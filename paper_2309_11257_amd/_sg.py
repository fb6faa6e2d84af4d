"""ctypes binding of the surrogate C ABI in include/sg.h (argument
marshalling only: every computation runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional

import numpy as np

from . import _rt
from ._rt import ALLOC_FN, FREE_FN, RT_DEVICE, RT_HOST, RT_OK, RTError


class SgConfig(C.Structure):
    _fields_ = [("n_members", C.c_int32), ("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_layers", C.c_int32),
                ("n_out", C.c_int32), ("max_batch", C.c_int32), ("seed", C.c_uint64), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("user", C.c_void_p), ("stream", C.c_void_p)]


_bound = False


def lib() -> C.CDLL:
    global _bound
    L = _rt.lib()
    if not _bound:
        P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        L.sg_create.argtypes = [C.POINTER(SgConfig), C.POINTER(P)]
        L.sg_destroy.argtypes = [P]
        L.sg_param_count.argtypes = [P]
        L.sg_param_count.restype = I64
        L.sg_get_params.argtypes = [P, I32, P, I32]
        L.sg_set_params.argtypes = [P, I32, P, I32]
        L.sg_forward.argtypes = [P, I32, P, P, I32]
        L.sg_train_step.argtypes = [P, I32, P, P, I32, F, P]
        L.sg_gradient.argtypes = [P, I32, P, P, I32, P, I32]
        L.sg_gate.argtypes = [P, P, P, P, P, I32, F, P, P]
        L.sg_standardize.argtypes = [P, P, P, P, P, I32, P]
        L.sg_apply_drag.argtypes = [P, P, P, P, P, I32, I32, P]
        L.sg_targets.argtypes = [P, P, P, P, I32, I32, P]
        L.sg_last_error.argtypes = [P]
        L.sg_last_error.restype = C.c_char_p
        for n in ("sg_create", "sg_destroy", "sg_get_params", "sg_set_params", "sg_forward", "sg_train_step",
                  "sg_gradient", "sg_gate", "sg_standardize", "sg_apply_drag", "sg_targets"):
            getattr(L, n).restype = C.c_int32
        _bound = True
    return L


def bf16_bits(x) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (round to nearest even), host side."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


class Surrogate:
    """An ensemble of column MLPs on one GPU (torch's current stream)."""

    def __init__(self, n_in: int, n_hidden: int, n_layers: int, n_out: int, n_members: int = 4,
                 max_batch: int = 4096, seed: int = 1, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.n_in, self.n_hidden, self.n_layers, self.n_out = n_in, n_hidden, n_layers, n_out
        self.n_members, self.max_batch = n_members, max_batch
        self._mem: Dict[int, object] = {}

        def _alloc(nbytes, user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            self._mem[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, user):
            self._mem.pop(int(ptr), None)

        self._a, self._f = ALLOC_FN(_alloc), FREE_FN(_free)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            cfg = SgConfig(n_members, n_in, n_hidden, n_layers, n_out, max_batch, seed, self._a, self._f, None,
                           C.c_void_p(self.stream.cuda_stream))
            h = C.c_void_p()
            st = lib().sg_create(C.byref(cfg), C.byref(h))
            if st != RT_OK:
                raise RTError(st, "sg_create failed")
        self.h = h
        self.P = int(lib().sg_param_count(h))

    def _check(self, st):
        if st != RT_OK:
            raise RTError(st, lib().sg_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().sg_destroy(self.h)
            self.h = None
            self._mem.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype):
        t = self.torch.as_tensor(a, device=self.device)
        if t.dtype != dtype:
            t = t.to(dtype)
        return t.contiguous()

    def get_params(self, member: int) -> np.ndarray:
        out = np.zeros(self.P, np.float32)
        self._check(lib().sg_get_params(self.h, member, out.ctypes.data, RT_HOST))
        return out

    def set_params(self, member: int, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (self.P,)
        self._check(lib().sg_set_params(self.h, member, p.ctypes.data, RT_HOST))

    def bf16_input(self, X):
        """Device bfloat16 tensor (as int16 bits) from host floats or a device bf16 tensor."""
        torch = self.torch
        if isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.bfloat16:
            return X.contiguous()
        return torch.from_numpy(bf16_bits(np.asarray(X, np.float32)).view(np.int16)).to(self.device).view(torch.bfloat16)

    def forward(self, X, member: int = -1):
        torch = self.torch
        Xd = self.bf16_input(X)
        B = Xd.shape[0]
        shape = (B, self.n_out) if member >= 0 else (self.n_members, B, self.n_out)
        Y = torch.empty(shape, dtype=torch.float32, device=self.device)
        self._check(lib().sg_forward(self.h, member, Xd.data_ptr(), Y.data_ptr(), B))
        return Y

    def gradient(self, member: int, X, T) -> np.ndarray:
        Xd = self.bf16_input(X)
        Td = self._dev(T, self.torch.float32)
        g = np.zeros(self.P, np.float32)
        self._check(lib().sg_gradient(self.h, member, Xd.data_ptr(), Td.data_ptr(), Xd.shape[0], g.ctypes.data, RT_HOST))
        return g

    def train_step(self, member: int, X, T, lr: float, loss=None):
        """One Adam step; `loss` may be a device float32 tensor of one element."""
        Xd = self.bf16_input(X)
        Td = self._dev(T, self.torch.float32)
        lp = loss.data_ptr() if loss is not None else None
        self._check(lib().sg_train_step(self.h, member, Xd.data_ptr(), Td.data_ptr(), Xd.shape[0], float(lr), lp))

    def gate(self, Yens, Xraw, fmin, fmax, tau: float):
        torch = self.torch
        # every operand stays referenced until the launch is enqueued
        Yd, Xd = self._dev(Yens, torch.float32), self._dev(Xraw, torch.float32)
        lo, hi = self._dev(fmin, torch.float32), self._dev(fmax, torch.float32)
        n = Xd.shape[0]
        spread = torch.empty(n, dtype=torch.float32, device=self.device)
        mask = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._check(lib().sg_gate(self.h, Yd.data_ptr(), Xd.data_ptr(), lo.data_ptr(), hi.data_ptr(), n, float(tau),
                                  spread.data_ptr(), mask.data_ptr()))
        return spread, mask

    def standardize(self, Xraw, mean, std, logfloor):
        torch = self.torch
        Xd = self._dev(Xraw, torch.float32)
        mu, sd, lg = (self._dev(a, torch.float32) for a in (mean, std, logfloor))
        n = Xd.shape[0]
        out = torch.empty((n, self.n_in), dtype=torch.bfloat16, device=self.device)
        self._check(lib().sg_standardize(self.h, Xd.data_ptr(), mu.data_ptr(), sd.data_ptr(), lg.data_ptr(), n,
                                         out.data_ptr()))
        return out

    def apply_drag(self, Yens, mean, std, mask, nz: int, drag):
        """Overwrite drag [2][nz][ncol] (device float64) in trusted columns
        with the ensemble mean of de-standardised outputs."""
        torch = self.torch
        Yd = self._dev(Yens, torch.float32)
        mu, sd = self._dev(mean, torch.float32), self._dev(std, torch.float32)
        mk = self._dev(mask, torch.uint8)
        assert drag.is_cuda and drag.dtype == torch.float64 and drag.is_contiguous()
        self._check(lib().sg_apply_drag(self.h, Yd.data_ptr(), mu.data_ptr(), sd.data_ptr(), mk.data_ptr(),
                                        mk.shape[0], nz, drag.data_ptr()))

    def targets(self, drag, mean, std, nz: int, out=None):
        """Standardised training targets [n_cols][2*nz] float32 from a device
        drag field [2][nz][n_cols] float64."""
        torch = self.torch
        assert drag.is_cuda and drag.dtype == torch.float64 and drag.is_contiguous()
        n = drag.numel() // (2 * nz)
        mu, sd = self._dev(mean, torch.float32), self._dev(std, torch.float32)
        T = torch.empty((n, 2 * nz), dtype=torch.float32, device=self.device) if out is None else out
        self._check(lib().sg_targets(self.h, drag.data_ptr(), mu.data_ptr(), sd.data_ptr(), n, nz, T.data_ptr()))
        return T
