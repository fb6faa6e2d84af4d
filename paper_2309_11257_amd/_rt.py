"""ctypes binding of the C ABI in include/rt.h (argument marshalling only).

Every step of the tracer runs in the HIP library librt.so; this module only
passes pointers, sizes and the stream.  Device memory for the library comes
from PyTorch's caching allocator through the rt_config alloc/free callbacks.
Importing this module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RT_LIBRARY may name another build of the same library (an A/B timing of two
# versions of the kernels in one process tree)
LIB_PATH = os.environ.get("RT_LIBRARY") or os.path.join(_HERE, "librt.so")

RT_OK, RT_E_ARG, RT_E_STATE, RT_E_NOMEM, RT_E_CAPACITY, RT_E_DEVICE, RT_E_NUMERIC, RT_E_UNSUPPORTED = range(8)
RT_CARTESIAN, RT_SPHERICAL = 0, 1
RT_FP64, RT_FP32 = 0, 1
RT_HOST, RT_DEVICE = 0, 1
RT_STEP_DEPOSIT, RT_STEP_SURROGATE, RT_STEP_SATURATE = 1, 2, 4
RT_MERGE, RT_CAP, RT_SPLIT_ONLY = 0, 1, 2

RAY_FIELDS = ("x", "y", "z", "k", "l", "m", "dx", "dy", "dz", "px", "py", "pz", "n")

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Config(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("precision", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("reserved", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("dz", C.c_double), ("a", C.c_double), ("capacity", C.c_int64), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("user", C.c_void_p), ("stream", C.c_void_p)]


class Rays(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in RAY_FIELDS] + [("id", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_active", "n_top", "n_bottom", "n_pole", "n_invalid", "n_split",
                                         "n_merged", "n_capped")] + \
               [(n, C.c_double) for n in ("sum_W", "sum_kW", "sum_lW", "sum_mW", "removed_W")] + \
               [("steps", C.c_int64), ("n_launched", C.c_int64), ("launched_W", C.c_double),
                ("first_bad_id", C.c_int64)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class LaunchParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("z_launch", "dt", "t_solstice", "F_s", "F_w", "lambda_h", "c_min",
                                          "c_max", "c_center", "c_width")] + \
               [("n_speeds", C.c_int32), ("where", C.c_int32), ("flux_col", C.c_void_p)]


class RTError(RuntimeError):
    def __init__(self, code: int, msg: str, stats: Optional[dict] = None):
        super().__init__(f"rt error {code}: {msg}")
        self.code = code
        self.stats = stats  # the full statistics, for RT_E_NUMERIC from rt_get_stats


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python paper_2309_11257_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.rt_create.argtypes = [C.POINTER(Config), C.POINTER(P)]
        L.rt_destroy.argtypes = [P]
        L.rt_init_background.argtypes = [P, P, P, P, P, P, I32]
        L.rt_set_rays.argtypes = [P, C.POINTER(Rays), I64, I32]
        L.rt_set_rays_host_noalloc.argtypes = [P, C.POINTER(Rays), I64]
        L.rt_get_rays.argtypes = [P, C.POINTER(Rays), C.POINTER(I64), I32]
        L.rt_step.argtypes = [P, D, I32]
        L.rt_deposit_flux.argtypes = [P, P, P, I32]
        L.rt_saturate.argtypes = [P, D, P, I32]
        L.rt_full_fluxes.argtypes = [P, P, P, I32, I32]
        L.rt_budget.argtypes = [P, P, P, I32, I32]
        L.rt_split_merge.argtypes = [P, D, I32, I32, C.POINTER(Stats)]
        L.rt_get_stats.argtypes = [P, C.POINTER(Stats)]
        L.rt_launch.argtypes = [P, C.POINTER(LaunchParams), C.POINTER(I64)]
        L.rt_set_scale_height.argtypes = [P, P, I32]
        L.rt_get_columns.argtypes = [P, P, C.POINTER(I64), I32]
        L.rt_profile.argtypes = [P, I32]
        L.rt_profile_read.argtypes = [P, P, P]
        L.rt_features.argtypes = [P, P, I32]
        L.rt_set_frozen_columns.argtypes = [P, P, I32]
        L.rt_last_error.argtypes = [P]
        L.rt_last_error.restype = C.c_char_p
        for name in ("rt_create", "rt_destroy", "rt_init_background", "rt_set_rays", "rt_set_rays_host_noalloc",
                     "rt_get_rays", "rt_step",
                     "rt_deposit_flux", "rt_split_merge", "rt_get_stats", "rt_profile", "rt_profile_read", "rt_get_columns",
                     "rt_features", "rt_set_frozen_columns", "rt_saturate", "rt_full_fluxes", "rt_budget", "rt_launch", "rt_set_scale_height"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


class Tracer:
    """One library context on one GPU (cuda:0 unless given) and torch's
    current stream.  Inputs may be numpy arrays (host) or CUDA tensors."""

    def __init__(self, geometry: int, precision: int, nx: int, ny: int, nz: int, dx: float, dy: float, dz: float,
                 capacity: int, a: float = 6.371e6, device: str = "cuda:0"):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.precision = precision
        self._mem: Dict[int, object] = {}

        self.n_alloc_calls = 0  # device allocations the library asked for

        def _alloc(nbytes, user):
            self.n_alloc_calls += 1
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            p = t.data_ptr()
            self._mem[p] = t
            return p

        def _free(ptr, user):
            self._mem.pop(int(ptr), None)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            cfg = Config(geometry, precision, nx, ny, nz, 0, dx, dy, dz, a, int(capacity), self._alloc_cb,
                         self._free_cb, None, C.c_void_p(stream.cuda_stream))
            h = C.c_void_p()
            st = lib().rt_create(C.byref(cfg), C.byref(h))
            if st != RT_OK:
                raise RTError(st, "rt_create failed")
        self.h = h
        self.stream = stream

    @classmethod
    def for_workload(cls, w, precision: int, capacity: Optional[int] = None, device: str = "cuda:0") -> "Tracer":
        cap = capacity if capacity is not None else max(w.n_rays, 1)
        return cls(w.geometry, precision, w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, cap, a=w.a, device=device)

    def _check(self, st: int):
        if st != RT_OK:
            raise RTError(st, lib().rt_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().rt_destroy(self.h)
            self.h = None
            self._mem.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- marshalling helpers -------------------------------------------------
    def _ptr_where(self, arrs):
        """Returns (pointers, where, keepalive) for a list of arrays that are
        either all numpy (host) or all CUDA tensors (device)."""
        torch = self.torch
        if all(isinstance(a, torch.Tensor) for a in arrs):
            keep = [a.contiguous() for a in arrs]
            for a in keep:
                assert a.device.type == "cuda"
            return [a.data_ptr() for a in keep], RT_DEVICE, keep
        keep = [np.ascontiguousarray(a) for a in arrs]
        return [a.ctypes.data for a in keep], RT_HOST, keep

    # -- API -------------------------------------------------------------------
    def init_background(self, U, V, N2, f, rho):
        arrs = [U, V, N2, rho] + ([f] if f is not None else [])
        torch = self.torch
        if all(isinstance(a, torch.Tensor) for a in arrs):
            arrs = [a.to(self.device, torch.float64) for a in arrs]
        else:
            arrs = [np.asarray(a, dtype=np.float64) for a in arrs]
        ptrs, where, keep = self._ptr_where(arrs)
        fp = ptrs[4] if f is not None else None
        self._check(lib().rt_init_background(self.h, ptrs[0], ptrs[1], ptrs[2], fp, ptrs[3], where))
        if where == RT_DEVICE:
            self._bg_keep = keep

    def init_background_from(self, w):
        self.init_background(w.U, w.V, w.N2, w.f, w.rho)
        if getattr(w, "G2", None) is not None:
            self.set_scale_height(w.G2)

    def set_scale_height(self, G2):
        """Gamma^2 [nz][ny][nx] (numpy or CUDA tensor), or None for Gamma = 0
        (rt_set_scale_height)."""
        if G2 is None:
            self._check(lib().rt_set_scale_height(self.h, None, RT_HOST))
            return
        torch = self.torch
        arr = G2.to(self.device, torch.float64) if isinstance(G2, torch.Tensor) else np.asarray(G2, np.float64)
        ptrs, where, keep = self._ptr_where([arr])
        self._check(lib().rt_set_scale_height(self.h, ptrs[0], where))
        if where == RT_DEVICE:
            self.stream.synchronize()

    def set_rays(self, rays: Dict[str, object]):
        torch = self.torch
        n = int(rays["x"].shape[0])
        if isinstance(rays["x"], torch.Tensor):
            arrs = [rays[f].to(self.device, torch.float64) for f in RAY_FIELDS] + [rays["id"].to(self.device, torch.int64)]
        else:
            arrs = [np.asarray(rays[f], dtype=np.float64) for f in RAY_FIELDS] + [np.asarray(rays["id"], dtype=np.int64)]
        ptrs, where, keep = self._ptr_where(arrs)
        r = Rays(*ptrs)
        self._check(lib().rt_set_rays(self.h, C.byref(r), n, where))
        if where == RT_DEVICE:
            self.stream.synchronize()

    def set_rays_host_noalloc(self, rays: Dict[str, np.ndarray]):
        """Load host (numpy) ray arrays through the library's fixed staging
        array (rt_set_rays_host_noalloc): no device allocation in the call."""
        n = int(rays["x"].shape[0])
        keep = [np.ascontiguousarray(rays[f], dtype=np.float64) for f in RAY_FIELDS] + \
            [np.ascontiguousarray(rays["id"], dtype=np.int64)]
        r = Rays(*[a.ctypes.data for a in keep])
        self._check(lib().rt_set_rays_host_noalloc(self.h, C.byref(r), n))

    def get_rays(self, device: bool = False) -> Dict[str, object]:
        n = C.c_int64(0)
        st = lib().rt_get_rays(self.h, None, C.byref(n), RT_HOST)
        if st not in (RT_OK, RT_E_ARG):
            self._check(st)
        cnt = n.value
        torch = self.torch
        if device:
            out = {f: torch.empty(max(cnt, 1), dtype=torch.float64, device=self.device) for f in RAY_FIELDS}
            out["id"] = torch.empty(max(cnt, 1), dtype=torch.int64, device=self.device)
            r = Rays(*[out[f].data_ptr() for f in RAY_FIELDS], out["id"].data_ptr())
            where = RT_DEVICE
        else:
            out = {f: np.empty(max(cnt, 1)) for f in RAY_FIELDS}
            out["id"] = np.empty(max(cnt, 1), dtype=np.int64)
            r = Rays(*[out[f].ctypes.data for f in RAY_FIELDS], out["id"].ctypes.data)
            where = RT_HOST
        n2 = C.c_int64(cnt)
        self._check(lib().rt_get_rays(self.h, C.byref(r), C.byref(n2), where))
        return {k: v[: n2.value] for k, v in out.items()}

    def get_columns(self) -> np.ndarray:
        """Parent-column key of each active ray, in get_rays() order."""
        n = C.c_int64(0)
        st = lib().rt_get_columns(self.h, None, C.byref(n), RT_HOST)
        if st not in (RT_OK, RT_E_ARG):
            self._check(st)
        out = np.empty(max(n.value, 1), dtype=np.uint32)
        n2 = C.c_int64(n.value)
        self._check(lib().rt_get_columns(self.h, out.ctypes.data, C.byref(n2), RT_HOST))
        return out[: n2.value]

    def step(self, dt: float, deposit: bool = False, surrogate: bool = False, saturate: bool = False):
        flags = ((RT_STEP_DEPOSIT if deposit else 0) | (RT_STEP_SURROGATE if surrogate else 0)
                 | (RT_STEP_SATURATE if saturate else 0))
        self._check(lib().rt_step(self.h, float(dt), flags))

    def saturate(self, dt: float, host: bool = False, kappa=None):
        """Spectral saturation of the current set (rt_saturate); returns the
        turbulent diffusivity [nz, ny, nx] float64 (a CUDA tensor, or numpy
        with host=True)."""
        shape = (self.nz, self.ny, self.nx)
        if host:
            K = np.zeros(shape) if kappa is None else kappa
            self._check(lib().rt_saturate(self.h, float(dt), K.ctypes.data, RT_HOST))
            return K
        torch = self.torch
        K = torch.empty(shape, dtype=torch.float64, device=self.device) if kappa is None else kappa
        self._check(lib().rt_saturate(self.h, float(dt), K.data_ptr(), RT_DEVICE))
        return K

    def set_frozen_columns(self, mask=None):
        """Column flags [ny*nx] (uint8, 1 = frozen) for step(surrogate=True):
        a numpy array or a CUDA tensor; None clears them."""
        torch = self.torch
        if mask is None:
            self._check(lib().rt_set_frozen_columns(self.h, None, RT_DEVICE))
        elif isinstance(mask, torch.Tensor):
            m = mask.to(device=self.device, dtype=torch.uint8).contiguous()
            assert m.numel() == self.nx * self.ny
            self._check(lib().rt_set_frozen_columns(self.h, m.data_ptr(), RT_DEVICE))
            self._frozen_ref = m  # alive until the stream has copied it
        else:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            assert m.size == self.nx * self.ny
            self._check(lib().rt_set_frozen_columns(self.h, m.ctypes.data, RT_HOST))

    def features(self, out=None, host: bool = False):
        """Surrogate input features [ny*nx][3*nz + 48] float32 of the current
        state: a CUDA tensor, or a numpy array with host=True."""
        torch = self.torch
        shape = (self.nx * self.ny, 3 * self.nz + 48)
        if host:
            X = np.zeros(shape, np.float32) if out is None else out
            self._check(lib().rt_features(self.h, X.ctypes.data, RT_HOST))
            return X
        X = torch.empty(shape, dtype=torch.float32, device=self.device) if out is None else out
        self._check(lib().rt_features(self.h, X.data_ptr(), RT_DEVICE))
        return X

    def deposit(self, flux=None, drag=None, host: bool = False):
        """Returns (flux [6, nz+1, ny, nx], drag [2, nz, ny, nx]) float64: CUDA
        tensors by default, numpy arrays with host=True."""
        torch = self.torch
        nz, ny, nx = self.nz, self.ny, self.nx
        if host:
            flux = np.zeros((6, nz + 1, ny, nx)) if flux is None else flux
            drag = np.zeros((2, nz, ny, nx)) if drag is None else drag
            self._check(lib().rt_deposit_flux(self.h, flux.ctypes.data, drag.ctypes.data, RT_HOST))
            return flux, drag
        if flux is None:
            flux = torch.empty((6, nz + 1, ny, nx), dtype=torch.float64, device=self.device)
        if drag is None:
            drag = torch.empty((2, nz, ny, nx), dtype=torch.float64, device=self.device)
        self._check(lib().rt_deposit_flux(self.h, flux.data_ptr(), drag.data_ptr(), RT_DEVICE))
        return flux, drag

    def _two_outputs(self, fn, shapes, smooth, host):
        torch = self.torch
        if host:
            outs = [np.zeros(s) for s in shapes]
            self._check(fn(self.h, outs[0].ctypes.data, outs[1].ctypes.data, 1 if smooth else 0, RT_HOST))
            return tuple(outs)
        outs = [torch.empty(s, dtype=torch.float64, device=self.device) for s in shapes]
        self._check(fn(self.h, outs[0].data_ptr(), outs[1].data_ptr(), 1 if smooth else 0, RT_DEVICE))
        return tuple(outs)

    def full_fluxes(self, smooth: bool = False, host: bool = False):
        """(flux [8, nz+1, ny, nx], tendencies [3, nz, ny, nx]) of the full
        flux formulation (rt_full_fluxes)."""
        nz, ny, nx = self.nz, self.ny, self.nx
        return self._two_outputs(lib().rt_full_fluxes, [(8, nz + 1, ny, nx), (3, nz, ny, nx)], smooth, host)

    def budget(self, smooth: bool = False, host: bool = False):
        """(fields [4, nz+1, ny, nx], terms [2, nz, ny, nx]) of the wave-action
        budget (rt_budget)."""
        nz, ny, nx = self.nz, self.ny, self.nx
        return self._two_outputs(lib().rt_budget, [(4, nz + 1, ny, nx), (2, nz, ny, nx)], smooth, host)

    def split_merge(self, alpha: float, n_max: int = 0, mode: int = RT_SPLIT_ONLY) -> dict:
        s = Stats()
        self._check(lib().rt_split_merge(self.h, float(alpha), int(n_max), int(mode), C.byref(s)))
        return s.as_dict()

    def launch(self, z_launch: float, dt: float, t_solstice: float = 0.0, F_s: float = 2.4e-3, F_w: float = 8e-3,
               lambda_h: float = 300e3, c_min: float = 2.0, c_max: float = 62.0, c_center: float = 25.0,
               c_width: float = 15.0, n_speeds: int = 8, flux_col=None) -> int:
        """Launch from the ghost layer (rt_launch); returns the count.
        flux_col ([ny*nx] Pa, numpy or CUDA tensor) is required on the box;
        on the sphere None selects the latitudinal background source."""
        p = LaunchParams(float(z_launch), float(dt), float(t_solstice), float(F_s), float(F_w), float(lambda_h),
                         float(c_min), float(c_max), float(c_center), float(c_width), int(n_speeds), RT_HOST, None)
        keep = None
        if flux_col is not None:
            torch = self.torch
            if isinstance(flux_col, torch.Tensor):
                arr = flux_col.to(self.device, torch.float64).contiguous().reshape(-1)
            else:
                arr = np.asarray(flux_col, dtype=np.float64).reshape(-1)
            ptrs, where, keep = self._ptr_where([arr])
            p.flux_col, p.where = ptrs[0], where
        cnt = C.c_int64(0)
        self._check(lib().rt_launch(self.h, C.byref(p), C.byref(cnt)))
        del keep
        return int(cnt.value)

    PROFILE_CLASSES = ("step", "sort", "deposit", "drag", "split_merge", "stats", "saturation", "c7")

    def profile(self, on: bool = True):
        self._check(lib().rt_profile(self.h, 1 if on else 0))

    def profile_read(self) -> dict:
        ms = np.zeros(8)
        n = np.zeros(8, dtype=np.int64)
        self._check(lib().rt_profile_read(self.h, ms.ctypes.data, n.ctypes.data))
        return {c: (float(ms[i]), int(n[i])) for i, c in enumerate(self.PROFILE_CLASSES) if n[i]}

    def stats(self) -> dict:
        """rt_get_stats; RT_E_NUMERIC (a volume was deactivated as
        non-finite or degenerate since the last call) raises RTError with the
        statistics attached, first_bad_id among them."""
        s = Stats()
        st = lib().rt_get_stats(self.h, C.byref(s))
        if st == RT_E_NUMERIC:
            raise RTError(st, lib().rt_last_error(self.h).decode(), s.as_dict())
        self._check(st)
        return s.as_dict()
