"""FP64 CPU oracle for the MS-GWaM-3D ray-volume hot path -- TEST INFRASTRUCTURE.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It is a ctypes wrapper around ``orc.c`` (plain
C, double precision, one ray at a time) plus the numpy reference of the
column surrogate in ``mlp.py``.  It shares no code with the GPU library and
never imports it.

Parity status: see ``orc.h``; every oracle function is pinned by the
``-m "not gpu"`` tests except the choice of merge partners (a reading),
which is "parity unpinned" beyond its conserved sums.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")

ACTIVE, GONE_TOP, GONE_BOTTOM, GONE_POLE, INVALID, MERGED, CAPPED = range(7)
RAY_FIELDS = ("x", "y", "z", "k", "l", "m", "dx", "dy", "dz", "px", "py", "pz", "n")


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so (gcc, -ffp-contract=off, OpenMP)."""
    src = os.path.join(_HERE, "orc.c")
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(src):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Bg(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("a", C.c_double)] + \
               [(n, C.c_void_p) for n in ("U", "V", "N2", "f2", "rho", "Ux", "Uy", "Uz", "Vx", "Vy", "Vz",
                                           "N2x", "N2y", "N2z", "f2y", "f", "G2", "G2x", "G2y", "G2z")]


class _Rays(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in RAY_FIELDS + ("id", "state", "col")]


class Tally(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_active", "n_top", "n_bottom", "n_pole", "n_invalid",
                                         "n_merged", "n_capped", "n_split")] + \
               [(n, C.c_double) for n in ("sum_W", "sum_kW", "sum_lW", "sum_mW", "removed_W")] + \
               [("n_launched", C.c_int64), ("launched_W", C.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class LaunchParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("z_launch", "dt", "t_solstice", "F_s", "F_w", "lambda_h", "c_min", "c_max",
                                          "c_center", "c_width")] + \
               [("n_speeds", C.c_int32), ("flux_col", C.c_void_p)]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _load(_LIB_PATH)
    return _lib


def build_variant(source_text: str, path: str) -> str:
    """Compile a modified copy of the oracle's C source (same flags as
    build()) into `path`.  Used only by the tests that plant a mistake in the
    oracle to show that its pins catch it."""
    src = os.path.splitext(path)[0] + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                    "-shared", "-w", "-I", _HERE, "-o", path, src, "-lm"], check=True)
    return path


def source_text() -> str:
    with open(os.path.join(_HERE, "orc.c")) as f:
        return f.read()


class using_library:
    """Context manager: route every oracle call through the library at
    `path` (a variant built by build_variant) and restore the real one."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _load(path: str) -> C.CDLL:
    L = C.CDLL(path)
    P = C.c_void_p
    L.orc_prepare.argtypes = [P]
    L.orc_interp.argtypes = [P, C.c_double, C.c_double, C.c_double, P]
    L.orc_dispersion.argtypes = [C.c_double] * 5 + [P]
    L.orc_dispersion_g.argtypes = [C.c_double] * 6 + [P]
    L.orc_interp_gamma.argtypes = [P, C.c_double, C.c_double, C.c_double, P]
    L.orc_rhs.argtypes = [P, P, P]
    L.orc_step.argtypes = [P, P, C.c_int64, C.c_double, P]
    L.orc_keys.argtypes = [P, P, C.c_int64]
    L.orc_deposit.argtypes = [P, P, C.c_int64, P]
    L.orc_drag.argtypes = [P, P, P]
    L.orc_split.argtypes = [P, P, C.c_int64, C.c_int64, C.c_double, P, P]
    L.orc_split.restype = C.c_int64
    L.orc_merge.argtypes = [P, P, C.c_int64, C.c_int32, P]
    L.orc_cap.argtypes = [P, P, C.c_int64, C.c_int32, P]
    L.orc_stats.argtypes = [P, C.c_int64, P]
    L.orc_features.argtypes = [P, P, C.c_int64, P]
    L.orc_saturation.argtypes = [P, P, C.c_int64, C.c_double, P, P, P, C.c_int]
    L.orc_full_fluxes.argtypes = [P, P, C.c_int64, P, C.c_int]
    L.orc_smooth.argtypes = [P, P, C.c_int, P]
    L.orc_divergence.argtypes = [P, P, P, P, P]
    L.orc_full_tendencies.argtypes = [P, P, P]
    L.orc_budget.argtypes = [P, P, C.c_int64, P, C.c_int]
    L.orc_budget_terms.argtypes = [P, P, P]
    L.orc_launch_flux.argtypes = [P, C.c_int, P]
    L.orc_launch_flux.restype = C.c_double
    L.orc_launch.argtypes = [P, P, C.c_int64, C.c_int64, P, P, P]
    L.orc_launch.restype = C.c_int64
    L.orc_num_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    return L


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class Background:
    """A grid plus resolved fields U, V, N2 [nz][ny][nx], Coriolis parameter
    f [ny], reference density rho [nz] and optionally the scale-height
    correction Gamma^2 [nz][ny][nx] (None: Gamma = 0); gradients are filled
    on creation."""

    def __init__(self, geometry, nx, ny, nz, dx, dy, dz, x0, y0, a, U, V, N2, f, rho, G2=None):
        c = lambda v: np.ascontiguousarray(v, dtype=np.float64)
        self.U, self.V, self.N2 = c(U), c(V), c(N2)
        f = c(f)
        self.f = f
        self.f2 = c(f * f)
        self.rho = c(rho)
        shape = (nz, ny, nx)
        for arr in (self.U, self.V, self.N2):
            assert arr.shape == shape
        assert self.f2.shape == (ny,) and self.rho.shape == (nz,)
        self.grads = {n: np.zeros(shape) for n in ("Ux", "Uy", "Uz", "Vx", "Vy", "Vz", "N2x", "N2y", "N2z")}
        self.f2y = np.zeros(ny)
        b = _Bg()
        b.geometry, b.nx, b.ny, b.nz = geometry, nx, ny, nz
        b.dx, b.dy, b.dz, b.x0, b.y0, b.a = dx, dy, dz, x0, y0, a
        b.U, b.V, b.N2, b.f2, b.rho = (_ptr(v) for v in (self.U, self.V, self.N2, self.f2, self.rho))
        for n, v in self.grads.items():
            setattr(b, n, _ptr(v))
        b.f2y = _ptr(self.f2y)
        b.f = _ptr(self.f)
        self.G2 = None
        if G2 is not None:
            self.G2 = c(G2)
            assert self.G2.shape == shape
            self.G2grads = {n: np.zeros(shape) for n in ("G2x", "G2y", "G2z")}
            b.G2 = _ptr(self.G2)
            for n, v in self.G2grads.items():
                setattr(b, n, _ptr(v))
        self._b = b
        self.geometry, self.nx, self.ny, self.nz = geometry, nx, ny, nz
        self.dx, self.dy, self.dz, self.x0, self.y0, self.a = dx, dy, dz, x0, y0, a
        lib().orc_prepare(C.byref(b))

    @classmethod
    def from_workload(cls, w) -> "Background":
        return cls(w.geometry, w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.x0, w.y0, w.a, w.U, w.V, w.N2, w.f, w.rho,
                   getattr(w, "G2", None))

    @property
    def ref(self):
        return C.byref(self._b)

    def interp(self, x, y, z) -> np.ndarray:
        out = np.zeros(14)
        lib().orc_interp(self.ref, float(x), float(y), float(z), _ptr(out))
        return out

    def interp_gamma(self, x, y, z) -> np.ndarray:
        """Gamma^2 and its x, y, z gradients at a point (zeros without Gamma)."""
        out = np.zeros(4)
        lib().orc_interp_gamma(self.ref, float(x), float(y), float(z), _ptr(out))
        return out

    def rhs(self, Y) -> np.ndarray:
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        F = np.zeros(9)
        lib().orc_rhs(self.ref, _ptr(Y), _ptr(F))
        return F


def dispersion(N2, f2, k, l, m, G2=None) -> np.ndarray:
    """(omega_hat, cg_x, cg_y, cg_z) intrinsic; G2 the scale-height
    correction Gamma^2 (None: Gamma = 0)."""
    out = np.zeros(4)
    if G2 is None:
        lib().orc_dispersion(float(N2), float(f2), float(k), float(l), float(m), _ptr(out))
    else:
        lib().orc_dispersion_g(float(N2), float(f2), float(G2), float(k), float(l), float(m), _ptr(out))
    return out


class RaySet:
    """SoA ray volumes with spare capacity for splitting.  Arrays are kept in
    ascending id order (splitting appends larger ids at the end)."""

    def __init__(self, rays: Dict[str, np.ndarray], capacity: Optional[int] = None):
        n = int(rays["x"].shape[0])
        cap = max(int(capacity or n), n, 1)
        self.cap = cap
        self.n = n
        self.a = {}
        for f in RAY_FIELDS:
            arr = np.zeros(cap)
            arr[:n] = rays[f]
            self.a[f] = arr
        self.a["id"] = np.zeros(cap, np.int64)
        self.a["id"][:n] = rays["id"]
        self.a["state"] = np.full(cap, 255, np.uint8)
        self.a["state"][:n] = ACTIVE
        self.a["col"] = np.full(cap, -1, np.int32)
        s = _Rays()
        for f in RAY_FIELDS + ("id", "state", "col"):
            setattr(s, f, _ptr(self.a[f]))
        self._s = s

    @property
    def ref(self):
        return C.byref(self._s)

    def __getitem__(self, f):
        return self.a[f][: self.n]

    def active(self) -> np.ndarray:
        return self.a["state"][: self.n] == ACTIVE

    def snapshot(self, only_active: bool = True) -> Dict[str, np.ndarray]:
        sel = self.active() if only_active else slice(None)
        return {f: self.a[f][: self.n][sel].copy() for f in RAY_FIELDS + ("id", "state", "col")}


def step(bg: Background, rs: RaySet, dt: float) -> dict:
    t = Tally()
    lib().orc_step(bg.ref, rs.ref, rs.n, float(dt), C.byref(t))
    return t.as_dict()


def keys(bg: Background, rs: RaySet) -> None:
    lib().orc_keys(bg.ref, rs.ref, rs.n)


def deposit(bg: Background, rs: RaySet, cols: Optional[np.ndarray] = None) -> np.ndarray:
    """Flux fields [6][nz+1][ny][nx].  The parent column of each active ray
    is computed from its position unless `cols` (one per ray of the set, -1
    for inactive) supplies that integer decision from elsewhere -- used to
    compare a lower-precision path whose rounding put a ray a hair's breadth
    across a cell face: both sides then take the same decision."""
    if cols is None:
        keys(bg, rs)
    else:
        cols = np.asarray(cols, dtype=np.int32)
        assert cols.shape == (rs.n,)
        rs.a["col"][: rs.n] = cols
    flux = np.zeros((6, bg.nz + 1, bg.ny, bg.nx))
    lib().orc_deposit(bg.ref, rs.ref, rs.n, _ptr(flux))
    return flux


def drag(bg: Background, flux: np.ndarray) -> np.ndarray:
    flux = np.ascontiguousarray(flux, dtype=np.float64)
    assert flux.shape == (6, bg.nz + 1, bg.ny, bg.nx)
    out = np.zeros((2, bg.nz, bg.ny, bg.nx))
    lib().orc_drag(bg.ref, _ptr(flux), _ptr(out))
    return out


def split(bg: Background, rs: RaySet, alpha: float, next_id: Optional[int] = None) -> dict:
    t = Tally()
    nid = C.c_int64(int(rs.a["id"][: rs.n].max()) + 1 if next_id is None and rs.n else (next_id or 0))
    out = lib().orc_split(bg.ref, rs.ref, rs.n, rs.cap, float(alpha), C.byref(nid), C.byref(t))
    if out < 0:
        raise RuntimeError("split exceeds capacity")
    rs.n = int(out)
    d = t.as_dict()
    d["next_id"] = nid.value
    return d


def merge(bg: Background, rs: RaySet, n_max: int) -> dict:
    t = Tally()
    lib().orc_merge(bg.ref, rs.ref, rs.n, int(n_max), C.byref(t))
    return t.as_dict()


def cap(bg: Background, rs: RaySet, n_max: int) -> dict:
    t = Tally()
    lib().orc_cap(bg.ref, rs.ref, rs.n, int(n_max), C.byref(t))
    return t.as_dict()


def stats(rs: RaySet) -> dict:
    t = Tally()
    lib().orc_stats(rs.ref, rs.n, C.byref(t))
    return t.as_dict()


def features(bg: Background, rs: RaySet, cols: Optional[np.ndarray] = None) -> np.ndarray:
    """Surrogate input features [nx*ny][3*nz + 48] of the current state
    (background profiles and per-sector ray-spectrum moments, see
    orc_features).  `cols` as in deposit()."""
    if cols is None:
        keys(bg, rs)
    else:
        cols = np.asarray(cols, dtype=np.int32)
        assert cols.shape == (rs.n,)
        rs.a["col"][: rs.n] = cols
    X = np.zeros((bg.nx * bg.ny, 3 * bg.nz + 48))
    lib().orc_features(bg.ref, rs.ref, rs.n, _ptr(X))
    return X


def saturation(bg: Background, rs: RaySet, dt: float, cols: Optional[np.ndarray] = None):
    """Spectral saturation of the current state (orc_saturation): returns
    (P, Q, kappa) on [nz][ny][nx] and damps the densities of the active
    volumes in place.  `cols` as in deposit()."""
    shape = (bg.nz, bg.ny, bg.nx)
    P, Q, K = np.zeros(shape), np.zeros(shape), np.zeros(shape)
    if cols is not None:
        cols = np.asarray(cols, dtype=np.int32)
        assert cols.shape == (rs.n,)
        rs.a["col"][: rs.n] = cols
    lib().orc_saturation(bg.ref, rs.ref, rs.n, float(dt), _ptr(P), _ptr(Q), _ptr(K), 0 if cols is None else 1)
    return P, Q, K


def _given_cols(rs: RaySet, cols) -> int:
    if cols is None:
        return 0
    cols = np.asarray(cols, dtype=np.int32)
    assert cols.shape == (rs.n,)
    rs.a["col"][: rs.n] = cols
    return 1


def full_fluxes(bg: Background, rs: RaySet, cols: Optional[np.ndarray] = None) -> np.ndarray:
    """Full flux formulation (orc_full_fluxes): [8][nz+1][ny][nx] = Fxu, Fxv,
    Fyu, Fyv, Bu, Bv (levels), Fzu, Fzv (interfaces).  `cols` as in
    deposit()."""
    out = np.zeros((8, bg.nz + 1, bg.ny, bg.nx))
    given = _given_cols(rs, cols)
    lib().orc_full_fluxes(bg.ref, rs.ref, rs.n, _ptr(out), given)
    return out


def smooth(bg: Background, fields: np.ndarray) -> np.ndarray:
    """3/2/1-weighted horizontal smoothing of every [ny][nx] slice."""
    f = np.ascontiguousarray(fields, dtype=np.float64)
    assert f.shape[-2:] == (bg.ny, bg.nx)
    out = np.zeros_like(f)
    lib().orc_smooth(bg.ref, _ptr(f), int(f.size // (bg.ny * bg.nx)), _ptr(out))
    return out


def divergence(bg: Background, Fx, Fy, Fz=None) -> np.ndarray:
    """div(Fx, Fy, Fz) on [nz][ny][nx]; Fx, Fy [nz+1][ny][nx] (levels), Fz on
    interfaces or None."""
    c = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    Fx, Fy = c(Fx), c(Fy)
    Fz = c(Fz) if Fz is not None else None
    out = np.zeros((bg.nz, bg.ny, bg.nx))
    lib().orc_divergence(bg.ref, _ptr(Fx), _ptr(Fy), _ptr(Fz) if Fz is not None else None, _ptr(out))
    return out


def full_tendencies(bg: Background, flux8: np.ndarray) -> np.ndarray:
    """du, dv, db [3][nz][ny][nx] of the full formulation (orc_full_tendencies)."""
    f = np.ascontiguousarray(flux8, dtype=np.float64)
    assert f.shape == (8, bg.nz + 1, bg.ny, bg.nx)
    out = np.zeros((3, bg.nz, bg.ny, bg.nx))
    lib().orc_full_tendencies(bg.ref, _ptr(f), _ptr(out))
    return out


def budget(bg: Background, rs: RaySet, cols: Optional[np.ndarray] = None) -> np.ndarray:
    """Wave-action budget fields [4][nz+1][ny][nx]: A, cgx A, cgy A (levels),
    cgz A (interfaces).  `cols` as in deposit()."""
    out = np.zeros((4, bg.nz + 1, bg.ny, bg.nx))
    given = _given_cols(rs, cols)
    lib().orc_budget(bg.ref, rs.ref, rs.n, _ptr(out), given)
    return out


def budget_terms(bg: Background, fields4: np.ndarray) -> np.ndarray:
    """Horizontal and vertical propagation terms [2][nz][ny][nx]."""
    f = np.ascontiguousarray(fields4, dtype=np.float64)
    out = np.zeros((2, bg.nz, bg.ny, bg.nx))
    lib().orc_budget_terms(bg.ref, _ptr(f), _ptr(out))
    return out


def launch_params(z_launch, dt, t_solstice=0.0, F_s=2.4e-3, F_w=8.0e-3, lambda_h=300e3, c_min=2.0, c_max=62.0,
                  c_center=25.0, c_width=15.0, n_speeds=8, flux_col=None):
    """Parameters of orc_launch; flux_col (numpy [ny*nx], Pa) is kept alive
    on the returned structure."""
    p = LaunchParams(z_launch, dt, t_solstice, F_s, F_w, lambda_h, c_min, c_max, c_center, c_width, n_speeds, None)
    if flux_col is not None:
        p._flux = np.ascontiguousarray(flux_col, dtype=np.float64)
        p.flux_col = _ptr(p._flux)
    return p


def launch_flux(bg: Background, j: int, p: LaunchParams) -> float:
    return float(lib().orc_launch_flux(bg.ref, int(j), C.byref(p)))


def launch(bg: Background, rs: RaySet, p: LaunchParams, next_id: Optional[int] = None) -> dict:
    """Append the volumes launched this step (orc_launch); returns the tally
    with the next free id."""
    t = Tally()
    nid = C.c_int64(int(rs.a["id"][: rs.n].max()) + 1 if next_id is None and rs.n else (next_id or 0))
    out = lib().orc_launch(bg.ref, rs.ref, rs.n, rs.cap, C.byref(p), C.byref(nid), C.byref(t))
    if out < 0:
        raise RuntimeError("launch exceeds capacity")
    rs.n = int(out)
    d = t.as_dict()
    d["next_id"] = nid.value
    return d


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())
