"""ctypes wrapper of the FP64 CPU oracle (``cbct_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and this package never imports the GPU library.

Geometries are duck-typed: any object with the attributes of a scan geometry
(nx, ny, nz, hx, hy, hz, nu, nv, pu, pv, sad, sdd, n_views, angles,
sample_ratio) works.  Arrays are float64, volumes (Nz, Ny, Nx), projections
(Nviews, Nv, Nu).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cbct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Geom(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("nu", C.c_int), ("nv", C.c_int), ("pu", C.c_double), ("pv", C.c_double),
                ("sad", C.c_double), ("sdd", C.c_double), ("nviews", C.c_int),
                ("angles", C.POINTER(C.c_double)), ("dtau", C.c_double)]


class Params(C.Structure):
    _fields_ = [("lam", C.c_double), ("step", C.c_double), ("tv_eps", C.c_double),
                ("armijo_c", C.c_double), ("backtrack", C.c_double), ("rof_tol", C.c_double),
                ("rof_max_iter", C.c_int), ("rof_max_backtrack", C.c_int), ("step1_eq6", C.c_int),
                ("conv_tol", C.c_double), ("projector", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("trace", C.POINTER(C.c_int)), ("trace_cap", C.c_int), ("trace_len", C.c_int),
                ("rof_e", C.POINTER(C.c_double)), ("energy", C.POINTER(C.c_double)),
                ("energy_cap", C.c_int), ("energy_len", C.c_int), ("t_used", C.c_double * 16)]


_D = C.POINTER(C.c_double)
_L = C.POINTER(C.c_long)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
            P = C.POINTER
            L.orc_forward.argtypes = [P(Geom), _D, _D]
            L.orc_forward_rays.argtypes = [P(Geom), _D, C.c_long, _L, _D]
            L.orc_adjoint.argtypes = [P(Geom), _D, _D]
            L.orc_adjoint_voxels.argtypes = [P(Geom), _D, C.c_long, _L, _D]
            L.orc_backproject_eq6.argtypes = [P(Geom), _D, _D]
            L.orc_forward_siddon.argtypes = [P(Geom), _D, _D]
            L.orc_adjoint_siddon.argtypes = [P(Geom), _D, _D]
            L.orc_forward_siddon_rays.argtypes = [P(Geom), _D, C.c_long, _L, _D]
            L.orc_adjoint_siddon_voxels.argtypes = [P(Geom), _D, C.c_long, _L, _D]
            L.orc_tv_energy.argtypes = [P(Geom), _D, C.c_double]
            L.orc_tv_energy.restype = C.c_double
            L.orc_tv_grad.argtypes = [P(Geom), _D, C.c_double, _D]
            L.orc_schur.argtypes = [P(Geom), _D, _D]
            L.orc_schur_step.argtypes = [P(Geom)]
            L.orc_schur_step.restype = C.c_double
            L.orc_fbs.argtypes = [P(Geom), _D, _D, C.c_int, P(Params), C.c_double, P(Stats), C.c_int]
            L.orc_rof.argtypes = [P(Geom), _D, _D, P(Params), C.c_double, P(Stats)]
            L.orc_prolong.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D]
            L.orc_restrict.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D]
            L.orc_bin_detector.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _D, _D]
            L.orc_level_geom.argtypes = [P(Geom), C.c_int, C.c_int, P(Geom)]
            L.orc_forward_level.argtypes = [P(Geom), C.c_int, C.c_int, _D, _D]
            L.orc_reconstruct.argtypes = [P(Geom), C.c_int, P(C.c_int), P(Params), C.c_int, _D, _D, _D,
                                          P(Stats)]
            L.orc_reconstruct.restype = C.c_int
            L.orc_set_fault.argtypes = [C.c_int]
            L.orc_set_threads.argtypes = [C.c_int]
            L.orc_get_threads.restype = C.c_int
            _lib = L
    return _lib


def set_fault(k: int) -> None:
    lib().orc_set_fault(int(k))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _GeomHolder:
    """Keeps the angle array alive with the ctypes struct."""

    def __init__(self, g):
        self.angles = None
        if getattr(g, "angles", None) is not None:
            self.angles = _f64(np.asarray(g.angles))
        dtau = float(getattr(g, "sample_ratio", 1.0)) * min(g.hx, g.hy)
        self.s = Geom(int(g.nx), int(g.ny), int(g.nz), float(g.hx), float(g.hy), float(g.hz),
                      int(g.nu), int(g.nv), float(g.pu), float(g.pv), float(g.sad), float(g.sdd),
                      int(g.n_views), _ptr(self.angles) if self.angles is not None else None, dtau)
        self.vol_shape = (g.nz, g.ny, g.nx)
        self.proj_shape = (g.n_views, g.nv, g.nu)

    def ref(self):
        return C.byref(self.s)


def forward(g, f) -> np.ndarray:
    """P f (Eq. 1 as the trilinear ray sum)."""
    h = _GeomHolder(g)
    f = _f64(f).reshape(h.vol_shape)
    y = np.empty(h.proj_shape)
    lib().orc_forward(h.ref(), _ptr(f), _ptr(y))
    return y


def forward_rays(g, f, rays) -> np.ndarray:
    h = _GeomHolder(g)
    f = _f64(f).reshape(h.vol_shape)
    rays = np.ascontiguousarray(rays, dtype=np.int64)
    out = np.empty(len(rays))
    lib().orc_forward_rays(h.ref(), _ptr(f), len(rays), rays.ctypes.data_as(_L), _ptr(out))
    return out


def adjoint(g, y) -> np.ndarray:
    """P^T y by the transposed scatter loop."""
    h = _GeomHolder(g)
    y = _f64(y).reshape(h.proj_shape)
    f = np.empty(h.vol_shape)
    lib().orc_adjoint(h.ref(), _ptr(y), _ptr(f))
    return f


def forward_siddon(g, f) -> np.ndarray:
    """Siddon's exact radiological path through the piecewise-constant volume."""
    h = _GeomHolder(g)
    f = _f64(f).reshape(h.vol_shape)
    y = np.empty(h.proj_shape)
    lib().orc_forward_siddon(h.ref(), _ptr(f), _ptr(y))
    return y


def adjoint_siddon(g, y) -> np.ndarray:
    """Transpose of forward_siddon by the scatter loop."""
    h = _GeomHolder(g)
    y = _f64(y).reshape(h.proj_shape)
    f = np.empty(h.vol_shape)
    lib().orc_adjoint_siddon(h.ref(), _ptr(y), _ptr(f))
    return f


def forward_siddon_rays(g, f, rays) -> np.ndarray:
    """forward_siddon at selected flat ray indices."""
    h = _GeomHolder(g)
    f = _f64(f).reshape(h.vol_shape)
    rays = np.ascontiguousarray(rays, dtype=np.int64)
    out = np.empty(len(rays))
    lib().orc_forward_siddon_rays(h.ref(), _ptr(f), len(rays), rays.ctypes.data_as(_L), _ptr(out))
    return out


def adjoint_siddon_voxels(g, y, voxels) -> np.ndarray:
    """adjoint_siddon at selected flat voxel indices, each from its cube's chords with the rays
    whose pixels lie in the cube's projected bounding box."""
    h = _GeomHolder(g)
    y = _f64(y).reshape(h.proj_shape)
    voxels = np.ascontiguousarray(voxels, dtype=np.int64)
    out = np.empty(len(voxels))
    lib().orc_adjoint_siddon_voxels(h.ref(), _ptr(y), len(voxels), voxels.ctypes.data_as(_L), _ptr(out))
    return out


def backproject_eq6(g, T) -> np.ndarray:
    """The voxel-driven Eq. 6 backprojector (bilinear T at (u*, v*), weight L^3/(L0 l^2)),
    scaled by hx hy hz / (pu pv)."""
    h = _GeomHolder(g)
    T = _f64(T).reshape(h.proj_shape)
    f = np.empty(h.vol_shape)
    lib().orc_backproject_eq6(h.ref(), _ptr(T), _ptr(f))
    return f


def adjoint_voxels(g, y, voxels) -> np.ndarray:
    h = _GeomHolder(g)
    y = _f64(y).reshape(h.proj_shape)
    voxels = np.ascontiguousarray(voxels, dtype=np.int64)
    out = np.empty(len(voxels))
    lib().orc_adjoint_voxels(h.ref(), _ptr(y), len(voxels), voxels.ctypes.data_as(_L), _ptr(out))
    return out


def forward_level(g, level: int, f, bin_detector: bool = True) -> np.ndarray:
    """P of multigrid level `level` of geometry g (the oracle's own level geometry: dims halved
    per level over the same box, detector binned, sample spacing scaled) applied to f."""
    h = _GeomHolder(g)
    k = 1 << level
    nz, ny, nx = g.nz // k, g.ny // k, g.nx // k
    nv, nu = (g.nv // k, g.nu // k) if bin_detector else (g.nv, g.nu)
    f = _f64(f).reshape(nz, ny, nx)
    y = np.empty((g.n_views, nv, nu))
    lib().orc_forward_level(h.ref(), int(level), int(bool(bin_detector)), _ptr(f), _ptr(y))
    return y


def tv_energy(g, f, eps: float = 1e-5) -> float:
    h = _GeomHolder(g)
    return float(lib().orc_tv_energy(h.ref(), _ptr(_f64(f).reshape(h.vol_shape)), eps))


def tv_grad(g, f, eps: float = 1e-5) -> np.ndarray:
    h = _GeomHolder(g)
    out = np.empty(h.vol_shape)
    lib().orc_tv_grad(h.ref(), _ptr(_f64(f).reshape(h.vol_shape)), eps, _ptr(out))
    return out


def schur(g):
    h = _GeomHolder(g)
    a, b = C.c_double(), C.c_double()
    lib().orc_schur(h.ref(), C.byref(a), C.byref(b))
    return a.value, b.value


def schur_step(g) -> float:
    h = _GeomHolder(g)
    return float(lib().orc_schur_step(h.ref()))


def prolong(coarse) -> np.ndarray:
    c = _f64(coarse)
    nz, ny, nx = c.shape
    out = np.empty((2 * nz, 2 * ny, 2 * nx))
    lib().orc_prolong(nx, ny, nz, _ptr(c), _ptr(out))
    return out


def restrict(fine) -> np.ndarray:
    f = _f64(fine)
    NZ, NY, NX = f.shape
    out = np.empty((NZ // 2, NY // 2, NX // 2))
    lib().orc_restrict(NX // 2, NY // 2, NZ // 2, _ptr(f), _ptr(out))
    return out


def bin_detector(Y, factor: int) -> np.ndarray:
    Y = _f64(Y)
    V, nv, nu = Y.shape
    out = np.empty((V, nv // factor, nu // factor))
    lib().orc_bin_detector(V, nv, nu, factor, _ptr(Y), _ptr(out))
    return out


DEFAULTS = dict(tv_eps=1e-5, armijo_c=0.01, backtrack=0.6, rof_tol=1e-3, rof_max_iter=50, rof_max_backtrack=30,
                step1_eq6=False, conv_tol=0.0, projector=0)


def _params(lam, step, **kw):
    p = dict(DEFAULTS)
    p.update(kw)
    return Params(float(lam), float(step), p["tv_eps"], p["armijo_c"], p["backtrack"], p["rof_tol"],
                  int(p["rof_max_iter"]), int(p["rof_max_backtrack"]), int(bool(p["step1_eq6"])),
                  float(p["conv_tol"]), int(p["projector"]))


class Result:
    def __init__(self, f, trace, rof_e, energy, t_used):
        self.f = f
        self.trace = trace          # (n, 4) int: level, outer, inner, m
        self.rof_e = rof_e          # (n, 3): E0, trial energy at the last tested step, G
        self.energy = energy        # E(f_k) per level, coarsest first
        self.t_used = t_used


def _stats(cap_trace: int, cap_energy: int):
    tr = np.zeros((cap_trace, 4), dtype=np.int32)
    re = np.zeros((cap_trace, 3))
    en = np.zeros(cap_energy)
    st = Stats(tr.ctypes.data_as(C.POINTER(C.c_int)), cap_trace, 0, _ptr(re), _ptr(en), cap_energy, 0)
    return st, tr, re, en


def reconstruct(g, Y, lam: float, iters, levels: int = 1, step: float = 0.0, bin_detector: bool = True,
                d_init=None, **kw) -> Result:
    """Algorithm A1 with the multigrid cascade; returns the finest-level volume and traces."""
    h = _GeomHolder(g)
    iters = list(iters)
    assert len(iters) == levels
    Y = _f64(Y).reshape(h.proj_shape)
    out = np.empty(h.vol_shape)
    cap_t = sum(iters) * 51 + 8
    st, tr, re, en = _stats(cap_t, sum(iters) + levels + 2)
    it = (C.c_int * levels)(*iters)
    pr = _params(lam, step, **kw)
    di = _f64(d_init).reshape(h.vol_shape) if d_init is not None else None
    rc = lib().orc_reconstruct(h.ref(), levels, it, C.byref(pr), int(bool(bin_detector)), _ptr(Y),
                               _ptr(di) if di is not None else None, _ptr(out), C.byref(st))
    if rc != 0:
        raise ValueError("oracle: invalid reconstruction arguments (grid not divisible by 2^(levels-1)?)")
    n = min(st.trace_len, cap_t)
    return Result(out, tr[:n].copy(), re[:n].copy(), en[:st.energy_len].copy(), list(st.t_used)[:levels])


def rof(g, gvol, lam: float, t: float, **kw) -> Result:
    h = _GeomHolder(g)
    gv = _f64(gvol).reshape(h.vol_shape)
    u = np.empty(h.vol_shape)
    cap = 64
    st, tr, re, en = _stats(cap, 4)
    pr = _params(lam, t, **kw)
    lib().orc_rof(h.ref(), _ptr(gv), _ptr(u), C.byref(pr), float(t), C.byref(st))
    n = min(st.trace_len, cap)
    return Result(u, tr[:n].copy(), re[:n].copy(), None, [t])


def fbs(g, Y, f0, lam: float, t: float, iters: int, **kw) -> Result:
    """Single-grid Algorithm A1 from f0 with a given t."""
    h = _GeomHolder(g)
    f = _f64(f0).reshape(h.vol_shape).copy()
    Y = _f64(Y).reshape(h.proj_shape)
    cap_t = iters * 51 + 8
    st, tr, re, en = _stats(cap_t, iters + 2)
    pr = _params(lam, t, **kw)
    lib().orc_fbs(h.ref(), _ptr(Y), _ptr(f), int(iters), C.byref(pr), float(t), C.byref(st), 0)
    n = min(st.trace_len, cap_t)
    return Result(f, tr[:n].copy(), re[:n].copy(), en[:st.energy_len].copy(), [t])
