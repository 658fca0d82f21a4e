"""Torch-facing wrappers of the libcbct entry points (device memory and streams only)."""
from __future__ import annotations

import ctypes as C

import torch

import numpy as np

from ._lib import GeometryDesc, SolveParams, SolveStats, check, context, lib


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require(t: torch.Tensor, shape, name: str, device) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 GPU tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if t.device != device:
        raise ValueError("%s is on %s, the plan on %s" % (name, t.device, device))


class Plan:
    """Geometry tables of a scan for `levels` multigrid levels (cbct_plan_create).

    `geom` is any object with the scan attributes (nx, ny, nz, hx, hy, hz, nu, nv,
    pu, pv, sad, sdd, n_views, angles, sample_ratio).  The plan lives on the
    current CUDA/HIP device."""

    def __init__(self, geom, levels: int = 1, bin_detector: bool = True):
        L = lib()
        self.geom = geom
        self.levels = int(levels)
        self.binned = bool(bin_detector)
        self.device = torch.device("cuda", torch.cuda.current_device())
        angles = getattr(geom, "angles", None)
        self._angles = (C.c_double * len(angles))(*angles) if angles is not None else None
        d = GeometryDesc(int(geom.nx), int(geom.ny), int(geom.nz), float(geom.hx), float(geom.hy), float(geom.hz),
                         int(geom.nu), int(geom.nv), float(geom.pu), float(geom.pv), float(geom.sad),
                         float(geom.sdd), int(geom.n_views),
                         C.cast(self._angles, C.POINTER(C.c_double)) if self._angles is not None else None,
                         float(getattr(geom, "sample_ratio", 1.0)))
        h = C.c_void_p()
        check(L.cbct_plan_create(context(self.device.index), C.byref(d), self.levels, int(self.binned), C.byref(h)))
        self._h = h
        self._dims = []
        for lvl in range(self.levels):
            out = (C.c_int * 6)()
            check(L.cbct_plan_level_dims(h, lvl, out))
            self._dims.append(tuple(out))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().cbct_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vol_shape(self, level: int = 0):
        nx, ny, nz, nu, nv, nviews = self._dims[level]
        return (nz, ny, nx)

    def proj_shape(self, level: int = 0):
        nx, ny, nz, nu, nv, nviews = self._dims[level]
        return (nviews, nv, nu)

    def forward_workspace_bytes(self, level: int = 0) -> int:
        n = C.c_size_t()
        check(lib().cbct_forward_workspace_size(self._h, level, C.byref(n)))
        return int(n.value)

    def forward(self, f: torch.Tensor, level: int = 0, out: torch.Tensor = None, workspace: torch.Tensor = None):
        """P f (cbct_forward)."""
        _require(f, self.vol_shape(level), "f", self.device)
        if out is None:
            out = torch.empty(self.proj_shape(level), dtype=torch.float32, device=self.device)
        _require(out, self.proj_shape(level), "out", self.device)
        nb = self.forward_workspace_bytes(level)
        if workspace is None or workspace.numel() * workspace.element_size() < nb:
            workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        check(lib().cbct_forward(self._h, level, f.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(), _stream_handle(self.device)))
        return out

    def forward_columns(self, f_cols: torch.Tensor, level: int = 0, out: torch.Tensor = None):
        """P of a volume stored [ny][nx][nz] (cbct_forward_columns)."""
        nz, ny, nx = self.vol_shape(level)
        _require(f_cols, (ny, nx, nz), "f_cols", self.device)
        if out is None:
            out = torch.empty(self.proj_shape(level), dtype=torch.float32, device=self.device)
        _require(out, self.proj_shape(level), "out", self.device)
        check(lib().cbct_forward_columns(self._h, level, f_cols.data_ptr(), out.data_ptr(),
                                         _stream_handle(self.device)))
        return out

    def adjoint_workspace_bytes(self, level: int = 0) -> int:
        n = C.c_size_t()
        check(lib().cbct_adjoint_workspace_size(self._h, level, C.byref(n)))
        return int(n.value)

    def adjoint(self, y: torch.Tensor, level: int = 0, out: torch.Tensor = None, workspace: torch.Tensor = None):
        """P^T y (cbct_adjoint)."""
        _require(y, self.proj_shape(level), "y", self.device)
        if out is None:
            out = torch.empty(self.vol_shape(level), dtype=torch.float32, device=self.device)
        _require(out, self.vol_shape(level), "out", self.device)
        nb = self.adjoint_workspace_bytes(level)
        if workspace is None or workspace.numel() * workspace.element_size() < nb:
            workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        check(lib().cbct_adjoint(self._h, level, y.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(), _stream_handle(self.device)))
        return out

    def backproject_eq6(self, y: torch.Tensor, level: int = 0, out: torch.Tensor = None):
        """The paper's Eq. 6 voxel-driven backprojector (cbct_backproject_eq6)."""
        _require(y, self.proj_shape(level), "y", self.device)
        if out is None:
            out = torch.empty(self.vol_shape(level), dtype=torch.float32, device=self.device)
        _require(out, self.vol_shape(level), "out", self.device)
        check(lib().cbct_backproject_eq6(self._h, level, y.data_ptr(), out.data_ptr(), _stream_handle(self.device)))
        return out

    def forward_siddon(self, f: torch.Tensor, level: int = 0, out: torch.Tensor = None,
                       workspace: torch.Tensor = None):
        """Siddon's exact-path projection (cbct_forward_siddon)."""
        _require(f, self.vol_shape(level), "f", self.device)
        if out is None:
            out = torch.empty(self.proj_shape(level), dtype=torch.float32, device=self.device)
        _require(out, self.proj_shape(level), "out", self.device)
        nb = self.forward_workspace_bytes(level)
        if workspace is None or workspace.numel() * workspace.element_size() < nb:
            workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        check(lib().cbct_forward_siddon(self._h, level, f.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                                        workspace.numel() * workspace.element_size(), _stream_handle(self.device)))
        return out

    def adjoint_siddon_workspace_bytes(self, level: int = 0) -> int:
        n = C.c_size_t()
        check(lib().cbct_adjoint_siddon_workspace_size(self._h, level, C.byref(n)))
        return int(n.value)

    def adjoint_siddon(self, y: torch.Tensor, level: int = 0, out: torch.Tensor = None,
                       workspace: torch.Tensor = None):
        """Transpose of the Siddon projection (cbct_adjoint_siddon)."""
        _require(y, self.proj_shape(level), "y", self.device)
        if out is None:
            out = torch.empty(self.vol_shape(level), dtype=torch.float32, device=self.device)
        _require(out, self.vol_shape(level), "out", self.device)
        nb = self.adjoint_siddon_workspace_bytes(level)
        if workspace is None or workspace.numel() * workspace.element_size() < nb:
            workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        check(lib().cbct_adjoint_siddon(self._h, level, y.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                                        workspace.numel() * workspace.element_size(), _stream_handle(self.device)))
        return out

    # ---- solver ----------------------------------------------------------------------------
    @staticmethod
    def solve_params(lam=0.05, iters=(20,), levels=None, step=0.0, replay=None, **kw):
        """cbct_solve_params with the library defaults, overridden by the arguments.
        Returns (params, keepalive) - the keepalive tuple owns the arrays."""
        p = SolveParams()
        lib().cbct_solve_params_default(C.byref(p))
        iters = list(iters)
        levels = len(iters) if levels is None else int(levels)
        it = (C.c_int * len(iters))(*iters)
        p.lam = float(lam)
        p.iters = C.cast(it, C.POINTER(C.c_int))
        p.levels = levels
        p.step = float(step)
        for k, v in kw.items():
            if not hasattr(p, k):
                raise TypeError("unknown solver parameter %r" % k)
            setattr(p, k, type(getattr(p, k))(v))
        rp = None
        if replay is not None:
            # records (m, ends_step2)
            flat = [int(v) for rec in replay for v in (rec[0], rec[1])]
            rp = (C.c_int * max(len(flat), 2))(*flat)
            p.replay = C.cast(rp, C.POINTER(C.c_int))
            p.replay_len = len(replay)
        return p, (it, rp)

    def reconstruct_workspace_bytes(self, params) -> int:
        n = C.c_size_t()
        check(lib().cbct_reconstruct_workspace_size(self._h, C.byref(params), C.byref(n)))
        return int(n.value)

    def reconstruct(self, y: torch.Tensor, lam=0.05, iters=(20,), step=0.0, init: torch.Tensor = None,
                    out: torch.Tensor = None, workspace: torch.Tensor = None, stats: bool = False, replay=None,
                    **kw):
        """Algorithm A1 with the multigrid cascade (cbct_reconstruct).  Returns the level-0 volume,
        and with stats=True also a dict with the ROF decision trace and the energy trace."""
        params, keep = self.solve_params(lam, iters, step=step, replay=replay, **kw)
        _require(y, self.proj_shape(0), "y", self.device)
        if init is not None:
            _require(init, self.vol_shape(0), "init", self.device)
        if out is None:
            out = torch.empty(self.vol_shape(0), dtype=torch.float32, device=self.device)
        _require(out, self.vol_shape(0), "out", self.device)
        nb = self.reconstruct_workspace_bytes(params)
        if workspace is None or workspace.numel() * workspace.element_size() < nb:
            workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        st, arrays = (self._stats(params) if stats else (None, None))
        check(lib().cbct_reconstruct(self._h, C.byref(params), y.data_ptr(),
                                     init.data_ptr() if init is not None else None, out.data_ptr(),
                                     workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                     _stream_handle(self.device), C.byref(st) if st is not None else None))
        if not stats:
            return out
        return out, self._stats_dict(st, arrays, params.levels)

    @staticmethod
    def _stats(params):
        total = sum(params.iters[l] for l in range(params.levels))
        cap = total * (params.rof_max_iter + 1) + 8
        tr = np.zeros((cap, 4), dtype=np.int32)
        re = np.zeros((cap, 3))
        en = np.zeros(total + params.levels + 2)
        st = SolveStats(tr.ctypes.data_as(C.POINTER(C.c_int)), cap, 0, re.ctypes.data_as(C.POINTER(C.c_double)),
                        en.ctypes.data_as(C.POINTER(C.c_double)), len(en), 0)
        return st, (tr, re, en)

    @staticmethod
    def _stats_dict(st, arrays, levels):
        tr, re, en = arrays
        n = min(st.trace_len, len(tr))
        return dict(trace=tr[:n].copy(), rof_e=re[:n].copy(), energy=en[:min(st.energy_len, len(en))].copy(),
                    t_used=list(st.t_used)[:levels], seconds=st.seconds, replay_used=st.replay_used)

    def tv_prox(self, g: torch.Tensor, lam: float, t: float, level: int = 0, replay=None, **kw):
        """Step 2 alone (cbct_tv_prox): u = ROF(g).  Returns (u, stats dict)."""
        params, keep = self.solve_params(lam, (0,), levels=1, step=t, replay=replay, **kw)
        _require(g, self.vol_shape(level), "g", self.device)
        u = torch.empty_like(g)
        n = C.c_size_t()
        check(lib().cbct_tv_prox_workspace_size(self._h, level, C.byref(n)))
        ws = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        tr = np.zeros((params.rof_max_iter + 2, 4), dtype=np.int32)
        re = np.zeros((params.rof_max_iter + 2, 3))
        st = SolveStats(tr.ctypes.data_as(C.POINTER(C.c_int)), len(tr), 0, re.ctypes.data_as(C.POINTER(C.c_double)),
                        None, 0, 0)
        check(lib().cbct_tv_prox(self._h, level, C.byref(params), g.data_ptr(), u.data_ptr(), ws.data_ptr(),
                                 int(n.value), _stream_handle(self.device), C.byref(st)))
        k = min(st.trace_len, len(tr))
        return u, dict(trace=tr[:k].copy(), rof_e=re[:k].copy(), replay_used=st.replay_used)

    def tv_energy_grad(self, f: torch.Tensor, tv_eps: float = 1e-5, level: int = 0, grad: torch.Tensor = None,
                       want_sum: bool = True, workspace: torch.Tensor = None):
        """S(f) = sum sqrt(|D f|^2 + eps^2) and dS/df (cbct_tv_energy_grad)."""
        _require(f, self.vol_shape(level), "f", self.device)
        if grad is None:
            grad = torch.empty_like(f)
        n = C.c_size_t()
        check(lib().cbct_tv_energy_grad_workspace_size(self._h, C.byref(n)))
        nb = int(n.value)
        if workspace is None or workspace.numel() * workspace.element_size() < nb:
            workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        h = C.c_double()
        check(lib().cbct_tv_energy_grad(self._h, level, float(tv_eps), f.data_ptr(), grad.data_ptr(),
                                        C.byref(h) if want_sum else None, workspace.data_ptr(),
                                        workspace.numel() * workspace.element_size(), _stream_handle(self.device)))
        return (h.value if want_sum else None), grad

    def prolong(self, c: torch.Tensor, coarse_level: int):
        _require(c, self.vol_shape(coarse_level), "c", self.device)
        out = torch.empty(self.vol_shape(coarse_level - 1), dtype=torch.float32, device=self.device)
        check(lib().cbct_prolong(self._h, coarse_level, c.data_ptr(), out.data_ptr(), _stream_handle(self.device)))
        return out

    def restrict(self, f: torch.Tensor, fine_level: int):
        _require(f, self.vol_shape(fine_level), "f", self.device)
        out = torch.empty(self.vol_shape(fine_level + 1), dtype=torch.float32, device=self.device)
        check(lib().cbct_restrict(self._h, fine_level, f.data_ptr(), out.data_ptr(), _stream_handle(self.device)))
        return out

    def bin_detector(self, y0: torch.Tensor, level: int):
        _require(y0, self.proj_shape(0), "y0", self.device)
        out = torch.empty(self.proj_shape(level), dtype=torch.float32, device=self.device)
        check(lib().cbct_bin_detector(self._h, level, y0.data_ptr(), out.data_ptr(), _stream_handle(self.device)))
        return out
