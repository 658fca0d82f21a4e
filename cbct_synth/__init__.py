"""Seeded synthetic inputs for cone-beam CT reconstruction tests and benchmarks.

What lives here: scan geometries of the benchmark workloads, random-ellipsoid
phantoms, their exact line integrals (closed-form chords), Poisson transmission
noise with the log transform, and random test vectors.

What does not live here: any part of the reconstruction method (no discrete
projector, adjoint, TV, prox or solver arithmetic).  Both the CPU oracle's
tests and the GPU path's tests and benchmark draw their inputs from this
module; neither of those two imports the other.

Conventions (the acquisition model of the paper, Eq. (1) and Fig. 1, with the
angle origin of its appendix, where the view at theta = 0 projects along +x):
  * x lateral, y anterior-posterior, z superior-inferior = rotation axis;
  * voxel centres x_a = (a - (Nx-1)/2) hx, likewise y, z; volume arrays are
    (Nz, Ny, Nx), x fastest;
  * view frame e_w = (cos t, sin t, 0), e_u = (sin t, -cos t, 0), e_v = z;
    source S = -SAD e_w; pixel (i, j) sits at S + SDD e_w + u_i e_u + v_j e_v
    with u_i = (i - (Nu-1)/2) pu, v_j = (j - (Nv-1)/2) pv;
  * projection arrays are (Nviews, Nv, Nu), u fastest.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Geometry", "Ellipsoid", "config_geometry", "CONFIGS", "view_angles",
    "make_phantom", "analytic_projections", "voxelize", "poisson_log",
    "random_volume", "random_projections", "serving_requests", "ray_endpoints",
    "level_geometry", "short_scan_angles", "mas_to_i0",
]


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Circular cone-beam scan: volume grid, flat detector, source orbit.

    Lengths are in mm.  ``angles`` (radians) may be None, meaning the equally
    spaced full orbit 2*pi*k/n_views.  ``sample_ratio`` is rho, the ray sample
    spacing along the transverse path in units of min(hx, hy).
    """
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    nu: int
    nv: int
    pu: float
    pv: float
    sad: float
    sdd: float
    n_views: int
    angles: Optional[tuple] = None
    sample_ratio: float = 1.0

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (self.n_views, self.nv, self.nu)

    def with_angles(self, angles: Sequence[float]) -> "Geometry":
        return dataclasses.replace(self, angles=tuple(float(a) for a in angles),
                                   n_views=len(angles))


def view_angles(g: Geometry) -> np.ndarray:
    if g.angles is not None:
        return np.asarray(g.angles, dtype=np.float64)
    return 2.0 * np.pi * np.arange(g.n_views, dtype=np.float64) / g.n_views


def level_geometry(g: Geometry, level: int, bin_detector: bool = True) -> Geometry:
    """Grid of multigrid level `level`: dims / 2^l over the same box, detector
    binned 2^l x 2^l when `bin_detector` (the recipe the benchmark inputs use)."""
    f = 1 << level
    kw = dict(nx=g.nx // f, ny=g.ny // f, nz=g.nz // f, hx=g.hx * f, hy=g.hy * f, hz=g.hz * f)
    if bin_detector:
        kw.update(nu=g.nu // f, nv=g.nv // f, pu=g.pu * f, pv=g.pv * f)
    return dataclasses.replace(g, **kw)


# --------------------------------------------------------------------------------------
# Short-scan acquisitions of the paper's physical experiments (Section III.B-C): a few hundred
# projections over a 200-degree arc (379 for the CatPhan scan, 363 for the head-and-neck and
# Rando scans), of which an equally spaced subset of 40 is reconstructed, at tube loads from
# 0.1 to 2.56 mAs per projection.
# --------------------------------------------------------------------------------------
def short_scan_angles(n_acquired: int = 363, n_used: int = 40, arc_deg: float = 200.0,
                      start_deg: float = 0.0) -> tuple:
    """Angles (radians) of an equally spaced subset of n_used among n_acquired projections spread
    evenly over [start, start + arc] (first and last at the arc's ends)."""
    if not (1 <= n_used <= n_acquired):
        raise ValueError("need 1 <= n_used <= n_acquired")
    step = arc_deg / (n_acquired - 1) if n_acquired > 1 else 0.0
    if n_used == 1:
        picks = [0]
    else:
        picks = [int(round(q * (n_acquired - 1) / (n_used - 1))) for q in range(n_used)]
    return tuple(math.radians(start_deg + k * step) for k in picks)


def mas_to_i0(mas: float, i0_ref: float = 1e5, mas_ref: float = 2.56) -> float:
    """Incident photons per detector pixel for a tube load (mAs per projection): proportional to
    the load, I0_ref at mas_ref (the CatPhan protocol)."""
    return i0_ref * mas / mas_ref


# --------------------------------------------------------------------------------------
# Workloads (sizes from the paper's NCAT experiment scaled to five
# workload definitions; the phantoms below stand in for NCAT/CatPhan/patient data).
# --------------------------------------------------------------------------------------
_CUBE32 = Geometry(32, 32, 32, 2.0, 2.0, 2.0, 64, 64, 1.5, 1.5, 1000.0, 1500.0, 16)
_WIDE512 = Geometry(512, 512, 64, 0.9, 0.9, 2.5, 512, 384, 0.78, 0.78, 1000.0, 1536.0, 40)
_BATCH128 = Geometry(128, 128, 128, 2.0, 2.0, 2.0, 256, 192, 2.0, 2.0, 1000.0, 1500.0, 60)

CONFIGS = {
    "cube32": dict(geometry=_CUBE32, levels=1, iters=[20], lam=0.05, I0=1e5, seeds=(11, 12)),
    "wide512x512x64": dict(geometry=_WIDE512, levels=2, iters=[20, 20], lam=0.05, I0=1e5, seeds=(21, 22)),
    "lowdose32": dict(geometry=_CUBE32, levels=3, iters=[100, 100, 100], lam=(0.02, 0.05, 0.1), I0=2e3,
                 seeds=(11, 32)),
    "batch8x128": dict(geometry=_BATCH128, batch=8, lam=0.05, I0=1e5, phantom_seeds=tuple(range(41, 49)),
                 noise_seed=49, perturb_seed=40, direction_seed=50),
    # the cube's grid scanned like the physical experiments: 40 of 363 projections over 200 deg,
    # tube loads from 0.1 to 2.56 mAs per projection
    "shortscan32": dict(geometry=dataclasses.replace(_CUBE32, n_views=40, angles=short_scan_angles(363, 40, 200.0)),
                        n_acquired=363, arc_deg=200.0,
                        mas=(0.1, 0.4, 1.0, 2.56), levels=1, iters=[20], lam=0.05, seeds=(11, 33)),
    "serving_mix": dict(n_requests=256, rate=4.0, vol_types=((64, 64, 64), (128, 128, 128), (256, 256, 96)),
                 h=2.0, views=(20, 120), iters=[30], lam=0.05, I0=1e5, budget_bytes=200 * 10**9,
                 seeds=dict(arrivals=51, mix=52, phantom0=5000, noise0=6000)),
}


def config_geometry(name: str) -> Geometry:
    return CONFIGS[name]["geometry"]


# --------------------------------------------------------------------------------------
# Ray endpoints (acquisition model)
# --------------------------------------------------------------------------------------
def ray_endpoints(g: Geometry, views=None):
    """Source points S (V,3) and pixel points D (V,Nv,Nu,3) for the selected views."""
    ang = view_angles(g)
    if views is not None:
        ang = ang[np.asarray(views)]
    c, s = np.cos(ang), np.sin(ang)
    ew = np.stack([c, s, np.zeros_like(c)], -1)
    eu = np.stack([s, -c, np.zeros_like(c)], -1)
    ev = np.array([0.0, 0.0, 1.0])
    u = (np.arange(g.nu) - (g.nu - 1) / 2.0) * g.pu
    v = (np.arange(g.nv) - (g.nv - 1) / 2.0) * g.pv
    S = -g.sad * ew
    D = (S + g.sdd * ew)[:, None, None, :] + u[None, None, :, None] * eu[:, None, None, :] \
        + v[None, :, None, None] * ev[None, None, None, :]
    return S, D


# --------------------------------------------------------------------------------------
# Ellipsoid phantom
# --------------------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Ellipsoid:
    center: tuple      # (x, y, z) mm
    axes: tuple        # semi-axes (a, b, c) mm, in the ellipsoid frame
    phi: float         # rotation about z (rad)
    dmu: float         # additive attenuation (1/mm)


def _body_axes(g: Geometry):
    r_fov = (g.nu * g.pu / 2.0) * g.sad / g.sdd
    rx = min(r_fov, g.nx * g.hx / 2.0)
    ry = min(r_fov, g.ny * g.hy / 2.0)
    hz = g.nz * g.hz / 2.0
    return np.array([0.9 * rx, 0.7 * ry, 0.9 * hz])


def _sphere_inside(c, rad, A):
    """Conservative test that the ball (c, rad) lies inside the axis-aligned
    ellipsoid with semi-axes A: bounds sum((c+rad n)_i^2/A_i^2) over unit n."""
    q = float(np.sum(c * c / (A * A)))
    lin = 2.0 * rad * math.sqrt(float(np.sum(c * c / A ** 4)))
    quad = rad * rad / float(np.min(A)) ** 2
    return q + lin + quad <= 1.0


def make_phantom(g: Geometry, seed: int, n_inner: int = 12, mu_body: float = 0.016) -> List[Ellipsoid]:
    """Body ellipsoid plus `n_inner` random inner ellipsoids (values in [0, 0.02] 1/mm).

    Draw order with numpy PCG64(seed): for each inner ellipsoid, 3 semi-axis
    factors U[0.06, 0.25], rotation U[0, pi), mu U[0, 0.02]; then centres by
    rejection sampling (3 uniforms in the body's bounding box per attempt) so
    that each bounding sphere is inside the body and pairwise disjoint.  After
    2000 failed attempts an ellipsoid's semi-axes shrink by 0.8 and sampling
    continues (deterministic given the seed).
    """
    rng = np.random.default_rng(seed)
    B = _body_axes(g)
    out = [Ellipsoid((0.0, 0.0, 0.0), tuple(B.tolist()), 0.0, mu_body)]
    specs = []
    for _ in range(n_inner):
        fac = rng.uniform(0.06, 0.25, size=3)
        phi = rng.uniform(0.0, np.pi)
        mu = rng.uniform(0.0, 0.02)
        specs.append([fac * B, phi, mu])
    placed = []  # (centre, radius)
    for spec in specs:
        axes, phi, mu = spec
        while True:
            rad = float(np.max(axes))
            ok = False
            for _ in range(2000):
                c = rng.uniform(-B, B)
                if not _sphere_inside(c, rad, B):
                    continue
                if all(np.linalg.norm(c - c2) > rad + r2 for c2, r2 in placed):
                    ok = True
                    break
            if ok:
                break
            axes = axes * 0.8
        placed.append((c, rad))
        out.append(Ellipsoid(tuple(c.tolist()), tuple(axes.tolist()), float(phi), float(mu - mu_body)))
    return out


def _ellipsoid_frame(e: Ellipsoid):
    c, s = math.cos(e.phi), math.sin(e.phi)
    # rows: ellipsoid-frame axes in world coordinates, scaled by 1/semi-axis
    R = np.array([[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]])
    return np.asarray(e.center, dtype=np.float64), R / np.asarray(e.axes)[:, None]


def chord_lengths(e: Ellipsoid, S: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Exact length of the segment S->D (extended to a full line) inside ellipsoid e.

    S broadcastable against D (..., 3).  The chord of a line through an
    ellipsoid is the root spacing of a quadratic in the world arc length."""
    c, M = _ellipsoid_frame(e)
    d = D - S
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    o = np.einsum("ij,...j->...i", M, S - c)
    dd = np.einsum("ij,...j->...i", M, d)
    a = np.sum(dd * dd, -1)
    b = 2.0 * np.sum(o * dd, -1)
    cc = np.sum(o * o, -1) - 1.0
    disc = b * b - 4.0 * a * cc
    return np.where(disc > 0.0, np.sqrt(np.maximum(disc, 0.0)) / a, 0.0)


def analytic_projections(g: Geometry, phantom: Sequence[Ellipsoid], views=None) -> np.ndarray:
    """Exact line integrals p = sum_e dmu_e * chord_e for every pixel-centre ray (float64)."""
    S, D = ray_endpoints(g, views)
    p = np.zeros(D.shape[:-1])
    for e in phantom:
        p += e.dmu * chord_lengths(e, S[:, None, None, :], D)
    return p


def analytic_projections_torch(g: Geometry, phantom: Sequence[Ellipsoid], device, dtype=None):
    """The same exact line integrals as analytic_projections, evaluated with torch on `device`
    (float64 by default): used to synthesise large request streams quickly."""
    import torch
    dtype = dtype or torch.float64
    S, D = ray_endpoints(g)
    S = torch.as_tensor(S, dtype=dtype, device=device)[:, None, None, :]
    D = torch.as_tensor(D, dtype=dtype, device=device)
    d = D - S
    d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    p = torch.zeros(D.shape[:-1], dtype=dtype, device=device)
    for e in phantom:
        c, M = _ellipsoid_frame(e)
        c = torch.as_tensor(c, dtype=dtype, device=device)
        M = torch.as_tensor(M, dtype=dtype, device=device)
        o = (S - c) @ M.T
        dd = d @ M.T
        a = (dd * dd).sum(-1)
        b = 2.0 * (o * dd).sum(-1)
        cc = (o * o).sum(-1) - 1.0
        disc = b * b - 4.0 * a * cc
        p += e.dmu * torch.where(disc > 0, torch.sqrt(torch.clamp(disc, min=0.0)) / a, torch.zeros_like(disc))
    return p


def poisson_log_torch(p, I0: float, seed: int):
    """Y = -ln(max(N, 1) / I0), N ~ Poisson(I0 exp(-p)), drawn with a seeded torch generator on
    p's device (a different stream of draws than poisson_log)."""
    import torch
    gen = torch.Generator(device=p.device)
    gen.manual_seed(int(seed))
    N = torch.poisson(I0 * torch.exp(-p), generator=gen)
    return -torch.log(torch.clamp(N, min=1.0) / I0)


def voxelize(g: Geometry, phantom: Sequence[Ellipsoid], supersample: int = 4) -> np.ndarray:
    """Ground-truth attenuation on the grid, each voxel the mean of supersample^3 points."""
    n = supersample
    off = (np.arange(n) + 0.5) / n - 0.5
    xs = (np.arange(g.nx) - (g.nx - 1) / 2.0) * g.hx
    ys = (np.arange(g.ny) - (g.ny - 1) / 2.0) * g.hy
    zs = (np.arange(g.nz) - (g.nz - 1) / 2.0) * g.hz
    vol = np.zeros((g.nz, g.ny, g.nx))
    for e in phantom:
        c, M = _ellipsoid_frame(e)
        rad = max(e.axes) + max(g.hx, g.hy, g.hz)
        ia = np.nonzero(np.abs(xs - c[0]) <= rad)[0]
        ib = np.nonzero(np.abs(ys - c[1]) <= rad)[0]
        ic = np.nonzero(np.abs(zs - c[2]) <= rad)[0]
        if len(ia) == 0 or len(ib) == 0 or len(ic) == 0:
            continue
        acc = np.zeros((len(ic), len(ib), len(ia)))
        for ox in off:
            for oy in off:
                for oz in off:
                    Z, Y, X = np.meshgrid(zs[ic] + oz * g.hz - c[2], ys[ib] + oy * g.hy - c[1],
                                          xs[ia] + ox * g.hx - c[0], indexing="ij")
                    P = np.stack([X, Y, Z], -1)
                    q = np.einsum("ij,...j->...i", M, P)
                    acc += (np.sum(q * q, -1) <= 1.0)
        vol[np.ix_(ic, ib, ia)] += e.dmu * acc / n ** 3
    return vol


def poisson_log(p: np.ndarray, I0: float, seed: int) -> np.ndarray:
    """Y = -ln(max(N, 1) / I0) with N ~ Poisson(I0 exp(-p)) (transmission counts)."""
    rng = np.random.default_rng(seed)
    N = rng.poisson(I0 * np.exp(-p))
    return -np.log(np.maximum(N, 1) / I0)


def random_volume(g: Geometry, seed: int, kind: str = "uniform") -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal(g.vol_shape)
    return rng.uniform(0.0, 1.0, g.vol_shape)


def random_projections(g: Geometry, seed: int, kind: str = "uniform") -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal(g.proj_shape)
    return rng.uniform(0.0, 1.0, g.proj_shape)


def serving_requests(n: Optional[int] = None):
    """The serving workload: arrival times and per-request geometry/seeds.

    Exponential inter-arrival times (rate 4/s, seed 51); volume type uniform
    over {64^3, 128^3, 256x256x96} at 2 mm and views uniform in [20, 120]
    (seed 52, drawn per request as type then views); detector Nu = 2 Nx,
    Nv = 2 Nz at 1.5 mm; SAD 1000 / SDD 1500."""
    cfg = CONFIGS["serving_mix"]
    n = cfg["n_requests"] if n is None else n
    s = cfg["seeds"]
    ra = np.random.default_rng(s["arrivals"])
    t = np.cumsum(ra.exponential(1.0 / cfg["rate"], size=n))
    rm = np.random.default_rng(s["mix"])
    reqs = []
    for r in range(n):
        ty = int(rm.integers(0, len(cfg["vol_types"])))
        nv_ = int(rm.integers(cfg["views"][0], cfg["views"][1] + 1))
        nx, ny, nz = cfg["vol_types"][ty]
        h = cfg["h"]
        geo = Geometry(nx, ny, nz, h, h, h, 2 * nx, 2 * nz, 1.5, 1.5, 1000.0, 1500.0, nv_)
        reqs.append(dict(index=r, arrival=float(t[r]), geometry=geo,
                         phantom_seed=s["phantom0"] + r, noise_seed=s["noise0"] + r))
    return reqs
