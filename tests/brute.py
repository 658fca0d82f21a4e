"""Independent brute-force forms used to pin the oracle (tiny problems only).

The forward operator is recomputed here by another route than the oracle's:
the scan geometry comes from rotating the theta = 0 configuration of the
paper's appendix (source at (-SAD, 0, 0), ray direction (L0, -u, v) as in
Eq. A2) with a rotation matrix; the closest approach of each ray's transverse
line to the axis is found numerically; and the zero-extended trilinear
interpolant is scipy's ``map_coordinates(order=1, mode='grid-constant')``.
The dense matrix has one column per voxel basis vector.
"""
import numpy as np
from scipy.ndimage import map_coordinates


def _angles(g):
    if g.angles is not None:
        return np.asarray(g.angles, dtype=np.float64)
    return 2 * np.pi * np.arange(g.n_views) / g.n_views


def sample_points(g):
    """Per ray: sample points (index coordinates) and the 3-D step length.

    Returns coords (3, n_rays, K) in (z, y, x) index order and w (n_rays,)."""
    dtau = g.sample_ratio * min(g.hx, g.hy)
    u = (np.arange(g.nu) - (g.nu - 1) / 2) * g.pu
    v = (np.arange(g.nv) - (g.nv - 1) / 2) * g.pv
    half = np.hypot((g.nx + 1) * g.hx / 2, (g.ny + 1) * g.hy / 2)
    K = int(np.ceil(half / dtau)) + 2
    ks = np.arange(-K, K + 1)
    pts, ws = [], []
    for th in _angles(g):
        R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
        src = R @ np.array([-g.sad, 0.0, 0.0])
        for vj in v:
            for ui in u:
                pix = R @ np.array([g.sdd - g.sad, -ui, vj])
                d = pix - src
                dxy = np.hypot(d[0], d[1])
                # parameter of the closest approach of the transverse line to the axis
                s_star = -(src[0] * d[0] + src[1] * d[1]) / (dxy * dxy)
                s = s_star + ks * dtau / dxy
                p = src[None, :] + s[:, None] * d[None, :]
                pts.append(p)
                ws.append(dtau * np.linalg.norm(d) / dxy)
    P = np.array(pts)  # (n_rays, K, 3) mm
    ix = P[..., 0] / g.hx + (g.nx - 1) / 2
    iy = P[..., 1] / g.hy + (g.ny - 1) / 2
    iz = P[..., 2] / g.hz + (g.nz - 1) / 2
    return np.stack([iz, iy, ix]), np.array(ws)


def forward(g, f):
    coords, w = sample_points(g)
    vals = map_coordinates(np.asarray(f, dtype=np.float64), coords.reshape(3, -1), order=1,
                           mode="grid-constant", cval=0.0, prefilter=False)
    return (w * vals.reshape(coords.shape[1:]).sum(-1)).reshape(g.n_views, g.nv, g.nu)


def matrix(g):
    """Dense system matrix A (n_rays, n_vox) built column by column."""
    coords, w = sample_points(g)
    flat = coords.reshape(3, -1)
    n_vox = g.nx * g.ny * g.nz
    A = np.zeros((coords.shape[1], n_vox))
    e = np.zeros((g.nz, g.ny, g.nx))
    for q in range(n_vox):
        e.flat[q] = 1.0
        vals = map_coordinates(e, flat, order=1, mode="grid-constant", cval=0.0, prefilter=False)
        A[:, q] = w * vals.reshape(coords.shape[1:]).sum(-1)
        e.flat[q] = 0.0
    return A


def appendix_uv(g, theta, point):
    """(u*, v*, l*, L) of Eq. (A6) for a world point, after rotating it into the theta = 0 frame."""
    c, s = np.cos(theta), np.sin(theta)
    x = c * point[0] + s * point[1]
    y = -s * point[0] + c * point[1]
    z = point[2]
    xs, ys, zs = -g.sad, 0.0, 0.0
    L0 = g.sdd
    us = -(y - ys) * L0 / (x - xs)
    vs = (z - zs) * L0 / (x - xs)
    L = np.sqrt(L0 ** 2 + us ** 2 + vs ** 2)
    ls = L * (x - xs) / L0
    return us, vs, ls, L


def box_chords(g, half_extent):
    """Chord length of every pixel-centre ray through the centred box |x_i| <= half_extent_i."""
    import cbct_synth
    S, D = cbct_synth.ray_endpoints(g)
    d = D - S[:, None, None, :]
    t0 = np.full(d.shape[:-1], -np.inf)
    t1 = np.full(d.shape[:-1], np.inf)
    for q in range(3):
        o = S[:, None, None, q]
        dq = d[..., q]
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (-half_extent[q] - o) / dq
            tb = (half_extent[q] - o) / dq
        lo, hi = np.minimum(ta, tb), np.maximum(ta, tb)
        inside = np.abs(o) < half_extent[q]
        lo = np.where(dq == 0, np.where(inside, -np.inf, np.inf), lo)
        hi = np.where(dq == 0, np.where(inside, np.inf, -np.inf), hi)
        t0, t1 = np.maximum(t0, lo), np.minimum(t1, hi)
    return np.maximum(t1 - t0, 0.0) * np.linalg.norm(d, axis=-1)


def cube_lengths(g):
    """Dense matrix of ray-in-voxel lengths: A[ray, voxel] = length of the segment S->D inside
    the voxel's cube [x_a - hx/2, x_a + hx/2] x ..., by clipping the segment against the cube's
    three slabs (a route independent of the oracle's sorted plane crossings).  A ray lying in a
    face plane belongs to the cube on the face's upper side (half-open slabs)."""
    import cbct_synth
    S, D = cbct_synth.ray_endpoints(g)
    d = (D - S[:, None, None, :]).reshape(-1, 3)
    Sr = np.repeat(S, g.nv * g.nu, axis=0)
    length = np.linalg.norm(d, axis=1)
    xs = (np.arange(g.nx) - (g.nx - 1) / 2) * g.hx
    ys = (np.arange(g.ny) - (g.ny - 1) / 2) * g.hy
    zs = (np.arange(g.nz) - (g.nz - 1) / 2) * g.hz
    A = np.zeros((len(d), g.n_vox))
    h = (g.hx, g.hy, g.hz)
    for c, zc in enumerate(zs):
        for b, yc in enumerate(ys):
            for a, xc in enumerate(xs):
                t0 = np.zeros(len(d))
                t1 = np.ones(len(d))
                for q, cen in enumerate((xc, yc, zc)):
                    lo, hi = cen - h[q] / 2, cen + h[q] / 2
                    dq, oq = d[:, q], Sr[:, q]
                    par = dq == 0
                    with np.errstate(divide="ignore", invalid="ignore"):
                        ta, tb = (lo - oq) / dq, (hi - oq) / dq
                    lo_t = np.where(par, np.where((oq >= lo) & (oq < hi), -np.inf, np.inf), np.minimum(ta, tb))
                    hi_t = np.where(par, np.where((oq >= lo) & (oq < hi), np.inf, -np.inf), np.maximum(ta, tb))
                    t0, t1 = np.maximum(t0, lo_t), np.minimum(t1, hi_t)
                A[:, (c * g.ny + b) * g.nx + a] = np.maximum(t1 - t0, 0.0) * length
    return A

