"""Pins of the FP64 oracle to facts outside itself (CPU only).

Every pin is a function returning (ok, detail) so that the mutation test at
the end can run them all with a deliberate mistake planted in the oracle and
check that each mistake is caught by at least one pin.
"""
import dataclasses
import json
import os

import numpy as np
import pytest
from scipy.optimize import nnls

import cbct_synth as S
import oracle as O
from tests import brute

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
G1 = S.config_geometry("cube32")
# tiny anisotropic grid, off-centre-sized detector, 3 views at irregular angles
TINY = dataclasses.replace(G1, nx=5, ny=4, nz=3, hx=2.0, hy=1.5, hz=2.5, nu=6, nv=4, pu=3.0, pv=4.0,
                           n_views=3, angles=(0.3, 2.1, 4.4))
SMALL = dataclasses.replace(G1, nx=16, ny=12, nz=10, nu=20, nv=14, n_views=5)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# ------------------------------------------------------------------ operator pins
def pin_brute_forward():
    """Oracle P = dense brute-force A x on a tiny anisotropic problem (1e-12)."""
    x = S.random_volume(TINY, 3, "normal")
    e = _rel(O.forward(TINY, x), brute.forward(TINY, x))
    return e < 1e-12, e


def pin_brute_adjoint():
    """Oracle P^T = A^T y with A the brute-force dense matrix (1e-12)."""
    A = brute.matrix(TINY)
    y = S.random_projections(TINY, 4, "normal")
    e = _rel(O.adjoint(TINY, y).ravel(), A.T @ y.ravel())
    return e < 1e-12, e


def pin_adjoint_identity():
    """<Px, y> = <x, P^T y> on random vectors (1e-12)."""
    worst = 0.0
    for g, seed in ((SMALL, 5), (G1, 6)):
        x = S.random_volume(g, seed, "normal")
        y = S.random_projections(g, seed + 100, "normal")
        a, b = np.vdot(O.forward(g, x), y), np.vdot(x, O.adjoint(g, y))
        worst = max(worst, abs(a - b) / abs(a))
    return worst < 1e-12, worst


_ELL = S.Ellipsoid((6.0, -4.0, 3.0), (22.0, 12.0, 15.0), 0.7, 0.01)
_BALL = S.Ellipsoid((5.0, -7.0, 4.0), (18.0, 18.0, 18.0), 0.0, 0.01)
_G1_FINE = dataclasses.replace(G1, nx=64, ny=64, nz=64, hx=1.0, hy=1.0, hz=1.0, nu=128, nv=128, pu=0.75, pv=0.75)


def _chord_err(g, body):
    f0 = S.voxelize(g, [body], 4)
    return _rel(O.forward(g, f0), S.analytic_projections(g, [body]))


def pin_chords():
    """P of a voxelised ball and of a rotated off-centre ellipsoid against their exact
    chords: rel-L2 <= 6 % at the 2 mm grid, and at least 1.6x smaller on a 2x finer grid."""
    out = {}
    ok = True
    for name, body in (("ball", _BALL), ("ellipsoid", _ELL)):
        e1, e2 = _chord_err(G1, body), _chord_err(_G1_FINE, body)
        out[name] = (e1, e2)
        ok &= (e1 < 0.06) and (e2 < e1 / 1.6)
    return ok, out


def pin_mass():
    """Detector-integrated projection per view equals the exact one (0.3 %):
    scale of P including the 3-D step weight."""
    f0 = S.voxelize(G1, [_ELL], 4)
    m1 = O.forward(G1, f0).sum(axis=(1, 2))
    m2 = S.analytic_projections(G1, [_ELL]).sum(axis=(1, 2))
    e = float(np.max(np.abs(m1 - m2) / m2))
    return e < 3e-3, e


def pin_box():
    """P 1 against the chord through the grid box (voxel centres +- h/2): 2 % at the 2 mm
    grid, smaller on the finer grid."""
    errs = []
    for g in (G1, _G1_FINE):
        half = np.array([g.nx * g.hx, g.ny * g.hy, g.nz * g.hz]) / 2
        errs.append(_rel(O.forward(g, np.ones(g.vol_shape)), brute.box_chords(g, half)))
    return errs[0] < 0.02 and errs[1] < errs[0], errs


def pin_centroid():
    """A small off-centre ball projects to (u*, v*) of Eq. (A6) at theta = 0 and 90 deg
    (within 1/20 pixel)."""
    g = dataclasses.replace(G1, nu=256, nv=256, pu=0.375, pv=0.375, n_views=2, angles=(0.0, np.pi / 2))
    c = np.array([15.0, -10.0, 8.0])
    f0 = S.voxelize(g, [S.Ellipsoid(tuple(c), (3.0, 3.0, 3.0), 0.0, 0.01)], 4)
    Pf = O.forward(g, f0)
    u = (np.arange(g.nu) - (g.nu - 1) / 2) * g.pu
    v = (np.arange(g.nv) - (g.nv - 1) / 2) * g.pv
    worst = 0.0
    for k, th in enumerate(g.angles):
        img = Pf[k]
        uc = (img.sum(0) * u).sum() / img.sum()
        vc = (img.sum(1) * v).sum() / img.sum()
        us, vs, _, _ = brute.appendix_uv(g, th, c)
        worst = max(worst, abs(uc - us) / g.pu, abs(vc - vs) / g.pv)
    return worst < 0.05, worst


def pin_continuum_adjoint():
    """P^T y of a smooth y against the closed-form gradient of Eq. (6) / Jacobian (A7):
    (hx hy hz / (pu pv)) sum_theta L^3/(L0 l^2) y(u*, v*) at interior voxels (3 % max, 0.6 % rms)."""
    g = dataclasses.replace(G1, nu=128, nv=128, pu=0.75, pv=0.75, n_views=4)
    u = (np.arange(g.nu) - (g.nu - 1) / 2) * g.pu
    v = (np.arange(g.nv) - (g.nv - 1) / 2) * g.pv

    def yfun(uu, vv):
        return 1 + 0.5 * np.cos(2 * np.pi * uu / 70.0) * np.cos(2 * np.pi * vv / 55.0 + 0.3)

    Y = np.broadcast_to(yfun(u[None, :], v[:, None]), g.proj_shape).copy()
    Pt = O.adjoint(g, Y)
    xs = (np.arange(g.nx) - (g.nx - 1) / 2) * g.hx
    ys = (np.arange(g.ny) - (g.ny - 1) / 2) * g.hy
    zs = (np.arange(g.nz) - (g.nz - 1) / 2) * g.hz
    Z, Yy, X = np.meshgrid(zs, ys, xs, indexing="ij")
    expect = np.zeros(g.vol_shape)
    for k in range(g.n_views):
        us, vs, ls, L = brute.appendix_uv(g, 2 * np.pi * k / g.n_views, (X, Yy, Z))
        expect += L ** 3 / (g.sdd * ls ** 2) * yfun(us, vs)
    expect *= g.hx * g.hy * g.hz / (g.pu * g.pv)
    sl = (slice(4, -4),) * 3
    err = np.abs(Pt[sl] - expect[sl]) / expect[sl]
    mx, rms = float(err.max()), float(np.sqrt((err ** 2).mean()))
    return mx < 0.03 and rms < 0.006, (mx, rms)


# ------------------------------------------------------------------ Siddon projector pins
# a wide cone (source 30 mm from the axis): rays cross several z planes inside the grid
_TINY_CONE = dataclasses.replace(TINY, sad=30.0, sdd=60.0, nv=5)


def pin_siddon_brute():
    """Siddon P and its transpose against the dense ray-in-voxel length matrix built by slab
    clipping (1e-12), on the tiny anisotropic problem and on a wide-cone copy of it."""
    out = []
    for g in (TINY, _TINY_CONE):
        A = brute.cube_lengths(g)
        x = S.random_volume(g, 13, "normal")
        y = S.random_projections(g, 14, "normal")
        out += [_rel(O.forward_siddon(g, x).ravel(), A @ x.ravel()),
                _rel(O.adjoint_siddon(g, y).ravel(), A.T @ y.ravel())]
    return max(out) < 1e-12, out


def pin_siddon_box_and_identity():
    """Siddon P 1 is exactly the chord through the grid box (1e-12), and <Px, y> = <x, P^T y>."""
    half = np.array([G1.nx * G1.hx, G1.ny * G1.hy, G1.nz * G1.hz]) / 2
    e1 = _rel(O.forward_siddon(G1, np.ones(G1.vol_shape)), brute.box_chords(G1, half))
    x = S.random_volume(G1, 15, "normal")
    y = S.random_projections(G1, 16, "normal")
    a, b = np.vdot(O.forward_siddon(G1, x), y), np.vdot(x, O.adjoint_siddon(G1, y))
    e2 = abs(a - b) / abs(a)
    return e1 < 1e-12 and e2 < 1e-12, (e1, e2)


def pin_siddon_sampled():
    """The sampled Siddon entry points (used at full size) equal the full ones (1e-12): P at
    selected rays, and P^T at selected voxels by per-cube chords over the projected footprint."""
    g = SMALL
    x = S.random_volume(g, 17, "normal")
    y = S.random_projections(g, 18, "normal")
    rays = np.arange(0, g.n_views * g.nv * g.nu, 7)
    vox = np.arange(0, g.n_vox, 5)
    e1 = _rel(O.forward_siddon_rays(g, x, rays), O.forward_siddon(g, x).ravel()[rays])
    e2 = _rel(O.adjoint_siddon_voxels(g, y, vox), O.adjoint_siddon(g, y).ravel()[vox])
    return max(e1, e2) < 1e-12, (e1, e2)


def pin_siddon_chords():
    """Siddon P of a voxelised ball against its exact chords: rel-L2 <= 8 % at 2 mm and at least
    1.6x smaller on the 2x finer grid (first order: the ray integral of a piecewise-constant
    voxelisation is exact for that image, so only the partial-volume error of the voxelisation
    remains, which halves with h)."""
    e1, e2 = (_rel(O.forward_siddon(g, S.voxelize(g, [_BALL], 4)), S.analytic_projections(g, [_BALL]))
              for g in (G1, _G1_FINE))
    return e1 < 0.08 and e2 < e1 / 1.6, (e1, e2)


# ------------------------------------------------------------------ "until convergence" per level
def pin_convergence_rule():
    """The per-level stop of Section II.C.3: a vanishing tolerance changes nothing (bitwise); a
    tolerance of 1 stops every level after one iteration; at 3e-3 every level ends at the first
    energy pair within the tolerance (or at its iteration bound)."""
    Y = S.poisson_log(S.analytic_projections(G1, S.make_phantom(G1, 11)), 2e3, 32)
    a = O.reconstruct(G1, Y, 0.05, [4, 4, 4], 3, conv_tol=1e-30)
    b = O.reconstruct(G1, Y, 0.05, [4, 4, 4], 3)
    ok1 = np.array_equal(a.f, b.f) and np.array_equal(a.energy, b.energy)
    c = O.reconstruct(G1, Y, 0.05, [4, 4, 4], 3, conv_tol=1.0)
    ok2 = len(c.energy) == 6 and sorted({(int(r[0]), int(r[1])) for r in c.trace}) == [(0, 0), (1, 0), (2, 0)]
    tol, bound = 3e-3, 40
    d = O.reconstruct(G1, Y, 0.05, [bound] * 3, 3, conv_tol=tol)
    tr = np.array(d.trace)
    ok3, pos = True, 0
    for lvl in (2, 1, 0):
        n_outer = int(tr[tr[:, 0] == lvl][:, 1].max()) + 1
        e = d.energy[pos:pos + n_outer + 1]
        pos += n_outer + 1
        rel = np.abs(np.diff(e)) / e[:-1]
        if n_outer < bound:
            ok3 &= bool(rel[-1] <= tol) and bool(np.all(rel[:-1] > tol))
        else:
            ok3 &= bool(np.all(rel > tol))
    return ok1 and ok2 and ok3, (ok1, ok2, ok3)


# ------------------------------------------------------------------ Eq. 6 backprojector pins
EQ6 = dataclasses.replace(G1, nx=12, ny=10, nz=8, nu=160, nv=128, pu=0.75, pv=0.75, n_views=5,
                          angles=(0.0, 0.7, 2.0, 3.6, 5.1))


def _eq6_expected(g, tfun):
    """hx hy hz/(pu pv) sum_theta L^3/(L0 l^2) T(u*, v*) by the appendix's rotated-frame formulas."""
    xs = (np.arange(g.nx) - (g.nx - 1) / 2) * g.hx
    ys = (np.arange(g.ny) - (g.ny - 1) / 2) * g.hy
    zs = (np.arange(g.nz) - (g.nz - 1) / 2) * g.hz
    Z, Yy, X = np.meshgrid(zs, ys, xs, indexing="ij")
    out = np.zeros(g.vol_shape)
    for th in g.angles:
        us, vs, ls, L = brute.appendix_uv(g, th, (X, Yy, Z))
        out += L ** 3 / (g.sdd * ls ** 2) * tfun(us, vs)
    return out * g.hx * g.hy * g.hz / (g.pu * g.pv)


def pin_eq6_affine():
    """Bilinear interpolation is exact for an affine T(u, v) = a + b u + c v, so the Eq. 6
    backprojector must equal the closed form through (A6)/(A7) everywhere (every voxel
    projects inside the imager here): 1e-12 relative."""
    u = (np.arange(EQ6.nu) - (EQ6.nu - 1) / 2) * EQ6.pu
    v = (np.arange(EQ6.nv) - (EQ6.nv - 1) / 2) * EQ6.pv

    def tfun(uu, vv):
        return 2.0 + 0.013 * uu - 0.021 * vv

    T = np.broadcast_to(tfun(u[None, :], v[:, None]), EQ6.proj_shape).copy()
    got = O.backproject_eq6(EQ6, T)
    e = _rel(got, _eq6_expected(EQ6, tfun))
    return e < 1e-12, e


def pin_eq6_near_adjoint():
    """For a smooth T the Eq. 6 backprojector and the exact P^T agree at interior voxels
    (both approximate the same continuum gradient): 3 % max, 0.6 % rms."""
    g = dataclasses.replace(G1, nu=128, nv=128, pu=0.75, pv=0.75, n_views=4)
    u = (np.arange(g.nu) - (g.nu - 1) / 2) * g.pu
    v = (np.arange(g.nv) - (g.nv - 1) / 2) * g.pv
    Y = np.broadcast_to(1 + 0.5 * np.cos(2 * np.pi * u[None, :] / 70.0) * np.cos(2 * np.pi * v[:, None] / 55.0 + 0.3),
                        g.proj_shape).copy()
    a, b = O.adjoint(g, Y), O.backproject_eq6(g, Y)
    sl = (slice(4, -4),) * 3
    err = np.abs(b[sl] - a[sl]) / a[sl]
    mx, rms = float(err.max()), float(np.sqrt((err ** 2).mean()))
    return mx < 0.03 and rms < 0.006, (mx, rms)


# ------------------------------------------------------------------ TV pins
TVG = dataclasses.replace(G1, nx=6, ny=5, nz=4, hx=1.0, hy=1.5, hz=2.5)


def pin_tv_gradient():
    """dR/df against FP64 central differences of R on a random volume (1e-6 rel)."""
    f = S.random_volume(TVG, 7) * 0.02
    grad = O.tv_grad(TVG, f, 1e-5)
    h = 1e-7
    num = np.zeros_like(f)
    for q in range(f.size):
        fp = f.copy(); fp.flat[q] += h
        fm = f.copy(); fm.flat[q] -= h
        num.flat[q] = (O.tv_energy(TVG, fp, 1e-5) - O.tv_energy(TVG, fm, 1e-5)) / (2 * h)
    e = _rel(grad, num)
    return e < 1e-6, e


def pin_tv_closed_forms():
    """R of special volumes in closed form: a constant volume (only the upper x and y faces
    jump, z is reflective) and a linear ramp along z (zero BC in x, y; reflective in z)."""
    g = TVG
    eps = 1e-5
    n = g.nx * g.ny * g.nz
    # constant 1: Dx = -1/hx on the last x column, Dy = -1/hy on the last y row, Dz = 0
    cnt_x = g.ny * g.nz - g.nz  # last-x but not last-y
    cnt_y = g.nx * g.nz - g.nz
    cnt_xy = g.nz
    cnt_0 = n - cnt_x - cnt_y - cnt_xy
    R1 = (cnt_0 * eps + cnt_x * np.hypot(1 / g.hx, eps) + cnt_y * np.hypot(1 / g.hy, eps)
          + cnt_xy * np.sqrt(1 / g.hx ** 2 + 1 / g.hy ** 2 + eps ** 2)) / n
    # ramp f = s*c along z: Dz = s/hz except at the last plane (0); x/y faces jump by -f
    s = 0.01
    f = np.broadcast_to((s * np.arange(g.nz))[:, None, None], g.vol_shape).copy()
    tot = 0.0
    for c in range(g.nz):
        dz = s / g.hz if c + 1 < g.nz else 0.0
        val = s * c
        for b in range(g.ny):
            for a in range(g.nx):
                dx = -val / g.hx if a == g.nx - 1 else 0.0
                dy = -val / g.hy if b == g.ny - 1 else 0.0
                tot += np.sqrt(dx * dx + dy * dy + dz * dz + eps * eps)
    R2 = tot / n
    e1 = abs(O.tv_energy(g, np.ones(g.vol_shape), eps) - R1) / R1
    e2 = abs(O.tv_energy(g, f, eps) - R2) / R2
    return max(e1, e2) < 1e-12, (e1, e2)


# ------------------------------------------------------------------ multigrid pins
def pin_transfers():
    """<Prol x, y> = 8 <x, R y>; R 1 = 1; Prol reproduces linear fields away from the clamped
    edges; Prol 1 = 1."""
    rng = np.random.default_rng(8)
    x = rng.standard_normal((3, 4, 5))
    y = rng.standard_normal((6, 8, 10))
    a, b = np.vdot(O.prolong(x), y), 8 * np.vdot(x, O.restrict(y))
    e_adj = abs(a - b) / abs(a)
    e_r1 = float(np.max(np.abs(O.restrict(np.ones((6, 8, 10))) - 1)))
    e_p1 = float(np.max(np.abs(O.prolong(np.ones((3, 4, 5))) - 1)))
    # linear field in coarse cell coordinates; fine cell C sits at coarse coordinate (C - 0.5)/2
    cz, cy, cx = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    lin = 0.3 * cx - 0.7 * cy + 1.1 * cz + 2.0
    fz, fy, fx = np.meshgrid((np.arange(8) - 0.5) / 2, (np.arange(10) - 0.5) / 2, (np.arange(12) - 0.5) / 2,
                             indexing="ij")
    want = 0.3 * fx - 0.7 * fy + 1.1 * fz + 2.0
    got = O.prolong(lin)
    e_lin = float(np.max(np.abs(got[1:-1, 1:-1, 1:-1] - want[1:-1, 1:-1, 1:-1])))
    ok = e_adj < 1e-12 and e_r1 < 1e-12 and e_p1 < 1e-12 and e_lin < 1e-12
    return ok, (e_adj, e_r1, e_p1, e_lin)


def pin_binning():
    """Detector binning = block mean."""
    Y = np.random.default_rng(9).standard_normal((2, 8, 6))
    want = Y.reshape(2, 4, 2, 3, 2).mean(axis=(2, 4))
    e = float(np.max(np.abs(O.bin_detector(Y, 2) - want)))
    return e < 1e-14, e


# ------------------------------------------------------------------ solver pins
def _cube32_data():
    ph = S.make_phantom(G1, 11)
    return S.poisson_log(S.analytic_projections(G1, ph), 1e5, 12)


def pin_rof_armijo():
    """Every ROF step obeys Eq. (5) with c = 0.01, alpha = 0.6: accepted steps satisfy
    E_new <= E0 - c t alpha^m G (so E_R strictly decreases); a refused search fails the test
    at m = 30.  Run with a large t so that backtracking occurs."""
    g = dataclasses.replace(G1, nx=12, ny=12, nz=8)
    gv = S.random_volume(g, 10) * 0.02
    t = 2.0
    res = O.rof(g, gv, 0.05, t)
    c, alpha = GOLD["armijo"]["c"], GOLD["armijo"]["alpha"]
    ok, backtracked = True, False
    for (lvl, outer, inner, m), (e0, enew, G) in zip(res.trace, res.rof_e):
        if m >= 0:
            s = t * alpha ** m
            ok &= bool(enew <= e0 - c * s * G) and bool(enew < e0)
            backtracked |= m > 0
        else:
            ok &= bool(enew > e0 - c * t * alpha ** 30 * G)
    return ok and backtracked and len(res.trace) > 0, (len(res.trace), res.trace[:, 3].tolist())


def pin_fbs_monotone():
    """E(f_k) = D + lambda R is non-increasing over 20 outer iterations on the 32^3
    workload (slack 1e-9 E)."""
    Y = _cube32_data()
    res = O.reconstruct(G1, Y, 0.05, [20], 1)
    e = res.energy
    viol = float(np.max(np.diff(e) - 1e-9 * e[:-1]))
    return viol <= 0 and e[-1] < 0.01 * e[0], (viol, e[0], e[-1])


def pin_nnls():
    """lambda = 0 reduces the method to projected gradient descent on D: after many
    iterations its objective matches scipy's NNLS on the dense brute-force matrix (1e-6)."""
    g = dataclasses.replace(G1, nx=4, ny=4, nz=3, hx=4.0, hy=4.0, hz=4.0, nu=8, nv=6, pu=3.0, pv=3.0, n_views=8)
    A = brute.matrix(g)
    rng = np.random.default_rng(13)
    ftrue = np.maximum(rng.standard_normal(g.n_vox), 0.0) * 0.02
    Y = A @ ftrue + 0.01 * rng.standard_normal(A.shape[0])
    xs, _ = nnls(A, Y, maxiter=10000)
    d_star = np.mean((A @ xs - Y) ** 2)
    res = O.reconstruct(g, Y.reshape(g.proj_shape), 0.0, [16000], 1)
    d = np.mean((A @ res.f.ravel() - Y) ** 2)
    e = abs(d - d_star) / d_star
    return e < 1e-6 and res.f.min() >= 0.0, e


def pin_fbs_siddon():
    """Algorithm A1 with the Siddon pair: E = D_s + lambda R non-increasing over 20 iterations on the
    32^3 workload, and with lambda = 0 projected gradient descent reaches scipy's NNLS objective on
    the slab-clipped ray-in-cube length matrix (1e-6)."""
    Y = _cube32_data()
    e = O.reconstruct(G1, Y, 0.05, [20], 1, projector=1).energy
    viol = float(np.max(np.diff(e) - 1e-9 * e[:-1]))
    g = dataclasses.replace(G1, nx=4, ny=4, nz=3, hx=4.0, hy=4.0, hz=4.0, nu=8, nv=6, pu=3.0, pv=3.0, n_views=8)
    A = brute.cube_lengths(g)
    rng = np.random.default_rng(17)
    ftrue = np.maximum(rng.standard_normal(g.n_vox), 0.0) * 0.02
    Yb = A @ ftrue + 0.01 * rng.standard_normal(A.shape[0])
    xs, _ = nnls(A, Yb, maxiter=10000)
    d_star = np.mean((A @ xs - Yb) ** 2)
    res = O.reconstruct(g, Yb.reshape(g.proj_shape), 0.0, [16000], 1, projector=1)
    en = abs(np.mean((A @ res.f.ravel() - Yb) ** 2) - d_star) / d_star
    return viol <= 0 and e[-1] < 0.01 * e[0] and en < 1e-6 and res.f.min() >= 0.0, (viol, e[0], e[-1], en)


def pin_resume():
    """10 + 10 outer iterations through d_init equal 20 iterations (oracle: 1e-15)."""
    Y = _cube32_data()
    t = O.schur_step(G1)
    a = O.reconstruct(G1, Y, 0.05, [20], 1, step=t).f
    b1 = O.reconstruct(G1, Y, 0.05, [10], 1, step=t).f
    b = O.reconstruct(G1, Y, 0.05, [10], 1, step=t, d_init=b1).f
    e = float(np.max(np.abs(a - b)) / np.max(np.abs(a)))
    return e <= 1e-15, e


def pin_constants():
    """The solver defaults are the paper's line-search constants."""
    d = O.DEFAULTS
    a = GOLD["armijo"]
    ok = d["armijo_c"] == a["c"] and d["backtrack"] == a["alpha"] and d["rof_tol"] == a["epsilon_relative"]
    ex = GOLD["appendix_example"]
    us, vs, ls, L = brute.appendix_uv(dataclasses.replace(G1, sad=-ex["S"][0], sdd=ex["L0"]), 0.0, ex["V"])
    ok &= abs(us - ex["u_star"]) < 1e-9 and abs(vs - ex["v_star"]) < 1e-9 and abs(ls - ex["l_star"]) < 1e-9
    ok &= abs(ex["L0"] * ls ** 2 / L ** 3 - ex["jacobian_L0_l2_over_L3"]) < 1e-12
    return ok, None


# ------------------------------------------------------------------ sampled entry points
def pin_sampled_operators():
    """The sampled entry points used as references at full size equal the full operators
    (1e-12): P at selected rays (forward_rays), and P^T at selected voxels (adjoint_voxels, which
    has its own detector-footprint window), on an anisotropic grid with an off-centre-sized detector
    and on the 32^3 workload geometry."""
    out = []
    for g, seed in ((SMALL, 31), (dataclasses.replace(G1, n_views=5), 33)):
        x = S.random_volume(g, seed, "normal")
        y = S.random_projections(g, seed + 1, "normal")
        rays = np.arange(0, g.n_views * g.nv * g.nu, 5)
        vox = np.arange(0, g.n_vox, 3)
        out += [_rel(O.forward_rays(g, x, rays), O.forward(g, x).ravel()[rays]),
                _rel(O.adjoint_voxels(g, y, vox), O.adjoint(g, y).ravel()[vox])]
    return max(out) < 1e-12, out


# ------------------------------------------------------------------ step size t (Schur bound)
def pin_schur():
    """max(P 1) and max(P^T 1) are the largest row and column sums of the dense brute-force matrix
    (1e-12); their product bounds sigma_max(A)^2 (Schur's test); and the step t is the reciprocal
    of kappa0 times that bound, kappa0 = 2 N_vox / N_rays being the scale of the normalised gradient
    N_vox dD/df = kappa0 A^T (A f - Y) (so t kappa0 sigma_max^2 <= 1: Step 1 is a stable gradient step)."""
    A = brute.matrix(TINY)
    a, b = O.schur(TINY)
    ea = abs(a - A.sum(axis=1).max()) / a
    eb = abs(b - A.sum(axis=0).max()) / b
    smax2 = np.linalg.norm(A, 2) ** 2
    kappa0 = 2.0 * A.shape[1] / A.shape[0]
    t = O.schur_step(TINY)
    et = abs(t * kappa0 * A.sum(axis=1).max() * A.sum(axis=0).max() - 1.0)
    ok = ea < 1e-12 and eb < 1e-12 and smax2 <= a * b * (1 + 1e-12) and et < 1e-12 and t * kappa0 * smax2 <= 1 + 1e-12
    return ok, (ea, eb, smax2 / (a * b), et)


# ------------------------------------------------------------------ ROF stop rule
def pin_rof_stop_rule():
    """The relative-decrease stop of Step 2 (the paper's 0.1 % rule after Eq. 5): in every ROF loop
    of a 32^3 solve, each accepted step that is not the loop's last changed E_R by at least 0.1 %;
    the last record is an accepted step below 0.1 %, a refused search (m = -1) or the 50th iteration."""
    Y = _cube32_data()
    res = O.reconstruct(G1, Y, 0.05, [6], 1)
    tol = GOLD["armijo"]["epsilon_relative"]
    groups = {}
    for rec, e in zip(res.trace, res.rof_e):
        groups.setdefault((int(rec[0]), int(rec[1])), []).append((int(rec[2]), int(rec[3]), e))
    ok, multi = True, 0
    for key, recs in groups.items():
        for n, (inner, m, (e0, enew, _)) in enumerate(recs):
            rel = abs(enew - e0) / e0
            if n + 1 < len(recs):
                ok &= m >= 0 and rel >= tol
            else:
                ok &= m == -1 or rel < tol or inner + 1 == O.DEFAULTS["rof_max_iter"]
        multi += len(recs) > 1
    return ok and multi > 0 and len(groups) == 6, (len(groups), multi)


# ------------------------------------------------------------------ Step-1 scale at lambda > 0
def pin_lambda_form_fixed_point():
    """Algorithm A1 minimises D + lambda R: on a tiny problem whose minimiser is positive (so the
    clamp of Step 3 is inactive), many outer iterations with an accurate Step 2 (rof_tol 1e-14)
    reach a point where the gradient of E = D + lambda R vanishes: |dD/df + lambda dR/df| <= 1e-6
    |dD/df|, with dD/df = (2/N_rays) A^T (A f - Y) from the dense brute-force matrix and dR/df by
    central differences of R.  A wrong Step-1 scale kappa0 (or a wrong weight between the two
    terms) moves the fixed point to the minimiser of another combination, where this fails."""
    g = dataclasses.replace(G1, nx=4, ny=4, nz=3, hx=4.0, hy=4.0, hz=4.0, nu=8, nv=6, pu=3.0, pv=3.0, n_views=8)
    A = brute.matrix(g)
    rng = np.random.default_rng(21)
    ftrue = 0.01 + 0.01 * rng.random(g.n_vox)
    Y = A @ ftrue + 0.0005 * rng.standard_normal(A.shape[0])
    lam, eps = 0.05, 1e-3
    res = O.reconstruct(g, Y.reshape(g.proj_shape), lam, [3000], 1, tv_eps=eps, rof_tol=1e-14)
    f = res.f.ravel()
    gD = 2.0 / A.shape[0] * A.T @ (A @ f - Y)
    h = 1e-7
    gR = np.zeros_like(f)
    for q in range(f.size):
        fp = f.copy(); fp[q] += h
        fm = f.copy(); fm[q] -= h
        gR[q] = (O.tv_energy(g, fp, eps) - O.tv_energy(g, fm, eps)) / (2 * h)
    e = float(np.linalg.norm(gD + lam * gR) / np.linalg.norm(gD))
    return e < 1e-6 and f.min() > 0.0, (e, f.min())


# ------------------------------------------------------------------ multigrid level geometry
def _binned_chords(g, l, half):
    """Chords through the centred box |x_q| <= half_q of the rays from the source to the centres of
    the 2^l x 2^l pixel blocks of the level-0 detector (block centre = mean of its pixel centres)."""
    k = 1 << l
    ub = ((np.arange(g.nu) - (g.nu - 1) / 2) * g.pu).reshape(-1, k).mean(1)
    vb = ((np.arange(g.nv) - (g.nv - 1) / 2) * g.pv).reshape(-1, k).mean(1)
    angles = g.angles if g.angles is not None else 2 * np.pi * np.arange(g.n_views) / g.n_views
    out = np.zeros((g.n_views, len(vb), len(ub)))
    for t, th in enumerate(angles):
        ew = np.array([np.cos(th), np.sin(th), 0.0])
        eu = np.array([np.sin(th), -np.cos(th), 0.0])
        src = -g.sad * ew
        for j, v in enumerate(vb):
            for i, u in enumerate(ub):
                d = g.sdd * ew + u * eu + np.array([0.0, 0.0, v])
                t0, t1 = -np.inf, np.inf
                for q in range(3):
                    if d[q] == 0.0:
                        if abs(src[q]) >= half[q]:
                            t0, t1 = 1.0, 0.0
                        continue
                    a, b = (-half[q] - src[q]) / d[q], (half[q] - src[q]) / d[q]
                    t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
                out[t, j, i] = max(t1 - t0, 0.0) * np.linalg.norm(d)
    return out


def pin_level_geometry():
    """Multigrid levels (Section II.C.3) cover the level-0 box: P_l 1 at levels 1 and 2 of the
    32^3 workload matches the chord through the level-0 grid box of the rays to the binned pixel
    centres (8 % and 12 %: the interpolant's one-voxel edge ramp is first order in the coarse
    pitch); and P_l equals the dense brute-force P of the grid with dims / 2^l, pitch x 2^l,
    detector binned (pitch x 2^l) and sample spacing min(h_l) (1e-12)."""
    half = np.array([G1.nx * G1.hx, G1.ny * G1.hy, G1.nz * G1.hz]) / 2
    ec = []
    for l in (1, 2):
        k = 1 << l
        P1 = O.forward_level(G1, l, np.ones((G1.nz // k, G1.ny // k, G1.nx // k)))
        ec.append(_rel(P1, _binned_chords(G1, l, half)))
    T = dataclasses.replace(G1, nx=8, ny=8, nz=4, hx=2.0, hy=2.0, hz=3.0, nu=8, nv=8, pu=3.0, pv=3.0, n_views=3,
                            angles=(0.2, 1.9, 4.0))
    eb = []
    for l in (1, 2):
        k = 1 << l
        Tl = dataclasses.replace(T, nx=T.nx // k, ny=T.ny // k, nz=T.nz // k, hx=T.hx * k, hy=T.hy * k,
                                 hz=T.hz * k, nu=T.nu // k, nv=T.nv // k, pu=T.pu * k, pv=T.pv * k)
        x = S.random_volume(Tl, 30 + l, "normal")
        eb.append(_rel(O.forward_level(T, l, x), brute.forward(Tl, x)))
    return ec[0] < 0.08 and ec[1] < 0.12 and max(eb) < 1e-12, (ec, eb)


PINS = [pin_brute_forward, pin_brute_adjoint, pin_adjoint_identity, pin_chords, pin_mass, pin_box,
        pin_centroid, pin_continuum_adjoint, pin_eq6_affine, pin_eq6_near_adjoint, pin_tv_gradient, pin_tv_closed_forms, pin_transfers,
        pin_binning, pin_rof_armijo, pin_fbs_monotone, pin_nnls, pin_resume, pin_constants, pin_convergence_rule,
        pin_siddon_brute, pin_siddon_box_and_identity, pin_siddon_sampled, pin_siddon_chords, pin_fbs_siddon,
        pin_sampled_operators, pin_schur, pin_rof_stop_rule, pin_lambda_form_fixed_point, pin_level_geometry]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(orc, pin):
    ok, detail = pin()
    assert ok, detail


# Each planted mistake (see the fault switch in the oracle) with the pins expected to catch it.
FAULTS = {
    1: "3-D step weight replaced by the transverse step",
    2: "detector u axis mirrored",
    3: "parallel-beam z slope",
    4: "transposed z weight wrong in P^T",
    5: "zero instead of reflective z boundary",
    6: "TV gradient misses the y terms",
    7: "prolongation weights 1/2, 1/2",
    8: "Armijo bound sign flipped",
    9: "Step 1 goes uphill",
    10: "restriction misses 1/8",
    11: "voxel grid shifted half a voxel in x",
    12: "Eq. 6 weight without the Jacobian's third power of L",
    13: "Siddon misses the z plane crossings",
    14: "P^T at sampled voxels: detector footprint window too narrow",
    15: "ROF relative-decrease stop test disabled",
    16: "Step 1 scale kappa0 halved",
    17: "coarse levels keep the level-0 detector pitch",
    18: "Schur step without the factor 2 of kappa0",
    19: "coarse levels keep the level-0 sample spacing",
}
QUICK = [pin_brute_forward, pin_brute_adjoint, pin_adjoint_identity, pin_centroid, pin_mass, pin_eq6_affine,
         pin_tv_gradient, pin_tv_closed_forms, pin_transfers, pin_rof_armijo, pin_fbs_monotone, pin_siddon_brute,
         pin_sampled_operators, pin_schur, pin_rof_stop_rule, pin_lambda_form_fixed_point, pin_level_geometry]


@pytest.mark.parametrize("fault", sorted(FAULTS), ids=[FAULTS[k] for k in sorted(FAULTS)])
def test_planted_mistake_is_caught(orc, fault):
    O.set_fault(fault)
    try:
        caught = []
        for pin in QUICK:
            try:
                ok, _ = pin()
            except Exception:
                ok = False
            if not ok:
                caught.append(pin.__name__)
                break
    finally:
        O.set_fault(0)
    assert caught, "planted mistake %d (%s) passed every pin" % (fault, FAULTS[fault])
