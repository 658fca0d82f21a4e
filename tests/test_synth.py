"""The seeded input generators: value ranges, determinism, noise statistics, exact chords."""
import dataclasses

import numpy as np

import cbct_synth as S


def test_phantom_values_and_seed():
    g = S.config_geometry("cube32")
    ph = S.make_phantom(g, 11)
    assert len(ph) == 13
    vol = S.voxelize(g, ph, 2)
    assert vol.min() >= -1e-12 and vol.max() <= 0.02 + 1e-12
    ph2 = S.make_phantom(g, 11)
    assert ph == ph2
    assert S.make_phantom(g, 12) != ph


def test_inner_ellipsoids_inside_and_disjoint():
    g = S.config_geometry("wide512x512x64")
    ph = S.make_phantom(g, 21)
    body = np.array(ph[0].axes)
    for i, e in enumerate(ph[1:]):
        c, r = np.array(e.center), max(e.axes)
        # bounding sphere inside the body: check points on it
        dirs = np.random.default_rng(0).standard_normal((2000, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        pts = c + r * dirs
        assert np.all(np.sum((pts / body) ** 2, 1) <= 1.0 + 1e-9)
        for e2 in ph[i + 2:]:
            assert np.linalg.norm(c - np.array(e2.center)) > r + max(e2.axes)
        assert 0.0 <= e.dmu + 0.016 <= 0.02


def test_ball_chord_closed_form():
    g = dataclasses.replace(S.config_geometry("cube32"), n_views=3)
    ball = S.Ellipsoid((3.0, -2.0, 1.0), (10.0, 10.0, 10.0), 0.4, 1.0)
    p = S.analytic_projections(g, [ball])
    Sx, D = S.ray_endpoints(g)
    d = D - Sx[:, None, None, :]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    w = np.array(ball.center) - Sx[:, None, None, :]
    dist2 = np.sum(w * w, -1) - np.sum(w * d, -1) ** 2
    want = 2 * np.sqrt(np.maximum(100.0 - dist2, 0.0))
    assert np.max(np.abs(p - want)) < 1e-9


def test_poisson_log_moments():
    p = np.full((4, 50, 50), 1.5)
    Y = S.poisson_log(p, 1e5, 3)
    N = 1e5 * np.exp(-Y)
    lam = 1e5 * np.exp(-1.5)
    assert abs(N.mean() - lam) / lam < 2e-3
    assert abs(N.var() - lam) / lam < 0.05
    assert np.array_equal(Y, S.poisson_log(p, 1e5, 3))
    # the floor max(N, 1) keeps the log finite for extinct rays
    assert np.isfinite(S.poisson_log(np.full((1, 2, 2), 60.0), 1e5, 1)).all()


def test_serving_mix():
    reqs = S.serving_requests(32)
    assert len(reqs) == 32
    assert all(b["arrival"] > a["arrival"] for a, b in zip(reqs, reqs[1:]))
    for r in reqs:
        g = r["geometry"]
        assert (g.nx, g.ny, g.nz) in ((64, 64, 64), (128, 128, 128), (256, 256, 96))
        assert 20 <= g.n_views <= 120 and g.nu == 2 * g.nx and g.nv == 2 * g.nz


def test_torch_projections_match_numpy():
    import torch
    g = dataclasses.replace(S.config_geometry("cube32"), n_views=3)
    ph = S.make_phantom(g, 11)
    a = S.analytic_projections(g, ph)
    b = S.analytic_projections_torch(g, ph, "cpu").numpy()
    assert np.max(np.abs(a - b)) < 1e-9  # rounding near tangent rays
    y = S.poisson_log_torch(torch.as_tensor(a), 1e5, 1)
    assert torch.isfinite(y).all()


def test_short_scan_angles():
    a = np.degrees(S.short_scan_angles(363, 40, 200.0))
    assert len(a) == 40 and a[0] == 0.0 and abs(a[-1] - 200.0) < 1e-12
    step = 200.0 / 362
    k = a / step
    assert np.allclose(k, np.round(k), atol=1e-9)          # a subset of the acquired angles
    assert np.all(np.diff(np.round(k)) >= 9) and np.all(np.diff(np.round(k)) <= 10)  # equally spaced picks
    assert S.mas_to_i0(2.56) == 1e5 and abs(S.mas_to_i0(0.1) - 1e5 * 0.1 / 2.56) < 1e-9
    g = S.config_geometry("shortscan32")
    assert g.n_views == 40 and len(g.angles) == 40
