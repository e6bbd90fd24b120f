"""Pins of the oracle's structural-similarity loss term (Sec. 3.5 trains with
SSIM and L1; the ablation's DSSIM = (1 - SSIM) / 2; SSIM as defined by Wang et
al. 2004: 11 x 11 Gaussian window of sigma 1.5, K1 = 0.01, K2 = 0.03, here
with dynamic range L = 1 and every fully contained window).

Pins: the window's closed form; SSIM(x, x) = 1; constant images (closed form
in their two values); y = 2 x in one window (closed form in the window's mean
and variance); a scalar brute-force twin over every window; the loss as the
mean of the map; the gradient against central differences.  Planted mistakes
(the two constants swapped, a wider window, a dropped factor 2) each fail one.
"""
import contextlib
import math

import numpy as np
import pytest

import oracle.glassnet_oracle as go

C1, C2 = 0.01 ** 2, 0.03 ** 2


def test_window_closed_form():
    G = go.ssim_window()
    assert G.shape == (11, 11)
    assert abs(G.sum() - 1.0) <= 1e-15
    assert np.allclose(G, G.T) and np.allclose(G, G[::-1, ::-1])
    assert np.linalg.matrix_rank(G) == 1                       # separable
    assert G[0, 0] / G[5, 5] == pytest.approx(math.exp(-50.0 / 4.5), rel=1e-12)
    assert G[5, 0] / G[5, 5] == pytest.approx(math.exp(-25.0 / 4.5), rel=1e-12)


def test_identical_images_give_one():
    x = np.random.default_rng(0).uniform(0, 2, size=(17, 19))
    assert np.max(np.abs(go.ssim_map(x, x) - 1.0)) <= 1e-12


def test_constant_images():
    for a, b in ((0.3, 0.7), (1.5, 0.0), (0.0, 0.0)):
        S = go.ssim_map(np.full((12, 13), a), np.full((12, 13), b))
        assert S.shape == (2, 3)
        assert np.allclose(S, (2 * a * b + C1) / (a * a + b * b + C1), rtol=1e-12, atol=0)


def test_doubled_image_in_one_window():
    """y = 2x: my = 2 mx, syy = 4 sxx, sxy = 2 sxx, so
    SSIM = (4 m^2 + C1)(4 s + C2) / ((5 m^2 + C1)(5 s + C2)), the window's
    mean m and variance s summed by hand from the Gaussian weights."""
    x = np.random.default_rng(1).uniform(0, 1, size=(11, 11))
    g = [math.exp(-(i - 5) ** 2 / 4.5) for i in range(11)]
    z = sum(g) ** 2
    m = sum(g[i] * g[j] * x[i, j] for i in range(11) for j in range(11)) / z
    s = sum(g[i] * g[j] * (x[i, j] - m) ** 2 for i in range(11) for j in range(11)) / z
    want = (4 * m * m + C1) * (4 * s + C2) / ((5 * m * m + C1) * (5 * s + C2))
    assert go.ssim_map(x, 2 * x)[0, 0] == pytest.approx(want, rel=1e-12)


def test_bruteforce_twin_and_symmetry():
    rng = np.random.default_rng(2)
    x, y = rng.uniform(0, 1, size=(13, 14)), rng.uniform(0, 1, size=(13, 14))
    g = [math.exp(-(i - 5) ** 2 / 4.5) for i in range(11)]
    z = sum(g) ** 2
    S = go.ssim_map(x, y)
    assert S.shape == (3, 4)
    for r in range(3):
        for c in range(4):
            acc = [0.0] * 5
            for i in range(11):
                for j in range(11):
                    wgt = g[i] * g[j] / z
                    a, b = x[r + i, c + j], y[r + i, c + j]
                    for k, v in enumerate((a, b, a * a, b * b, a * b)):
                        acc[k] += wgt * v
            mx, my, ex2, ey2, exy = acc
            want = ((2 * mx * my + C1) * (2 * (exy - mx * my) + C2) /
                    ((mx * mx + my * my + C1) * (ex2 - mx * mx + ey2 - my * my + C2)))
            assert S[r, c] == pytest.approx(want, rel=1e-12)
    assert np.allclose(go.ssim_map(y, x), S, rtol=1e-14, atol=0)


def test_loss_is_half_one_minus_the_mean_map():
    rng = np.random.default_rng(3)
    out, tgt = rng.uniform(0, 1, size=(2, 3, 15, 16)), rng.uniform(0, 1, size=(2, 3, 15, 16))
    loss, _ = go.dssim_loss(out, tgt)
    maps = [go.ssim_map(out[f, c], tgt[f, c]) for f in range(2) for c in range(3)]
    assert loss == pytest.approx((1.0 - np.mean(maps)) / 2.0, rel=1e-13)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    out = rng.uniform(0, 1, size=(1, 3, 13, 14))
    tgt = np.clip(out + 0.2 * rng.normal(size=out.shape), 0, 1)
    _, g = go.dssim_loss(out, tgt)
    eps = 1e-6
    worst = 0.0
    for idx in np.ndindex(out.shape):
        p, m = out.copy(), out.copy()
        p[idx] += eps
        m[idx] -= eps
        fd = (go.dssim_loss(p, tgt)[0] - go.dssim_loss(m, tgt)[0]) / (2 * eps)
        worst = max(worst, abs(fd - g[idx]) / (1e-9 + 1e-6 * abs(g[idx])))
    assert worst <= 1.0


# ---------------------------------------------------------------- mutations
@contextlib.contextmanager
def patched(**kw):
    old = {k: getattr(go, k) for k in kw}
    for k, v in kw.items():
        setattr(go, k, v)
    try:
        yield
    finally:
        for k, v in old.items():
            setattr(go, k, v)


_orig_map = go.ssim_map


def _map_no_factor2(x, y):
    G = go.ssim_window()
    mx, my = go._local(x, G), go._local(y, G)
    sxx = go._local(x * x, G) - mx * mx
    syy = go._local(y * y, G) - my * my
    sxy = go._local(x * y, G) - mx * my
    return ((2 * mx * my + C1) * (sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


@pytest.mark.parametrize("mutation", [dict(SSIM_K1=0.03, SSIM_K2=0.01), dict(SSIM_SIGMA=2.0),
                                      dict(ssim_map=_map_no_factor2)])
def test_pins_catch_planted_mistakes(mutation):
    caught = 0
    with patched(**mutation):
        for t in (test_window_closed_form, test_identical_images_give_one, test_constant_images,
                  test_doubled_image_in_one_window, test_bruteforce_twin_and_symmetry):
            try:
                t()
            except AssertionError:
                caught += 1
    assert caught > 0
