"""Pins of the oracle's x2 super-sampling network (Sec. 3.4 raises GlassNet's
render to twice its resolution with a small CNN fed by full-resolution
G-buffers; the layers are this implementation's reading).

Pins: the bilinear upsample against torch's (align_corners=False, the
half-pixel convention) and closed forms (a constant image, a linear ramp away
from the clamped edges); the 3x3 convolution against torch's conv2d in float64;
the whole network against a scalar brute-force twin; zero weights (output =
upsample + last bias); a channel-routing network whose every ReLU is the
identity (output = upsample + a chosen G-buffer channel, in closed form).
Planted mistakes (corner-aligned upsampling, transposed kernel taps, edge
replication instead of zero padding, a dropped residual) each fail one.
"""
import contextlib

import numpy as np
import pytest

import oracle.sr_oracle as so

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _weights(seed, scale=0.2):
    return np.random.default_rng(seed).normal(size=so.sr_n_params()) * scale


def test_param_count():
    assert so.sr_n_params() == 32 * 17 * 9 + 32 + 32 * 32 * 9 + 32 + 3 * 32 + 3 == 14275


def test_upsample_matches_torch_bilinear():
    x = np.random.default_rng(1).uniform(-1, 1, size=(2, 3, 5, 7))
    ref = F.interpolate(torch.from_numpy(x), scale_factor=2, mode="bilinear",
                        align_corners=False).numpy()
    assert np.max(np.abs(so.upsample2x(x) - ref)) <= 1e-14


def test_upsample_closed_forms():
    assert np.array_equal(so.upsample2x(np.full((4, 6), 0.37)), np.full((8, 12), 0.37))
    ramp = np.tile(np.arange(6, dtype=np.float64) * 1.5, (4, 1))     # value = 1.5 x
    up = so.upsample2x(ramp)
    X = np.arange(1, 11)                                              # interior columns
    assert np.allclose(up[:, 1:11], 1.5 * ((X + 0.5) / 2 - 0.5), rtol=0, atol=1e-14)
    assert np.allclose(up[:, 0], 0.0) and np.allclose(up[:, 11], 7.5)  # clamped edges


def test_conv_matches_torch():
    rng = np.random.default_rng(2)
    x, W, b = rng.normal(size=(5, 6, 9)), rng.normal(size=(4, 5, 3, 3)), rng.normal(size=4)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(W), torch.from_numpy(b),
                   padding=1).numpy()[0]
    assert np.max(np.abs(so.conv3x3(x, W, b) - ref)) <= 1e-12


def test_bruteforce_twin():
    rng = np.random.default_rng(3)
    w = _weights(3)
    lo, g = rng.uniform(0, 1, size=(2, 3, 3, 4)), rng.uniform(-1, 1, size=(2, 14, 6, 8))
    a, b = so.sr_forward(w, lo, g), so.sr_forward_bruteforce(w, lo, g)
    assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))


def test_zero_weights_give_upsample_plus_bias():
    w = np.zeros(so.sr_n_params())
    w[-3:] = (0.5, -1.0, 2.0)
    rng = np.random.default_rng(4)
    lo, g = rng.uniform(0, 1, size=(1, 3, 4, 5)), rng.uniform(size=(1, 14, 8, 10))
    want = so.upsample2x(lo[0]) + np.array([0.5, -1.0, 2.0])[:, None, None]
    assert np.allclose(so.sr_forward(w, lo, g)[0], want, rtol=0, atol=1e-15)


def test_channel_routing_closed_form():
    """conv1 copies input channel 3 + 2o into hidden channel o (centre tap),
    conv2 is the centre-tap identity, conv3 sends hidden channel o(k) to
    output k: with non-negative G-buffers every ReLU passes, so output k =
    upsample_k + G[2 o(k)]."""
    p = {name: np.zeros(shp) for name, shp in so.sr_shapes()}
    for o in range(7):
        p["w1"][o, 3 + 2 * o, 1, 1] = 1.0
    for o in range(32):
        p["w2"][o, o, 1, 1] = 1.0
    route = (4, 0, 6)
    for k, o in enumerate(route):
        p["w3"][k, o] = 1.0
    w = np.concatenate([p[name].ravel() for name, _ in so.sr_shapes()])
    rng = np.random.default_rng(5)
    lo, g = rng.uniform(0, 1, size=(1, 3, 3, 5)), rng.uniform(0, 1, size=(1, 14, 6, 10))
    want = so.upsample2x(lo[0]) + g[0, [2 * o for o in route]]
    assert np.allclose(so.sr_forward(w, lo, g)[0], want, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- mutations
@contextlib.contextmanager
def patched(**kw):
    old = {k: getattr(so, k) for k in kw}
    for k, v in kw.items():
        setattr(so, k, v)
    try:
        yield
    finally:
        for k, v in old.items():
            setattr(so, k, v)


_up, _conv, _fwd = so.upsample2x, so.conv3x3, so.sr_forward


def _up_corner_aligned(img):
    img = np.asarray(img, dtype=np.float64)
    h, w = img.shape[-2:]
    ys, xs = np.linspace(0, h - 1, 2 * h), np.linspace(0, w - 1, 2 * w)
    y0, x0 = np.floor(ys).astype(int), np.floor(xs).astype(int)
    y1, x1 = np.minimum(y0 + 1, h - 1), np.minimum(x0 + 1, w - 1)
    fy, fx = ys - y0, xs - x0
    rows = img[..., y0, :] * (1 - fy)[:, None] + img[..., y1, :] * fy[:, None]
    return rows[..., x0] * (1 - fx) + rows[..., x1] * fx


def _conv_transposed_taps(x, W, b):
    return _conv(x, np.swapaxes(W, 2, 3), b)


def _conv_edge_replicate(x, W, b):
    cin, H, Wd = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)), mode="edge")
    y = np.zeros((W.shape[0], H, Wd)) + b[:, None, None]
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oc,chw->ohw", W[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + Wd])
    return y


def _fwd_no_residual(w, lowres, gbuf_hi, C=so.SR_WIDTH):
    return _fwd(w, lowres, gbuf_hi, C) - _up(np.asarray(lowres, dtype=np.float64))


@pytest.mark.parametrize("mutation", [dict(upsample2x=_up_corner_aligned),
                                      dict(conv3x3=_conv_transposed_taps),
                                      dict(conv3x3=_conv_edge_replicate),
                                      dict(sr_forward=_fwd_no_residual)])
def test_pins_catch_planted_mistakes(mutation):
    caught = 0
    with patched(**mutation):
        for t in (test_upsample_matches_torch_bilinear, test_upsample_closed_forms,
                  test_conv_matches_torch, test_bruteforce_twin,
                  test_zero_weights_give_upsample_plus_bias, test_channel_routing_closed_form):
            try:
                t()
            except AssertionError:
                caught += 1
    assert caught > 0


# ---------------------------------------------------------------- gradient
def _torch_sr_grad(w, lo, g, dy):
    """The same network in torch float64 with autograd (library convolution,
    interpolation and their backward)."""
    p = {k: torch.tensor(v, requires_grad=True) for k, v in so.sr_unpack(w).items()}
    up = F.interpolate(torch.from_numpy(lo), scale_factor=2, mode="bilinear", align_corners=False)
    x = torch.cat([up, torch.from_numpy(g)], dim=1)
    a1 = torch.relu(F.conv2d(x, p["w1"], p["b1"], padding=1))
    a2 = torch.relu(F.conv2d(a1, p["w2"], p["b2"], padding=1))
    y = up + F.conv2d(a2, p["w3"][:, :, None, None], p["b3"])
    (y * torch.from_numpy(dy)).sum().backward()
    return np.concatenate([p[name].grad.numpy().ravel() for name, _ in so.sr_shapes()])


def test_grad_matches_torch_autograd():
    rng = np.random.default_rng(6)
    w = _weights(6)
    lo, g = rng.uniform(0, 2, size=(2, 3, 4, 5)), rng.uniform(-1, 1, size=(2, 14, 8, 10))
    dy = rng.normal(size=(2, 3, 8, 10))
    ref = _torch_sr_grad(w, lo, g, dy)
    got = so.sr_grad(w, lo, g, dy)
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_grad_matches_central_differences():
    rng = np.random.default_rng(8)
    w = _weights(8)
    lo, g = rng.uniform(0, 2, size=(1, 3, 2, 3)), rng.uniform(-1, 1, size=(1, 14, 4, 6))
    dy = rng.normal(size=(1, 3, 4, 6))
    gr = so.sr_grad(w, lo, g, dy)
    f = lambda ww: float(np.sum(so.sr_forward(ww, lo, g) * dy))  # noqa: E731
    eps = 1e-6
    idx = np.concatenate([rng.choice(4896, 40, replace=False), 4896 + np.arange(32),
                          4928 + rng.choice(9216, 40, replace=False), 14144 + np.arange(131)])
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        fd = (f(wp) - f(wm)) / (2 * eps)
        assert abs(fd - gr[i]) <= 1e-6 * max(1.0, abs(gr[i])), i


def _grad_no_relu_mask(w, lowres, gbuf_hi, dy, C=so.SR_WIDTH):
    """The chain rule with the ReLU derivatives dropped (masks of ones)."""
    p = so.sr_unpack(w, C)
    out = {k: np.zeros_like(v) for k, v in p.items()}
    for f in range(lowres.shape[0]):
        x = np.concatenate([so.upsample2x(lowres[f]), gbuf_hi[f]], axis=0)
        H, Wd = x.shape[1:]
        a1 = np.maximum(so.conv3x3(x, p["w1"], p["b1"]), 0.0)
        a2 = np.maximum(so.conv3x3(a1, p["w2"], p["b2"]), 0.0)
        d = dy[f].reshape(3, -1)
        out["w3"] += d @ a2.reshape(C, -1).T
        out["b3"] += d.sum(axis=1)
        dW2, db2, da1 = so.conv3x3_backward(a1, p["w2"], (p["w3"].T @ d).reshape(C, H, Wd))
        dW1, db1, _ = so.conv3x3_backward(x, p["w1"], da1)
        for k, v in (("w2", dW2), ("b2", db2), ("w1", dW1), ("b1", db1)):
            out[k] += v
    return np.concatenate([out[name].ravel() for name, _ in so.sr_shapes(C)])


def _bwd_taps_transposed(x, W, dz):
    dW, db, dx = _bwd(x, np.swapaxes(W, 2, 3), dz)
    return np.swapaxes(dW, 2, 3), db, dx


_grad, _bwd = so.sr_grad, so.conv3x3_backward


@pytest.mark.parametrize("mutation", [dict(sr_grad=_grad_no_relu_mask),
                                      dict(conv3x3_backward=_bwd_taps_transposed)])
def test_grad_pins_catch_planted_mistakes(mutation):
    caught = 0
    with patched(**mutation):
        for t in (test_grad_matches_torch_autograd, test_grad_matches_central_differences):
            try:
                t()
            except AssertionError:
                caught += 1
    assert caught > 0
