"""Pins of the FP64 spatial-network oracle (oracle/spatial_oracle.py).

Each ties the oracle to something other than itself: torch's float64
convolution, pooling and upsampling (library routines), a scalar brute-force
twin, the per-pixel oracle (which the spatial networks reduce to when every
3 x 3 kernel has only its centre tap and the U-Nets' lower branch is off),
invariants of Eq. (5) over whole transparency buffers, translation
equivariance away from the borders, and closed forms.
"""
import itertools

import numpy as np
import pytest
import torch
import torch.nn.functional as tf

import oracle
import oracle.spatial_oracle as so
from paper_2405_19056_amd import synth


def tiny(n=1, h=4, w=6, k=2, W=4, seed=3):
    s = synth.streams(seed)
    wts = synth.make_spatial_weights(W, s["weights"])
    fr = synth.Frame(synth.make_gbuf(n, h, w, s["gbuf"]),
                     synth.make_layers(n, k, h, w, s["slots"], s["active"], "uniform_count"),
                     synth.make_scene(n, s["gbuf"]))
    return wts, fr


def test_param_count():
    for W in (4, 64, 128):
        assert so.n_params(W) == synth.make_spatial_weights(W, np.random.default_rng(0)).size
    assert so.n_params(128) == sum(o * i * k * k + o for o, i, k in synth.spatial_layer_shapes(128))


@pytest.mark.parametrize("k", [1, 3])
def test_conv_equals_torch_conv2d(k):
    rng = np.random.default_rng(k)
    x = rng.normal(size=(5, 7, 9))
    A = rng.normal(size=(4, 5, k, k))
    c = rng.normal(size=4)
    got = so.conv(x, (A, c))
    ref = tf.conv2d(torch.from_numpy(x)[None], torch.from_numpy(A), torch.from_numpy(c),
                    padding=(k - 1) // 2)[0].numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12


def test_pool_and_upsample_equal_torch():
    x = np.random.default_rng(0).normal(size=(3, 6, 8))
    t = torch.from_numpy(x)[None]
    assert np.allclose(so.avgpool2(x), tf.avg_pool2d(t, 2)[0].numpy(), atol=1e-15)
    assert np.array_equal(so.upsample2(x), tf.interpolate(t, scale_factor=2, mode="nearest")[0].numpy())
    with pytest.raises(ValueError):
        so.avgpool2(x[:, :5])


@pytest.mark.parametrize("pool", ["mean", "sum"])
def test_vectorised_matches_bruteforce(pool):
    wts, fr = tiny(n=1, h=4, w=4, k=2, W=3)
    a = so.forward(wts, 3, fr.gbuf, fr.layers, fr.scene, pool=pool)
    b = so.forward_bruteforce(wts, 3, fr.gbuf, fr.layers, fr.scene, pool=pool)
    assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))


def test_whole_buffer_permutations_leave_the_image_unchanged():
    W = 4
    wts, fr = tiny(n=1, h=4, w=6, k=3, W=W)
    y0 = so.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
    for p in itertools.permutations(range(3)):
        y = so.forward(wts, W, fr.gbuf, fr.layers[:, list(p)], fr.scene)
        assert np.max(np.abs(y - y0)) <= 1e-13 * np.max(np.abs(y0))


def test_alpha_zero_buffer_equals_absent_buffer():
    W = 4
    wts, fr = tiny(n=1, h=4, w=6, k=3, W=W)
    L = fr.layers.copy()
    L[:, 1, 9] = 0.0
    a = so.forward(wts, W, fr.gbuf, L, fr.scene)
    b = so.forward(wts, W, fr.gbuf, L[:, [0, 2]], fr.scene)
    assert np.array_equal(a, b)


def _centre_only(P):
    """Zero every off-centre tap."""
    out = {}
    for net, layers in P.items():
        out[net] = []
        for A, c in layers:
            A = A.copy()
            if A.shape[2] == 3:
                keep = A[:, :, 1, 1].copy()
                A[:] = 0.0
                A[:, :, 1, 1] = keep
            out[net].append((A, c.copy()))
    return out


@pytest.mark.parametrize("pool", ["mean", "sum"])
def test_reduces_to_the_per_pixel_networks(pool):
    """Centre taps only and the U-Nets' lower branch switched off (its conv
    zero): F, B become per-pixel 3-layer MLPs (x -> e1 -> e2 -> out with e2's
    weights on e1), h and R per-pixel MLPs, so the spatial forward equals the
    per-pixel oracle's forward with those matrices."""
    W = 5
    wts, fr = tiny(n=2, h=4, w=6, k=3, W=W, seed=9)
    P = _centre_only(so.unpack(wts, W))
    for net in ("F", "B"):
        A, c = P[net][1]
        P[net][1] = (0 * A, 0 * c)
    flat = {}
    for net in so.NETS:
        L = P[net]
        if net in ("F", "B"):
            mats = [L[0], (L[2][0][:, :W], L[2][1]), L[3]]
        else:
            mats = L
        flat[net] = [(A[:, :, A.shape[2] // 2, A.shape[3] // 2], c) for A, c in mats]
    w_pp = oracle.pack(flat)
    a = so.forward(so.pack(P), W, fr.gbuf, fr.layers, fr.scene, pool=pool)
    b = oracle.forward(w_pp, W, fr.gbuf, fr.layers, fr.scene, pool=pool)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_translation_equivariance_away_from_borders():
    """Shifting every input by 2 pixels along x (one step of the U-Net's
    pooling grid) shifts the output, outside the receptive field of the frame
    edges and of the wrapped columns (the chain F, h, B, R sees well under
    24 pixels either side)."""
    W = 3
    wts, fr = tiny(n=1, h=4, w=64, k=2, W=W, seed=5)
    y = so.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
    ys = so.forward(wts, W, np.roll(fr.gbuf, 2, axis=3), np.roll(fr.layers, 2, axis=4), fr.scene)
    a, b = ys[..., 26:38], y[..., 24:36]
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(y))
    assert np.max(np.abs(ys - y)) > 1e-3          # the shift does change the image


def test_zero_weights_give_the_last_bias():
    W = 4
    wts, fr = tiny(n=1, h=4, w=4, k=2, W=W)
    P = so.unpack(np.zeros(so.n_params(W)), W)
    P["R"][2] = (P["R"][2][0], np.array([0.25, -1.5, 3.0]))
    y = so.forward(so.pack(P), W, fr.gbuf, fr.layers, fr.scene)
    assert np.array_equal(y, np.broadcast_to(np.array([0.25, -1.5, 3.0])[None, :, None, None],
                                             y.shape))


def test_mean_times_count_is_the_sum():
    W = 4
    wts, fr = tiny(n=1, h=4, w=6, k=3, W=W)
    _, la = so.forward(wts, W, fr.gbuf, fr.layers, fr.scene, pool="mean", return_latents=True)
    _, ls = so.forward(wts, W, fr.gbuf, fr.layers, fr.scene, pool="sum", return_latents=True)
    m, s = la[0], ls[0]
    assert np.allclose(m["tau"] * np.maximum(m["count"], 1.0)[None], s["tau"], rtol=1e-13,
                       atol=1e-13)
    assert np.array_equal(m["sigma"], s["sigma"])


# ------------------------------------------------- planted mistakes are caught
def _pins():
    return [lambda: test_conv_equals_torch_conv2d(3),
            lambda: test_pool_and_upsample_equal_torch(),
            lambda: test_vectorised_matches_bruteforce("mean"),
            lambda: test_reduces_to_the_per_pixel_networks("mean"),
            lambda: test_alpha_zero_buffer_equals_absent_buffer(),
            lambda: test_translation_equivariance_away_from_borders()]


def _conv_edge(x, layer):
    A, c = layer
    o, i, k, _ = A.shape
    r = (k - 1) // 2
    xp = np.pad(x, ((0, 0), (r, r), (r, r)), mode="edge")
    H, Wd = x.shape[1:]
    y = np.zeros((o, H, Wd))
    for dy in range(k):
        for dx in range(k):
            y += np.tensordot(A[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + Wd], axes=(1, 0))
    return y + c[:, None, None]


_ORIG_CONV = so.conv


def _conv_flipped(x, layer):
    A, c = layer
    return _ORIG_CONV(x, (A[:, :, ::-1, ::-1].copy(), c))


def _unet_swapped(layers, x):
    e1 = so.relu(so.conv(x, layers[0]))
    m = so.relu(so.conv(so.avgpool2(e1), layers[1]))
    e2 = so.relu(so.conv(np.concatenate([so.upsample2(m), e1]), layers[2]))
    return so.conv(e2, layers[3])


def _up_shifted(x):
    return np.roll(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 1, axis=2)


def _pool_max(x):
    C, H, Wd = x.shape
    return x.reshape(C, H // 2, 2, Wd // 2, 2).max(axis=(2, 4))


SPATIAL_MUTATIONS = {
    "edge-replicated instead of zero padding": ("conv", _conv_edge),
    "convolution instead of correlation (flipped taps)": ("conv", _conv_flipped),
    "skip join [u; e1] instead of [e1; u]": ("unet", _unet_swapped),
    "upsample shifted by one pixel": ("upsample2", _up_shifted),
    "max pooling instead of the 2 x 2 average": ("avgpool2", _pool_max),
}


@pytest.mark.parametrize("name", sorted(SPATIAL_MUTATIONS))
def test_some_spatial_pin_catches_the_planted_mistake(name):
    attr, fn = SPATIAL_MUTATIONS[name]
    old = getattr(so, attr)
    setattr(so, attr, fn)
    caught = 0
    try:
        for t in _pins():
            try:
                t()
            except (AssertionError, ValueError):
                caught += 1
    finally:
        setattr(so, attr, old)
    assert caught, f"no spatial pin caught: {name}"
