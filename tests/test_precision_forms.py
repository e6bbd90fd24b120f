"""Error of the reduced-precision forms against the FP64 oracle, by CPU
emulation of their rounding (no GPU).

The library builds GN_BF16 and GN_FP8_T and rejects GN_FP8_ALL with
GN_E_UNSUPPORTED.  This file measures why: every layer's inputs and weights
rounded as the form rounds them (bf16 round-to-nearest-even; OCP E4M3FN with
round-to-nearest-even and saturation at 448, per-output-channel weight scales
max |W[n, :]| / 448 and one static activation scale per layer, amax / 448 from
a separate calibration frame), products accumulated exactly, biases and the
pool of Eq. (5) in full precision.  The FP8_T form puts h's second layer (the
per-slot W x W layer) in FP8 and the rest in bf16; FP8_ALL puts every layer in
FP8.  On the 512^2, K = 8 workload's input distribution the first two meet
their bars (2e-2 and 6e-2 relative Frobenius error) and FP8_ALL does not: its
error is bound by E4M3's 3 mantissa bits compounding over the 12 layers of
the chain F, h, B, R, not by the scales.
"""
import numpy as np
import pytest

import oracle
from oracle import glassnet_oracle as go
from paper_2405_19056_amd import synth

W = 128
K = 8


def bf16(x):
    """Round to bf16 (nearest, ties to even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3(x):
    """Round to OCP E4M3FN (3 mantissa bits, bias 7, subnormal step 2^-9,
    largest finite 448), nearest with ties to even, saturating."""
    a = np.minimum(np.abs(x), 448.0)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -6)))
    q = 2.0 ** (e - 3)
    return np.sign(x) * np.minimum(np.round(a / q) * q, 448.0)


def test_e4m3_grid():
    """The E4M3FN grid: every representable magnitude is a fixed point, the
    midpoints between neighbours round to the even one, and values beyond
    448 saturate."""
    grid = [m * 2.0 ** -9 for m in range(8)]                        # subnormals
    grid += [(1 + m / 8) * 2.0 ** e for e in range(-6, 9) for m in range(8)]
    grid = np.array([g for g in grid if g <= 448.0])
    assert grid.size == 127 and grid.max() == 448.0
    assert np.array_equal(e4m3(grid), grid) and np.array_equal(e4m3(-grid), -grid)
    mid = (grid[:-1] + grid[1:]) / 2
    # the neighbour whose 3-bit mantissa (or subnormal count) is even
    even = np.where(np.arange(grid.size - 1) % 2 == 0, grid[:-1], grid[1:])
    assert np.array_equal(e4m3(mid), even)
    assert e4m3(np.array([500.0, 1e6, -1e6])).tolist() == [448.0, 448.0, -448.0]


def test_bf16_rounding():
    assert bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0                  # tie to even (down)
    assert bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6  # tie to even (up)
    assert bf16(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)) == 1.0 + 2.0 ** -7


def _forward(P, G, L, S, layer, pool="mean"):
    """The per-pixel forward of Eq. (5) with every linear map computed by
    layer(name, A, c, x); the pool and the mean in full precision."""
    def mlp(net, x):
        (A1, c1), (A2, c2), (A3, c3) = P[net]
        a = np.maximum(layer(net + "1", A1, c1, x), 0.0)
        a = np.maximum(layer(net + "2", A2, c2, a), 0.0)
        return layer(net + "3", A3, c3, a)
    sigma = mlp("F", np.concatenate([G, S]))
    Z = np.zeros_like(sigma)
    cnt = np.zeros(sigma.shape[1])
    for i in range(L.shape[0]):
        m = (L[i][9] > 0).astype(np.float64)
        Z += m * mlp("T", np.concatenate([L[i], sigma]))
        cnt += m
    tau = Z / np.maximum(cnt, 1.0) if pool == "mean" else Z
    phi = mlp("B", np.concatenate([sigma, tau]))
    return mlp("R", np.concatenate([phi, G[11:14]]))


def exact(name, A, c, x):
    return A @ x + c[:, None]


def rounded_bf16(name, A, c, x):
    return bf16(A) @ bf16(x) + c[:, None]


def fp8_layer(scales):
    def f(name, A, c, x):
        sw = np.abs(A).max(axis=1) / 448.0
        sw = np.where(sw > 0, sw, 1.0)
        sa = scales[name]
        return (e4m3(A / sw[:, None]) @ e4m3(x / sa)) * (sa * sw)[:, None] + c[:, None]
    return f


def calibrate(P, G, L, S):
    """amax / 448 of every layer's input over a calibration frame."""
    amax = {}

    def rec(name, A, c, x):
        amax[name] = max(amax.get(name, 0.0), float(np.abs(x).max()))
        return exact(name, A, c, x)
    _forward(P, G, L, S, rec)
    return {k: (v / 448.0 if v > 0 else 1.0) for k, v in amax.items()}


@pytest.fixture(scope="module")
def errors():
    w = synth.make_weights(W, synth.streams(2)["weights"])
    P = go.unpack(w, W)
    fr = synth.make_frame(1, 48, 48, K, seed=2)
    cal = synth.make_frame(1, 48, 48, K, seed=999)
    G, L, S, _ = go._pixels(fr.gbuf, fr.layers, fr.scene)
    Gc, Lc, Sc, _ = go._pixels(cal.gbuf, cal.layers, cal.scene)
    scales = calibrate(P, Gc, Lc, Sc)
    ref = _forward(P, G, L, S, exact)
    # the emulation's exact arithmetic is the oracle's forward
    y0 = oracle.forward(w, W, fr.gbuf, fr.layers, fr.scene)
    assert np.max(np.abs(np.moveaxis(y0, 1, 0).reshape(3, -1) - ref)) <= 1e-12 * np.abs(ref).max()
    fp8 = fp8_layer(scales)

    def fp8_t(name, A, c, x):
        return fp8(name, A, c, x) if name == "T2" else rounded_bf16(name, A, c, x)
    rel = lambda y: float(np.linalg.norm(y - ref) / np.linalg.norm(ref))  # noqa: E731
    return {"bf16": rel(_forward(P, G, L, S, rounded_bf16)),
            "fp8_t": rel(_forward(P, G, L, S, fp8_t)),
            "fp8_all": rel(_forward(P, G, L, S, fp8))}


def test_bf16_and_fp8_t_meet_their_bars_and_fp8_all_does_not(errors):
    print({k: f"{v:.3e}" for k, v in errors.items()})
    assert errors["bf16"] <= 2e-2
    assert errors["fp8_t"] <= 6e-2
    assert errors["fp8_all"] > 6e-2
    assert errors["bf16"] < errors["fp8_t"] < errors["fp8_all"]
