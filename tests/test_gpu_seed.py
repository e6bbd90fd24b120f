"""Seeded initialisation through the C ABI: glassnet_create with no host
weights draws them from gn_config.seed (He et al.'s uniform initialisation
for ReLU layers; biases within 1/sqrt(fan_in)).  The values are checked
against SplitMix64 written out here from its published definition (Steele,
Lea and Flood 2014), and a seeded handle's forward against the oracle on
the weights it reports."""
import math

import numpy as np
import pytest

import oracle
from paper_2405_19056_amd import synth
from paper_2405_19056_amd.glassnet import GlassNet

from gpu_util import dev, gate, host, torch_dev

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1


def splitmix64(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def expected(W, seed, pe=0):
    """The documented draw, in the flat layout (nets F, T, B, R; per layer
    matrix [out][in] then bias)."""
    out = []
    e = 0
    for (o, i) in synth.layer_shapes(W, pe):
        for count, bound in ((o * i, math.sqrt(6.0 / i)), (o, 1.0 / math.sqrt(i))):
            for _ in range(count):
                x = splitmix64((seed + (e + 1) * 0x9E3779B97F4A7C15) & M64)
                u = (x >> 11) * 2.0 ** -53
                out.append(np.float32((2.0 * u - 1.0) * bound))
                e += 1
    return np.asarray(out, dtype=np.float32)


@pytest.mark.parametrize("W,pe,seed", [(64, 0, 0), (128, 0, 12345), (64, 2, 2 ** 63 + 7)])
def test_seeded_weights_follow_the_documented_draw(W, pe, seed):
    torch_dev()
    with GlassNet(None, W, precision="bf16", pe_levels=pe, seed=seed) as net:
        got = net.get_weights()
    want = expected(W, seed, pe)
    assert got.size == oracle.n_params(W, pe) == want.size
    assert np.array_equal(got, want)


def test_seeds_differ_and_bounds_hold():
    torch_dev()
    W = 128
    with GlassNet(None, W, seed=1) as a, GlassNet(None, W, seed=2) as b, \
            GlassNet(None, W, seed=1) as c:
        wa, wb, wc = a.get_weights(), b.get_weights(), c.get_weights()
    assert np.array_equal(wa, wc) and not np.array_equal(wa, wb)
    P = oracle.unpack(wa, W)
    for net in ("F", "T", "B", "R"):
        for A, bias in P[net]:
            fan_in = A.shape[1]
            assert np.max(np.abs(A)) <= math.sqrt(6.0 / fan_in)
            assert np.max(np.abs(bias)) <= 1.0 / math.sqrt(fan_in)
            # uniform on +-bound: variance bound^2 / 3
            assert abs(A.var() / (6.0 / fan_in / 3.0) - 1.0) < 0.1


def test_seeded_handle_forward_matches_oracle():
    torch = torch_dev()
    W = 128
    fr = synth.make_frame(1, 33, 47, 4, seed=5)
    with GlassNet(None, W, k_max=8, precision="bf16", seed=77) as net:
        w = net.get_weights()
        y = net.forward(dev(fr.gbuf), dev(fr.layers), dev(fr.scene))
        torch.cuda.synchronize()
        y = host(y)
    ref = oracle.forward(w, W, fr.gbuf, fr.layers, fr.scene, pool="mean")
    gate(y, ref, 2e-2, "seeded bf16")
