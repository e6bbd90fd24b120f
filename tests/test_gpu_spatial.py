"""GPU parity of the spatial networks (U-Net F and B, 3 x 3 CNNs h and R)
through the C ABI, against the FP64 spatial oracle.

The kernels compute in bf16 on the matrix cores with fp32 accumulation; the
gate is the bf16 output tolerance of the per-pixel networks (relative
Frobenius error 2e-2, largest element 4e-2, per-pixel p99 6e-2).  Small and
ragged frames are compared whole; the 512^2, K = 8 frame on a crop whose
central part lies beyond the receptive field of the crop's edges (the chain
F, h, B, R sees fewer than 16 pixels either side).
"""
import numpy as np
import pytest

import oracle.spatial_oracle as so
from paper_2405_19056_amd import synth
from paper_2405_19056_amd.glassnet import GN_E_INVAL, GlassNet, GlassNetError

from gpu_util import dev, gate, host, log, relF, torch_dev

pytestmark = pytest.mark.gpu

TOL = 2e-2


def frame(n, h, w, k, W, seed):
    s = synth.streams(seed)
    wts = synth.make_spatial_weights(W, s["weights"])
    fr = synth.Frame(synth.make_gbuf(n, h, w, s["gbuf"]),
                     synth.make_layers(n, k, h, w, s["slots"], s["active"], "uniform_count"),
                     synth.make_scene(n, s["gbuf"]))
    return wts, fr


def run(net, wts, fr):
    torch = torch_dev()
    L = dev(fr.layers) if fr.k > 0 else None
    y = net.spatial_forward(dev(wts), dev(fr.gbuf), L, dev(fr.scene))
    torch.cuda.synchronize()
    return host(y)


@pytest.mark.parametrize("W,n,h,w,k,pool", [(64, 1, 16, 24, 3, "mean"), (128, 2, 10, 34, 2, "sum"),
                                            (128, 1, 32, 70, 5, "mean"), (64, 1, 6, 8, 0, "mean")])
def test_spatial_forward_matches_oracle(W, n, h, w, k, pool):
    wts, fr = frame(n, h, w, k, W, seed=200 + h + k)
    log(f"spatial W={W} {n}x{h}x{w} K={k} {pool}")
    ref = so.forward(wts, W, fr.gbuf, fr.layers, fr.scene, pool=pool)
    with GlassNet(synth.make_weights(W, np.random.default_rng(0)), W, k_max=8, pool=pool,
                  precision="bf16") as net:
        assert net.spatial_num_params() == so.n_params(W) == wts.size
        y = run(net, wts, fr)
    gate(y, ref, TOL, f"spatial W={W} {n}x{h}x{w} K={k}")


def test_spatial_256sq_k4_whole_frame():
    W = 128
    wts, fr = frame(1, 256, 256, 4, W, seed=301)
    ref = so.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
    with GlassNet(synth.make_weights(W, np.random.default_rng(0)), W, k_max=8,
                  precision="bf16") as net:
        y = run(net, wts, fr)
    gate(y, ref, TOL, "spatial 256^2 K=4 whole frame")


def test_spatial_512sq_k8_central_crop():
    """The 512^2, K = 8 frame on the GPU; the oracle on a 96 x 96 crop of its
    inputs: the crop's central 64 x 64 pixels see none of the crop's edges."""
    W = 128
    wts, fr = frame(1, 512, 512, 8, W, seed=302)
    with GlassNet(synth.make_weights(W, np.random.default_rng(0)), W, k_max=8,
                  precision="bf16") as net:
        y = run(net, wts, fr)
    assert np.all(np.isfinite(y))
    for (r0, c0) in [(200, 304), (0, 416)]:          # an interior crop and a corner crop
        crop = synth.Frame(fr.gbuf[:, :, r0:r0 + 96, c0:c0 + 96],
                           fr.layers[:, :, :, r0:r0 + 96, c0:c0 + 96], fr.scene)
        ref = so.forward(wts, W, crop.gbuf, crop.layers, crop.scene)
        # rows/cols away from the crop's cut edges (frame edges are real edges)
        rs = slice(16 if r0 > 0 else 0, 80 if r0 + 96 < 512 else 96)
        cs = slice(16 if c0 > 0 else 0, 80 if c0 + 96 < 512 else 96)
        got = y[:, :, r0:r0 + 96, c0:c0 + 96][:, :, rs, cs]
        gate(got, ref[:, :, rs, cs], TOL, f"spatial 512^2 K=8 crop at ({r0}, {c0})")


def test_spatial_buffer_permutations_and_alpha_zero():
    """Whole-buffer permutations agree up to the pool's fp32 summation order;
    a buffer with alpha = 0 everywhere is the same as no buffer, bitwise."""
    W = 64
    wts, fr = frame(1, 24, 32, 4, W, seed=303)
    with GlassNet(synth.make_weights(W, np.random.default_rng(0)), W, k_max=8,
                  precision="bf16") as net:
        y0 = run(net, wts, fr)
        yp = run(net, wts, synth.Frame(fr.gbuf, fr.layers[:, [2, 0, 3, 1]], fr.scene))
        L = fr.layers.copy()
        L[:, 1, 9] = 0.0
        ya = run(net, wts, synth.Frame(fr.gbuf, L, fr.scene))
        yb = run(net, wts, synth.Frame(fr.gbuf, np.ascontiguousarray(L[:, [0, 2, 3]]), fr.scene))
    assert relF(yp, y0) <= 1e-3
    assert np.array_equal(ya, yb)


def test_spatial_rejects_odd_sizes():
    torch = torch_dev()
    W = 64
    wts, fr = frame(1, 9, 12, 2, W, seed=304)
    with GlassNet(synth.make_weights(W, np.random.default_rng(0)), W, k_max=8) as net:
        with pytest.raises(GlassNetError) as e:
            run(net, wts, fr)
        assert e.value.status == GN_E_INVAL
        torch.cuda.synchronize()
