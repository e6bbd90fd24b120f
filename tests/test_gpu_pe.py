"""GPU parity of the positionally encoded network (Sec. 3.4: every network
input is encoded; L levels widen F's input to 30 (1 + 2 L) columns and h's
slot input to 12 (1 + 2 L)) against the FP64 oracle, through the C ABI.

Forward tolerances are those of the unencoded forward (relative Frobenius
error: fp32 1e-4, bf16 2e-2, fp8_t 6e-2).  Object streaming of an encoded
handle is bitwise its fused forward; the FP32 form stays bitwise invariant
under slot permutations; the backward (fp32) meets 1e-4 per tensor on pixels
away from ReLU kinks, as the unencoded backward does.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2405_19056_amd import synth
from paper_2405_19056_amd.glassnet import GlassNet, GlassNetError, GN_E_UNSUPPORTED

from gpu_util import KINK, dev, host, log, relF, torch_dev
from test_gpu_backward import gpu_grad

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 2e-2, "fp8_t": 6e-2}


def frame(n, h, w, k, W, pe, seed):
    s = synth.streams(seed)
    wts = synth.make_weights(W, s["weights"], pe_levels=pe)
    fr = synth.Frame(synth.make_gbuf(n, h, w, s["gbuf"]),
                     synth.make_layers(n, k, h, w, s["slots"], s["active"], "uniform_count"),
                     synth.make_scene(n, s["gbuf"]))
    return wts, fr, s


def open_net(wts, W, precision, pe, pool="mean", k_max=8, slot_order="canonical"):
    net = GlassNet(wts, W, k_max=k_max, pool=pool, precision=precision, pe_levels=pe,
                   slot_order=slot_order)
    if precision == "fp8_t":
        _, cal, _ = frame(1, 64, 64, 4, W, pe, seed=999)
        net.calibrate(dev(cal.gbuf), dev(cal.layers), dev(cal.scene))
    return net


def run(net, fr, k=None):
    torch = torch_dev()
    k = fr.k if k is None else k
    L = dev(fr.layers[:, :k]) if k > 0 else None
    y = net.forward(dev(fr.gbuf), L, dev(fr.scene))
    torch.cuda.synchronize()
    return host(y)


@pytest.mark.parametrize("precision,W,pe,pool", [
    ("fp32", 128, 2, "mean"), ("fp32", 64, 4, "sum"), ("fp32", 128, 1, "mean"),
    ("bf16", 128, 1, "mean"), ("bf16", 128, 2, "sum"), ("bf16", 128, 3, "mean"),
    ("bf16", 128, 4, "mean"), ("bf16", 64, 2, "mean"), ("bf16", 64, 4, "sum"),
    ("fp8_t", 128, 2, "mean"), ("fp8_t", 128, 4, "sum")])
def test_encoded_forward_matches_oracle(precision, W, pe, pool):
    wts, fr, _ = frame(2, 37, 41, 5, W, pe, seed=90 + pe)
    log(f"encoded forward {precision} W={W} L={pe} {pool} 2x37x41 K=5")
    ref = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene, pool=pool, pe_levels=pe)
    with open_net(wts, W, precision, pe, pool) as net:
        y = run(net, fr)
        y0 = run(net, fr, k=0)
    e = relF(y, ref)
    log(f"  relF {e:.3e}")
    assert e <= TOL[precision]
    ref0 = oracle.forward(wts, W, fr.gbuf, fr.layers[:, :0], fr.scene, pool=pool, pe_levels=pe)
    assert relF(y0, ref0) <= TOL[precision]


def test_unencoded_weights_in_an_encoded_handle():
    """Zero sin/cos columns: the encoded handle reproduces the unencoded
    handle's result (up to the different summation of F1's K-steps)."""
    W, pe = 128, 3
    wts, fr, _ = frame(1, 30, 33, 4, W, 0, seed=97)
    from test_oracle_pe import _widen
    wide = _widen(wts.astype(np.float64), W, pe).astype(np.float32)
    with open_net(wts, W, "bf16", 0) as a, open_net(wide, W, "bf16", pe) as b:
        ya, yb = run(a, fr), run(b, fr)
    assert relF(yb, ya) <= 1e-2


@pytest.mark.parametrize("precision", ["bf16", "fp8_t", "fp32"])
def test_encoded_stream_is_the_fused_forward_bitwise(precision):
    torch = torch_dev()
    W, pe = 128, 2
    wts, fr, _ = frame(2, 29, 31, 5, W, pe, seed=98)
    with open_net(wts, W, precision, pe, slot_order="input") as net:
        y_ref = run(net, fr)
        g, sc = dev(fr.gbuf), dev(fr.scene)
        st = net.stream_state(fr.n, fr.h, fr.w)
        net.stream_begin(g, sc, st)
        for a, b in ((0, 2), (2, 3), (3, 5)):
            net.stream_accumulate(dev(fr.layers[:, a:b]), st)
        y = host(net.stream_finish(g, st))
        torch.cuda.synchronize()
        net.stream_release(st)
    assert np.array_equal(y, y_ref)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8_t"])
def test_encoded_forward_is_bitwise_permutation_invariant(precision):
    """Canonical slot order: per-pixel shuffles of the slots leave every
    output bit unchanged (Eq. (5) is symmetric in the slots)."""
    W, pe = (64, 2) if precision != "fp8_t" else (128, 2)
    wts, fr, s = frame(1, 40, 40, 6, W, pe, seed=99)
    rng = np.random.default_rng(99)
    with open_net(wts, W, precision, pe) as net:
        y0 = run(net, fr)
        for _ in range(4):
            p = synth.slot_shuffles(1, 6, 40, 40, 1, rng)[0]
            y = run(net, synth.Frame(fr.gbuf, synth.apply_slot_permutation(fr.layers, p),
                                     fr.scene))
            assert np.array_equal(y, y0)


@pytest.mark.parametrize("W,pe", [(128, 2), (64, 4), (128, 4)])
def test_encoded_backward_matches_oracle(W, pe):
    wts, fr, s = frame(2, 17, 21, 3, W, pe, seed=60 + pe)
    dy = s["noise"].normal(size=(2, 3, 17, 21)).astype(np.float32)
    ok = oracle.relu_margins(wts, W, fr.gbuf, fr.layers, fr.scene, pool="mean",
                             pe_levels=pe) >= KINK
    dy *= ok[:, None]
    log(f"encoded backward W={W} L={pe}: {int((~ok).sum())} of {ok.size} pixels near a kink")
    ref = oracle.grad_from_dy(wts, W, fr.gbuf, fr.layers, fr.scene, dy, pool="mean",
                              pe_levels=pe)
    with GlassNet(wts, W, k_max=8, precision="fp32", pe_levels=pe) as net:
        g = gpu_grad(net, fr, dy)
    off, worst = 0, 0.0
    for o, i in synth.layer_shapes(W, pe):
        for n in (o * i, o):
            a, b = g[off:off + n], ref[off:off + n]
            off += n
            if np.linalg.norm(b) == 0.0:
                assert np.all(a == 0.0)
                continue
            worst = max(worst, relF(a, b))
    log(f"  worst per-tensor relF {worst:.3e}")
    assert off == g.size == synth.num_params(W, pe)
    assert worst <= 1e-4


def test_encoded_serving_equals_the_forward():
    torch = torch_dev()
    W, pe = 128, 2
    wts, fr, _ = frame(1, 70, 90, 4, W, pe, seed=101)
    with open_net(wts, W, "bf16", pe) as net:
        y_ref = run(net, fr)
        g, L, sc = dev(fr.gbuf), dev(fr.layers), dev(fr.scene)
        out = torch.empty((1, 3, 70, 90), device="cuda:0")
        torch.cuda.synchronize()
        t = net.serve_submit(g, L, sc, out)
        deadline = time.time() + 60
        while not net.serve_poll(t)[0]:
            assert time.time() < deadline, "serving did not finish"
            time.sleep(0.0005)
        net.serve_drain()
        assert np.array_equal(host(out), y_ref)


def test_encoding_level_limits():
    W = 64
    with pytest.raises(GlassNetError) as e:
        GlassNet(np.zeros(synth.num_params(W, 5), np.float32), W, pe_levels=5)
    assert e.value.status == GN_E_UNSUPPORTED
    with pytest.raises(GlassNetError):            # weights sized for another level count
        GlassNet(np.zeros(synth.num_params(W, 1), np.float32), W, pe_levels=2)
