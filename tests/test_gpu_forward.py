"""GPU parity of the forward pass against the FP64 oracle, through the C ABI.

Tolerances (relative Frobenius error on output radiance): fp32 1e-4, bf16
2e-2.  Small frames are compared element by element; the full 256^2/K=4 and
512^2/K=8 workloads are compared on sampled pixels the oracle evaluates one
by one (pixels are independent).
"""
import numpy as np
import pytest

import oracle
from paper_2405_19056_amd import synth
from paper_2405_19056_amd.glassnet import GlassNet, GlassNetError, GN_E_INVAL

from gpu_util import (dev, gate, gpu_on_sample, host, log, oracle_on_sample, relF,
                      sample_every_tile, torch_dev)

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 2e-2, "fp8_t": 6e-2}


def frame(n, h, w, k, W, seed, alpha_mode="uniform_count"):
    s = synth.streams(seed)
    wts = synth.make_weights(W, s["weights"])
    fr = synth.Frame(synth.make_gbuf(n, h, w, s["gbuf"]),
                     synth.make_layers(n, k, h, w, s["slots"], s["active"], alpha_mode),
                     synth.make_scene(n, s["gbuf"]))
    return wts, fr


def canonical_slot_order(layers):
    """The library's canonical order of every pixel's slots, on the host:
    active slots by alpha's bits, ties by planes 0..11's bits, then index;
    inactive slots after them by index.  Returns perm [n][k][h][w]."""
    bits = np.ascontiguousarray(layers, dtype=np.float32).view(np.uint32).astype(np.int64)
    active = layers[:, :, 9] > 0
    idx = np.broadcast_to(np.arange(layers.shape[1])[None, :, None, None], active.shape)
    keys = [idx] + [np.where(active, bits[:, :, c], 0) for c in range(11, -1, -1)]
    keys.append(np.where(active, bits[:, :, 9], 2 ** 33))       # primary key last
    return np.lexsort(keys, axis=1)


def calibrate(net, W, k, seed=999):
    """FP8 activation scale from a separate seeded calibration frame."""
    _, cal = frame(1, 64, 64, k, W, seed=seed)
    net.calibrate(dev(cal.gbuf), dev(cal.layers) if k else None, dev(cal.scene))


def run(net, fr):
    torch = torch_dev()
    L = dev(fr.layers) if fr.k > 0 else None
    y = net.forward(dev(fr.gbuf), L, dev(fr.scene))
    torch.cuda.synchronize()
    return host(y)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_config0_64sq_k2_w64_elementwise(precision):
    w, fr, _ = synth.config_inputs("c0_64sq_k2_w64")
    log(f"config c0 {precision}")
    ref = oracle.forward(w, 64, fr.gbuf, fr.layers, fr.scene, pool="mean")
    with GlassNet(w, 64, k_max=2, pool="mean", precision=precision) as net:
        y = run(net, fr)
    gate(y, ref, TOL[precision], f"c0 {precision}")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("pool", ["mean", "sum"])
@pytest.mark.parametrize("W", [64, 128])
def test_ragged_multi_frame(precision, pool, W):
    """3 frames of 37 x 53 (several tiles and a ragged tail), K=5."""
    w, fr = frame(3, 37, 53, 5, W, seed=100 + W)
    log(f"ragged {precision} {pool} W={W}")
    ref = oracle.forward(w, W, fr.gbuf, fr.layers, fr.scene, pool=pool)
    with GlassNet(w, W, k_max=8, pool=pool, precision=precision) as net:
        y = run(net, fr)
    gate(y, ref, TOL[precision], f"ragged {precision} {pool} W={W}")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_edge_shapes(precision):
    W = 128
    for (n, h, w_, k) in [(1, 1, 1, 1), (1, 1, 7, 0), (2, 3, 5, 3), (1, 16, 16, 8), (1, 5, 61, 2)]:
        wts, fr = frame(n, h, w_, k, W, seed=7 + h + k)
        log(f"edge {precision} n={n} h={h} w={w_} k={k}")
        ref = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
        with GlassNet(wts, W, k_max=8, precision=precision) as net:
            y = run(net, fr)
        gate(y, ref, TOL[precision], f"edge {(n, h, w_, k)}")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8_t"])
def test_maximum_slot_count(precision):
    """k = GN_MAX_K = 64 slots (the largest a handle accepts) on a ragged frame;
    one more is rejected before any launch."""
    W, K = 128, 64
    wts, fr = frame(1, 19, 27, K, W, seed=12)
    log(f"max slots {precision}: 1x19x27 K={K}")
    ref = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
    with GlassNet(wts, W, k_max=K, precision=precision) as net:
        if precision == "fp8_t":
            calibrate(net, W, 4)
        y = run(net, fr)
        L65 = np.concatenate([fr.layers, fr.layers[:, :1]], axis=1)
        with pytest.raises(GlassNetError) as e:
            run(net, synth.Frame(fr.gbuf, L65, fr.scene))
        assert e.value.status == GN_E_INVAL
    gate(y, ref, TOL[precision], f"max slots {precision}")
    with pytest.raises(GlassNetError):
        GlassNet(wts, W, k_max=K + 1, precision=precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_all_slots_inactive_equals_no_slots(precision):
    W = 128
    wts, fr = frame(1, 24, 24, 4, W, seed=5)
    L0 = fr.layers.copy()
    L0[:, :, 9] = 0.0
    with GlassNet(wts, W, k_max=8, precision=precision) as net:
        y_dead = run(net, synth.Frame(fr.gbuf, L0, fr.scene))
        y_none = run(net, synth.Frame(fr.gbuf, fr.layers[:, :0], fr.scene))
    assert np.array_equal(y_dead, y_none)
    ref = oracle.forward(wts, W, fr.gbuf, fr.layers[:, :0], fr.scene)
    gate(y_none, ref, TOL[precision], "no slots")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8_t"])
def test_coherent_coverage_matches_oracle(precision):
    """Discs of coverage per slot (a labelled variant): many waves see slots in
    which none of their pixels is active, which the fused kernel skips."""
    W = 128
    wts, fr = frame(2, 64, 80, 6, W, seed=8, alpha_mode="discs")
    log(f"coherent coverage {precision}: active fraction {(fr.layers[:, :, 9] > 0).mean():.3f}")
    ref = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
    with GlassNet(wts, W, k_max=8, precision=precision) as net:
        if precision == "fp8_t":
            calibrate(net, W, 4)
        y = run(net, fr)
        # a slot of zero alpha everywhere, inserted: bitwise the same result
        L = np.concatenate([fr.layers[:, :2], 0 * fr.layers[:, :1], fr.layers[:, 2:]], axis=1)
        y_ins = run(net, synth.Frame(fr.gbuf, L, fr.scene))
    gate(y, ref, TOL[precision], f"coherent {precision}")
    assert np.array_equal(y, y_ins)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_one_active_slot_equals_k1(precision):
    W = 128
    wts, fr = frame(1, 32, 32, 8, W, seed=9)
    rng = np.random.default_rng(1)
    L = fr.layers.copy()
    L[:, :, 9] = 0.0
    pos = rng.integers(0, 8, size=(32, 32))
    single = np.empty((1, 1, 12, 32, 32), np.float32)
    for r in range(32):
        for c in range(32):
            L[0, pos[r, c], 9, r, c] = 0.1 + 0.9 * rng.uniform()
            single[0, 0, :, r, c] = L[0, pos[r, c], :, r, c]
    with GlassNet(wts, W, k_max=8, precision=precision) as net:
        y8 = run(net, synth.Frame(fr.gbuf, L, fr.scene))
        y1 = run(net, synth.Frame(fr.gbuf, single, fr.scene))
    assert np.array_equal(y8, y1)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8_t"])
@pytest.mark.parametrize("k", [2, 5, 8, 12])
def test_slot_permutations_are_bitwise(precision, k):
    """Per-pixel shuffles of the slots leave every output bit unchanged: each
    pixel's slots are pooled in canonical order (Eq. (5) is symmetric; the
    order-inversion table of Sec. 4.3 reports no difference).  k = 12 takes
    the general ranking path of the fused kernel, k <= 8 the register one."""
    W = 128
    wts, fr = frame(1, 48, 40, k, W, seed=21 + k)
    perms = synth.slot_shuffles(1, k, 48, 40, 6, np.random.default_rng(2))
    with GlassNet(wts, W, k_max=16, precision=precision) as net:
        if precision == "fp8_t":
            calibrate(net, W, 4)
        y0 = run(net, fr)
        for p in perms:
            y = run(net, synth.Frame(fr.gbuf, synth.apply_slot_permutation(fr.layers, p), fr.scene))
            assert np.array_equal(y, y0)
    gate(y0, oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene), TOL[precision],
         f"{precision} k={k}")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8_t"])
@pytest.mark.parametrize("k,W,pe,order", [(8, 128, 0, "canonical"), (3, 64, 0, "canonical"),
                                          (12, 128, 0, "canonical"), (6, 128, 2, "canonical"),
                                          (8, 128, 0, "input")])
def test_pixel_permutations_are_bitwise(precision, k, W, pe, order):
    """Pixels are independent (Sec. 3.4), and every path computes each one
    the same whichever lane, wave and tile it lands in: moving pixels around
    the frame (tail tile included) changes which pixels share a wave, its
    slot-skip decisions and the tail lanes' duplicates, but no output bit.
    Canonical order with the register ranking (k <= 8) and the general one
    (k = 12), encoded inputs, input order and the plane pipeline."""
    if precision == "fp8_t" and W != 128:
        pytest.skip("fp8_t is built for W = 128")
    h, w = 48, 44                     # 2112 px: 8 full tiles and a ragged one
    wts, fr = frame(2, h, w, k, W, seed=40 + k + pe, alpha_mode="uniform_count")
    if pe:
        wts = synth.make_weights(W, synth.streams(40 + k)["weights"], pe_levels=pe)
    rng = np.random.default_rng(k * 7 + pe)
    with GlassNet(wts, W, k_max=16, precision=precision, pe_levels=pe, slot_order=order) as net:
        if precision == "fp8_t":
            calibrate(net, W, 4)
        y0 = run(net, fr)
        for _ in range(3):
            perm = rng.permutation(h * w)
            g = fr.gbuf.reshape(2, -1, h * w)[:, :, perm].reshape(fr.gbuf.shape)
            L = fr.layers.reshape(2, k, -1, h * w)[:, :, :, perm].reshape(fr.layers.shape)
            y = run(net, synth.Frame(g, L, fr.scene))
            back = np.empty_like(y.reshape(2, 3, h * w))
            back[:, :, perm] = y.reshape(2, 3, h * w)
            assert np.array_equal(back.reshape(y0.shape), y0)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8_t"])
def test_equal_alphas_take_the_full_record_order(precision):
    """Active slots of equal alpha are ordered by their other planes: a frame
    whose slots share a handful of alpha values (and some fully duplicated
    records) still gives bitwise the same image under every shuffle."""
    W, k, h, w = 128, 6, 32, 36
    wts, fr = frame(1, h, w, k, W, seed=27)
    L = fr.layers.copy()
    rng = np.random.default_rng(27)
    act = L[:, :, 9] > 0
    L[:, :, 9] = np.where(act, rng.choice([0.25, 0.5, 0.75], size=act.shape), 0.0)
    L[:, 3] = L[:, 1]                        # slot 3 duplicates slot 1 everywhere
    fr = synth.Frame(fr.gbuf, L.astype(np.float32), fr.scene)
    with GlassNet(wts, W, k_max=8, precision=precision) as net:
        if precision == "fp8_t":
            calibrate(net, W, 4)
        y0 = run(net, fr)
        for p in synth.slot_shuffles(1, k, h, w, 6, rng):
            y = run(net, synth.Frame(fr.gbuf, synth.apply_slot_permutation(fr.layers, p), fr.scene))
            assert np.array_equal(y, y0)
    gate(y0, oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene), TOL[precision], "equal alphas")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8_t"])
def test_input_order_handle(precision):
    """slot_order="input" pools in slot order: it matches the oracle, agrees
    with the canonical handle up to the pool's fp32 rounding, and equals it
    bitwise when the slots already sit in canonical order."""
    W, k = 128, 5
    wts, fr = frame(1, 40, 44, k, W, seed=28)
    with GlassNet(wts, W, k_max=8, precision=precision) as a, \
            GlassNet(wts, W, k_max=8, precision=precision, slot_order="input") as b:
        if precision == "fp8_t":
            calibrate(a, W, 4)
            calibrate(b, W, 4)
        ya, yb = run(a, fr), run(b, fr)
        order = canonical_slot_order(fr.layers)
        yc = run(b, synth.Frame(fr.gbuf, synth.apply_slot_permutation(fr.layers, order), fr.scene))
    ref = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
    gate(yb, ref, TOL[precision], f"input order {precision}")
    assert relF(ya, yb) <= (1e-6 if precision == "fp32" else 1e-2)
    assert np.array_equal(yc, ya)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_run_to_run_bitwise(precision):
    W = 128
    wts, fr = frame(2, 40, 40, 4, W, seed=31)
    with GlassNet(wts, W, k_max=8, precision=precision) as net:
        a = run(net, fr)
        b = run(net, fr)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("cfg,precision", [("c1_256sq_k4_w128", "bf16"),
                                           ("c1_256sq_k4_w128", "fp32"),
                                           ("c2_512sq_k8_w128", "bf16"),
                                           ("c2_512sq_k8_w128", "fp32")])
def test_full_size_on_sampled_pixels(cfg, precision):
    c = synth.CONFIGS[cfg]
    w, fr, _ = synth.config_inputs(cfg)
    log(f"full-size {cfg} {precision}")
    with GlassNet(w, c["width"], k_max=c["k"], pool=c["pool"], precision=precision) as net:
        y = run(net, fr)
    assert np.all(np.isfinite(y))
    flat = sample_every_tile(fr, 3 if fr.h * fr.w > 100000 else 8, np.random.default_rng(0))
    ref = oracle_on_sample(w, c["width"], fr, flat, c["pool"])
    got = gpu_on_sample(y, fr, flat)
    gate(got, ref, TOL[precision], f"{cfg} {precision} sampled ({len(flat)} px, every tile)")
    if precision != "fp32":
        # the whole frame against the fp32 path (itself oracle-checked): no tile
        # anywhere may stray beyond the precision's tolerance
        with GlassNet(w, c["width"], k_max=c["k"], pool=c["pool"], precision="fp32") as net32:
            y32 = run(net32, fr)
        gate(y, y32, TOL[precision], f"{cfg} {precision} whole frame vs fp32 path")


def test_invalid_arguments_are_rejected():
    torch = torch_dev()
    W = 64
    wts, fr = frame(1, 8, 8, 3, W, seed=1)
    with GlassNet(wts, W, k_max=2) as net:
        with pytest.raises(GlassNetError) as e:
            run(net, fr)                     # k=3 > k_max=2
        assert e.value.status == GN_E_INVAL
        g = dev(fr.gbuf)
        with pytest.raises(GlassNetError):
            net.forward(g, dev(fr.layers[:, :2]), dev(fr.scene), out=g.view(-1)[:3 * 64].view(1, 3, 8, 8))
        # the handle still works after rejected calls
        y = net.forward(g, dev(fr.layers[:, :2]), dev(fr.scene))
        torch.cuda.synchronize()
        assert np.all(np.isfinite(host(y)))


def test_fp32_plane_workspace_reused_across_sizes_and_with_backward():
    """One fp32 handle: a small frame, a larger one (the plane workspace grows),
    the small one again (planes re-zeroed for the shorter rows), then a backward
    on a third size and the small forward once more: every result matches the
    oracle, and the repeated small forwards are bitwise equal."""
    torch = torch_dev()
    W = 64
    wts, fr_a = frame(2, 19, 23, 3, W, seed=61)
    _, fr_b = frame(1, 80, 80, 5, W, seed=62)
    _, fr_c = frame(1, 30, 33, 2, W, seed=63)
    with GlassNet(wts, W, k_max=8, precision="fp32") as net:
        ya = run(net, fr_a)
        yb = run(net, fr_b)
        ya2 = run(net, fr_a)
        dy = np.random.default_rng(3).normal(size=(1, 3, 30, 33)).astype(np.float32)
        g = net.backward(dev(fr_c.gbuf), dev(fr_c.layers), dev(fr_c.scene), dev(dy))
        torch.cuda.synchronize()
        ya3 = run(net, fr_a)
    for y, fr in ((ya, fr_a), (yb, fr_b)):
        gate(y, oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene), TOL["fp32"])
    assert np.array_equal(ya, ya2) and np.array_equal(ya, ya3)
    assert np.all(np.isfinite(host(g)))


def test_fp32_forward_rejects_more_pixels_than_it_addresses():
    """The fp32 plane pipeline covers at most 3 * 2^20 pixels per call; beyond
    that the forward is an argument error raised before any launch."""
    torch = torch_dev()
    W, n, h, w = 64, 1, 1025, 3072
    wts = synth.make_weights(W, np.random.default_rng(0))
    g = torch.zeros((n, 14, h, w), device="cuda:0")
    sc = torch.zeros((n, 16), device="cuda:0")
    with GlassNet(wts, W, k_max=2, precision="fp32") as net:
        with pytest.raises(GlassNetError) as e:
            net.forward(g, None, sc)
        assert e.value.status == GN_E_INVAL
    del g
    torch.cuda.empty_cache()


def test_workspace_does_not_depend_on_k():
    W = 128
    wts, _ = frame(1, 4, 4, 1, W, seed=0)
    sizes = []
    for kmax in (1, 2, 4, 8, 16):
        with GlassNet(wts, W, k_max=kmax, precision="bf16") as net:
            sizes.append(net.workspace_bytes())
    assert len(set(sizes)) == 1, sizes


# ------------------------------------------------------------------ fp8 form
def test_fp8_small_frames_elementwise():
    W = 128
    for (n, h, w_, k, pool) in [(1, 37, 53, 8, "mean"), (2, 16, 40, 4, "sum"), (1, 5, 7, 0, "mean")]:
        wts, fr = frame(n, h, w_, k, W, seed=50 + k)
        log(f"fp8 n={n} h={h} w={w_} k={k} {pool}")
        ref = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene, pool=pool)
        with GlassNet(wts, W, k_max=8, pool=pool, precision="fp8_t") as net:
            calibrate(net, W, max(k, 1))
            y = run(net, fr)
        gate(y, ref, TOL["fp8_t"], f"fp8 {(n, h, w_, k, pool)}")


def test_fp8_full_size_on_sampled_pixels_and_permutations():
    cfg = "c2_512sq_k8_w128"
    c = synth.CONFIGS[cfg]
    w, fr, st = synth.config_inputs(cfg)
    with GlassNet(w, 128, k_max=8, pool=c["pool"], precision="fp8_t") as net:
        calibrate(net, 128, 8)
        y = run(net, fr)
        flat = sample_every_tile(fr, 3, np.random.default_rng(0))
        ref = oracle_on_sample(w, 128, fr, flat, c["pool"])
        gate(gpu_on_sample(y, fr, flat), ref, TOL["fp8_t"], "fp8 512^2 K=8 sampled, every tile")
        perms = synth.slot_shuffles(1, 8, fr.h, fr.w, 4, st["shuffles"])
        for p in perms:
            yp = run(net, synth.Frame(fr.gbuf, synth.apply_slot_permutation(fr.layers, p), fr.scene))
            assert np.array_equal(yp, y)
        with GlassNet(w, 128, k_max=8, pool=c["pool"], precision="fp32") as net32:
            y32 = run(net32, fr)
        gate(y, y32, TOL["fp8_t"], "fp8 512^2 K=8 whole frame vs fp32 path")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8_t"])
def test_permutation_sweep_512sq_k8_32_shuffles(precision):
    """The 512^2, K=8 workload under 32 independent per-pixel shuffles of its
    eight layers (Eq. (5) is symmetric in the layers): with each pixel's
    slots pooled in canonical order every output is bitwise unchanged in
    every precision (Sec. 4.3's order-inversion table: difference 0).  The
    shuffles are applied on the device."""
    torch = torch_dev()
    cfg = "c2_512sq_k8_w128"
    c = synth.CONFIGS[cfg]
    w, fr, st = synth.config_inputs(cfg)
    g, L, s = dev(fr.gbuf), dev(fr.layers), dev(fr.scene)
    with GlassNet(w, 128, k_max=8, pool=c["pool"], precision=precision) as net:
        if precision == "fp8_t":
            calibrate(net, 128, 8)
        y0 = net.forward(g, L, s).clone()
        ymax = float(y0.abs().max())
        out = torch.empty_like(y0)
        worst, worst_rel = 0.0, 0.0
        y0n = float(torch.linalg.vector_norm(y0.double()))
        for _ in range(32):
            p = torch.from_numpy(synth.slot_shuffles(1, 8, fr.h, fr.w, 1, st["shuffles"])[0])
            p = p.to("cuda:0")[:, :, None].expand_as(L)
            net.forward(g, torch.gather(L, 1, p).contiguous(), s, out=out)
            d = (out - y0).double()
            worst = max(worst, float(d.abs().max()) / ymax)
            worst_rel = max(worst_rel, float(torch.linalg.vector_norm(d)) / y0n)
        torch.cuda.synchronize()
    log(f"  {precision} 512^2 K=8, 32 shuffles: worst relF {worst_rel:.3e}, "
        f"worst element {worst:.3e}")
    assert worst == 0.0 and worst_rel == 0.0


def test_fp8_calibration_sets_a_positive_scale_and_rejects_bad_scales():
    W = 128
    wts, fr = frame(1, 8, 8, 2, W, seed=3)
    with GlassNet(wts, W, k_max=8, precision="fp8_t") as net:
        calibrate(net, W, 2)
        net.set_act_scale(0.02)
        with pytest.raises(GlassNetError):
            net.set_act_scale(-1.0)
