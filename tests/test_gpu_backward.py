"""GPU backward (dL/dw) against the FP64 oracle's hand-written backprop.

The backward runs in fp32 for every handle precision, so the bar is the fp32
one: relative Frobenius error <= 1e-4 per weight/bias tensor.  The oracle's
own gradient is pinned to central finite differences in the CPU suite.

A pixel with a ReLU input within fp32 rounding of the kink may take the other
(equally valid) branch of ReLU' in fp32 than in fp64, which changes that
pixel's whole contribution; dL/dy is therefore zero on pixels closer than
KINK to a kink (both sides use the same dL/dy).
"""
import numpy as np
import pytest

import oracle
from paper_2405_19056_amd import synth
from paper_2405_19056_amd.glassnet import GlassNet

from gpu_util import dev, host, kink_free, log, relF, torch_dev

pytestmark = pytest.mark.gpu

TOL = 1e-4


def tensors(W):
    """(name, start, stop) of every matrix and bias in the flat layout."""
    shapes = synth.layer_shapes(W)
    names = [f"{n}{j}" for n in "FTBR" for j in (1, 2, 3)]
    out, off = [], 0
    for nm, (o, i) in zip(names, shapes):
        out.append((nm + ".w", off, off + o * i))
        off += o * i
        out.append((nm + ".b", off, off + o))
        off += o
    return out


def check(g, ref, W, tol=TOL):
    worst = 0.0
    for nm, a, b in tensors(W):
        if np.linalg.norm(ref[a:b]) == 0.0:
            assert np.all(g[a:b] == 0.0), nm
            continue
        e = relF(g[a:b], ref[a:b])
        worst = max(worst, e)
        assert e <= tol, (nm, e)
    return worst


def frame(n, h, w, k, W, seed):
    s = synth.streams(seed)
    wts = synth.make_weights(W, s["weights"])
    fr = synth.Frame(synth.make_gbuf(n, h, w, s["gbuf"]),
                     synth.make_layers(n, k, h, w, s["slots"], s["active"]),
                     synth.make_scene(n, s["gbuf"]))
    return wts, fr, s


def redraw_near_kinks(wts, W, fr, pool, s):
    """Redraw the inputs of pixels with a ReLU input near its kink (see the
    module docstring) until none is left; other pixels keep their inputs."""
    g, L = fr.gbuf.copy(), fr.layers.copy()
    for _ in range(50):
        bad = ~kink_free(wts, W, synth.Frame(g, L, fr.scene), pool)
        if not bad.any():
            return synth.Frame(g, L, fr.scene)
        n, k, h, w = fr.n, fr.k, fr.h, fr.w
        g2 = synth.make_gbuf(n, h, w, s["gbuf"])
        L2 = synth.make_layers(n, k, h, w, s["slots"], s["active"])
        np.moveaxis(g, 1, 3)[bad] = np.moveaxis(g2, 1, 3)[bad]
        np.moveaxis(L, (1, 2), (3, 4))[bad] = np.moveaxis(L2, (1, 2), (3, 4))[bad]
    raise AssertionError("could not move every pixel away from the kinks")


def gpu_grad(net, fr, dy):
    torch = torch_dev()
    L = dev(fr.layers) if fr.k > 0 else None
    g = net.backward(dev(fr.gbuf), L, dev(fr.scene), dev(dy))
    torch.cuda.synchronize()
    return host(g)


@pytest.mark.parametrize("W", [64, 128])
@pytest.mark.parametrize("pool", ["mean", "sum"])
@pytest.mark.parametrize("k", [0, 3])
def test_backward_matches_oracle(W, pool, k):
    wts, fr, s = frame(2, 19, 23, k, W, seed=40 + k)
    dy = s["noise"].normal(size=(2, 3, 19, 23)).astype(np.float32)
    ok = kink_free(wts, W, fr, pool)
    dy *= ok[:, None]
    log(f"backward W={W} {pool} k={k}: {int((~ok).sum())} of {ok.size} pixels near a kink")
    ref = oracle.grad_from_dy(wts, W, fr.gbuf, fr.layers, fr.scene, dy, pool=pool)
    with GlassNet(wts, W, k_max=8, pool=pool, precision="fp32") as net:
        g = gpu_grad(net, fr, dy)
    worst = check(g, ref, W)
    log(f"  worst per-tensor relF {worst:.3e}, whole {relF(g, ref):.3e}")


def test_backward_rejects_more_pixels_than_it_addresses():
    """One call covers at most 3 * 2^20 pixels; beyond that it is an argument
    error raised before any launch (buffers are real, so nothing could fault)."""
    torch = torch_dev()
    from paper_2405_19056_amd.glassnet import GlassNetError
    W, n, h, w = 64, 1, 1025, 3072
    wts = synth.make_weights(W, np.random.default_rng(0))
    g = torch.zeros((n, 14, h, w), device="cuda:0")
    sc = torch.zeros((n, 16), device="cuda:0")
    dy = torch.zeros((n, 3, h, w), device="cuda:0")
    with GlassNet(wts, W, k_max=2, precision="fp32") as net:
        with pytest.raises(GlassNetError):
            net.backward(g, None, sc, dy)
    del g, dy
    torch.cuda.empty_cache()


def test_backward_is_deterministic_and_precision_independent():
    W = 128
    wts, fr, s = frame(1, 32, 40, 4, W, seed=3)
    dy = s["noise"].normal(size=(1, 3, 32, 40)).astype(np.float32)
    with GlassNet(wts, W, k_max=8, precision="fp32") as n32, \
            GlassNet(wts, W, k_max=8, precision="bf16") as n16:
        a = gpu_grad(n32, fr, dy)
        b = gpu_grad(n32, fr, dy)
        c = gpu_grad(n16, fr, dy)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)


def test_training_workload_with_sparse_seed():
    """16 crops of 128^2, K=4, W=128.  dL/dy is non-zero on 2048 sampled pixels
    only, so dL/dw depends on those pixels alone and the oracle evaluates
    them one by one."""
    c = synth.CONFIGS["c3_train_16x128sq_k4_w128"]
    w, fr, s = synth.config_inputs("c3_train_16x128sq_k4_w128")
    n, h, wd, W = fr.n, fr.h, fr.w, c["width"]
    rng = np.random.default_rng(8)
    cand = rng.choice(n * h * wd, size=3072, replace=False)
    flat = np.sort(cand[kink_free(w, W, fr, c["pool"], cand)][:2048])
    assert len(flat) == 2048
    dy = np.zeros((n, 3, h * wd), np.float32)
    vals = rng.normal(size=(len(flat), 3)).astype(np.float32)
    dy[flat // (h * wd), :, flat % (h * wd)] = vals
    dy = dy.reshape(n, 3, h, wd)
    ref = np.zeros(synth.num_params(W))
    for f in np.unique(flat // (h * wd)):
        sel = flat[flat // (h * wd) == f] % (h * wd)
        g = fr.gbuf[f].reshape(14, -1)[:, sel][None, :, None, :]
        L = fr.layers[f].reshape(fr.k, 12, -1)[:, :, sel][None, :, :, None, :]
        d = dy[f].reshape(3, -1)[:, sel][None, :, None, :]
        ref += oracle.grad_from_dy(w, W, g, L, fr.scene[f:f + 1], d, pool=c["pool"])
    with GlassNet(w, W, k_max=c["k"], pool=c["pool"], precision="bf16") as net:
        gg = gpu_grad(net, fr, dy)
    worst = check(gg, ref, W)
    log(f"  training workload worst per-tensor relF {worst:.3e}")


def test_l1_gradient_matches_central_differences_on_an_8x8_crop():
    """The training workload's gradient check: dL/dw of the L1 loss on an 8x8
    crop, K=4, W=128, from the library (forward, L1 kernel, fp32 backward),
    against FP64 central differences of the oracle's loss (h = 1e-6) on 160
    coordinates whose +-h perturbation leaves every branch (ReLU sign, L1
    sign) unchanged.  Targets sit 0.5 from the output, so the L1 sign is the
    same in fp32 and fp64; pixels near a ReLU kink are redrawn."""
    torch = torch_dev()
    W = 128
    wts, fr, s = frame(1, 8, 8, 4, W, seed=90)
    fr = redraw_near_kinks(wts, W, fr, "mean", s)
    rng = np.random.default_rng(90)
    y = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
    target = y + rng.choice([-0.5, 0.5], size=y.shape)
    with GlassNet(wts, W, k_max=8, precision="fp32") as net:
        gd, Ld, sd = dev(fr.gbuf), dev(fr.layers), dev(fr.scene)
        yy = net.forward(gd, Ld, sd)
        dy = torch.empty_like(yy)
        net.l1_loss(yy, dev(target), grad_out=dy)
        g = host(net.backward(gd, Ld, sd, dy)).astype(np.float64)
        torch.cuda.synchronize()
    w64 = wts.astype(np.float64)
    eps, fds = 1e-6, []
    for i in rng.choice(w64.size, size=160, replace=False):
        wp, wm = w64.copy(), w64.copy()
        wp[i] += eps
        wm[i] -= eps
        if not np.array_equal(oracle.relu_signature(wp, W, fr.gbuf, fr.layers, fr.scene, target),
                              oracle.relu_signature(wm, W, fr.gbuf, fr.layers, fr.scene, target)):
            continue
        lp = oracle.l1_loss(oracle.forward(wp, W, fr.gbuf, fr.layers, fr.scene), target)[0]
        lm = oracle.l1_loss(oracle.forward(wm, W, fr.gbuf, fr.layers, fr.scene), target)[0]
        fds.append((i, (lp - lm) / (2 * eps)))
    assert len(fds) >= 144
    scale = max(abs(f) for _, f in fds)
    # fp32 backward: ~1e-6 relative per coordinate; the loss's fp64 rounding
    # over 2h contributes ~1e-10 absolute
    worst = max(abs(g[i] - f) / (1e-4 * abs(f) + 1e-6 * scale) for i, f in fds)
    log(f"  8x8 crop: {len(fds)} coordinates, worst |g - fd| / bound {worst:.3f}")
    assert worst <= 1.0


def test_l1_loss_kernel():
    torch = torch_dev()
    rng = np.random.default_rng(0)
    y = rng.normal(size=(3, 3, 37, 41)).astype(np.float32)
    t = rng.normal(size=y.shape).astype(np.float32)
    t.ravel()[:50] = y.ravel()[:50]                 # ties: subgradient 0
    wts = synth.make_weights(64, rng)
    with GlassNet(wts, 64, k_max=2) as net:
        grad = torch.empty(y.shape, dtype=torch.float32, device="cuda:0")
        loss = net.l1_loss(dev(y), dev(t), grad_out=grad)
        torch.cuda.synchronize()
        ref_loss, ref_grad = oracle.l1_loss(y, t)
        assert abs(float(host(loss)) - ref_loss) <= 1e-5 * ref_loss
        assert np.array_equal(np.sign(host(grad)), np.sign(ref_grad))
        assert np.allclose(host(grad), ref_grad, rtol=1e-6, atol=0)


def test_autograd_training_step_matches_oracle_l1_gradient():
    torch = torch_dev()
    from paper_2405_19056_amd.autograd import GlassNetFunction, L1Function, train_step
    W = 64
    wts, fr, s = frame(2, 16, 16, 4, W, seed=77)
    fr = redraw_near_kinks(wts, W, fr, "mean", s)
    teacher = synth.make_weights(W, s["teacher"])
    target = (oracle.forward(teacher, W, fr.gbuf, fr.layers, fr.scene)
              + 0.01 * s["noise"].normal(size=(2, 3, 16, 16))).astype(np.float32)
    ref_loss, ref = oracle.grad(wts, W, fr.gbuf, fr.layers, fr.scene, target)
    with GlassNet(wts, W, k_max=8, precision="fp32") as net:
        w = torch.tensor(wts, device="cuda:0", requires_grad=True)
        g, L, sc, t = dev(fr.gbuf), dev(fr.layers), dev(fr.scene), dev(target)
        y = GlassNetFunction.apply(net, g, L, sc, w)
        loss = L1Function.apply(net, y, t)
        loss.backward()
        torch.cuda.synchronize()
        assert abs(float(loss.detach().cpu()) - ref_loss) <= 1e-5 * ref_loss
        check(host(w.grad), ref, W)
        loss2, gw = train_step(net, g, L, sc, t, w.detach())
        torch.cuda.synchronize()
        assert np.array_equal(host(gw), host(w.grad))


def test_l1_gradient_scaled_by_a_device_scalar():
    """grad_scale (a device scalar) multiplies the subgradient on the device:
    sign(y - t) * (1 / n) * s in fp32, element for element."""
    torch = torch_dev()
    rng = np.random.default_rng(1)
    y = rng.normal(size=(2, 3, 19, 23)).astype(np.float32)
    t = rng.normal(size=y.shape).astype(np.float32)
    t.ravel()[:7] = y.ravel()[:7]
    with GlassNet(synth.make_weights(64, rng), 64, k_max=2) as net:
        grad = torch.empty(y.shape, dtype=torch.float32, device="cuda:0")
        s = torch.tensor(-2.75, dtype=torch.float32, device="cuda:0")
        net.l1_loss(dev(y), dev(t), grad_out=grad, grad_scale=s)
        torch.cuda.synchronize()
    want = np.sign(y - t).astype(np.float32) * (np.float32(1.0 / y.size) * np.float32(-2.75))
    assert np.array_equal(host(grad), want)


def test_autograd_scaled_loss_and_weights_changed_before_backward():
    """(a) A non-unit upstream gradient, 2.5 L, gives 2.5 times the oracle's
    gradient.  (b) Two forwards on one handle with different weights (a
    teacher, then a student) before the backward: each gradient is taken at
    the weights of its own forward."""
    torch = torch_dev()
    from paper_2405_19056_amd.autograd import GlassNetFunction, L1Function
    W = 64
    wts, fr, s = frame(1, 16, 16, 3, W, seed=78)
    fr = redraw_near_kinks(wts, W, fr, "mean", s)
    target = s["noise"].normal(size=(1, 3, 16, 16)).astype(np.float32)
    _, ref = oracle.grad(wts, W, fr.gbuf, fr.layers, fr.scene, target)
    other = synth.make_weights(W, s["teacher"])
    with GlassNet(wts, W, k_max=8, precision="fp32") as net:
        g, L, sc, t = dev(fr.gbuf), dev(fr.layers), dev(fr.scene), dev(target)
        w = torch.tensor(wts, device="cuda:0", requires_grad=True)
        w2 = torch.tensor(other, device="cuda:0", requires_grad=True)
        y = GlassNetFunction.apply(net, g, L, sc, w)
        y2 = GlassNetFunction.apply(net, g, L, sc, w2)     # the handle now holds w2
        loss = 2.5 * L1Function.apply(net, y, t) + 0.0 * y2.sum()
        loss.backward()
        torch.cuda.synchronize()
    check(host(w.grad) / 2.5, ref, W)
