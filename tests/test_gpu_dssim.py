"""GPU DSSIM loss term (glassnet_dssim_loss; Sec. 3.5 trains with SSIM and
L1) against the FP64 oracle, through the C ABI.

Bars: the loss within 2e-6 absolute of the oracle's (it is a mean of fp32
window terms of magnitude <= 1); the gradient within relF 1e-4 (the local
variances are differences of fp32 moments).  Images span several 16 x 16
tiles with ragged edges; 11 x 11 is the one-window case.
"""
import numpy as np
import pytest

import oracle
from paper_2405_19056_amd import synth
from paper_2405_19056_amd.glassnet import GlassNet, GlassNetError, GN_E_INVAL

from gpu_util import dev, host, log, relF, torch_dev

pytestmark = pytest.mark.gpu


def images(n, h, w, seed, noise=0.1):
    rng = np.random.default_rng(seed)
    out = rng.uniform(0, 1, size=(n, 3, h, w)).astype(np.float32)
    tgt = np.clip(out + noise * rng.normal(size=out.shape), 0, 1).astype(np.float32)
    return out, tgt


def net64():
    return GlassNet(synth.make_weights(64, np.random.default_rng(0)), 64, precision="bf16")


@pytest.mark.parametrize("n,h,w", [(2, 37, 41), (1, 11, 11), (1, 11, 30), (3, 64, 17)])
def test_dssim_matches_oracle(n, h, w):
    torch = torch_dev()
    out, tgt = images(n, h, w, seed=h * w)
    ref_loss, ref_grad = oracle.dssim_loss(out, tgt)
    with net64() as net:
        g = torch.full((n, 3, h, w), float("nan"), device="cuda:0")
        loss = net.dssim_loss(dev(out), dev(tgt), grad_out=g)
        torch.cuda.synchronize()
        l, gg = float(loss.cpu()), host(g)
    log(f"dssim {n}x3x{h}x{w}: loss {l:.6f} vs {ref_loss:.6f}, grad relF {relF(gg, ref_grad):.2e}")
    assert abs(l - ref_loss) <= 2e-6
    assert relF(gg, ref_grad) <= 1e-4


def test_dssim_accumulates_onto_l1():
    torch = torch_dev()
    out, tgt = images(2, 40, 50, seed=5)
    _, dl1 = oracle.l1_loss(out, tgt)
    _, dds = oracle.dssim_loss(out, tgt)
    with net64() as net:
        g = torch.empty((2, 3, 40, 50), device="cuda:0")
        o, t = dev(out), dev(tgt)
        net.l1_loss(o, t, grad_out=g)
        net.dssim_loss(o, t, grad_out=g, accumulate=True)
        torch.cuda.synchronize()
        assert relF(host(g), dl1 + dds) <= 1e-5


def test_identical_images_have_zero_loss_and_gradient():
    torch = torch_dev()
    out, _ = images(1, 30, 33, seed=6)
    with net64() as net:
        g = torch.empty((1, 3, 30, 33), device="cuda:0")
        loss = net.dssim_loss(dev(out), dev(out), grad_out=g)
        torch.cuda.synchronize()
        assert abs(float(loss.cpu())) <= 1e-6
        assert float(np.max(np.abs(host(g)))) <= 1e-9


def test_training_batch_shape_sampled():
    """16 crops of 128^2 (the training workload's output): the loss against the
    oracle's, and the gradient on every pixel of two crops."""
    torch = torch_dev()
    out, tgt = images(16, 128, 128, seed=7, noise=0.05)
    with net64() as net:
        g = torch.empty((16, 3, 128, 128), device="cuda:0")
        loss = net.dssim_loss(dev(out), dev(tgt), grad_out=g)
        torch.cuda.synchronize()
        l, gg = float(loss.cpu()), host(g)
    ref_loss, _ = oracle.dssim_loss(out, tgt)
    assert abs(l - ref_loss) <= 2e-6
    # per-crop gradients scale with 1 / (number of crops): compare two crops
    _, ref2 = oracle.dssim_loss(out[[3, 11]], tgt[[3, 11]])
    assert relF(gg[[3, 11]] * 8.0, ref2) <= 1e-4


def test_dssim_rejects_small_images_and_aliasing():
    torch = torch_dev()
    with net64() as net:
        x = torch.zeros((1, 3, 10, 20), device="cuda:0")
        with pytest.raises(GlassNetError) as e:
            net.dssim_loss(x, x)
        assert e.value.status == GN_E_INVAL
        y = torch.zeros((1, 3, 12, 12), device="cuda:0")
        t = torch.zeros((1, 3, 12, 12), device="cuda:0")
        for kw in (dict(loss=y.view(-1)[5]), dict(grad_out=y), dict(grad_out=t)):
            with pytest.raises(GlassNetError) as e:
                net.dssim_loss(y, t, **kw)
            assert e.value.status == GN_E_INVAL
