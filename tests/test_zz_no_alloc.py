"""The allocation-free DSSIM entry point (glassnet_dssim_loss_noalloc),
through the C ABI: its loss and gradient equal glassnet_dssim_loss's, bit for
bit (same kernels, a fixed device workspace instead of the handle's), on two
calls in a row, the second on a smaller input; sizes beyond its workspace
are rejected before any launch."""
import numpy as np
import pytest

from paper_2405_19056_amd import synth
from paper_2405_19056_amd.glassnet import GN_E_INVAL, GlassNet, GlassNetError

from gpu_util import dev, host, log, torch_dev

pytestmark = pytest.mark.gpu


def _pair(net, out, tgt, accumulate, seed):
    torch = torch_dev()
    rng = np.random.default_rng(seed)
    g0 = rng.normal(size=out.shape).astype(np.float32)
    res = []
    for noalloc in (False, True):
        loss = torch.full((), float("nan"), device="cuda:0")
        grad = dev(g0)
        net.dssim_loss(out, tgt, loss=loss, grad_out=grad, accumulate=accumulate,
                       noalloc=noalloc)
        torch.cuda.synchronize()
        res.append((host(loss), host(grad)))
    return res


def test_noalloc_dssim_equals_the_allocating_entry_point():
    torch = torch_dev()
    rng = np.random.default_rng(3)
    with GlassNet(synth.make_weights(64, rng), 64, k_max=2) as net:
        # the training batch's shape, then a smaller one: the fixed workspace
        # keeps the first call's contents, which the second must not read
        for i, (n, h, w, acc) in enumerate([(16, 128, 128, True), (2, 37, 53, False)]):
            o = dev(rng.uniform(0, 2, size=(n, 3, h, w)).astype(np.float32))
            t = dev(rng.uniform(0, 2, size=(n, 3, h, w)).astype(np.float32))
            (la, ga), (lb, gb) = _pair(net, o, t, acc, seed=10 + i)
            log(f"  dssim noalloc {n}x3x{h}x{w}: loss {float(lb):.6f}")
            assert np.isfinite(la) and np.array_equal(la, lb)
            assert np.array_equal(ga, gb)
        # a size whose workspace exceeds the fixed array: rejected
        big = torch.zeros((1, 3, 1024, 1024), device="cuda:0")
        with pytest.raises(GlassNetError) as e:
            net.dssim_loss(big, big, grad_out=torch.empty_like(big), noalloc=True)
        assert e.value.status == GN_E_INVAL
