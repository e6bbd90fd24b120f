"""GPU optimiser step (glassnet_adam_step, Sec. 4: Adam with weight decay)
against the FP64 oracle's step, through the C ABI.

The update runs in fp32 on the handle's master weights; after three steps the
weights and both moment vectors agree with the oracle's to fp32 rounding
(max |error| <= 1e-6 on weights of magnitude <= 1, relF <= 1e-5 on the moments;
the hyperparameters are the fp32 values that cross the ABI, on both sides).
The packed forms are re-derived: the stepped handle's forward equals that of a
fresh handle made from its weights, bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2405_19056_amd import synth
from paper_2405_19056_amd.glassnet import GlassNet, GlassNetError, GN_E_INVAL

from gpu_util import dev, host, log, relF, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,W,pe", [("bf16", 128, 0), ("fp32", 64, 2), ("fp8_t", 128, 0)])
def test_adam_steps_match_oracle_and_repack(precision, W, pe):
    torch = torch_dev()
    s = synth.streams(31)
    w0 = synth.make_weights(W, s["weights"], pe_levels=pe)
    n = w0.size
    rng = np.random.default_rng(31)
    # the hyperparameters cross the ABI as fp32: both sides use those values
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    lr, betas, eps, wd = f32(1e-3), (f32(0.9), f32(0.999)), f32(1e-8), f32(1e-4)
    fr = synth.make_frame(1, 21, 23, 3, seed=32)
    with GlassNet(w0, W, k_max=4, precision=precision, pe_levels=pe) as net:
        if precision == "fp8_t":
            net.calibrate(dev(fr.gbuf), dev(fr.layers), dev(fr.scene))
        state = net.adam_state()
        w, m, v = w0.astype(np.float64), np.zeros(n), np.zeros(n)
        for t in range(1, 4):
            g = (rng.normal(size=n) * 10.0 ** rng.uniform(-4, 0, size=n)).astype(np.float32)
            net.adam_step(dev(g), state, t, lr=lr, betas=betas, eps=eps, weight_decay=wd)
            w, m, v = oracle.adam_step(w, g, m, v, t, lr=lr, beta1=betas[0], beta2=betas[1],
                                       eps=eps, weight_decay=wd)
        torch.cuda.synchronize()
        wg = net.get_weights()
        st = host(state)
        err = float(np.max(np.abs(wg - w)))
        log(f"adam {precision} W={W} L={pe}: max |w - w_ref| {err:.2e}, "
            f"moments relF {relF(st[:n], m):.2e} {relF(st[n:], v):.2e}")
        assert err <= 1e-6
        assert relF(st[:n], m) <= 1e-5 and relF(st[n:], v) <= 1e-5
        if precision == "fp8_t":
            # the step keeps the activation scale; recalibrate as the fresh handle does
            net.calibrate(dev(fr.gbuf), dev(fr.layers), dev(fr.scene))
        y = net.forward(dev(fr.gbuf), dev(fr.layers), dev(fr.scene))
        torch.cuda.synchronize()
        y = host(y)
    with GlassNet(wg, W, k_max=4, precision=precision, pe_levels=pe) as fresh:
        if precision == "fp8_t":
            fresh.calibrate(dev(fr.gbuf), dev(fr.layers), dev(fr.scene))
        y2 = host(fresh.forward(dev(fr.gbuf), dev(fr.layers), dev(fr.scene)))
        torch.cuda.synchronize()
    assert np.array_equal(y, y2)


def test_adam_argument_errors():
    torch = torch_dev()
    W = 64
    w0 = synth.make_weights(W, np.random.default_rng(0))
    with GlassNet(w0, W, precision="bf16") as net:
        state = net.adam_state()
        g = torch.zeros(net.nparams, device="cuda:0")
        for kw in (dict(step=0), dict(step=1, lr=-1.0), dict(step=1, betas=(1.0, 0.999)),
                   dict(step=1, eps=0.0), dict(step=1, weight_decay=-0.1)):
            step = kw.pop("step")
            with pytest.raises(GlassNetError) as e:
                net.adam_step(g, state, step, **kw)
            assert e.value.status == GN_E_INVAL
        with pytest.raises(GlassNetError) as e:          # gradient inside the state
            net.adam_step(state[: net.nparams], state, 1)
        assert e.value.status == GN_E_INVAL
        torch.cuda.synchronize()
        assert np.array_equal(net.get_weights(), w0)      # nothing ran
