"""Pins of the oracle's optimiser step (Sec. 4: the networks are trained with
Adam and weight decay; Kingma & Ba's algorithm).

The pins are closed forms derived by hand from the algorithm (the first step,
and any number of steps under a constant gradient, where the bias corrections
make both moment estimates exact) and a library implementation of the same
algorithm (torch.optim.Adam on the CPU in float64, whose weight_decay is the
same L2 term added to the gradient).  Planted mistakes in the oracle's step
(no bias correction, decoupled decay, eps under the square root) each fail
one of them.
"""
import contextlib

import numpy as np
import pytest

import oracle.glassnet_oracle as go


def test_first_step_closed_form():
    """m_hat = g', v_hat = g'^2 at t = 1: the step is lr g' / (|g'| + eps)."""
    rng = np.random.default_rng(1)
    w, g = rng.normal(size=50), rng.normal(size=50)
    lr, eps, wd = 1e-3, 1e-8, 0.01
    w1, m1, v1 = go.adam_step(w, g, np.zeros(50), np.zeros(50), 1, lr=lr, eps=eps,
                              weight_decay=wd)
    gp = g + wd * w
    assert np.allclose(w1, w - lr * gp / (np.abs(gp) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * gp, rtol=1e-15, atol=0)
    assert np.allclose(v1, 0.001 * gp * gp, rtol=1e-12, atol=0)


def test_constant_gradient_moves_linearly():
    """With a constant gradient and no decay, the corrected moments equal g and
    g^2 at every step, so each step moves by lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    w0, g = rng.normal(size=20), rng.normal(size=20)
    w, m, v = w0.copy(), np.zeros(20), np.zeros(20)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 8):
        w, m, v = go.adam_step(w, g, m, v, t, lr=lr, eps=eps)
        assert np.allclose(w, w0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)


def test_matches_torch_adam():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    n, lr, betas, eps, wd = 64, 3e-3, (0.8, 0.99), 1e-6, 0.05
    w0 = rng.normal(size=n)
    p = torch.nn.Parameter(torch.tensor(w0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=lr, betas=betas, eps=eps, weight_decay=wd)
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.normal(size=n)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        w, m, v = go.adam_step(w, g, m, v, t, lr=lr, beta1=betas[0], beta2=betas[1], eps=eps,
                               weight_decay=wd)
        assert np.max(np.abs(w - p.detach().numpy())) <= 1e-14


def test_zero_gradient_without_decay_is_a_fixed_point():
    w = np.linspace(-1, 1, 9)
    w1, m1, v1 = go.adam_step(w, np.zeros(9), np.zeros(9), np.zeros(9), 1)
    assert np.array_equal(w1, w) and not m1.any() and not v1.any()


# ---------------------------------------------------------------- mutations
_orig = go.adam_step


def _no_bias_correction(w, g, m, v, t, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8,
                        weight_decay=0.0):
    g = np.asarray(g, float) + weight_decay * np.asarray(w, float)
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    return w - lr * m / (np.sqrt(v) + eps), m, v


def _decoupled_decay(w, g, m, v, t, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8,
                     weight_decay=0.0):
    w1, m1, v1 = _orig(w, g, m, v, t, lr, beta1, beta2, eps, 0.0)
    return w1 - lr * weight_decay * np.asarray(w, float), m1, v1


def _eps_inside(w, g, m, v, t, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    g = np.asarray(g, float) + weight_decay * np.asarray(w, float)
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    return w - lr * (m / (1 - beta1 ** t)) / np.sqrt(v / (1 - beta2 ** t) + eps), m, v


@contextlib.contextmanager
def planted(fn):
    go.adam_step = fn
    try:
        yield
    finally:
        go.adam_step = _orig


@pytest.mark.parametrize("fn", [_no_bias_correction, _decoupled_decay, _eps_inside])
def test_pins_catch_planted_mistakes(fn):
    caught = 0
    with planted(fn):
        for t in (test_first_step_closed_form, test_constant_gradient_moves_linearly,
                  test_matches_torch_adam):
            try:
                t()
            except AssertionError:
                caught += 1
    assert caught > 0
