"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in the oracle (on the CPU, by patching a private
function for the duration of the case) and runs the pin tests of
test_oracle_pins.py; at least one pin must fail.  This is evidence that the
pins tie the oracle to the paper rather than to itself.
"""
import contextlib

import numpy as np
import pytest

import oracle.glassnet_oracle as go
import test_oracle_pe as pe_pins
import test_oracle_pins as pins

PIN_TESTS = [
    lambda: pins.test_vectorised_matches_bruteforce("mean", 3),
    lambda: pins.test_affine_regime_equals_composed_matrix_products(),
    lambda: pins.test_hand_worked_width1_example(),
    lambda: pins.test_zero_weights_give_the_last_bias(),
    lambda: pins.test_alpha_zero_slot_equals_absent_slot("mean"),
    lambda: pins.test_one_active_slot_equals_k1_frame(),
    lambda: pins.test_empty_slot_set_gives_zero_tau(),
    lambda: pins.test_mean_sum_closed_forms(),
    lambda: pins.test_every_slot_order_gives_the_same_image("sum"),
    lambda: pins.test_frames_use_their_own_scene_vector(),
    lambda: pe_pins.test_encoding_identities(),
    lambda: pe_pins.test_encoding_exact_values(),
    lambda: pe_pins.test_encoded_vectorised_matches_bruteforce(2, "mean"),
    lambda: pe_pins.test_zero_encoding_columns_reduce_to_the_raw_network(1),
    lambda: pe_pins.test_column_layout_of_the_encoded_inputs(),
]


def _forward_cols_variant(P, G, L, S, W, pool, keep=False, pe=0, *, cat_h=None,
                          ld=slice(11, 14), active=lambda a: a > 0.0, sign=1.0,
                          mean_over_k=False, cat_b=None, use_scene=True, encode_slots=True):
    relu = go._relu
    x = go.encode(np.concatenate([G, S if use_scene else 0 * S], axis=0), pe)
    sigma = go._mlp(P["F"], x)
    Ssum = np.zeros_like(sigma)
    cnt = np.zeros(sigma.shape[1])
    for i in range(L.shape[0]):
        b = L[i]
        be = go.encode(b, pe) if encode_slots else np.concatenate([b] + [0 * b] * (2 * pe))
        inp = cat_h(be, sigma) if cat_h else np.concatenate([be, sigma], axis=0)
        h = go._mlp(P["T"], inp)
        m = active(b[9]).astype(np.float64)
        Ssum += sign * m[None, :] * h
        cnt += m
    if pool == "sum":
        tau = Ssum
    else:
        tau = Ssum / (max(L.shape[0], 1) if mean_over_k else np.maximum(cnt, 1.0)[None, :])
    binp = cat_b(sigma, tau) if cat_b else np.concatenate([sigma, tau], axis=0)
    phi = go._mlp(P["B"], binp)
    y = go._mlp(P["R"], np.concatenate([phi, G[ld]], axis=0))
    del relu
    if keep:
        return y, dict(sigma=sigma, tau=tau, phi=phi, count=cnt, S=Ssum)
    return y


def _mlp_no_bias2(layers, x):
    (A1, c1), (A2, c2), (A3, c3) = layers
    a = go._relu(A1 @ x + c1[:, None])
    a = go._relu(A2 @ a)
    return A3 @ a + c3[:, None]


def _mlp_relu_out(layers, x):
    return go._relu(_orig_mlp(layers, x))


_orig_mlp = go._mlp
_orig_unpack = go.unpack
_orig_fc = go._forward_cols
_orig_encode = go.encode


def _encode_variant(x, levels, *, freq=lambda k: np.pi * 2.0 ** k, cos_first=False):
    x = np.asarray(x, dtype=np.float64)
    blocks = [x]
    for k in range(levels):
        s, c = np.sin(freq(k) * x), np.cos(freq(k) * x)
        blocks += [c, s] if cos_first else [s, c]
    return np.concatenate(blocks, axis=0)


def enc(**kw):
    return lambda x, levels: _encode_variant(x, levels, **kw)


def _unpack_transposed(w, W, pe_levels=0):
    P = _orig_unpack(w, W, pe_levels)
    return {n: [(A.T if A.shape[0] == A.shape[1] else A, c) for A, c in layers]
            for n, layers in P.items()}


def fc(**kw):
    return lambda *a, **k: _forward_cols_variant(*a, **k, **kw)


MUTATIONS = {
    "transposed square weights": ("unpack", _unpack_transposed),
    "dropped hidden bias": ("_mlp", _mlp_no_bias2),
    "ReLU on every output layer": ("_mlp", _mlp_relu_out),
    "h input [sigma; b] instead of [b; sigma]": (
        "_forward_cols", fc(cat_h=lambda b, s: np.concatenate([s, b], axis=0))),
    "L_d taken from planes 8..10": ("_forward_cols", fc(ld=slice(8, 11))),
    "mean over all K slots": ("_forward_cols", fc(mean_over_k=True)),
    "inactive slots included (alpha >= 0)": ("_forward_cols", fc(active=lambda a: a >= 0.0)),
    "pool subtracts h": ("_forward_cols", fc(sign=-1.0)),
    "B input [tau; sigma]": ("_forward_cols", fc(cat_b=lambda s, t: np.concatenate([t, s], axis=0))),
    "scene vector ignored": ("_forward_cols", fc(use_scene=False)),
    "encoding frequencies 2^k instead of pi 2^k": ("encode", enc(freq=lambda k: 2.0 ** k)),
    "encoding frequencies pi (k + 1)": ("encode", enc(freq=lambda k: np.pi * (k + 1))),
    "encoding frequencies 2 pi 2^k": ("encode", enc(freq=lambda k: 2 * np.pi * 2.0 ** k)),
    "cos block before sin block": ("encode", enc(cos_first=True)),
    "slot input left unencoded": ("_forward_cols", fc(encode_slots=False)),
}


@contextlib.contextmanager
def planted(name):
    attr, fn = MUTATIONS[name]
    old = getattr(go, attr)
    setattr(go, attr, fn)
    try:
        yield
    finally:
        setattr(go, attr, old)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_some_pin_catches_the_planted_mistake(name):
    caught = []
    with planted(name):
        for t in PIN_TESTS:
            try:
                t()
            except (AssertionError, ValueError):
                caught.append(t)
    assert caught, f"no pin caught: {name}"


def test_pins_pass_without_mistakes():
    for t in PIN_TESTS:
        t()


# ---------------------------------------------------------------- gradient
GRAD_PIN_TESTS = [
    lambda: pins.test_grad_from_dy_equals_l1_gradient_at_its_seed(),
    lambda: pins.test_grad_from_dy_matches_central_differences("mean"),
    lambda: pins.test_gradient_matches_central_differences("sum"),
]


def _mlp_bwd_variant(layers, cache, dout, grads, *, mask2=True, bias1_from=None):
    (A1, _), (A2, _), (A3, _) = layers
    x, z1, a1, z2, a2 = cache
    grads[2][0] += dout @ a2.T
    grads[2][1] += dout.sum(axis=1)
    d = (A3.T @ dout) * ((z2 > 0.0) if mask2 else 1.0)
    grads[1][0] += d @ a1.T
    grads[1][1] += d.sum(axis=1)
    d2 = d
    d = (A2.T @ d) * (z1 > 0.0)
    grads[0][0] += d @ x.T
    grads[0][1] += (d2 if bias1_from == "layer2" else d).sum(axis=1)
    return A1.T @ d


def _backprop_dy(transform):
    old = go._backprop

    def f(*a, dy=None, **k):
        return old(*a, dy=None if dy is None else transform(np.asarray(dy)), **k)
    return f


GRAD_MUTATIONS = {
    "ReLU mask of the second hidden layer dropped": (
        "_mlp_bwd", lambda *a: _mlp_bwd_variant(*a, mask2=False)),
    "first bias gradient from the second layer's delta": (
        "_mlp_bwd", lambda *a: _mlp_bwd_variant(*a, bias1_from="layer2")),
    "dy with its sign flipped": ("_backprop", _backprop_dy(lambda d: -d)),
    "dy channels reversed": ("_backprop", _backprop_dy(lambda d: d[:, ::-1])),
    "dy image transposed": ("_backprop", _backprop_dy(lambda d: np.swapaxes(d, 2, 3)
                                                      .reshape(d.shape))),
}


@pytest.mark.parametrize("name", sorted(GRAD_MUTATIONS))
def test_some_gradient_pin_catches_the_planted_mistake(name):
    attr, fn = GRAD_MUTATIONS[name]
    old = getattr(go, attr)
    setattr(go, attr, fn)
    caught = []
    try:
        for t in GRAD_PIN_TESTS:
            try:
                t()
            except (AssertionError, ValueError):
                caught.append(t)
    finally:
        setattr(go, attr, old)
    assert caught, f"no gradient pin caught: {name}"


def test_gradient_pins_pass_without_mistakes():
    for t in GRAD_PIN_TESTS:
        t()
