"""Pins of the oracle's positional encoding (Sec. 3.4: every input of the
networks is positionally encoded; the frequency count is left open).

With L levels an input vector x becomes [x; sin(pi x); cos(pi x); ...;
sin(2^(L-1) pi x); cos(2^(L-1) pi x)] (blocks of the raw width), applied to
F's input [G; s] and to h's slot input b_i.  The pins tie the encoding to
trigonometric identities and exact values (not to its own formula), the
encoded network to its scalar brute-force twin, to the unencoded network (an
encoded network whose sin/cos columns are zero is the raw one), to the column
layout of the packed weights, and its gradient to finite differences.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.glassnet_oracle as go
from paper_2405_19056_amd import synth

from test_oracle_pins import rel


def tiny_pe(pe, n=1, h=3, w=2, k=3, W=8, seed=11, alpha_mode="p0.3"):
    s = synth.streams(seed)
    wts = synth.make_weights(W, s["weights"], pe_levels=pe)
    fr = synth.Frame(synth.make_gbuf(n, h, w, s["gbuf"]),
                     synth.make_layers(n, k, h, w, s["slots"], s["active"], alpha_mode),
                     synth.make_scene(n, s["gbuf"]))
    return wts, fr


# ------------------------------------------------------------- the encoding
def test_encoding_identities():
    """Raw block first; each level's (sin, cos) on the unit circle; each level
    the double angle of the one before (frequencies 2^k); period 2 in x."""
    x = np.random.default_rng(5).uniform(-3, 3, size=(7, 50))
    L = 5
    e = go.encode(x, L)
    assert e.shape == (7 * (1 + 2 * L), 50)
    assert np.array_equal(e[:7], x)
    sin = [e[7 * (1 + 2 * k):7 * (2 + 2 * k)] for k in range(L)]
    cos = [e[7 * (2 + 2 * k):7 * (3 + 2 * k)] for k in range(L)]
    for k in range(L):
        assert np.max(np.abs(sin[k] ** 2 + cos[k] ** 2 - 1.0)) <= 1e-14
    for k in range(L - 1):
        assert np.max(np.abs(sin[k + 1] - 2.0 * sin[k] * cos[k])) <= 1e-12
        assert np.max(np.abs(cos[k + 1] - (cos[k] ** 2 - sin[k] ** 2))) <= 1e-12
    assert np.max(np.abs(go.encode(x + 2.0, L)[7:] - e[7:])) <= 1e-12


def test_encoding_exact_values():
    """Level 0 is sin(pi x), cos(pi x): known values at 0, 1/2, 1/3, 1/6, 1."""
    x = np.array([[0.0, 0.5, 1.0 / 3.0, 1.0 / 6.0, 1.0]])
    e = go.encode(x, 2)
    s3 = math.sqrt(3.0) / 2.0
    want_sin0 = [0.0, 1.0, s3, 0.5, 0.0]
    want_cos0 = [1.0, 0.0, 0.5, s3, -1.0]
    want_sin1 = [0.0, 0.0, s3, s3, 0.0]          # sin(2 pi x)
    want_cos1 = [1.0, -1.0, -0.5, 0.5, 1.0]
    for row, want in zip(e[1:], (want_sin0, want_cos0, want_sin1, want_cos1)):
        assert np.max(np.abs(row - np.array(want))) <= 1e-15
    assert np.array_equal(go.encode(x, 0), x)


# -------------------------------------------------------- the encoded network
@pytest.mark.parametrize("pe", [1, 2])
@pytest.mark.parametrize("pool", ["mean", "sum"])
def test_encoded_vectorised_matches_bruteforce(pe, pool):
    wts, fr = tiny_pe(pe, n=2, h=2, w=2, k=3, W=8)
    y = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, pool=pool, pe_levels=pe)
    yb = oracle.forward_bruteforce(wts, 8, fr.gbuf, fr.layers, fr.scene, pool=pool,
                                   pe_levels=pe)
    assert rel(y, yb) <= 1e-12


def _widen(w_raw, W, pe):
    """Weights of the encoded network that ignore every sin/cos column: F1's
    and T1's raw columns (and T1's sigma columns) copied, the rest zero."""
    P = oracle.unpack(w_raw, W)
    Q = {net: [(A.copy(), c.copy()) for A, c in P[net]] for net in P}
    e = 1 + 2 * pe
    A, c = P["F"][0]
    AF = np.zeros((W, 30 * e))
    AF[:, :30] = A
    Q["F"][0] = (AF, c)
    A, c = P["T"][0]
    AT = np.zeros((W, 12 * e + W))
    AT[:, :12] = A[:, :12]
    AT[:, 12 * e:] = A[:, 12:]
    Q["T"][0] = (AT, c)
    w = oracle.pack(Q)
    assert w.size == oracle.n_params(W, pe) == synth.num_params(W, pe)
    return w


@pytest.mark.parametrize("pe", [1, 3])
def test_zero_encoding_columns_reduce_to_the_raw_network(pe):
    wts, fr = tiny_pe(0, n=1, h=3, w=3, k=3, W=8, alpha_mode="uniform_count")
    y0 = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene)
    y = oracle.forward(_widen(wts, 8, pe), 8, fr.gbuf, fr.layers, fr.scene, pe_levels=pe)
    assert rel(y, y0) <= 1e-14


def test_column_layout_of_the_encoded_inputs():
    """F1 reading one encoded column, F2 = F3 = identity: sigma_0 is the ReLU of
    that column's function of that channel (block order raw, sin 0, cos 0,
    sin 1, cos 1, ...; G channels before the scene within a block).  Likewise
    for T1's slot columns through h's first layer (via tau with one slot)."""
    W, pe = 8, 2
    rng = np.random.default_rng(9)
    gbuf = rng.uniform(-1, 1, size=(1, 14, 1, 1))
    scene = rng.uniform(-1, 1, size=(1, 16))
    layers = rng.uniform(0.1, 1, size=(1, 1, 12, 1, 1))       # alpha > 0: active
    x = np.concatenate([gbuf[0, :, 0, 0], scene[0]])
    b = layers[0, 0, :, 0, 0]
    funcs = [lambda v: v] + [f for k in range(pe) for f in
                             (lambda v, k=k: math.sin(math.pi * 2 ** k * v),
                              lambda v, k=k: math.cos(math.pi * 2 ** k * v))]
    base = oracle.unpack(np.zeros(oracle.n_params(W, pe)), W, pe)
    eye = (np.eye(W), np.zeros(W))
    for blk in range(1 + 2 * pe):
        for ch in (0, 13, 14, 29):
            P = {net: [(A.copy(), c.copy()) for A, c in base[net]] for net in base}
            AF = np.zeros((W, 30 * (1 + 2 * pe)))
            AF[0, 30 * blk + ch] = 1.0
            P["F"] = [(AF, np.zeros(W)), eye, eye]
            _, lat = oracle.forward(oracle.pack(P), W, gbuf, layers, scene, pool="sum",
                                    return_latents=True, pe_levels=pe)
            assert lat["sigma"][0, 0, 0, 0] == pytest.approx(max(funcs[blk](x[ch]), 0.0),
                                                             abs=1e-15)
        for ch in (0, 9, 11):
            P = {net: [(A.copy(), c.copy()) for A, c in base[net]] for net in base}
            AT = np.zeros((W, 12 * (1 + 2 * pe) + W))
            AT[0, 12 * blk + ch] = 1.0
            P["T"] = [(AT, np.zeros(W)), eye, eye]
            _, lat = oracle.forward(oracle.pack(P), W, gbuf, layers, scene, pool="sum",
                                    return_latents=True, pe_levels=pe)
            assert lat["tau"][0, 0, 0, 0] == pytest.approx(max(funcs[blk](b[ch]), 0.0),
                                                           abs=1e-15)


def test_mask_reads_the_raw_alpha():
    """Encoding does not change which slots are active: a slot with alpha = 0
    is still absent (its encoded alpha columns hold sin 0 = 0, cos 0 = 1)."""
    wts, fr = tiny_pe(2, n=1, h=3, w=3, k=3, W=8, alpha_mode="uniform_count")
    L = fr.layers.copy()
    L[:, 1, 9] = 0.0
    y = oracle.forward(wts, 8, fr.gbuf, L, fr.scene, pe_levels=2)
    y2 = oracle.forward(wts, 8, fr.gbuf, L[:, [0, 2]], fr.scene, pe_levels=2)
    assert rel(y, y2) <= 1e-14


def test_encoded_gradient_matches_central_differences():
    W, pe, eps = 8, 2, 1e-6
    wts, fr = tiny_pe(pe, n=1, h=3, w=3, k=3, W=W, seed=23, alpha_mode="uniform_count")
    rng = np.random.default_rng(23)
    target = rng.normal(size=(1, 3, 3, 3))
    w64 = wts.astype(np.float64)
    _, g = oracle.grad(w64, W, fr.gbuf, fr.layers, fr.scene, target, pe_levels=pe)
    P = oracle.unpack(np.arange(w64.size, dtype=np.float64), W, pe)
    f1 = P["F"][0][0].ravel().astype(int)
    t1 = P["T"][0][0].ravel().astype(int)
    coords = set(rng.choice(f1, 150, replace=False).tolist())
    coords |= set(rng.choice(t1, 150, replace=False).tolist())
    checked, worst = 0, 0.0
    for i in sorted(coords):
        wp, wm = w64.copy(), w64.copy()
        wp[i] += eps
        wm[i] -= eps
        sp = oracle.relu_signature(wp, W, fr.gbuf, fr.layers, fr.scene, target, pe_levels=pe)
        sm = oracle.relu_signature(wm, W, fr.gbuf, fr.layers, fr.scene, target, pe_levels=pe)
        if not np.array_equal(sp, sm):
            continue
        lp = oracle.l1_loss(oracle.forward(wp, W, fr.gbuf, fr.layers, fr.scene, pe_levels=pe),
                            target)[0]
        lm = oracle.l1_loss(oracle.forward(wm, W, fr.gbuf, fr.layers, fr.scene, pe_levels=pe),
                            target)[0]
        fd = (lp - lm) / (2 * eps)
        worst = max(worst, abs(fd - g[i]) / (1e-9 + 1e-6 * abs(g[i])))
        checked += 1
    assert checked >= 0.9 * len(coords)
    assert worst <= 1.0
