"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties the oracle to something other than itself: a scalar brute-force
twin, invariants of Eq. (5), special cases with closed forms (derived by hand or
reducing to plain matrix products), finite differences for the gradient and the
paper's printed order-inversion table.  A plausible slip in the oracle (dropped
term, wrong sign or index, transposed operand, misplaced ReLU) fails one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2405_19056_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(n=1, h=3, w=2, k=3, W=8, seed=11, alpha_mode="p0.3"):
    s = synth.streams(seed)
    wts = synth.make_weights(W, s["weights"])
    fr = synth.Frame(synth.make_gbuf(n, h, w, s["gbuf"]),
                     synth.make_layers(n, k, h, w, s["slots"], s["active"], alpha_mode),
                     synth.make_scene(n, s["gbuf"]))
    return wts, fr


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("pool", ["mean", "sum"])
@pytest.mark.parametrize("k", [0, 1, 3])
def test_vectorised_matches_bruteforce(pool, k):
    wts, fr = tiny(n=2, h=3, w=2, k=k, W=8)
    y = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, pool=pool)
    yb = oracle.forward_bruteforce(wts, 8, fr.gbuf, fr.layers, fr.scene, pool=pool)
    assert y.shape == (2, 3, 3, 2)
    assert rel(y, yb) <= 1e-12


def test_chunking_is_transparent():
    wts, fr = tiny(n=1, h=5, w=7, k=2, W=8)
    a = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, chunk=3)
    b = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, chunk=1 << 20)
    assert rel(a, b) <= 1e-14   # BLAS may block differently per chunk width


# --------------------------------------------------------- Eq. (5) invariants
@pytest.mark.parametrize("pool", ["mean", "sum"])
def test_every_slot_order_gives_the_same_image(pool):
    wts, fr = tiny(n=1, h=4, w=3, k=4, W=8, alpha_mode="uniform_count")
    y0 = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, pool=pool)
    for order in oracle.all_slot_orders(4):
        y = oracle.forward(wts, 8, fr.gbuf, fr.layers[:, list(order)], fr.scene, pool=pool)
        assert rel(y, y0) <= 1e-14


def test_per_pixel_shuffles_give_the_same_image():
    wts, fr = tiny(n=2, h=4, w=4, k=5, W=8, alpha_mode="uniform_count")
    y0 = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene)
    perms = synth.slot_shuffles(2, 5, 4, 4, 8, np.random.default_rng(5))
    for p in perms:
        y = oracle.forward(wts, 8, fr.gbuf, synth.apply_slot_permutation(fr.layers, p), fr.scene)
        assert rel(y, y0) <= 1e-14


def test_alpha_blending_is_order_dependent_negative_control():
    # Eqs. (3)-(4) by hand: front (C=1, a=0.5) over back (C=0, a=0.5) gives 0.5;
    # the reversed stack gives 0 + 0.5 * 0.5 * 1 = 0.25.
    c = np.array([[1.0], [0.0]])
    a = np.array([[0.5], [0.5]])
    assert oracle.alpha_blend(c, a)[0] == pytest.approx(0.5)
    assert oracle.alpha_blend(c[::-1], a[::-1])[0] == pytest.approx(0.25)
    # A random stack changes under permutation: the comparison used for the
    # network would have flagged an order-dependent blend.
    rng = np.random.default_rng(0)
    col = rng.uniform(size=(4, 3, 10))
    alp = rng.uniform(0.1, 0.9, size=(4, 10))
    base = oracle.alpha_blend(col, alp)
    worst = max(rel(oracle.alpha_blend(col[list(o)], alp[list(o)]), base)
                for o in itertools.permutations(range(4)))
    assert worst > 1e-2


@pytest.mark.parametrize("pool", ["mean", "sum"])
def test_alpha_zero_slot_equals_absent_slot(pool):
    wts, fr = tiny(n=1, h=3, w=4, k=4, W=8, alpha_mode="uniform_count")
    y = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, pool=pool)
    for r in range(3):
        for c in range(4):
            keep = [i for i in range(4) if fr.layers[0, i, 9, r, c] > 0.0]
            g = fr.gbuf[:, :, r:r + 1, c:c + 1]
            L = fr.layers[:, keep, :, r:r + 1, c:c + 1]
            yp = oracle.forward(wts, 8, g, L, fr.scene, pool=pool)
            assert rel(yp[0, :, 0, 0], y[0, :, r, c]) <= 1e-13


def test_one_active_slot_equals_k1_frame():
    wts, fr = tiny(n=1, h=4, w=4, k=8, W=8, alpha_mode="uniform_count")
    rng = np.random.default_rng(3)
    L = fr.layers.copy()
    L[:, :, 9] = 0.0
    pos = rng.integers(0, 8, size=(4, 4))
    single = np.empty((1, 1, 12, 4, 4), dtype=np.float32)
    for r in range(4):
        for c in range(4):
            L[0, pos[r, c], 9, r, c] = 0.25 + 0.5 * rng.uniform()
            single[0, 0, :, r, c] = L[0, pos[r, c], :, r, c]
    for pool in ("mean", "sum"):
        y8 = oracle.forward(wts, 8, fr.gbuf, L, fr.scene, pool=pool)
        y1 = oracle.forward(wts, 8, fr.gbuf, single, fr.scene, pool=pool)
        assert rel(y8, y1) <= 1e-14
    # with one active slot, mean and sum pooling coincide
    ym = oracle.forward(wts, 8, fr.gbuf, single, fr.scene, pool="mean")
    ys = oracle.forward(wts, 8, fr.gbuf, single, fr.scene, pool="sum")
    assert np.array_equal(ym, ys)


def test_empty_slot_set_gives_zero_tau():
    wts, fr = tiny(n=1, h=3, w=3, k=4, W=8)
    L = fr.layers.copy()
    L[:, :, 9] = 0.0
    y, lat = oracle.forward(wts, 8, fr.gbuf, L, fr.scene, return_latents=True)
    assert np.all(lat["tau"] == 0.0)
    y0 = oracle.forward(wts, 8, fr.gbuf, fr.layers[:, :0], fr.scene)
    assert np.array_equal(y, y0)


def test_mean_sum_closed_forms():
    wts, fr = tiny(n=1, h=4, w=4, k=4, W=8, alpha_mode="uniform_count")
    _, lm = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, pool="mean", return_latents=True)
    _, ls = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, pool="sum", return_latents=True)
    c = np.maximum(lm["count"], 1.0)[:, None]
    assert rel(lm["tau"] * c, ls["tau"]) <= 1e-14
    # duplicating every slot doubles the sum and leaves the mean unchanged
    dup = np.concatenate([fr.layers, fr.layers], axis=1)
    _, ls2 = oracle.forward(wts, 8, fr.gbuf, dup, fr.scene, pool="sum", return_latents=True)
    assert rel(ls2["tau"], 2.0 * ls["tau"]) <= 1e-14
    ym = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene, pool="mean")
    ym2 = oracle.forward(wts, 8, fr.gbuf, dup, fr.scene, pool="mean")
    assert rel(ym2, ym) <= 1e-13
    assert np.array_equal(lm["count"] * 2, _count(dup))


def _count(layers):
    return (layers[:, :, 9] > 0).sum(axis=1).astype(np.float64)


# --------------------------------------------------------------- closed forms
def _test_side_pack(mats, W):
    """Pack per-layer (matrix, bias) lists in the documented flat order.

    Written independently of the oracle: nets F, T, B, R; layers 1..3; the
    [out][in] matrix row by row, then the bias.
    """
    flat = []
    for net in ("F", "T", "B", "R"):
        for A, c in mats[net]:
            for row in A:
                flat.extend(float(v) for v in row)
            flat.extend(float(v) for v in c)
    return np.array(flat)


def test_affine_regime_equals_composed_matrix_products():
    """Non-negative weights, biases and inputs keep every ReLU at identity, so
    the network reduces to composed affine maps (plain matrix products)."""
    W, k = 6, 3
    rng = np.random.default_rng(7)
    fin = {"F": [30, W, W], "T": [12 + W, W, W], "B": [2 * W, W, W], "R": [W + 3, W, W]}
    fout = {"F": [W, W, W], "T": [W, W, W], "B": [W, W, W], "R": [W, W, 3]}
    mats = {net: [(rng.uniform(0, 0.3, (fout[net][j], fin[net][j])),
                   rng.uniform(0, 0.3, fout[net][j])) for j in range(3)]
            for net in fin}
    wts = _test_side_pack(mats, W)
    h, w = 2, 3
    g = rng.uniform(0, 1, (1, 14, h, w))
    L = rng.uniform(0, 1, (1, k, 12, h, w))
    L[0, 1, 9, 0, 0] = 0.0          # one inactive slot
    s = rng.uniform(0, 1, (1, 16))

    def compose(net):
        (A1, c1), (A2, c2), (A3, c3) = mats[net]
        return A3 @ A2 @ A1, A3 @ (A2 @ c1 + c2) + c3

    MF, cF = compose("F")
    MT, cT = compose("T")
    MB, cB = compose("B")
    MR, cR = compose("R")
    for pool in ("mean", "sum"):
        y = oracle.forward(wts, W, g, L, s, pool=pool)
        for r in range(h):
            for c in range(w):
                x = np.concatenate([g[0, :, r, c], s[0]])
                sigma = MF @ x + cF
                act = [i for i in range(k) if L[0, i, 9, r, c] > 0]
                tau = sum(MT @ np.concatenate([L[0, i, :, r, c], sigma]) + cT for i in act)
                if pool == "mean":
                    tau = tau / len(act)
                phi = MB @ np.concatenate([sigma, tau]) + cB
                exp = MR @ np.concatenate([phi, g[0, 11:14, r, c]]) + cR
                assert rel(y[0, :, r, c], exp) <= 1e-12


def test_zero_weights_give_the_last_bias():
    W = 4
    n = oracle.n_params(W)
    wts = np.zeros(n)
    wts[-3:] = [0.3, -0.7, 1.1]     # R's last bias; a stray output ReLU would clip -0.7
    wts32, fr = tiny(W=W)
    y = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene)
    assert np.all(y[:, 0] == 0.3) and np.all(y[:, 1] == -0.7) and np.all(y[:, 2] == 1.1)


def test_hand_worked_width1_example():
    """W = 1 network whose every weight is chosen by hand; values derived on paper.

    sigma = F3*relu(F2*relu(pos_x)) + 0.5 with F2 = 2, F3 = 1; pos_x = 0.25 -> 1.0
    h(b, sigma) = 3*relu(alpha + sigma) - 1 = 3*alpha + 2
    alphas 0.5, 0.25 and 0 (inactive): h = 3.5, 2.75
        mean tau = 3.125, sum tau = 6.25
    phi = 2*relu(sigma - tau + 4) + 0.1: mean 3.85, sum 0.1
    r = relu(phi + L_d,red) with L_d,red = 0.15: mean 4.0, sum 0.25
    y = (r, -r, 0.5 r - 0.2): mean (4, -4, 1.8), sum (0.25, -0.25, -0.075)
    """
    W = 1
    z = lambda o, i: np.zeros((o, i))  # noqa: E731
    F1 = z(1, 30); F1[0, 0] = 1.0
    T1 = z(1, 13); T1[0, 9] = 1.0; T1[0, 12] = 1.0
    B1 = np.array([[1.0, -1.0]])
    R1 = np.array([[1.0, 1.0, 0.0, 0.0]])
    mats = {
        "F": [(F1, [0.0]), ([[2.0]], [0.0]), ([[1.0]], [0.5])],
        "T": [(T1, [0.0]), ([[1.0]], [0.0]), ([[3.0]], [-1.0])],
        "B": [(B1, [4.0]), ([[1.0]], [0.0]), ([[2.0]], [0.1])],
        "R": [(R1, [0.0]), ([[1.0]], [0.0]), ([[1.0], [-1.0], [0.5]], [0.0, 0.0, -0.2])],
    }
    wts = _test_side_pack(mats, W)
    g = np.zeros((1, 14, 1, 1)); g[0, 0] = 0.25; g[0, 11] = 0.15; g[0, 12] = 9.0
    L = np.zeros((1, 3, 12, 1, 1))
    L[0, 0, 9] = 0.5; L[0, 1, 9] = 0.25; L[0, 2, 9] = 0.0; L[0, 2, 0] = 5.0
    s = np.zeros((1, 16))
    ym = oracle.forward(wts, W, g, L, s, pool="mean")[0, :, 0, 0]
    ys = oracle.forward(wts, W, g, L, s, pool="sum")[0, :, 0, 0]
    np.testing.assert_allclose(ym, [4.0, -4.0, 1.8], rtol=0, atol=1e-14)
    np.testing.assert_allclose(ys, [0.25, -0.25, -0.075], rtol=0, atol=1e-14)
    yb = oracle.forward_bruteforce(wts, W, g, L, s, pool="mean")[0, :, 0, 0]
    np.testing.assert_allclose(yb, [4.0, -4.0, 1.8], rtol=0, atol=1e-14)


def test_pixels_are_independent():
    wts, fr = tiny(n=1, h=5, w=6, k=3, W=8)
    y = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene)
    # transposing the image transposes the output
    yt = oracle.forward(wts, 8, fr.gbuf.transpose(0, 1, 3, 2), fr.layers.transpose(0, 1, 2, 4, 3),
                        fr.scene)
    assert rel(yt, y.transpose(0, 1, 3, 2)) <= 1e-15
    # a crop of the input gives the crop of the output
    yc = oracle.forward(wts, 8, fr.gbuf[:, :, 1:4, 2:5], fr.layers[:, :, :, 1:4, 2:5], fr.scene)
    assert rel(yc, y[:, :, 1:4, 2:5]) <= 1e-15


def test_frames_use_their_own_scene_vector():
    wts, fr = tiny(n=2, h=2, w=2, k=2, W=8)
    y = oracle.forward(wts, 8, fr.gbuf, fr.layers, fr.scene)
    y1 = oracle.forward(wts, 8, fr.gbuf[1:], fr.layers[1:], fr.scene[1:])
    assert rel(y1[0], y[1]) <= 1e-15


# ------------------------------------------------------------------ gradient
def _fd_check(W, n, h, w, k, pool, n_coords, seed):
    wts, fr = tiny(n=n, h=h, w=w, k=k, W=W, seed=seed, alpha_mode="uniform_count")
    rng = np.random.default_rng(seed)
    target = rng.normal(size=(n, 3, h, w))
    w64 = wts.astype(np.float64)
    loss, g = oracle.grad(w64, W, fr.gbuf, fr.layers, fr.scene, target, pool=pool)
    y = oracle.forward(w64, W, fr.gbuf, fr.layers, fr.scene, pool=pool)
    assert loss == pytest.approx(oracle.l1_loss(y, target)[0], rel=1e-13)
    npar = w64.size
    coords = set(rng.choice(npar, size=min(n_coords, npar), replace=False).tolist())
    coords |= set(range(npar - 3, npar))          # R's output biases
    eps = 1e-6
    checked, skipped, worst = 0, 0, 0.0
    for i in sorted(coords):
        wp, wm = w64.copy(), w64.copy()
        wp[i] += eps
        wm[i] -= eps
        sp = oracle.relu_signature(wp, W, fr.gbuf, fr.layers, fr.scene, target, pool)
        sm = oracle.relu_signature(wm, W, fr.gbuf, fr.layers, fr.scene, target, pool)
        if not np.array_equal(sp, sm):
            skipped += 1
            continue
        lp = oracle.l1_loss(oracle.forward(wp, W, fr.gbuf, fr.layers, fr.scene, pool=pool), target)[0]
        lm = oracle.l1_loss(oracle.forward(wm, W, fr.gbuf, fr.layers, fr.scene, pool=pool), target)[0]
        fd = (lp - lm) / (2 * eps)
        # rounding of the loss contributes ~eps*|L|/h ~ 1e-10 absolute
        err = abs(fd - g[i]) / (1e-9 + 1e-6 * abs(g[i]))
        worst = max(worst, err)
        checked += 1
    assert checked >= 0.9 * len(coords)
    return worst, checked, skipped


@pytest.mark.parametrize("pool", ["mean", "sum"])
def test_gradient_matches_central_differences(pool):
    worst, checked, skipped = _fd_check(W=8, n=1, h=4, w=4, k=3, pool=pool, n_coords=400, seed=21)
    assert worst <= 1.0, (worst, checked, skipped)


def test_gradient_matches_central_differences_w128_crop():
    """The 8x8 crop, K=4, W=128 check of the training workload (subset of coordinates)."""
    worst, checked, skipped = _fd_check(W=128, n=1, h=8, w=8, k=4, pool="mean", n_coords=160,
                                        seed=3)
    assert worst <= 1.0, (worst, checked, skipped)


def test_gradient_is_zero_for_inactive_only_slot_weights():
    """With every alpha = 0 no gradient reaches T."""
    wts, fr = tiny(n=1, h=3, w=3, k=2, W=8)
    L = fr.layers.copy()
    L[:, :, 9] = 0.0
    t = np.zeros((1, 3, 3, 3))
    _, g = oracle.grad(wts, 8, fr.gbuf, L, fr.scene, t)
    P = oracle.unpack(g, 8)
    assert all(np.all(A == 0) and np.all(c == 0) for A, c in P["T"])
    assert any(np.any(A != 0) for A, c in P["F"])


# ------------------------------------------------------------- kink margins
def test_relu_margin_vanishes_at_a_planted_kink():
    """One hidden unit of F gets the bias that puts its input exactly at the
    kink for one pixel (fp64 weights): that pixel's margin drops to rounding
    level while every other pixel keeps a margin far above it."""
    W = 8
    wts, fr = tiny(n=1, h=3, w=2, k=2, W=W)
    P = oracle.unpack(wts, W)
    G = fr.gbuf.reshape(14, -1).astype(np.float64)
    x = np.concatenate([G, np.repeat(fr.scene.reshape(16, 1).astype(np.float64), G.shape[1], 1)])
    base = oracle.relu_margins(wts, W, fr.gbuf, fr.layers, fr.scene).ravel()
    assert np.all((base > 0) & (base <= 1.0))
    p, j = 4, 3
    A1, c1 = P["F"][0]
    c1 = c1.copy()
    c1[j] = -(A1[j] @ x[:, p])
    P["F"][0] = (A1, c1)
    m = oracle.relu_margins(oracle.pack(P), W, fr.gbuf, fr.layers, fr.scene).ravel()
    assert m[p] < 1e-14
    assert np.all(np.delete(m, p) > 1e-9)


def test_relu_margin_ignores_inactive_slots():
    """A slot with alpha = 0 never reaches the output, so its h units cannot
    set a pixel's margin: with every alpha zeroed the margins equal those of
    the same frame without slots."""
    W = 8
    wts, fr = tiny(n=1, h=3, w=3, k=3, W=W)
    L = fr.layers.copy()
    L[:, :, 9] = 0.0
    a = oracle.relu_margins(wts, W, fr.gbuf, L, fr.scene)
    b = oracle.relu_margins(wts, W, fr.gbuf, L[:, :0], fr.scene)
    assert np.array_equal(a, b)
    c = oracle.relu_margins(wts, W, fr.gbuf, fr.layers, fr.scene)
    assert not np.array_equal(a, c)


# ------------------------------------------------------ the paper's own table
def test_order_inversion_table():
    """Tab. OrderLoss: inverting the transparency-buffer order leaves the MAE
    unchanged to the printed five decimals on every scene."""
    with open(os.path.join(GOLDEN, "order_loss_table.json")) as f:
        tab = json.load(f)
    for row in tab["rows"]:
        assert f"{row['mae'] - row['mae_inverted']:.5f}" in ("0.00000", "-0.00000")
        assert row["difference"] == 0.0
    wts, fr = tiny(n=1, h=8, w=8, k=4, W=16, alpha_mode="uniform_count")
    t = np.random.default_rng(1).uniform(size=(1, 3, 8, 8))
    mae = oracle.l1_loss(oracle.forward(wts, 16, fr.gbuf, fr.layers, fr.scene), t)[0]
    mae_inv = oracle.l1_loss(oracle.forward(wts, 16, fr.gbuf, fr.layers[:, ::-1], fr.scene), t)[0]
    assert f"{abs(mae - mae_inv):.5f}" == "0.00000"
    assert abs(mae - mae_inv) <= 1e-15


def test_param_count_formula():
    for W in (1, 8, 64, 128):
        assert oracle.n_params(W) == 11 * W * W + 59 * W + 3 == synth.num_params(W)
    assert math.isclose(oracle.n_params(128) * 4 / 1024, 733.51171875)


# ------------------------------------------- the vector-Jacobian product
# grad_from_dy is the checker of every GPU backward test; its dy branch is
# pinned here to the L1 branch, to finite differences of sum(dy * y) and to
# linearity in dy.
def test_grad_from_dy_equals_l1_gradient_at_its_seed():
    """With dL/dy = sign(y - t) / N (the L1 term's derivative, Sec. 3.5) the
    vector-Jacobian product is the L1 gradient itself."""
    W = 8
    wts, fr = tiny(n=2, h=3, w=4, k=3, W=W, seed=5, alpha_mode="uniform_count")
    t = np.random.default_rng(5).normal(size=(2, 3, 3, 4))
    for pool in ("mean", "sum"):
        y = oracle.forward(wts, W, fr.gbuf, fr.layers, fr.scene, pool=pool)
        dy = np.sign(y - t) / y.size
        g_l1 = oracle.grad(wts, W, fr.gbuf, fr.layers, fr.scene, t, pool=pool)[1]
        g_dy = oracle.grad_from_dy(wts, W, fr.gbuf, fr.layers, fr.scene, dy, pool=pool)
        assert np.max(np.abs(g_dy - g_l1)) <= 1e-15 * max(1.0, np.max(np.abs(g_l1)))
        assert np.any(g_dy != 0)


def test_grad_from_dy_is_linear_in_dy():
    W = 8
    wts, fr = tiny(n=1, h=4, w=3, k=2, W=W, seed=6, alpha_mode="uniform_count")
    rng = np.random.default_rng(6)
    d1, d2 = rng.normal(size=(2, 1, 3, 4, 3))
    g = lambda d: oracle.grad_from_dy(wts, W, fr.gbuf, fr.layers, fr.scene, d)  # noqa: E731
    lhs = g(2.0 * d1 - 3.0 * d2)
    rhs = 2.0 * g(d1) - 3.0 * g(d2)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))
    assert np.array_equal(g(np.zeros_like(d1)), np.zeros(oracle.n_params(W)))


def _fd_vjp(W, pe, pool, seed, n_coords):
    """Central differences (h = 1e-6) of J(w) = sum(dy * y(w)) against
    grad_from_dy, skipping coordinates whose +-h evaluations lie on
    different pieces of the ReLU network (their branch signatures differ)."""
    s = synth.streams(seed)
    wts = synth.make_weights(W, s["weights"], pe_levels=pe).astype(np.float64)
    fr = synth.Frame(synth.make_gbuf(1, 3, 3, s["gbuf"]),
                     synth.make_layers(1, 3, 3, 3, s["slots"], s["active"], "uniform_count"),
                     synth.make_scene(1, s["gbuf"]))
    rng = np.random.default_rng(seed)
    dy = rng.normal(size=(1, 3, 3, 3))
    g = oracle.grad_from_dy(wts, W, fr.gbuf, fr.layers, fr.scene, dy, pool=pool, pe_levels=pe)
    ny = dy.size
    zero_t = np.zeros_like(dy)

    def J(w):
        y = oracle.forward(w, W, fr.gbuf, fr.layers, fr.scene, pool=pool, pe_levels=pe)
        return float((dy * y).sum())

    def sig(w):   # ReLU and mask branches only (the trailing y > t part is dropped)
        return oracle.relu_signature(w, W, fr.gbuf, fr.layers, fr.scene, zero_t, pool,
                                     pe_levels=pe)[:-ny]

    coords = set(rng.choice(wts.size, size=min(n_coords, wts.size), replace=False).tolist())
    coords |= set(range(wts.size - 3, wts.size))
    eps, worst, checked = 1e-6, 0.0, 0
    for i in sorted(coords):
        wp, wm = wts.copy(), wts.copy()
        wp[i] += eps
        wm[i] -= eps
        if not np.array_equal(sig(wp), sig(wm)):
            continue
        fd = (J(wp) - J(wm)) / (2 * eps)
        worst = max(worst, abs(fd - g[i]) / (1e-8 + 1e-6 * abs(g[i])))
        checked += 1
    assert checked >= 0.9 * len(coords)
    return worst


@pytest.mark.parametrize("pool", ["mean", "sum"])
def test_grad_from_dy_matches_central_differences(pool):
    assert _fd_vjp(W=8, pe=0, pool=pool, seed=31, n_coords=300) <= 1.0


def test_grad_from_dy_matches_central_differences_encoded():
    assert _fd_vjp(W=8, pe=2, pool="mean", seed=32, n_coords=300) <= 1.0
