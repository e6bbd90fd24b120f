"""The seeded input generator: determinism, shapes and distributions."""
import numpy as np

from paper_2405_19056_amd import synth


def test_same_seed_same_arrays():
    a = synth.config_inputs("c0_64sq_k2_w64")
    b = synth.config_inputs("c0_64sq_k2_w64")
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1].gbuf, b[1].gbuf)
    assert np.array_equal(a[1].layers, b[1].layers)
    assert np.array_equal(a[1].scene, b[1].scene)


def test_shapes_and_dtypes():
    w, fr, _ = synth.config_inputs("c0_64sq_k2_w64")
    assert w.dtype == np.float32 and w.size == 11 * 64 * 64 + 59 * 64 + 3
    assert fr.gbuf.shape == (1, 14, 64, 64) and fr.gbuf.dtype == np.float32
    assert fr.layers.shape == (1, 2, 12, 64, 64)
    assert fr.scene.shape == (1, 16)
    for arr in (fr.gbuf, fr.layers, fr.scene):
        assert arr.flags["C_CONTIGUOUS"]


def test_gbuffer_distributions():
    g = synth.make_gbuf(2, 32, 32, np.random.default_rng(0)).astype(np.float64)
    assert np.all(np.abs(g[:, 0:3]) <= 1)
    nrm = np.sqrt((g[:, 3:6] ** 2).sum(axis=1))
    assert np.allclose(nrm, 1.0, atol=1e-6)
    assert np.all((g[:, 6:10] >= 0) & (g[:, 6:10] <= 1))
    assert set(np.unique(g[:, 10])) <= {0.0, 1.0}
    assert 0.25 < g[:, 10].mean() < 0.35
    assert np.all((g[:, 11:14] >= 0) & (g[:, 11:14] <= 2))


def test_uniform_active_count_rule():
    k = 8
    L = synth.make_layers(1, k, 64, 64, np.random.default_rng(1), np.random.default_rng(2))
    a = L[0, :, 9]
    cnt = (a > 0).sum(axis=0)
    assert cnt.min() == 0 and cnt.max() == k
    hist = np.bincount(cnt.ravel(), minlength=k + 1) / cnt.size
    assert np.all(np.abs(hist - 1 / (k + 1)) < 0.02)
    assert np.all(a[a > 0] <= 1.0)
    # inactive slots still carry drawn geometry
    assert np.any(L[0, :, 0][a == 0] != 0)
    # each slot position is equally likely to be active
    frac = (a > 0).mean(axis=(1, 2))
    assert np.all(np.abs(frac - 0.5) < 0.03)
    assert np.all((L[0, :, 10] >= 1) & (L[0, :, 10] <= 2))


def test_p03_alpha_rule():
    L = synth.make_layers(1, 2, 64, 64, np.random.default_rng(1), np.random.default_rng(2), "p0.3")
    z = (L[0, :, 9] == 0).mean()
    assert 0.27 < z < 0.33


def test_weight_init_bounds():
    W = 128
    w = synth.make_weights(W, np.random.default_rng(0)).astype(np.float64)
    off = 0
    for fo, fi in synth.layer_shapes(W):
        A = w[off:off + fo * fi]
        off += fo * fi
        b = w[off:off + fo]
        off += fo
        assert np.all(np.abs(A) <= np.sqrt(6 / fi)) and np.all(np.abs(b) <= 1 / np.sqrt(fi))
        assert np.abs(A).max() > 0.9 * np.sqrt(6 / fi)
    assert off == w.size


def test_shuffles_are_permutations():
    p = synth.slot_shuffles(1, 8, 4, 4, 32, np.random.default_rng(0))
    assert p.shape == (32, 1, 8, 4, 4)
    assert np.all(np.sort(p, axis=2) == np.arange(8)[None, None, :, None, None])
    L = synth.make_layers(1, 8, 4, 4, np.random.default_rng(1), np.random.default_rng(2))
    Lp = synth.apply_slot_permutation(L, p[0])
    for r in range(4):
        for c in range(4):
            assert np.array_equal(Lp[0, :, :, r, c], L[0, p[0, 0, :, r, c], :, r, c])


def test_poisson_arrivals_rate():
    t = synth.poisson_arrivals(200.0, 60.0, np.random.default_rng(4))
    assert abs(len(t) - 12000) < 400
    assert np.all(np.diff(t) > 0)
