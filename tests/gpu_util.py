"""Helpers shared by the GPU tests: device transfer, sampling, error metrics."""
import sys

import numpy as np

import oracle
from paper_2405_19056_amd import synth


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def host(t):
    return t.detach().to("cpu").numpy()


def relF(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((y - ref).ravel()) / np.linalg.norm(ref.ravel()))


def relInf(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))


def sample_pixels(fr: synth.Frame, count, rng):
    """Pick `count` pixels (frame index, flat pixel) and gather them into a
    one-row frame per source frame (pixels are independent, Sec. 3.4)."""
    n, hw = fr.n, fr.h * fr.w
    flat = rng.choice(n * hw, size=min(count, n * hw), replace=False)
    flat.sort()
    return flat


def oracle_on_sample(w, W, fr: synth.Frame, flat, pool):
    """Oracle output [len(flat)][3] for the sampled pixels."""
    hw = fr.h * fr.w
    out = np.empty((len(flat), 3))
    for f in np.unique(flat // hw):
        sel = flat[flat // hw == f] % hw
        g = fr.gbuf[f].reshape(14, hw)[:, sel][None, :, None, :]
        L = fr.layers[f].reshape(fr.k, 12, hw)[:, :, sel][None, :, :, None, :]
        y = oracle.forward(w, W, g, L, fr.scene[f:f + 1], pool=pool)
        out[flat // hw == f] = y[0, :, 0, :].T
    return out


def gpu_on_sample(y_dev_np, fr: synth.Frame, flat):
    hw = fr.h * fr.w
    f, q = flat // hw, flat % hw
    yy = y_dev_np.reshape(fr.n, 3, hw)
    return yy[f, :, q]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# A ReLU input closer to its kink than this fraction of the absolute-value sum
# that bounds its rounding error may take the other branch in fp32 than in
# the fp64 oracle (fp32 evaluation errors measure about 1e-6 of that sum).
# Gradient parity is compared on pixels away from such kinks.
KINK = 1e-5


def kink_free(w, W, fr: synth.Frame, pool, flat=None):
    """Boolean mask of pixels (all [n][h][w], or the sampled `flat` indices)
    whose every ReLU input is at least KINK away from its kink."""
    if flat is None:
        return oracle.relu_margins(w, W, fr.gbuf, fr.layers, fr.scene, pool=pool) >= KINK
    hw = fr.h * fr.w
    ok = np.empty(len(flat), dtype=bool)
    for f in np.unique(flat // hw):
        at = flat // hw == f
        sel = flat[at] % hw
        g = fr.gbuf[f].reshape(14, hw)[:, sel][None, :, None, :]
        L = fr.layers[f].reshape(fr.k, 12, hw)[:, :, sel][None, :, :, None, :]
        ok[at] = oracle.relu_margins(w, W, g, L, fr.scene[f:f + 1], pool=pool).ravel() >= KINK
    return ok


def pixel_p99(y, ref):
    """99th percentile over pixels of |y_p - y*_p|_2 / rms_q |y*_q|_2, for
    outputs [n][3][h][w] (or sampled [P][3]).  Its mean square is relF^2."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if y.ndim == 4:
        y = np.moveaxis(y, 1, -1).reshape(-1, y.shape[1])
        ref = np.moveaxis(ref, 1, -1).reshape(-1, ref.shape[1])
    e = np.linalg.norm(y - ref, axis=1)
    rms = np.sqrt(np.mean(np.sum(ref * ref, axis=1)))
    return float(np.percentile(e, 99) / rms)


def gate(y, ref, tol, what=""):
    """Output-radiance parity: relative Frobenius error <= tol, the largest
    element error <= 2 tol of the largest reference element, and the
    per-pixel error's 99th percentile <= 3 tol of the rms pixel.  Returns the
    three figures (logged)."""
    f, i, p = relF(y, ref), relInf(y, ref), pixel_p99(y, ref)
    log(f"  {what} relF={f:.3e} relInf={i:.3e} p99={p:.3e} (tol {tol:g})")
    assert np.all(np.isfinite(y)), what
    assert f <= tol, (what, "relF", f)
    assert i <= 2 * tol, (what, "relInf", i)
    assert p <= 3 * tol, (what, "p99", p)
    return f, i, p


def sample_every_tile(fr: synth.Frame, per_tile, rng, tile=256):
    """Flat pixel indices covering every 256-pixel tile of every frame
    (`per_tile` random pixels each, the ragged last tile included) plus each
    frame's four corners and its last pixel: a wrong tile anywhere shows."""
    hw = fr.h * fr.w
    picks = []
    for f in range(fr.n):
        base = f * hw
        for t0 in range(0, hw, tile):
            t1 = min(hw, t0 + tile)
            picks.append(base + rng.choice(np.arange(t0, t1), size=min(per_tile, t1 - t0),
                                           replace=False))
        corners = [0, fr.w - 1, (fr.h - 1) * fr.w, hw - 1]
        picks.append(base + np.asarray(corners))
    flat = np.unique(np.concatenate(picks))
    return flat
