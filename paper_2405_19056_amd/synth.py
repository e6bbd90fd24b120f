"""Seeded synthetic inputs for GlassNet: buffers, scene vectors, weights, targets.

This module only draws random numbers and lays them out.  It holds none of the
network's arithmetic, so both the FP64 oracle (through the tests) and the HIP
path consume the very same arrays.

Buffer schema (the paper's Fig. "Inputs" lists the kind of per-pixel planes a
rasterizer provides for the opaque G-buffer and for each transparency buffer,
Sec. 3.2; the exact channel set used here is fixed by this library):

  G-buffer, 14 fp32 planes:  position(3) U(-1,1), unit normal(3) from a
      normalised N(0,1)^3 draw, albedo(3) U(0,1), roughness U(0,1),
      metallic Bernoulli(0.3), direct light L_d(3) U(0,2).
  Transparency layer, 12 fp32 planes: position(3), unit normal(3) as above,
      tint(3) U(0,1), alpha, IOR U(1,2), depth U(0,1).
  Scene vector, 16 fp32 U(-1,1)  (the variable scene parameters of the
      appendix table: roughness, position, lighting, colour).

Alpha rules:
  "p0.3":          alpha ~ U(0,1), then set to 0 with probability 0.3.
  "uniform_count": per pixel an active count n ~ U{0..K}; a uniformly random
                   subset of n slots is active with alpha ~ U(0,1] (strictly
                   positive), the others get alpha = 0 while their other 11
                   planes are still drawn (so masking is really exercised).

Everything is stored as C-contiguous fp32 in struct-of-arrays order:
  gbuf   [n][14][h][w]
  layers [n][k][12][h][w]
  scene  [n][16]

Weights: one flat fp32 vector.  Networks in the order F, T, B, R; within a
network layers 1, 2, 3; within a layer the matrix (row-major [out][in]) then
the bias.  Kaiming-uniform matrices U(+-sqrt(6/fan_in)) and biases
U(+-1/sqrt(fan_in)).
"""
from __future__ import annotations

import dataclasses

import numpy as np

N_G = 14
N_L = 12
N_S = 16
N_OUT = 3

# Child-stream order of a config's SeedSequence.
_STREAMS = ("weights", "gbuf", "slots", "active", "shuffles", "teacher",
            "noise", "arrivals")


def layer_shapes(width: int, pe_levels: int = 0):
    """(fan_out, fan_in) of the 12 linear layers in packing order.  With
    positional encoding of L levels, F's input and h's slot input are
    (1 + 2 L) times wider."""
    W = width
    e = 1 + 2 * pe_levels
    return [
        (W, (N_G + N_S) * e), (W, W), (W, W),    # F
        (W, N_L * e + W), (W, W), (W, W),        # T (shared per-layer MLP h)
        (W, 2 * W), (W, W), (W, W),              # B
        (W, W + 3), (W, W), (N_OUT, W),          # R
    ]


def num_params(width: int, pe_levels: int = 0) -> int:
    return sum(o * i + o for o, i in layer_shapes(width, pe_levels))


def streams(seed: int) -> dict:
    """Independent generators for every random quantity of one config."""
    children = np.random.SeedSequence(seed).spawn(len(_STREAMS))
    return {name: np.random.default_rng(c) for name, c in zip(_STREAMS, children)}


def make_weights(width: int, rng: np.random.Generator, pe_levels: int = 0) -> np.ndarray:
    parts = []
    for fan_out, fan_in in layer_shapes(width, pe_levels):
        wb = np.sqrt(6.0 / fan_in)
        bb = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-wb, wb, size=fan_out * fan_in))
        parts.append(rng.uniform(-bb, bb, size=fan_out))
    return np.concatenate(parts).astype(np.float32)


SR_WIDTH, SR_IN, SR_OUT = 32, 3 + N_G, 3


def sr_layer_shapes():
    """(fan_out, fan_in, taps) of the super-sampling network's three convs."""
    return [(SR_WIDTH, SR_IN, 9), (SR_WIDTH, SR_WIDTH, 9), (SR_OUT, SR_WIDTH, 1)]


def make_sr_weights(rng: np.random.Generator) -> np.ndarray:
    """Packed super-sampling weights (each conv's W then b), initialised like
    make_weights with fan_in = input channels x taps."""
    parts = []
    for fan_out, cin, taps in sr_layer_shapes():
        fan_in = cin * taps
        parts.append(rng.uniform(-np.sqrt(6.0 / fan_in), np.sqrt(6.0 / fan_in),
                                 size=fan_out * fan_in))
        parts.append(rng.uniform(-1.0 / np.sqrt(fan_in), 1.0 / np.sqrt(fan_in), size=fan_out))
    return np.concatenate(parts).astype(np.float32)


def spatial_layer_shapes(width: int):
    """(fan_out, cin, k) of the spatial networks' convolutions in packing
    order: F (U-Net, 4), T (3), B (U-Net, 4), R (3); k x k kernels."""
    W = width
    return [(W, N_G + N_S, 3), (W, W, 3), (W, 2 * W, 3), (W, W, 1),
            (W, N_L + W, 3), (W, W, 1), (W, W, 1),
            (W, 2 * W, 3), (W, W, 3), (W, 2 * W, 3), (W, W, 1),
            (W, W + 3, 3), (W, W, 3), (N_OUT, W, 1)]


def make_spatial_weights(width: int, rng: np.random.Generator) -> np.ndarray:
    """Packed spatial-network weights (each conv's W [out][in][k][k], then b),
    initialised like make_weights with fan_in = input channels x taps."""
    parts = []
    for fan_out, cin, k in spatial_layer_shapes(width):
        fan_in = cin * k * k
        parts.append(rng.uniform(-np.sqrt(6.0 / fan_in), np.sqrt(6.0 / fan_in),
                                 size=fan_out * fan_in))
        parts.append(rng.uniform(-1.0 / np.sqrt(fan_in), 1.0 / np.sqrt(fan_in), size=fan_out))
    return np.concatenate(parts).astype(np.float32)


def make_sr_inputs(n: int, h: int, w: int, seed: int):
    """A render [n][3][h][w] (radiance-like values in [0, 2)) and a G-buffer at
    twice its resolution, [n][14][2h][2w]."""
    rng = np.random.default_rng(seed)
    lowres = rng.uniform(0.0, 2.0, size=(n, 3, h, w)).astype(np.float32)
    return lowres, make_gbuf(n, 2 * h, 2 * w, rng)


def _unit_normals(rng, shape):
    v = rng.standard_normal(size=(3,) + shape)
    n = np.sqrt((v * v).sum(axis=0, keepdims=True))
    n = np.where(n == 0.0, 1.0, n)
    return v / n


def make_gbuf(n: int, h: int, w: int, rng: np.random.Generator) -> np.ndarray:
    g = np.empty((n, N_G, h, w), dtype=np.float64)
    shp = (n, h, w)
    g[:, 0:3] = np.moveaxis(rng.uniform(-1.0, 1.0, size=(3,) + shp), 0, 1)
    g[:, 3:6] = np.moveaxis(_unit_normals(rng, shp), 0, 1)
    g[:, 6:9] = np.moveaxis(rng.uniform(0.0, 1.0, size=(3,) + shp), 0, 1)
    g[:, 9] = rng.uniform(0.0, 1.0, size=shp)
    g[:, 10] = (rng.uniform(0.0, 1.0, size=shp) < 0.3).astype(np.float64)
    g[:, 11:14] = np.moveaxis(rng.uniform(0.0, 2.0, size=(3,) + shp), 0, 1)
    return np.ascontiguousarray(g.astype(np.float32))


def make_layers(n: int, k: int, h: int, w: int, rng_slots: np.random.Generator,
                rng_active: np.random.Generator, alpha_mode: str = "uniform_count"
                ) -> np.ndarray:
    L = np.empty((n, k, N_L, h, w), dtype=np.float64)
    shp = (n, k, h, w)
    L[:, :, 0:3] = np.moveaxis(rng_slots.uniform(-1.0, 1.0, size=(3,) + shp), 0, 2)
    L[:, :, 3:6] = np.moveaxis(_unit_normals(rng_slots, shp), 0, 2)
    L[:, :, 6:9] = np.moveaxis(rng_slots.uniform(0.0, 1.0, size=(3,) + shp), 0, 2)
    L[:, :, 10] = rng_slots.uniform(1.0, 2.0, size=shp)
    L[:, :, 11] = rng_slots.uniform(0.0, 1.0, size=shp)
    if alpha_mode == "p0.3":
        a = rng_active.uniform(0.0, 1.0, size=shp)
        a[rng_active.uniform(0.0, 1.0, size=shp) < 0.3] = 0.0
    elif alpha_mode == "uniform_count":
        cnt = rng_active.integers(0, k + 1, size=(n, h, w))
        # a uniformly random subset of size cnt: rank slots by a random key
        keys = rng_active.uniform(size=(n, k, h, w))
        rank = np.argsort(np.argsort(keys, axis=1), axis=1)
        active = rank < cnt[:, None]
        a = np.where(active, 1.0 - rng_active.uniform(0.0, 1.0, size=shp), 0.0)
    elif alpha_mode == "discs":
        # spatially coherent coverage (a labelled variant, not a workload of
        # the configs): slot i of a frame covers one disc, centre uniform in
        # the frame, radius U(0.1, 0.35) of the shorter side; alpha U(0, 1]
        # inside, 0 outside
        yy, xx = np.mgrid[0:h, 0:w]
        a = np.zeros(shp)
        for f in range(n):
            for i in range(k):
                cy, cx = rng_active.uniform(0, h), rng_active.uniform(0, w)
                r = rng_active.uniform(0.1, 0.35) * min(h, w)
                inside = (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
                a[f, i] = np.where(inside, 1.0 - rng_active.uniform(0.0, 1.0, size=(h, w)), 0.0)
    else:
        raise ValueError(f"unknown alpha_mode {alpha_mode!r}")
    L[:, :, 9] = a
    return np.ascontiguousarray(L.astype(np.float32))


def make_scene(n: int, rng: np.random.Generator) -> np.ndarray:
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(n, N_S)).astype(np.float32))


@dataclasses.dataclass
class Frame:
    gbuf: np.ndarray
    layers: np.ndarray
    scene: np.ndarray

    @property
    def n(self):
        return self.gbuf.shape[0]

    @property
    def h(self):
        return self.gbuf.shape[2]

    @property
    def w(self):
        return self.gbuf.shape[3]

    @property
    def k(self):
        return self.layers.shape[1]


def make_frame(n, h, w, k, seed, alpha_mode="uniform_count") -> Frame:
    s = streams(seed)
    return Frame(make_gbuf(n, h, w, s["gbuf"]),
                 make_layers(n, k, h, w, s["slots"], s["active"], alpha_mode),
                 make_scene(n, s["gbuf"]))


def slot_shuffles(n, k, h, w, count, rng: np.random.Generator) -> np.ndarray:
    """`count` independent per-pixel permutations of the k slots: [count][n][k][h][w]."""
    keys = rng.uniform(size=(count, n, k, h, w))
    return np.argsort(keys, axis=2).astype(np.int64)


def apply_slot_permutation(layers: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Reorder slots per pixel: out[:, i] = layers[:, perm[:, i]] for every pixel."""
    idx = np.broadcast_to(perm[:, :, None], layers.shape)
    return np.ascontiguousarray(np.take_along_axis(layers, idx, axis=1))


def noise(shape, sigma, rng: np.random.Generator) -> np.ndarray:
    return (sigma * rng.standard_normal(size=shape)).astype(np.float32)


def poisson_arrivals(rate_hz: float, duration_s: float, rng: np.random.Generator):
    """Arrival times of a Poisson process on [0, duration)."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return np.asarray(out)
        out.append(t)


# The benchmark workloads: sizes and input rules.
CONFIGS = {
    "c0_64sq_k2_w64": dict(n=1, h=64, w=64, k=2, width=64, alpha_mode="p0.3",
                           pool="mean", seed=0),
    "c1_256sq_k4_w128": dict(n=1, h=256, w=256, k=4, width=128,
                             alpha_mode="uniform_count", pool="mean", seed=1),
    "c2_512sq_k8_w128": dict(n=1, h=512, w=512, k=8, width=128,
                             alpha_mode="uniform_count", pool="mean", seed=2),
    "c3_train_16x128sq_k4_w128": dict(n=16, h=128, w=128, k=4, width=128,
                                      alpha_mode="uniform_count", pool="mean", seed=3),
}
SERVE_RESOLUTIONS = [(256, 256), (512, 512), (360, 640), (576, 1024)]


def config_inputs(name: str):
    """(weights, Frame, streams) for one named workload."""
    c = CONFIGS[name]
    s = streams(c["seed"])
    w = make_weights(c["width"], s["weights"])
    fr = Frame(make_gbuf(c["n"], c["h"], c["w"], s["gbuf"]),
               make_layers(c["n"], c["k"], c["h"], c["w"], s["slots"], s["active"],
                           c["alpha_mode"]),
               make_scene(c["n"], s["gbuf"]))
    return w, fr, s
