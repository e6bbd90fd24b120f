"""FP64 CPU oracle for the spatial GlassNet networks.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The HIP library never calls it and shares no code with it.

The paper's networks are convolutional (Sec. 3.4): the scene encoder F and the
blending network B are U-Nets, the per-buffer network h of T and the rendering
network R are multi-layer CNNs, R ending in 1x1 kernels with larger kernels
before them; T pools h over the transparency buffers with the symmetric sum of
Eq. (5).  Widths, depths and the U-Net's resolution levels are not given.  The
readings taken here (each listed in the design notes):

  * conv3 / conv1: 3 x 3 (zero padding of one pixel, stride 1) and 1 x 1
    convolutions with bias; ReLU after every layer but a network's last;
  * U-Net (F and B), one level down: e1 = relu(conv3(x)), d = the 2 x 2
    average of e1 (frames of even height and width), m = relu(conv3(d)) at
    half resolution, u = m upsampled by repeating each pixel 2 x 2,
    e2 = relu(conv3([e1; u])), output = conv1(e2): width W throughout;
  * h(b_i, sigma) = conv1(relu(conv1(relu(conv3([b_i; sigma]))))): one 3 x 3
    layer on the buffer and sigma, then two 1 x 1 layers;
  * the pool of Eq. (5) per pixel over the buffers whose alpha > 0 there (sum,
    or mean over them: 0 where none is), as in the per-pixel networks;
  * R = conv1(relu(conv3(relu(conv3([phi; L_d]))))) with 3 outputs;
  * F's input [G; s]: the 14 G-buffer planes and the 16 scene values as
    constant planes; B's input [sigma; tau].
A permutation of the transparency buffers is a permutation of whole images:
h sees a buffer's neighbourhood, so per-pixel reshuffles are not symmetries.

Parameters, one flat vector: nets F (4 convolutions), T (3), B (4), R (3);
per convolution the weight [out][in][kh][kw] row-major, then the bias.
Everything is evaluated in float64 from the float32 inputs, literally in the
order above.  `forward_bruteforce` is a scalar Python-loop twin for tiny
inputs.
"""
from __future__ import annotations

import numpy as np

NG, NL, NS, NOUT = 14, 12, 16, 3
NETS = ("F", "T", "B", "R")


def layer_shapes(W):
    """(out, in, k) of every convolution in packing order."""
    return {
        "F": [(W, NG + NS, 3), (W, W, 3), (W, 2 * W, 3), (W, W, 1)],
        "T": [(W, NL + W, 3), (W, W, 1), (W, W, 1)],
        "B": [(W, 2 * W, 3), (W, W, 3), (W, 2 * W, 3), (W, W, 1)],
        "R": [(W, W + 3, 3), (W, W, 3), (NOUT, W, 1)],
    }


def n_params(W):
    return sum(o * i * k * k + o for net in NETS for (o, i, k) in layer_shapes(W)[net])


def unpack(w, W):
    """Flat vector -> {net: [(A [out][in][k][k], c [out]), ...]} in float64."""
    w = np.asarray(w, dtype=np.float64).ravel()
    if w.size != n_params(W):
        raise ValueError(f"expected {n_params(W)} weights for W={W}, got {w.size}")
    out, off = {}, 0
    for net in NETS:
        layers = []
        for (o, i, k) in layer_shapes(W)[net]:
            A = w[off:off + o * i * k * k].reshape(o, i, k, k)
            off += o * i * k * k
            layers.append((A, w[off:off + o]))
            off += o
        out[net] = layers
    return out


def pack(params):
    return np.concatenate([np.concatenate([np.ravel(A), np.ravel(c)])
                           for net in NETS for A, c in params[net]])


def relu(x):
    return np.maximum(x, 0.0)


def conv(x, layer):
    """x [C, H, W] -> [out, H, W]: k x k correlation, zero padding (k - 1) / 2."""
    A, c = layer
    o, i, k, _ = A.shape
    C, H, Wd = x.shape
    if C != i:
        raise ValueError(f"conv expects {i} input channels, got {C}")
    r = (k - 1) // 2
    xp = np.pad(x, ((0, 0), (r, r), (r, r)))
    y = np.zeros((o, H, Wd))
    for dy in range(k):
        for dx in range(k):
            y += np.tensordot(A[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + Wd], axes=(1, 0))
    return y + c[:, None, None]


def avgpool2(x):
    C, H, Wd = x.shape
    if H % 2 or Wd % 2:
        raise ValueError("the U-Net needs even frame sizes")
    return x.reshape(C, H // 2, 2, Wd // 2, 2).mean(axis=(2, 4))


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def unet(layers, x):
    e1 = relu(conv(x, layers[0]))
    m = relu(conv(avgpool2(e1), layers[1]))
    e2 = relu(conv(np.concatenate([e1, upsample2(m)]), layers[2]))
    return conv(e2, layers[3])


def h_net(layers, b, sigma):
    z = relu(conv(np.concatenate([b, sigma]), layers[0]))
    z = relu(conv(z, layers[1]))
    return conv(z, layers[2])


def r_net(layers, phi, ld):
    z = relu(conv(np.concatenate([phi, ld]), layers[0]))
    z = relu(conv(z, layers[1]))
    return conv(z, layers[2])


def forward(w, W, gbuf, layers, scene, pool="mean", return_latents=False):
    """gbuf [n][14][H][W], layers [n][k][12][H][W], scene [n][16] -> y [n][3][H][W]."""
    P = unpack(w, W)
    g = np.asarray(gbuf, dtype=np.float64)
    L = np.asarray(layers, dtype=np.float64)
    s = np.asarray(scene, dtype=np.float64)
    n, _, H, Wd = g.shape
    k = L.shape[1]
    ys, lats = [], []
    for f in range(n):
        x = np.concatenate([g[f], np.broadcast_to(s[f][:, None, None], (NS, H, Wd))])
        sigma = unet(P["F"], x)
        S = np.zeros_like(sigma)
        cnt = np.zeros((H, Wd))
        for i in range(k):
            m = (L[f, i, 9] > 0.0).astype(np.float64)          # alpha > 0, per pixel
            S += m[None] * h_net(P["T"], L[f, i], sigma)
            cnt += m
        if pool == "sum":
            tau = S
        elif pool == "mean":
            tau = S / np.maximum(cnt, 1.0)[None]
        else:
            raise ValueError(pool)
        phi = unet(P["B"], np.concatenate([sigma, tau]))
        ys.append(r_net(P["R"], phi, g[f, 11:14]))
        lats.append(dict(sigma=sigma, tau=tau, phi=phi, count=cnt))
    y = np.stack(ys)
    return (y, lats) if return_latents else y


# ---------------------------------------------------------------- brute force
def forward_bruteforce(w, W, gbuf, layers, scene, pool="mean"):
    """Scalar loops over pixels, channels and taps (tiny inputs only)."""
    P = unpack(w, W)
    g = np.asarray(gbuf, dtype=np.float64)
    L = np.asarray(layers, dtype=np.float64)
    s = np.asarray(scene, dtype=np.float64)
    n, _, H, Wd = g.shape
    k = L.shape[1]

    def conv_s(img, layer, act):
        A, c = layer
        o, i, kk, _ = A.shape
        r = (kk - 1) // 2
        hh, ww = len(img[0]), len(img[0][0])
        out = [[[0.0] * ww for _ in range(hh)] for _ in range(o)]
        for oc in range(o):
            for y in range(hh):
                for x in range(ww):
                    acc = float(c[oc])
                    for ic in range(i):
                        for dy in range(kk):
                            for dx in range(kk):
                                yy, xx = y + dy - r, x + dx - r
                                if 0 <= yy < hh and 0 <= xx < ww:
                                    acc += float(A[oc, ic, dy, dx]) * img[ic][yy][xx]
                    out[oc][y][x] = max(acc, 0.0) if act else acc
        return out

    def pool2(img):
        return [[[(img[c][2 * y][2 * x] + img[c][2 * y][2 * x + 1] + img[c][2 * y + 1][2 * x]
                   + img[c][2 * y + 1][2 * x + 1]) / 4.0 for x in range(len(img[0][0]) // 2)]
                 for y in range(len(img[0]) // 2)] for c in range(len(img))]

    def up2(img):
        return [[[img[c][y // 2][x // 2] for x in range(2 * len(img[0][0]))]
                 for y in range(2 * len(img[0]))] for c in range(len(img))]

    def unet_s(layers_, x):
        e1 = conv_s(x, layers_[0], True)
        m = conv_s(pool2(e1), layers_[1], True)
        e2 = conv_s(e1 + up2(m), layers_[2], True)
        return conv_s(e2, layers_[3], False)

    y = np.zeros((n, NOUT, H, Wd))
    for f in range(n):
        x = [[[float(g[f, c, yy, xx]) for xx in range(Wd)] for yy in range(H)] for c in range(NG)]
        x += [[[float(s[f, c])] * Wd for _ in range(H)] for c in range(NS)]
        sigma = unet_s(P["F"], x)
        tau = [[[0.0] * Wd for _ in range(H)] for _ in range(W)]
        cnt = [[0] * Wd for _ in range(H)]
        for i in range(k):
            b = [[[float(L[f, i, c, yy, xx]) for xx in range(Wd)] for yy in range(H)]
                 for c in range(NL)]
            z = conv_s(b + sigma, P["T"][0], True)
            z = conv_s(z, P["T"][1], True)
            hi = conv_s(z, P["T"][2], False)
            for yy in range(H):
                for xx in range(Wd):
                    if b[9][yy][xx] > 0.0:
                        cnt[yy][xx] += 1
                        for c in range(W):
                            tau[c][yy][xx] += hi[c][yy][xx]
        if pool == "mean":
            for c in range(W):
                for yy in range(H):
                    for xx in range(Wd):
                        if cnt[yy][xx] > 0:
                            tau[c][yy][xx] /= cnt[yy][xx]
        phi = unet_s(P["B"], sigma + tau)
        ld = [[[float(g[f, 11 + c, yy, xx]) for xx in range(Wd)] for yy in range(H)]
              for c in range(3)]
        z = conv_s(phi + ld, P["R"][0], True)
        z = conv_s(z, P["R"][1], True)
        out = conv_s(z, P["R"][2], False)
        y[f] = np.asarray(out)
    return y
