"""FP64 CPU oracle for the x2 super-sampling network.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The HIP library never calls it and shares no code with it.

What is computed (Sec. 3.4, end, and Sec. 4.1 of Zhang & Simo-Serra): GlassNet
renders at the training resolution, and a small multi-layer CNN raises its
result to twice that resolution, helped by textures and a G-buffer that the
rasterizer produces cheaply at the higher resolution.  The paper fixes neither
the layers nor the width; the readings (each listed in the design notes) are

  * input at the output resolution (2h x 2w): the rendered image upsampled x2
    bilinearly (sample centres at half-pixel offsets, sources clamped at the
    image edge), then the 14 G-buffer channels at full resolution: 17 channels;
  * conv 3x3 (17 -> 32) + ReLU, conv 3x3 (32 -> 32) + ReLU, conv 1x1 (32 -> 3),
    each 3x3 conv zero-padded to keep the size (the paper puts 1x1 kernels at
    the end of its rendering CNNs and larger kernels before them);
  * output = upsampled image + the last conv (a residual on the upsample);
  * weights packed as conv1 W [32][17][3][3], b [32]; conv2 W [32][32][3][3],
    b [32]; conv3 W [3][32], b [3]: 14,275 floats.

Everything is evaluated in float64 from the float32 inputs; a conv is the sum
over its taps of a channel matrix times the shifted zero-padded input.
"""
import numpy as np

SR_WIDTH = 32
SR_IN = 3 + 14
SR_OUT = 3


def sr_shapes(C=SR_WIDTH):
    """(name, shape) of each packed tensor, in packing order."""
    return [("w1", (C, SR_IN, 3, 3)), ("b1", (C,)), ("w2", (C, C, 3, 3)), ("b2", (C,)),
            ("w3", (SR_OUT, C)), ("b3", (SR_OUT,))]


def sr_n_params(C=SR_WIDTH) -> int:
    return int(sum(np.prod(s) for _, s in sr_shapes(C)))


def sr_unpack(w, C=SR_WIDTH):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == sr_n_params(C)
    out, o = {}, 0
    for name, shp in sr_shapes(C):
        n = int(np.prod(shp))
        out[name] = w[o:o + n].reshape(shp)
        o += n
    return out


def upsample2x(img):
    """Bilinear x2 of [..., h, w]: output sample (Y, X) sits at source position
    ((Y + 0.5) / 2 - 0.5, (X + 0.5) / 2 - 0.5); the two nearest source rows and
    columns (clamped into the image) are blended by the fractional distances."""
    img = np.asarray(img, dtype=np.float64)
    h, w = img.shape[-2:]

    def taps(n_out, n_in):
        s = (np.arange(n_out) + 0.5) / 2.0 - 0.5
        i0 = np.floor(s).astype(np.int64)
        f = s - i0
        return np.clip(i0, 0, n_in - 1), np.clip(i0 + 1, 0, n_in - 1), f

    y0, y1, fy = taps(2 * h, h)
    x0, x1, fx = taps(2 * w, w)
    rows = img[..., y0, :] * (1.0 - fy)[:, None] + img[..., y1, :] * fy[:, None]
    return rows[..., x0] * (1.0 - fx) + rows[..., x1] * fx


def conv3x3(x, W, b):
    """Zero-padded 'same' 3x3 convolution (cross-correlation, as CNN layers
    compute it) of x [cin][H][W] with W [cout][cin][3][3], plus b."""
    cin, H, Wd = x.shape
    xp = np.zeros((cin, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((W.shape[0], H, Wd)) + b[:, None, None]
    for dy in range(3):
        for dx in range(3):
            shifted = xp[:, dy:dy + H, dx:dx + Wd].reshape(cin, -1)
            y += (W[:, :, dy, dx] @ shifted).reshape(-1, H, Wd)
    return y


def sr_forward(w, lowres, gbuf_hi, C=SR_WIDTH):
    """lowres [n][3][h][w], gbuf_hi [n][14][2h][2w] -> [n][3][2h][2w]."""
    p = sr_unpack(w, C)
    lowres = np.asarray(lowres, dtype=np.float64)
    gbuf_hi = np.asarray(gbuf_hi, dtype=np.float64)
    n, _, h, wd = lowres.shape
    assert gbuf_hi.shape == (n, SR_IN - 3, 2 * h, 2 * wd)
    out = np.empty((n, SR_OUT, 2 * h, 2 * wd))
    for f in range(n):
        up = upsample2x(lowres[f])
        x = np.concatenate([up, gbuf_hi[f]], axis=0)
        a1 = np.maximum(conv3x3(x, p["w1"], p["b1"]), 0.0)
        a2 = np.maximum(conv3x3(a1, p["w2"], p["b2"]), 0.0)
        y = (p["w3"] @ a2.reshape(C, -1)).reshape(SR_OUT, 2 * h, 2 * wd) + p["b3"][:, None, None]
        out[f] = up + y
    return out


def conv3x3_backward(x, W, dz):
    """Gradients of conv3x3(x, W, b) for the upstream gradient dz [cout][H][W]:
    dW[o][c][dy][dx] = sum_p dz[o][p] xpad[c][p + (dy, dx)], db = sum_p dz,
    and dx, each padded input position collecting W[o][c][tap] dz[o][p] from
    every output p whose window holds it (the padding's share dropped)."""
    cin, H, Wd = x.shape
    cout = W.shape[0]
    xp = np.zeros((cin, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    d = dz.reshape(cout, -1)
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            dW[:, :, dy, dx] = d @ xp[:, dy:dy + H, dx:dx + Wd].reshape(cin, -1).T
            dxp[:, dy:dy + H, dx:dx + Wd] += (W[:, :, dy, dx].T @ d).reshape(cin, H, Wd)
    return dW, d.sum(axis=1), dxp[:, 1:-1, 1:-1]


def sr_grad(w, lowres, gbuf_hi, dy, C=SR_WIDTH):
    """Packed gradient of sum(dy * sr_forward(w, ...)) with respect to w: the
    chain rule through the head, conv2, its ReLU, conv1 and its ReLU (the
    derivative of ReLU taken as 0 at 0).  The residual and the inputs carry
    no weights."""
    p = sr_unpack(w, C)
    g = {k: np.zeros_like(v) for k, v in p.items()}
    lowres = np.asarray(lowres, dtype=np.float64)
    gbuf_hi = np.asarray(gbuf_hi, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    for f in range(lowres.shape[0]):
        x = np.concatenate([upsample2x(lowres[f]), gbuf_hi[f]], axis=0)
        H, Wd = x.shape[1:]
        z1 = conv3x3(x, p["w1"], p["b1"])
        a1 = np.maximum(z1, 0.0)
        z2 = conv3x3(a1, p["w2"], p["b2"])
        a2 = np.maximum(z2, 0.0)
        d = dy[f].reshape(SR_OUT, -1)
        g["w3"] += d @ a2.reshape(C, -1).T
        g["b3"] += d.sum(axis=1)
        dz2 = (p["w3"].T @ d).reshape(C, H, Wd) * (z2 > 0)
        dW2, db2, da1 = conv3x3_backward(a1, p["w2"], dz2)
        dz1 = da1 * (z1 > 0)
        dW1, db1, _ = conv3x3_backward(x, p["w1"], dz1)
        g["w2"] += dW2
        g["b2"] += db2
        g["w1"] += dW1
        g["b1"] += db1
    return np.concatenate([g[name].ravel() for name, _ in sr_shapes(C)])


def sr_forward_bruteforce(w, lowres, gbuf_hi, C=SR_WIDTH):
    """Scalar Python-loop twin of sr_forward for tiny inputs."""
    p = sr_unpack(w, C)
    n, _, h, wd = np.shape(lowres)
    H, Wd = 2 * h, 2 * wd

    def up(f, c, Y, X):
        def tap(i, n_in):
            s = (i + 0.5) / 2.0 - 0.5
            i0 = int(np.floor(s))
            return min(max(i0, 0), n_in - 1), min(max(i0 + 1, 0), n_in - 1), s - i0
        a0, a1, fy = tap(Y, h)
        c0, c1, fx = tap(X, wd)
        v = 0.0
        for r, wy in ((a0, 1 - fy), (a1, fy)):
            for q, wx in ((c0, 1 - fx), (c1, fx)):
                v += wy * wx * float(lowres[f][c][r][q])
        return v

    out = np.zeros((n, SR_OUT, H, Wd))
    for f in range(n):
        x = [[[up(f, c, Y, X) if c < 3 else float(gbuf_hi[f][c - 3][Y][X]) for X in range(Wd)]
              for Y in range(H)] for c in range(SR_IN)]
        a1 = [[[0.0] * Wd for _ in range(H)] for _ in range(C)]
        for o in range(C):
            for Y in range(H):
                for X in range(Wd):
                    s = p["b1"][o]
                    for c in range(SR_IN):
                        for dy in range(3):
                            for dx in range(3):
                                yy, xx = Y + dy - 1, X + dx - 1
                                if 0 <= yy < H and 0 <= xx < Wd:
                                    s += p["w1"][o, c, dy, dx] * x[c][yy][xx]
                    a1[o][Y][X] = max(s, 0.0)
        for Y in range(H):
            for X in range(Wd):
                a2 = []
                for o in range(C):
                    s = p["b2"][o]
                    for c in range(C):
                        for dy in range(3):
                            for dx in range(3):
                                yy, xx = Y + dy - 1, X + dx - 1
                                if 0 <= yy < H and 0 <= xx < Wd:
                                    s += p["w2"][o, c, dy, dx] * a1[c][yy][xx]
                    a2.append(max(s, 0.0))
                for k in range(SR_OUT):
                    out[f, k, Y, X] = x[k][Y][X] + p["b3"][k] + sum(p["w3"][k, o] * a2[o]
                                                                  for o in range(C))
    return out
