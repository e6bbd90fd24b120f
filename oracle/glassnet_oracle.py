"""FP64 CPU oracle for GlassNet's per-pixel evaluation.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The HIP library never calls it and shares no code with it.

What is computed (Zhang & Simo-Serra, "Neural Scene Baking for Permutation
Invariant Transparency Rendering with Real-time Global Illumination"):

  Sec. 3.4  F, the scene encoder, maps the opaque G-buffer plus the variable
            scene parameters to the scene representation sigma.
  Sec. 3.3, Eq. (5)
            tau = g(h(b_1, sigma), ..., h(b_t, sigma)) with g = addition: one
            network h shared by every transparency buffer b_i, followed by a
            symmetric pool, hence permutation invariant.
  Sec. 3.4  B blends sigma and tau into the neural buffer phi; R maps phi and
            the direct light L_d to the output radiance.
  Sec. 3.5  Training uses an L1 term (the SSIM term is not part of this oracle).

Readings where the paper leaves details open (each listed in the design notes):
  * every network is a per-pixel 3-layer MLP (Linear-ReLU-Linear-ReLU-Linear),
    hidden and latent width W, R has 3 linear outputs;
  * h takes the concatenation [b_i ; sigma] (slot channels first);
  * slot i participates iff alpha_i > 0 (hard mask, no gradient through it);
  * pool "sum" is Eq. (5) literally; pool "mean" divides by max(#active, 1);
    no active slot gives tau = 0;
  * B takes [sigma ; tau]; R takes [phi ; L_d] with L_d = G-buffer planes 11..13;
  * L1 loss = mean |y - t| over every output element, with subgradient 0 at
    y == t and ReLU'(0) = 0;
  * positional encoding (Sec. 3.4 encodes every input; the frequency count is
    not given): with L levels, an input vector x becomes
    [x; sin(pi x); cos(pi x); sin(2 pi x); cos(2 pi x); ...;
     sin(2^(L-1) pi x); cos(2^(L-1) pi x)], blocks of the raw width in that
    order.  It applies to F's input [G; s] and to h's slot input b_i; sigma
    (internal) and R's L_d stay raw, and the mask reads the raw alpha.  L = 0
    is the unencoded network of the workloads.

Everything is evaluated in float64 from the float32 inputs, literally in the
order above: no hoisting of sigma out of h, no fusion.  `forward_bruteforce`
is a scalar Python-loop twin used to pin `forward` on tiny inputs.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

NG, NL, NS, NOUT = 14, 12, 16, 3
NETS = ("F", "T", "B", "R")


def encode(x, levels):
    """Positional encoding of the rows of x [C, P] -> [(1 + 2 levels) C, P]."""
    x = np.asarray(x, dtype=np.float64)
    blocks = [x]
    for k in range(levels):
        arg = np.pi * (2.0 ** k) * x
        blocks.append(np.sin(arg))
        blocks.append(np.cos(arg))
    return np.concatenate(blocks, axis=0)


def _shapes(W, pe_levels=0):
    e = 1 + 2 * pe_levels
    fan_in = {"F": ((NG + NS) * e, W, W), "T": (NL * e + W, W, W), "B": (2 * W, W, W),
              "R": (W + 3, W, W)}
    fan_out = {"F": (W, W, W), "T": (W, W, W), "B": (W, W, W), "R": (W, W, NOUT)}
    return fan_in, fan_out


def n_params(W: int, pe_levels: int = 0) -> int:
    fi, fo = _shapes(W, pe_levels)
    return sum(fo[n][j] * fi[n][j] + fo[n][j] for n in NETS for j in range(3))


def unpack(w, W: int, pe_levels: int = 0):
    """Flat float vector -> {net: [(A1, c1), (A2, c2), (A3, c3)]} in float64.

    Order: nets F, T, B, R; layers 1..3; matrix row-major [out][in], then bias.
    """
    w = np.asarray(w, dtype=np.float64).ravel()
    if w.size != n_params(W, pe_levels):
        raise ValueError(f"expected {n_params(W, pe_levels)} weights for W={W}, "
                         f"{pe_levels} encoding levels, got {w.size}")
    fi, fo = _shapes(W, pe_levels)
    out, off = {}, 0
    for net in NETS:
        layers = []
        for j in range(3):
            o, i = fo[net][j], fi[net][j]
            A = w[off:off + o * i].reshape(o, i)
            off += o * i
            c = w[off:off + o]
            off += o
            layers.append((A, c))
        out[net] = layers
    return out


def pack(params) -> np.ndarray:
    """Inverse of `unpack` (used to build gradients in the same layout)."""
    parts = []
    for net in NETS:
        for A, c in params[net]:
            parts.append(np.asarray(A, dtype=np.float64).ravel())
            parts.append(np.asarray(c, dtype=np.float64).ravel())
    return np.concatenate(parts)


def _relu(x):
    return np.maximum(x, 0.0)


def _mlp(layers, x):
    """x: [in, P] -> [out, P]; ReLU after layers 1 and 2, none after layer 3."""
    (A1, c1), (A2, c2), (A3, c3) = layers
    a = _relu(A1 @ x + c1[:, None])
    a = _relu(A2 @ a + c2[:, None])
    return A3 @ a + c3[:, None]


def _pixels(gbuf, layers, scene):
    """Flatten frames to pixel columns.  Returns G [14,P], L [k,12,P], S [16,P]."""
    g = np.asarray(gbuf, dtype=np.float64)
    L = np.asarray(layers, dtype=np.float64)
    s = np.asarray(scene, dtype=np.float64)
    n, _, h, w = g.shape
    k = L.shape[1]
    G = np.moveaxis(g, 1, 0).reshape(NG, n * h * w)
    Lp = np.moveaxis(L, (1, 2), (0, 1)).reshape(k, NL, n * h * w)
    S = np.repeat(s.T, h * w, axis=1)  # [16, P]
    return G, Lp, S, (n, h, w)


def _forward_cols(P, G, L, S, W, pool, keep=False, pe=0):
    """Column-wise forward over pixels.  P = unpacked params."""
    x = encode(np.concatenate([G, S], axis=0), pe)          # [30 (1 + 2 pe), P]
    sigma = _mlp(P["F"], x)                                 # [W, P]
    k = L.shape[0]
    Ssum = np.zeros_like(sigma)
    cnt = np.zeros(sigma.shape[1])
    for i in range(k):
        b = L[i]                                            # [12, P]
        h = _mlp(P["T"], np.concatenate([encode(b, pe), sigma], axis=0))  # Eq. (5): h(b_i, sigma)
        m = (b[9] > 0.0).astype(np.float64)                 # alpha > 0
        Ssum += m[None, :] * h
        cnt += m
    if pool == "sum":
        tau = Ssum
    elif pool == "mean":
        tau = Ssum / np.maximum(cnt, 1.0)[None, :]
    else:
        raise ValueError(pool)
    phi = _mlp(P["B"], np.concatenate([sigma, tau], axis=0))
    y = _mlp(P["R"], np.concatenate([phi, G[11:14]], axis=0))
    if keep:
        return y, dict(sigma=sigma, tau=tau, phi=phi, count=cnt, S=Ssum)
    return y


def forward(w, W, gbuf, layers, scene, pool="mean", chunk=16384, return_latents=False,
            pe_levels=0):
    """Vectorised FP64 forward.  Returns y [n][3][h][w] (float64).

    With return_latents=True also returns dict of sigma, tau, phi [n][W][h][w]
    and the active count [n][h][w].
    """
    P = unpack(w, W, pe_levels)
    G, L, S, (n, h, wd) = _pixels(gbuf, layers, scene)
    npx = G.shape[1]
    y = np.empty((NOUT, npx))
    lat = {key: np.empty((W, npx)) for key in ("sigma", "tau", "phi", "S")}
    lat["count"] = np.empty(npx)
    for a in range(0, npx, chunk):
        b = min(npx, a + chunk)
        if return_latents:
            yy, d = _forward_cols(P, G[:, a:b], L[:, :, a:b], S[:, a:b], W, pool, keep=True,
                                  pe=pe_levels)
            for key in lat:
                lat[key][..., a:b] = d[key]
        else:
            yy = _forward_cols(P, G[:, a:b], L[:, :, a:b], S[:, a:b], W, pool, pe=pe_levels)
        y[:, a:b] = yy

    def img(v):
        return np.moveaxis(v.reshape(v.shape[0], n, h, wd), 0, 1)

    out = img(y)
    if return_latents:
        lat_img = {key: img(v) for key, v in lat.items() if key != "count"}
        lat_img["count"] = lat["count"].reshape(n, h, wd)
        return out, lat_img
    return out


def forward_bruteforce(w, W, gbuf, layers, scene, pool="mean", pe_levels=0):
    """Scalar Python loops over pixels, slots and neurons (tiny inputs only)."""
    P = unpack(w, W, pe_levels)

    def enc(v):
        out = list(v)
        for k in range(pe_levels):
            f = math.pi * 2 ** k
            out += [math.sin(f * t) for t in v]
            out += [math.cos(f * t) for t in v]
        return out

    def dense(layer, v, act):
        A, c = layer
        res = []
        for r in range(A.shape[0]):
            acc = float(c[r])
            for q in range(A.shape[1]):
                acc += float(A[r, q]) * v[q]
            res.append(max(acc, 0.0) if act else acc)
        return res

    def net(name, v):
        v = dense(P[name][0], v, True)
        v = dense(P[name][1], v, True)
        return dense(P[name][2], v, False)

    g = np.asarray(gbuf, dtype=np.float64)
    L = np.asarray(layers, dtype=np.float64)
    s = np.asarray(scene, dtype=np.float64)
    n, _, h, wd = g.shape
    k = L.shape[1]
    y = np.zeros((n, NOUT, h, wd))
    for f in range(n):
        for r in range(h):
            for c in range(wd):
                gp = [float(g[f, ch, r, c]) for ch in range(NG)]
                sigma = net("F", enc(gp + [float(v) for v in s[f]]))
                tau = [0.0] * W
                active = 0
                for i in range(k):
                    b = [float(L[f, i, ch, r, c]) for ch in range(NL)]
                    if b[9] > 0.0:
                        hi = net("T", enc(b) + sigma)
                        tau = [t + v for t, v in zip(tau, hi)]
                        active += 1
                if pool == "mean" and active > 0:
                    tau = [t / active for t in tau]
                phi = net("B", sigma + tau)
                out = net("R", phi + gp[11:14])
                for ch in range(NOUT):
                    y[f, ch, r, c] = out[ch]
    return y


def l1_loss(y, target):
    """Sec. 3.5 L1 term: mean absolute error over every element, and dL/dy."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    d = y - t
    return float(np.abs(d).mean()), np.sign(d) / d.size


def _mlp_fwd_keep(layers, x):
    (A1, c1), (A2, c2), (A3, c3) = layers
    z1 = A1 @ x + c1[:, None]
    a1 = _relu(z1)
    z2 = A2 @ a1 + c2[:, None]
    a2 = _relu(z2)
    return A3 @ a2 + c3[:, None], (x, z1, a1, z2, a2)


def _mlp_bwd(layers, cache, dout, grads):
    """Backprop through one MLP.  Accumulates into grads [(dA, dc)]*3, returns dx."""
    (A1, _), (A2, _), (A3, _) = layers
    x, z1, a1, z2, a2 = cache
    grads[2][0] += dout @ a2.T
    grads[2][1] += dout.sum(axis=1)
    d = (A3.T @ dout) * (z2 > 0.0)
    grads[1][0] += d @ a1.T
    grads[1][1] += d.sum(axis=1)
    d = (A2.T @ d) * (z1 > 0.0)
    grads[0][0] += d @ x.T
    grads[0][1] += d.sum(axis=1)
    return A1.T @ d


def grad(w, W, gbuf, layers, scene, target, pool="mean", chunk=16384, pe_levels=0):
    """L1 loss and its gradient w.r.t. the flat weight vector (FP64 backprop).

    The transparency mask alpha > 0 is a hard selection (no gradient flows
    through it); gradients flow into sigma through every active slot's h.
    """
    return _backprop(w, W, gbuf, layers, scene, pool, chunk, target=target, pe=pe_levels)


def grad_from_dy(w, W, gbuf, layers, scene, dy, pool="mean", chunk=16384, pe_levels=0):
    """dL/dw for a given dL/dy [n][3][h][w] (the vector-Jacobian product)."""
    return _backprop(w, W, gbuf, layers, scene, pool, chunk, dy=dy, pe=pe_levels)[1]


def _backprop(w, W, gbuf, layers, scene, pool, chunk, target=None, dy=None, pe=0):
    P = unpack(w, W, pe)
    G, L, S, (n, h, wd) = _pixels(gbuf, layers, scene)
    if target is not None:
        t = np.asarray(target, dtype=np.float64)
        T = np.moveaxis(t, 1, 0).reshape(NOUT, -1)
    else:
        DY = np.moveaxis(np.asarray(dy, dtype=np.float64), 1, 0).reshape(NOUT, -1)
    npx = G.shape[1]
    total = NOUT * npx
    grads = {net: [[np.zeros_like(A), np.zeros_like(c)] for A, c in P[net]] for net in NETS}
    loss = 0.0
    for a0 in range(0, npx, chunk):
        b0 = min(npx, a0 + chunk)
        Gc, Lc, Sc = G[:, a0:b0], L[:, :, a0:b0], S[:, a0:b0]
        x = encode(np.concatenate([Gc, Sc], axis=0), pe)
        sigma, cF = _mlp_fwd_keep(P["F"], x)
        k = Lc.shape[0]
        Ssum = np.zeros_like(sigma)
        cnt = np.zeros(sigma.shape[1])
        cT, ms = [], []
        for i in range(k):
            hi, ci = _mlp_fwd_keep(P["T"], np.concatenate([encode(Lc[i], pe), sigma], axis=0))
            m = (Lc[i][9] > 0.0).astype(np.float64)
            Ssum += m[None, :] * hi
            cnt += m
            cT.append(ci)
            ms.append(m)
        if pool == "sum":
            tau, scale = Ssum, np.ones_like(cnt)
        else:
            scale = 1.0 / np.maximum(cnt, 1.0)
            tau = Ssum * scale[None, :]
        phi, cB = _mlp_fwd_keep(P["B"], np.concatenate([sigma, tau], axis=0))
        y, cR = _mlp_fwd_keep(P["R"], np.concatenate([phi, Gc[11:14]], axis=0))
        if target is not None:
            diff = y - T[:, a0:b0]
            loss += np.abs(diff).sum()
            dyc = np.sign(diff) / total
        else:
            dyc = DY[:, a0:b0]
        dR_in = _mlp_bwd(P["R"], cR, dyc, grads["R"])
        dphi = dR_in[:W]
        dB_in = _mlp_bwd(P["B"], cB, dphi, grads["B"])
        dsigma = dB_in[:W].copy()
        dS = dB_in[W:] * scale[None, :]
        for i in range(k):
            dh = dS * ms[i][None, :]
            dv = _mlp_bwd(P["T"], cT[i], dh, grads["T"])
            dsigma += dv[NL * (1 + 2 * pe):]
        _mlp_bwd(P["F"], cF, dsigma, grads["F"])
    flat = pack({net: [(gA, gc) for gA, gc in grads[net]] for net in NETS})
    return loss / total, flat


def relu_signature(w, W, gbuf, layers, scene, target, pool="mean", pe_levels=0):
    """Every branch decision of the loss (ReLU signs, slot masks, L1 signs).

    Two parameter vectors with equal signatures lie on the same smooth piece
    of the loss, where central finite differences are valid.
    """
    P = unpack(w, W, pe_levels)
    G, L, S, _ = _pixels(gbuf, layers, scene)
    T = np.moveaxis(np.asarray(target, dtype=np.float64), 1, 0).reshape(NOUT, -1)
    sig = []

    def run(name, x):
        out, (_, z1, _, z2, _) = _mlp_fwd_keep(P[name], x)
        sig.append(z1 > 0.0)
        sig.append(z2 > 0.0)
        return out

    x = encode(np.concatenate([G, S], axis=0), pe_levels)
    sigma = run("F", x)
    Ssum = np.zeros_like(sigma)
    cnt = np.zeros(sigma.shape[1])
    for i in range(L.shape[0]):
        hi = run("T", np.concatenate([encode(L[i], pe_levels), sigma], axis=0))
        m = (L[i][9] > 0.0).astype(np.float64)
        Ssum += m * hi
        cnt += m
    tau = Ssum if pool == "sum" else Ssum / np.maximum(cnt, 1.0)
    phi = run("B", np.concatenate([sigma, tau], axis=0))
    y = run("R", np.concatenate([phi, G[11:14]], axis=0))
    sig.append(y > T)
    return np.concatenate([s.ravel() for s in sig])


def relu_margins(w, W, gbuf, layers, scene, pool="mean", pe_levels=0):
    """Per pixel, how far every ReLU input lies from the kink at 0.

    For each hidden pre-activation z = a . x + c of F, of h for every active
    slot, of B and of R, the ratio |z| / (|a| . |x| + |c|) is the relative
    distance from the kink measured against the absolute-value sum that
    bounds the rounding error of evaluating z.  Returns the minimum ratio per
    pixel, shape [n, h, w].  Where it is of the order of the working
    precision's unit roundoff, a lower-precision evaluation may take the other
    branch of ReLU' (a different but equally valid subgradient choice), so
    gradient parity is only meaningful away from such pixels.
    """
    P = unpack(w, W, pe_levels)
    G, L, S, (n, h, wd) = _pixels(gbuf, layers, scene)
    marg = np.full(G.shape[1], np.inf)

    def run(name, x, active=None):
        nonlocal marg
        (A1, c1), (A2, c2), (A3, c3) = P[name]
        z1 = A1 @ x + c1[:, None]
        a1 = _relu(z1)
        z2 = A2 @ a1 + c2[:, None]
        for z, A, c, v in ((z1, A1, c1, x), (z2, A2, c2, a1)):
            r = (np.abs(z) / (np.abs(A) @ np.abs(v) + np.abs(c)[:, None] + 1e-300)).min(axis=0)
            if active is not None:
                r = np.where(active, r, np.inf)
            marg = np.minimum(marg, r)
        return A3 @ _relu(z2) + c3[:, None]

    sigma = run("F", encode(np.concatenate([G, S], axis=0), pe_levels))
    Ssum = np.zeros_like(sigma)
    cnt = np.zeros(sigma.shape[1])
    for i in range(L.shape[0]):
        m = L[i][9] > 0.0
        hi = run("T", np.concatenate([encode(L[i], pe_levels), sigma], axis=0), active=m)
        Ssum += m * hi
        cnt += m
    tau = Ssum if pool == "sum" else Ssum / np.maximum(cnt, 1.0)
    phi = run("B", np.concatenate([sigma, tau], axis=0))
    run("R", np.concatenate([phi, G[11:14]], axis=0))
    return marg.reshape(n, h, wd)


SSIM_K1, SSIM_K2, SSIM_RANGE, SSIM_SIZE, SSIM_SIGMA = 0.01, 0.03, 1.0, 11, 1.5


def ssim_window():
    """Wang et al.'s 11 x 11 Gaussian window, sigma 1.5, normalised to sum 1."""
    r = np.arange(SSIM_SIZE) - (SSIM_SIZE - 1) / 2.0
    g = np.exp(-r * r / (2.0 * SSIM_SIGMA ** 2))
    G = np.outer(g, g)
    return G / G.sum()


def _local(img, G):
    """Gaussian-weighted local mean over every fully contained window ('valid')."""
    win = np.lib.stride_tricks.sliding_window_view(img, G.shape)
    return np.einsum("abij,ij->ab", win, G)


def ssim_map(x, y):
    """SSIM index map of two single-channel images (Wang et al. 2004, the
    paper's loss term, Sec. 3.5): local Gaussian statistics, then
    ((2 mx my + C1)(2 sxy + C2)) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2))
    with C1 = (0.01 L)^2, C2 = (0.03 L)^2 and dynamic range L = 1."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    G = ssim_window()
    C1, C2 = (SSIM_K1 * SSIM_RANGE) ** 2, (SSIM_K2 * SSIM_RANGE) ** 2
    mx, my = _local(x, G), _local(y, G)
    sxx = _local(x * x, G) - mx * mx
    syy = _local(y * y, G) - my * my
    sxy = _local(x * y, G) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def dssim_loss(out, target):
    """Structural dissimilarity term of the loss (Sec. 3.5; the ablation's
    DSSIM): (1 - mean SSIM) / 2 over every valid window of every channel of
    every frame of [n][3][h][w] images, and its gradient w.r.t. out.

    The gradient is the chain rule through the local statistics: with
    S = A1 A2 / (B1 B2), A1 = 2 mx my + C1, A2 = 2 (E[xy] - mx my) + C2,
    B1 = mx^2 + my^2 + C1, B2 = E[x^2] - mx^2 + E[y^2] - my^2 + C2, the partial
    derivatives of S with respect to mx, E[x^2] and E[xy] at each window are
    spread back over the window's pixels by its Gaussian weights.
    """
    out = np.asarray(out, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    G = ssim_window()
    C1, C2 = (SSIM_K1 * SSIM_RANGE) ** 2, (SSIM_K2 * SSIM_RANGE) ** 2
    n, c, h, w = out.shape
    k = SSIM_SIZE
    if h < k or w < k:
        raise ValueError("images smaller than the SSIM window")
    count = n * c * (h - k + 1) * (w - k + 1)
    total = 0.0
    grad = np.zeros_like(out)
    for f in range(n):
        for ch in range(c):
            x, y = out[f, ch], target[f, ch]
            mx, my = _local(x, G), _local(y, G)
            ex2, ey2, exy = _local(x * x, G), _local(y * y, G), _local(x * y, G)
            A1 = 2 * mx * my + C1
            A2 = 2 * (exy - mx * my) + C2
            B1 = mx * mx + my * my + C1
            B2 = (ex2 - mx * mx) + (ey2 - my * my) + C2
            S = A1 * A2 / (B1 * B2)
            total += S.sum()
            dmx = S * (2 * my / A1 - 2 * my / A2 - 2 * mx / B1 + 2 * mx / B2)
            dex2 = -S / B2
            dexy = 2 * S / A2
            # scatter each window's partials back over its pixels
            for i in range(k):
                for j in range(k):
                    sl = (slice(i, i + h - k + 1), slice(j, j + w - k + 1))
                    grad[f, ch][sl] += G[i, j] * (dmx + 2 * x[sl] * dex2 + y[sl] * dexy)
    loss = (1.0 - total / count) / 2.0
    return loss, -grad / (2.0 * count)


def adam_step(w, g, m, v, t, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One optimiser step (Sec. 4: Adam with weight decay), float64.

    Kingma & Ba's update in its published order: biased first and second
    moment estimates, their bias corrections for step t >= 1, then the
    parameter step.  Weight decay is read as an L2 term added to the gradient
    first (the coupled form).  Returns the new (w, m, v).
    """
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64) + weight_decay * w
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def alpha_blend(colors, alphas):
    """Order-dependent alpha compositing of Eqs. (3)-(4), front-to-back.

    colors [t][...], alphas [t][...]; slot 0 is the front-most surface and
    z_i is the transmittance of the surfaces in front of slot i.
    """
    colors = np.asarray(colors, dtype=np.float64)
    alphas = np.asarray(alphas, dtype=np.float64)
    out = np.zeros(colors.shape[1:])
    trans = np.ones(alphas.shape[1:])
    for i in range(colors.shape[0]):
        out = out + alphas[i] * colors[i] * trans
        trans = trans * (1.0 - alphas[i])
    return out


def all_slot_orders(k):
    """Every permutation of k slots (small k only)."""
    return list(itertools.permutations(range(k)))
