"""Element-wise error bounds of the surrogate's device arithmetic against the
FP64 reference (imported by test modules only).

The device network stores its matrices (W1b, W1d, W2, W3), its dense inputs
and its hidden activations in BF16, accumulates in FP32 and keeps biases and
the output layer in FP32; the backward pass stores dz3, dz2 and dz1 in BF16.
The FP64 reference (oracle/mlp.py) evaluates the same function on the same
BF16 values, rounding the hidden activations where the device stores them.
Every device quantity then differs from the reference's only by

  * FP32 sums and products of the same values: a dot product or sum of n
    terms is off by at most gamma(n) sum |terms|, gamma(n) = n u / (1 - n u),
    u = 2^-24, in any order of summation;
  * BF16 roundings (RNE, unit roundoff 2^-8) of values that differ: since
    bf16(relu(.)) and bf16(.) are monotone, a value known to lie in
    [z - E, z + E] rounds into [bf16(z - E), bf16(z + E)], which is usually
    a single BF16 value (no difference at all) and one BF16 step where the
    interval straddles a rounding point;
  * ReLU masks that may flip where the interval straddles zero.

The bounds below propagate these intervals layer by layer, element by
element, in FP64 with absolute values.  They use the reference's values
(never the device's) and hold for any summation order.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
TINY = 1e-30     # absorbs flushed subnormal operands


def gamma(n: int) -> float:
    return n * U32 / (1.0 - n * U32)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even) through FP32, as float64."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def _fl32_interval(z, E):
    """[lo, hi] containing every FP32 value within E of z (z's own FP32
    rounding included)."""
    w = E + np.abs(z) * U32 + TINY
    return z - w, z + w


def act_interval(z, E):
    """Bound of |bf16(relu(z_dev)) - bf16(relu(z))| for |z_dev - z| <= E
    (z_dev an FP32 value); also returns whether the ReLU mask may differ."""
    lo, hi = _fl32_interval(z, E)
    ref = bf16(np.maximum(z, 0.0))
    a_lo, a_hi = bf16(np.maximum(lo, 0.0)), bf16(np.maximum(hi, 0.0))
    err = np.maximum(np.abs(a_hi - ref), np.abs(ref - a_lo))
    flip = (lo <= 0.0) & (hi > 0.0)
    return err, flip


def masked_bf16_interval(g, Eg, mask_ref, mask_flip):
    """Bound of |dev - ref| for dev = bf16(g_dev) * mask_dev against
    ref = g * mask_ref (unrounded), |g_dev - g| <= Eg, where the device mask
    equals mask_ref unless mask_flip."""
    lo, hi = _fl32_interval(g, Eg)
    r = np.where(mask_ref, g, 0.0)
    d_on = np.maximum(np.abs(bf16(hi) - r), np.abs(r - bf16(lo)))
    d_off = np.abs(r)
    return np.where(mask_flip, np.maximum(d_on, d_off), np.where(mask_ref, d_on, d_off))


def forward_bounds(q, rows, dense, cache):
    """Per-element bounds of the device forward against the reference with
    BF16-rounded activations.  q: parameters as the device uses them (BF16
    matrices, FP32 biases and output layer, in float64); rows: bit lists;
    dense: BF16 values [B, d]; cache: oracle.mlp.forward's cache (z1..h3).
    Returns dict with E_z1..E_z3, E_h1..E_h3, flip1..flip3 and E_y."""
    B = len(rows)
    H = q["b1"].shape[0]
    d = dense.shape[1] if dense.ndim == 2 else 0
    out = {}
    # layer 1: zd = dense W1d on the MFMA (exact products, FP32 sum over d),
    # then b1 + zd + the row's W1b entries summed one by one in FP32
    if d:
        zd = dense @ q["W1d"]
        Ezd = gamma(d) * (np.abs(dense) @ np.abs(q["W1d"]))
    else:
        zd = np.zeros((B, H))
        Ezd = np.zeros((B, H))
    mag = np.abs(q["b1"])[None, :] + np.abs(zd) + Ezd
    nb = np.array([len(r) for r in rows])
    for b in range(B):
        for i in rows[b]:
            mag[b] += np.abs(q["W1b"][int(i)])
    Ez1 = Ezd + gamma(nb.max() + 2) * mag
    Eh1, f1 = act_interval(cache["z1"], Ez1)
    out.update(E_z1=Ez1, E_h1=Eh1, flip1=f1)
    # layers 2 and 3: MFMA (exact BF16 products, FP32 sum over H) + bias
    h_prev, Eh_prev = cache["h1"], Eh1
    for l, (W, bias, z) in enumerate([(q["W2"], q["b2"], cache["z2"]),
                                      (q["W3"], q["b3"], cache["z3"])], start=2):
        aW = np.abs(W)
        Ez = Eh_prev @ aW + gamma(H + 1) * ((np.abs(h_prev) + Eh_prev) @ aW
                                            + np.abs(bias)[None, :])
        Eh, fl = act_interval(z, Ez)
        out.update({f"E_z{l}": Ez, f"E_h{l}": Eh, f"flip{l}": fl})
        h_prev, Eh_prev = cache[f"h{l}"], Eh
    # output layer: FP32 products and sums over H, + b4
    aW4 = np.abs(q["W4"])
    out["E_y"] = Eh_prev @ aW4 + gamma(H + 2) * ((np.abs(h_prev) + Eh_prev) @ aW4
                                                 + np.abs(q["b4"])[None, :]) + TINY
    return out


def gradient_bounds(q, rows, dense, cache, y, t, fb, d_bits):
    """Per-element bounds of the device gradients against oracle.mlp.backward
    on the same reference forward (y: reference outputs, t: targets, fb:
    forward_bounds).  Returns a dict keyed like the parameters."""
    B = y.shape[0]
    H = q["b1"].shape[0]
    d = dense.shape[1] if dense.ndim == 2 else 0
    aW4 = np.abs(q["W4"])
    # dy = (y - t) / B in FP32
    r = y - t
    Edy = (fb["E_y"] + 2 * U32 * (np.abs(r) + fb["E_y"])) / B + TINY
    dy = r / B
    G = {}
    # output layer weights: FP32 products, two-stage FP32 sums over the batch
    h3, Eh3 = cache["h3"], fb["E_h3"]
    G["W4"] = (Eh3.T @ np.abs(dy) + (np.abs(h3) + Eh3).T @ Edy
               + gamma(B + 2) * ((np.abs(h3) + Eh3).T @ (np.abs(dy) + Edy)))
    G["b4"] = Edy.sum(axis=0) + gamma(B + 1) * (np.abs(dy) + Edy).sum(axis=0)
    # dz3 = bf16(dy W4^T) where h3 > 0
    g3 = dy @ q["W4"].T
    Eg3 = Edy @ aW4.T + gamma(3) * ((np.abs(dy) + Edy) @ aW4.T)
    m3 = cache["z3"] > 0
    dz3 = np.where(m3, g3, 0.0)
    Edz3 = masked_bf16_interval(g3, Eg3, m3, fb["flip3"])
    layers = [("W3", "b3", "h2", "E_h2", "W3", "flip2", "z2"),
              ("W2", "b2", "h1", "E_h1", "W2", "flip1", "z1")]
    dz, Edz = dz3, Edz3
    for wname, bname, hname, ehname, wn, flipname, zname in layers:
        h, Eh = cache[hname], fb[ehname]
        # weight gradient h^T dz on the MFMA (BF16 operands: exact products)
        G[wname] = (Eh.T @ np.abs(dz) + (np.abs(h) + Eh).T @ Edz
                    + gamma(B) * ((np.abs(h) + Eh).T @ (np.abs(dz) + Edz)))
        G[bname] = Edz.sum(axis=0) + gamma(B + 1) * (np.abs(dz) + Edz).sum(axis=0)
        # next dz = bf16((dz W^T) * [h > 0])
        aW = np.abs(q[wn])
        gp = dz @ q[wn].T
        Egp = Edz @ aW.T + gamma(H) * ((np.abs(dz) + Edz) @ aW.T)
        m = cache[zname] > 0
        Edz_new = masked_bf16_interval(gp, Egp, m, fb[flipname])
        dz, Edz = np.where(m, gp, 0.0), Edz_new
    # layer 1: b1 and W1b from dz1 sums, W1d = dense^T dz1 on the MFMA
    G["b1"] = Edz.sum(axis=0) + gamma(B + 1) * (np.abs(dz) + Edz).sum(axis=0)
    Ew = np.zeros((d_bits, H))
    cnt = np.zeros(d_bits, np.int64)
    mag = np.zeros((d_bits, H))
    for b in range(B):
        for i in rows[b]:
            i = int(i)
            Ew[i] += Edz[b]
            mag[i] += np.abs(dz[b]) + Edz[b]
            cnt[i] += 1
    G["W1b"] = Ew + np.array([gamma(int(c) + 1) for c in cnt])[:, None] * mag
    if d:
        ad = np.abs(dense)
        G["W1d"] = ad.T @ Edz + gamma(B) * (ad.T @ (np.abs(dz) + Edz))
    else:
        G["W1d"] = np.zeros((0, H))
    return {k: v + TINY for k, v in G.items()}


def adam_bounds(p, g_dev, m, v, Em, Ev, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step, FP64, on the device's gradient g_dev, with per-element
    bounds of the device's FP32 step (FP32 master weights and moments, FP32
    constants beta1, beta2, 1 - beta^step from powf) against it.

    p, m, v: the reference's weights and moments (dicts of float64 arrays);
    Em, Ev: bounds of |m_dev - m|, |v_dev - v| before the step (zeros for a
    fresh optimiser).  Returns (p_new, m_new, v_new, Ew, Em_new, Ev_new), Ew
    bounding |w_dev - p_new| given a device weight equal to p before the
    step.  The FP32 constants are the roundings of 0.9 and 0.999; their
    relative offsets from the FP64 constants enter linearly, the bias
    corrections are taken good to 8 FP32 ulps."""
    b1f = float(np.float32(beta1))
    b2f = float(np.float32(beta2))
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    dc1 = abs((1.0 - b1f ** step) - c1) / c1 + 8 * U32 / c1
    dc2 = abs((1.0 - b2f ** step) - c2) / c2 + 8 * U32 / c2
    P, M, V, EW, EM, EV = {}, {}, {}, {}, {}, {}
    for k in p:
        gk = g_dev[k]
        mk = beta1 * m[k] + (1 - beta1) * gk
        vk = beta2 * v[k] + (1 - beta2) * gk * gk
        # device moments: b1f m_dev + (1 - b1f) g, three FP32 roundings
        em = (b1f * Em[k] + abs(b1f - beta1) * np.abs(m[k])
              + abs((1 - b1f) - (1 - beta1)) * np.abs(gk)
              + 3 * U32 * (np.abs(mk) + b1f * Em[k]))
        ev = (b2f * Ev[k] + abs(b2f - beta2) * v[k]
              + abs((1 - b2f) - (1 - beta2)) * gk * gk
              + 4 * U32 * (vk + b2f * Ev[k]))
        mh = mk / c1
        vh = vk / c2
        den = np.sqrt(vh) + eps
        upd = lr * mh / den
        # relative error of m-hat / (sqrt(v-hat) + eps): numerator and the
        # square root's argument perturbed, then five FP32 operations
        rm = (em / np.maximum(np.abs(mk), 1e-300)) + dc1 + U32
        rv = (ev / np.maximum(vk, 1e-300)) + dc2 + U32
        rq = rm + 0.5 * rv / (1.0 - rv) + 6 * U32
        upd_err = np.where(np.abs(mk) > 0, np.abs(upd) * rq,
                           lr * em / c1 / np.maximum(den - np.sqrt(ev / c2), eps))
        P[k] = p[k] - upd
        M[k], V[k] = mk, vk
        EW[k] = upd_err + 2 * U32 * (np.abs(p[k]) + np.abs(upd)) + TINY
        EM[k], EV[k] = em + TINY, ev + TINY
    return P, M, V, EW, EM, EV
