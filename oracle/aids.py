"""FP64 CPU oracle for the steps either side of the rasteriser that the paper uses to make the
fit work, and for its layer export (DiffBMP, arXiv 2602.22625):

  gaussian_blur          soft rasterisation: every bitmap blurred once before the fit
                         (Sec. 3.2.1; blur_sigma = 1 in Supp. Table S1)
  local_variance, nlv    structure-aware initialisation's complexity map: variance of the
                         target over a 7 x 7 window, normalised to [0, 1] (Sec. 3.2.2)
  sa_init                its sampler: lattice points with probability proportional to
                         0.1 + 0.9 NLV, scale s_max - (s_max - s_min) NLV, colour from the
                         target plus N(0, sigma_c^2) noise, fixed opacity logit, uniform angle
  philox4x64, noise_canvas  the uniform-noise background of Eq. (8), one draw per iteration
  constraint_loss        the spatial-constraint objective of Eq. (9) and its gradients
  reinit_transparent     re-initialisation of primitives whose opacity fell below a threshold
                         (Supp. Sec. S1.4.2)
  export_layers          one alpha layer per primitive at an export scale rho (Sec. 3.1.3 and
                         Supp. "PSD export")

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg are the only
callers. It shares no code with the GPU path. Random numbers the method draws are inputs here
(uniforms and normals passed by the caller), except the noise canvas, whose generator (Philox,
Salmon et al., SC 2011) is implemented from its published definition.

Readings of points the paper leaves open are stated in each function's docstring.
"""
from __future__ import annotations

import math

import numpy as np

# ------------------------------------------------------------------------------------------
# Soft rasterisation (Sec. 3.2.1)
# ------------------------------------------------------------------------------------------


def gaussian_weights(sigma=1.0, truncate=3.0):
    """Normalised 1-D Gaussian taps w(d) ~ exp(-d^2 / (2 sigma^2)), d = -r..r, with radius
    r = floor(truncate * sigma + 0.5). Reading: the paper gives only sigma; the window is cut at
    three standard deviations and renormalised."""
    r = int(truncate * sigma + 0.5)
    d = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-d * d / (2.0 * sigma * sigma))
    return w / w.sum(), r


def gaussian_blur(atlas, sigma=1.0, truncate=3.0):
    """Blurred bitmaps [B, Hb, Wb] (float64): out[y, x] = sum_{dy, dx} w(dy) w(dx) P[y+dy, x+dx],
    texels outside the bitmap read 0 (the sampler's zero padding). Reading: the bitmap keeps its
    size (its support and the primitive's footprint do not change); texels that the blur would
    carry past the border are dropped."""
    a = np.asarray(atlas, dtype=np.float64)
    if a.ndim == 2:
        a = a[None]
    w, r = gaussian_weights(sigma, truncate)
    B, Hb, Wb = a.shape
    pad = np.zeros((B, Hb + 2 * r, Wb + 2 * r))
    pad[:, r:r + Hb, r:r + Wb] = a
    out = np.zeros_like(a)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            out += w[dy + r] * w[dx + r] * pad[:, r + dy:r + dy + Hb, r + dx:r + dx + Wb]
    return out


# ------------------------------------------------------------------------------------------
# Structure-aware initialisation (Sec. 3.2.2)
# ------------------------------------------------------------------------------------------


def local_variance(img, win=7):
    """[H, W] map of the local variance of the target [3, H, W]: per channel, the (population)
    variance of the values in the win x win window centred on the pixel, then the mean over the
    three channels. Reading: the window is clipped at the image border (only pixels inside it
    count), and "across RGB channels" is the mean of the per-channel variances."""
    img = np.asarray(img, dtype=np.float64)
    _, H, W = img.shape
    h = win // 2
    out = np.zeros((H, W))
    for y in range(H):
        y0, y1 = max(0, y - h), min(H, y + h + 1)
        for x in range(W):
            x0, x1 = max(0, x - h), min(W, x + h + 1)
            blk = img[:, y0:y1, x0:x1].reshape(3, -1)
            mean = blk.mean(axis=1, keepdims=True)
            out[y, x] = np.mean(np.mean((blk - mean) ** 2, axis=1))
    return out


def nlv(lv):
    """Normalised local variance (LV - min) / (max - min), all zeros for a constant map."""
    lv = np.asarray(lv, dtype=np.float64)
    lo, hi = lv.min(), lv.max()
    if not hi > lo:
        return np.zeros_like(lv)
    return (lv - lo) / (hi - lo)


WEIGHT_BITS = 24  # sampling weights are integers w * 2^24 (exact cumulative sums)


def sampling_weights(nlv_map, base=0.1):
    """Integer weights floor((base + (1 - base) NLV) * 2^24) of every lattice point, row-major.
    Reading: the probability proportional to 0.1 + 0.9 NLV is quantised to 2^-24 of the largest
    weight, so that the cumulative sums that invert it are exact integers."""
    v = np.asarray(nlv_map, dtype=np.float64).reshape(-1)
    w = base + (1.0 - base) * v
    return np.floor(w * float(1 << WEIGHT_BITS)).astype(np.int64)


def sample_lattice(weights, u):
    """Inverse-CDF sampling: for each uniform u in [0, 1), the first lattice point p whose
    cumulative weight exceeds floor(u * total)."""
    cdf = np.cumsum(np.asarray(weights, dtype=np.int64))
    total = int(cdf[-1])
    t = np.floor(np.asarray(u, dtype=np.float64) * float(total)).astype(np.int64)
    return np.searchsorted(cdf, t, side="right")


def sa_init(nlv_map, img, u_pos, u_theta, z_col, s_min, s_max, nu_init=-2.0, sigma_c=0.02,
            base=0.1):
    """Primitive parameters [N, 8] (x, y, log s, theta, nu, colour logits) from the NLV map
    [H, W], the target [3, H, W] and the caller's random draws: u_pos, u_theta ~ U[0, 1) [N],
    z_col ~ N(0, 1) [N, 3].
      position  the sampled lattice point (x, y) = (p mod W, p div W)
      scale     s = s_max - (s_max - s_min) NLV(x, y)          (learned as log s)
      angle     theta = 2 pi u_theta
      colour    c_hat = clip(I(x, y) + sigma_c z, 1e-3, 1 - 1e-3), logit c = log(c / (1 - c))
      opacity   nu = nu_init (Sec. 3.2.2 fixes -2; Supp. Table S1 lists -4: an input here)"""
    nlv_map = np.asarray(nlv_map, dtype=np.float64)
    img = np.asarray(img, dtype=np.float64)
    H, W = nlv_map.shape
    p = sample_lattice(sampling_weights(nlv_map, base), u_pos)
    x, y = p % W, p // W
    n = nlv_map.reshape(-1)[p]
    s = s_max - (s_max - s_min) * n
    out = np.zeros((len(p), 8))
    out[:, 0] = x
    out[:, 1] = y
    out[:, 2] = np.log(s)
    out[:, 3] = 2.0 * math.pi * np.asarray(u_theta, dtype=np.float64)
    out[:, 4] = nu_init
    ch = img[:, y, x].T + sigma_c * np.asarray(z_col, dtype=np.float64)
    ch = np.clip(ch, 1e-3, 1.0 - 1e-3)
    out[:, 5:8] = np.log(ch / (1.0 - ch))
    return out


# ------------------------------------------------------------------------------------------
# Noise canvas (Eq. 8): Philox4x64-10 counter-based generator
# ------------------------------------------------------------------------------------------
_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def philox4x64(counter, key, rounds=10):
    """Philox4x64-R (Salmon, Moraes, Dror, Shaw, SC 2011): 4 x 64-bit counter, 2 x 64-bit key.
    Each round multiplies words 0 and 2 by the constants M0, M1 (128-bit products), mixes the
    high halves with the other words and the key, and the key is bumped by the Weyl constants
    between rounds."""
    c = [int(v) & _MASK for v in counter]
    k = [int(v) & _MASK for v in key]
    for _ in range(rounds):
        p0, p1 = _M0 * c[0], _M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & _MASK, (p0 >> 64) ^ c[3] ^ k[1], p0 & _MASK]
        k = [(k[0] + _W0) & _MASK, (k[1] + _W1) & _MASK]
    return c


def u01_from_u64(x):
    """Uniform float32 in [0, 1) from the top 24 bits of a 64-bit word (exact in float32)."""
    return float(int(x) >> 40) * 2.0 ** -24


def noise_canvas(H, W, seed, iteration):
    """[3, H, W] background b ~ U[0, 1)^3 per pixel for one iteration (Eq. 8): pixel p of
    iteration t uses the Philox block with counter (p, t, 0, 0) and key (seed, 0); its words
    0, 1, 2 give the red, green and blue values."""
    out = np.zeros((3, H, W))
    for p in range(H * W):
        w = philox4x64((p, iteration, 0, 0), (seed, 0))
        for ch in range(3):
            out[ch, p // W, p % W] = u01_from_u64(w[ch])
    return out


# ------------------------------------------------------------------------------------------
# Spatial constraint (Eq. 9) and re-initialisation (Supp. Sec. S1.4.2)
# ------------------------------------------------------------------------------------------


def constraint_loss(I, A, target, target_alpha, lam):
    """Eq. (9): L = mean over 3HW of [A_t > 0] (I - I_t)^2 + lam * mean over HW of (A - A_t)^2.
    Reading: the squared norms are taken as means (the `mse` convention of Supp. Table S1).
    Returns (L, dL/dI [3, H, W], dL/dA [H, W])."""
    I = np.asarray(I, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    ta = np.asarray(target_alpha, dtype=np.float64)
    m = (ta > 0).astype(np.float64)
    d = m[None] * (I - t)
    e = A - ta
    L = float(np.sum(d * d) / I.size + lam * np.sum(e * e) / A.size)
    return L, 2.0 * d / I.size, 2.0 * lam * e / A.size


def reinit_transparent(params, m, v, proposal, threshold=0.3):
    """Rows whose opacity sigmoid(nu) is below the threshold take the proposal's row (a fresh
    structure-aware draw) and restart their Adam moments at zero; returns (params, m, v, count).
    Reading: the moments of a re-initialised primitive restart, as for a new parameter."""
    params = np.array(params, dtype=np.float64, copy=True)
    m = np.array(m, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    sel = 1.0 / (1.0 + np.exp(-params[:, 4])) < threshold
    params[sel] = np.asarray(proposal, dtype=np.float64)[sel]
    m[sel] = 0.0
    v[sel] = 0.0
    return params, m, v, int(sel.sum())


# ------------------------------------------------------------------------------------------
# Layer export (Sec. 3.1.3, Supp. "PSD export")
# ------------------------------------------------------------------------------------------


def export_alpha(p, bitmap, X, Y, rho, alpha_max=1.0):
    """Alpha of one primitive (parameter row p) at export pixels (X, Y) of the canvas scaled by
    rho: the export pixel centre sits at canvas point ((X + 0.5) / rho - 0.5, (Y + 0.5) / rho -
    0.5) (reading: the export grid covers the same canvas, rho x rho export pixels per pixel),
    then Eqs. (1)-(3) with zero padding outside the bitmap."""
    bm = np.asarray(bitmap, dtype=np.float64)
    Hb, Wb = bm.shape
    x = (np.asarray(X, dtype=np.float64) + 0.5) / rho - 0.5
    y = (np.asarray(Y, dtype=np.float64) + 0.5) / rho - 0.5
    s = math.exp(p[2])
    ct, st = math.cos(p[3]), math.sin(p[3])
    dx, dy = x - p[0], y - p[1]
    U = ((ct * dx + st * dy) / s + 1.0) / 2.0 * (Wb - 1)
    V = ((-st * dx + ct * dy) / s + 1.0) / 2.0 * (Hb - 1)
    u0, v0 = np.floor(U), np.floor(V)
    wu, wv = U - u0, V - v0
    iu, iv = u0.astype(np.int64), v0.astype(np.int64)

    def tex(r, c):
        ok = (r >= 0) & (r < Hb) & (c >= 0) & (c < Wb)
        return np.where(ok, bm[np.clip(r, 0, Hb - 1), np.clip(c, 0, Wb - 1)], 0.0)

    M = ((1 - wu) * (1 - wv) * tex(iv, iu) + wu * (1 - wv) * tex(iv, iu + 1)
         + (1 - wu) * wv * tex(iv + 1, iu) + wu * wv * tex(iv + 1, iu + 1))
    return alpha_max / (1.0 + math.exp(-p[4])) * M


def export_layers(params, idx, atlas, H, W, rho, alpha_max=1.0):
    """Per primitive: (bbox (x0, y0, w, h) of the export pixels where its alpha is non-zero,
    found by testing every export pixel; the alpha over that box; its colour sigmoid(c)).
    An empty layer has w = h = 0."""
    params = np.asarray(params, dtype=np.float64).reshape(-1, 8)
    atlas = np.asarray(atlas, dtype=np.float64)
    if atlas.ndim == 2:
        atlas = atlas[None]
    HH, WW = int(round(H * rho)), int(round(W * rho))
    Y, X = np.meshgrid(np.arange(HH), np.arange(WW), indexing="ij")
    out = []
    for k in range(params.shape[0]):
        a = export_alpha(params[k], atlas[int(idx[k])], X, Y, rho, alpha_max)
        nz = np.argwhere(a != 0.0)
        col = 1.0 / (1.0 + np.exp(-params[k, 5:8]))
        if len(nz) == 0:
            out.append(((0, 0, 0, 0), np.zeros((0, 0)), col))
            continue
        y0, x0 = nz.min(axis=0)
        y1, x1 = nz.max(axis=0)
        out.append(((int(x0), int(y0), int(x1 - x0 + 1), int(y1 - y0 + 1)),
                    a[y0:y1 + 1, x0:x1 + 1].copy(), col))
    return out
