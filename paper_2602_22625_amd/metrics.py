"""Host-side measurement helpers (NumPy, float64), independent of the GPU path.

support_pairs: exact count of (pixel, primitive) pairs at which the primitive's bilinear
footprint reads at least one texel inside its bitmap (Eq. 1-2: floor(U) in [-1, Wb-1] and
floor(V) in [-1, Hb-1]), or, with `tight`, at least one NON-ZERO texel (floor(U) in
[xlo-1, xhi], floor(V) in [ylo-1, yhi] for the bitmap's non-zero box). The tight count is the
work the rasteriser performs; outside it M and its derivatives are exactly zero.
"""
from __future__ import annotations

import math

import numpy as np


def nonzero_boxes(atlas: np.ndarray):
    """[B, 4] int: xlo, xhi, ylo, yhi of the non-zero texels of each bitmap (xlo > xhi: empty)."""
    atlas = np.asarray(atlas)
    if atlas.ndim == 2:
        atlas = atlas[None]
    out = np.zeros((atlas.shape[0], 4), dtype=np.int64)
    for b in range(atlas.shape[0]):
        nz = np.nonzero(atlas[b] != 0)
        if len(nz[0]) == 0:
            out[b] = (1, 0, 1, 0)
        else:
            out[b] = (nz[1].min(), nz[1].max(), nz[0].min(), nz[0].max())
    return out


def support_pairs(params, Hb, Wb, H, W, crop=None, idx=None, boxes=None):
    """Count as described in the module docstring. `boxes` (from nonzero_boxes) together with
    `idx` selects the tight count."""
    p = np.asarray(params, dtype=np.float64).reshape(-1, 8)
    x0, y0, w, h = crop if crop is not None else (0, 0, W, H)
    cu, cv = 0.5 * (Wb - 1), 0.5 * (Hb - 1)
    total = 0
    for k in range(p.shape[0]):
        if boxes is not None:
            xlo, xhi, ylo, yhi = boxes[int(idx[k])]
            if xlo > xhi:
                continue
            ulo, uhi, vlo, vhi = xlo - 1, xhi, ylo - 1, yhi
        else:
            ulo, uhi, vlo, vhi = -1, Wb - 1, -1, Hb - 1
        s = math.exp(p[k, 2])
        ct, st = math.cos(p[k, 3]), math.sin(p[k, 3])
        # bounding box of the parallelogram floor(U) in [ulo, uhi], floor(V) in [vlo, vhi]
        us = [ulo, uhi + 1]
        vs = [vlo, vhi + 1]
        xs, ys = [], []
        for U in us:
            for V in vs:
                u, v = U / cu - 1.0, V / cv - 1.0
                xs.append(p[k, 0] + s * (ct * u - st * v))
                ys.append(p[k, 1] + s * (st * u + ct * v))
        ax0 = max(int(math.floor(min(xs))) - 1, x0)
        ax1 = min(int(math.ceil(max(xs))) + 1, x0 + w - 1)
        ay0 = max(int(math.floor(min(ys))) - 1, y0)
        ay1 = min(int(math.ceil(max(ys))) + 1, y0 + h - 1)
        if ax0 > ax1 or ay0 > ay1:
            continue
        X = np.arange(ax0, ax1 + 1, dtype=np.float64)[None, :] - p[k, 0]
        Y = np.arange(ay0, ay1 + 1, dtype=np.float64)[:, None] - p[k, 1]
        U = ((ct * X + st * Y) / s + 1.0) / 2.0 * (Wb - 1)
        V = ((-st * X + ct * Y) / s + 1.0) / 2.0 * (Hb - 1)
        fu, fv = np.floor(U), np.floor(V)
        total += int(np.count_nonzero((fu >= ulo) & (fu <= uhi) & (fv >= vlo) & (fv <= vhi)))
    return total


# Arithmetic the method performs per evaluated (pixel, primitive) pair, in floating-point
# operations (an FMA counts 2; floor/fraction and the reciprocal count 1 each), for the
# algorithmic side of the roofline. Culling tests, addressing and loop control are excluded.
FWD_FLOP_PER_PAIR = (
    8      # Eq. (1)-(2): U', V' = a x + b y + e, two FMAs each
    + 4    # integer part and fraction of U', V'
    + 9    # Supp. Eqs. (S1)-(S3): two differences, three lerps (FMA) and one difference
    + 1    # Eq. (3): alpha = alpha_max sigma(nu) M
    + 1    # w = T alpha
    + 6    # Eq. (5): C += w c, three FMAs
    + 2    # Eq. (4): T *= (1 - alpha)
)  # = 31
BWD_FLOP_PER_PAIR = (
    8 + 4 + 12  # coordinates, fraction, bilinear value and both derivatives
    + 3         # alpha, 1 - alpha, T_j = T_{j+1} / (1 - alpha_j)
    + 12        # Supp. Eq. (S5): g . (c - G) + g_A B, times T_j
    + 7         # Supp. Eq. (S4): T alpha, then g_c (T alpha) c (1 - c) per channel
    + 3         # dL/dnu and dL/dM
    + 4         # dL/dU', dL/dV' and the centred coordinates
    + 14        # Eq. (7): x, y, log s, theta
    + 10        # back-to-front recurrences G and B
    + 8         # summing the 8 partials over pixels
)  # = 85


def bwd_algorithmic_bytes(H, W, N, atlas_bytes):
    """HBM bytes the MSE-fused backward must move: the forward's image and the target (12 B per
    pixel each), the forward's per-pixel (K, T_K) (8 B), every primitive's 8 parameters in and 8
    gradients out (32 B each) and the atlas once. Tile list ids (4 B per tile-primitive pair,
    under 2 % of the total at these workloads) are not counted."""
    return 32 * H * W + 64 * N + atlas_bytes


def fused_algorithmic_bytes(H, W, N, atlas_bytes):
    """HBM bytes of the fused fit step (forward + MSE backward in one launch): the target in,
    the image and the per-pixel (K, T_K) out (12 + 12 + 8 B per pixel), parameters in and
    gradients out (32 + 32 B per primitive) and the atlas once; tile list ids not counted."""
    return 32 * H * W + 64 * N + atlas_bytes
