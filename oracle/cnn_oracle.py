"""FP64 CPU oracle for the learned initialiser's layers: 3x3 stride-2 convolution (zero padding
1) forward, input gradient and weight gradient; dense layers; the parameter regression loss.

TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU kernels; it shares no code with
them. Layouts follow the kernels' ABI: activations NHWC [B][H][W][C], convolution weights
[Cout][3][3][Cin], dense weights [N][K].

Each function is the plain definition: a sum over the nine filter taps of products of shifted,
strided views (the convolution's own definition, output (oy, ox) reads input (2oy+ky-1,
2ox+kx-1)), with NumPy einsum as the per-tap contraction.
"""
from __future__ import annotations

import numpy as np


def _pad(x):
    return np.pad(np.asarray(x, dtype=np.float64), ((0, 0), (1, 1), (1, 1), (0, 0)))


def _tap(xp, ky, kx, OH, OW):
    """Input values under tap (ky, kx) for every output pixel: [B][OH][OW][C]."""
    return xp[:, ky:ky + 2 * OH:2, kx:kx + 2 * OW:2, :]


def conv_forward(x, w, bias=None, relu=False):
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    B, H, W, C = x.shape
    OH, OW = H // 2, W // 2
    xp = _pad(x)
    y = np.zeros((B, OH, OW, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("bhwc,oc->bhwo", _tap(xp, ky, kx, OH, OW), w[:, ky, kx, :])
    if bias is not None:
        y += np.asarray(bias, np.float64)
    return np.maximum(y, 0.0) if relu else y


def conv_backward_data(dz, w, H, W, mask=None):
    """dL/dx for y = conv(x): each output gradient flows back to the input pixel each tap read."""
    dz = np.asarray(dz, np.float64)
    w = np.asarray(w, np.float64)
    B, OH, OW, _ = dz.shape
    dxp = np.zeros((B, H + 2, W + 2, w.shape[3]))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + 2 * OH:2, kx:kx + 2 * OW:2, :] += np.einsum(
                "bhwo,oc->bhwc", dz, w[:, ky, kx, :])
    dx = dxp[:, 1:H + 1, 1:W + 1, :]
    if mask is not None:
        dx = dx * (np.asarray(mask, np.float64) > 0)
    return dx


def conv_backward_weight(x, dz):
    x = np.asarray(x, np.float64)
    dz = np.asarray(dz, np.float64)
    B, H, W, C = x.shape
    OH, OW = H // 2, W // 2
    xp = _pad(x)
    dw = np.zeros((dz.shape[3], 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = np.einsum("bhwo,bhwc->oc", dz, _tap(xp, ky, kx, OH, OW))
    return dw, dz.sum(axis=(0, 1, 2))


def linear_forward(x, w, bias=None, relu=False):
    y = np.asarray(x, np.float64) @ np.asarray(w, np.float64).T
    if bias is not None:
        y = y + np.asarray(bias, np.float64)
    return np.maximum(y, 0.0) if relu else y


def linear_backward_data(dz, w, mask=None):
    dx = np.asarray(dz, np.float64) @ np.asarray(w, np.float64)
    if mask is not None:
        dx = dx * (np.asarray(mask, np.float64) > 0)
    return dx


def linear_backward_weight(x, dz):
    dz = np.asarray(dz, np.float64)
    return dz.T @ np.asarray(x, np.float64), dz.sum(axis=0)


def param_loss(pred, target, weights8, scale):
    """Rows of 8: weighted squared error, the angle column (3) as w (1 - cos(difference))."""
    p = np.asarray(pred, np.float64).reshape(-1, 8)
    t = np.asarray(target, np.float64).reshape(-1, 8)
    w = np.asarray(weights8, np.float64)
    d = p - t
    L = w * d * d
    G = 2.0 * w * d
    L[:, 3] = w[3] * (1.0 - np.cos(d[:, 3]))
    G[:, 3] = w[3] * np.sin(d[:, 3])
    return float(L.sum() * scale), (G * scale).reshape(np.shape(pred))


def code_params(x, slots, grid, block, cell, scale8, bias8, clip, decode):
    """Per-column affine coding of parameter rows (the initialiser's output coding): row r is
    slot r % slots of a grid x grid template whose cell centre offsets x (column 0) and y
    (column 1); every column but the angle (3) is clipped to [-clip, clip] in code space.
    Slots are numbered block x block cells at a time: slot k sits at position k % block^2
    (row-major) of block k // block^2, the blocks taken row-major over the grid."""
    x = np.asarray(x, np.float64).reshape(-1, 8)
    r = np.arange(x.shape[0]) % slots
    centre = np.zeros_like(x)
    col = np.zeros(x.shape[0], np.int64)
    row = np.zeros(x.shape[0], np.int64)
    for k in range(x.shape[0]):  # one slot at a time, as the definition reads
        blk, pos = divmod(int(r[k]), block * block)
        brow, bcol = divmod(blk, grid // block)
        row[k] = brow * block + pos // block
        col[k] = bcol * block + pos % block
    centre[:, 0] = (col + 0.5) * cell
    centre[:, 1] = (row + 0.5) * cell
    s = np.asarray(scale8, np.float64)
    b = np.asarray(bias8, np.float64)
    keep = np.arange(8) != 3
    if decode:
        t = x.copy()
        t[:, keep] = np.clip(t[:, keep], -clip, clip)
        return t * s + b + centre
    t = (x - b - centre) / s
    t[:, keep] = np.clip(t[:, keep], -clip, clip)
    return t
