"""Seeded synthetic inputs: target images, bitmap atlases and initial primitive parameters.

This module is shared by the GPU path's tests/benchmark and by the CPU oracle's tests. It holds
no arithmetic of the rendering method itself: it only draws inputs with the shapes and value
distributions of the paper's workloads (Sec. 3.1.1 parameterisation; Sec. 4.1 resolutions).
Everything is NumPy with PCG64 generators seeded explicitly, so both sides see identical bytes.

Parameter layout (one row of 8 float32 per primitive, front-to-back = increasing row index):
    x, y          canvas position of the primitive centre, pixels (pixel centres are integers)
    log_s         natural log of the half-extent s in pixels (Eq. 1 divides by s)
    theta         rotation in radians
    nu            opacity logit
    c_r, c_g, c_b colour logits
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import numpy as np

PARAM_NAMES = ("x", "y", "log_s", "theta", "nu", "c_r", "c_g", "c_b")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# --------------------------------------------------------------------------------------------
# bf16 storage helpers (round-to-nearest-even), pure bit manipulation
# --------------------------------------------------------------------------------------------
def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (RNE) and return the 16-bit patterns as uint16."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(a)
    if nan.any():
        r[nan] = 0x7FC0
    return r


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Widen bfloat16 bit patterns to float32 (exact)."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


# --------------------------------------------------------------------------------------------
# Target images: low-passed Gaussian random field plus anti-aliased opaque ellipses
# --------------------------------------------------------------------------------------------
def _lowpass_field(g: np.random.Generator, H: int, W: int, sigma: float) -> np.ndarray:
    noise = g.standard_normal((3, H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    # Gaussian of spatial std `sigma` px has frequency response exp(-2 pi^2 sigma^2 f^2)
    resp = np.exp(-2.0 * math.pi ** 2 * sigma ** 2 * (fx ** 2 + fy ** 2))
    out = np.fft.irfft2(np.fft.rfft2(noise, axes=(1, 2)) * resp, s=(H, W), axes=(1, 2))
    lo = out.min(axis=(1, 2), keepdims=True)
    hi = out.max(axis=(1, 2), keepdims=True)
    return (out - lo) / np.maximum(hi - lo, 1e-12)


def target_image(H: int, W: int, n_ellipses: int, seed: int) -> np.ndarray:
    """3xHxW float32 RGB target in [0,1]: smooth random field with `n_ellipses` filled ellipses.

    Ellipses: centre ~ U[0,W)xU[0,H), semi-axes ~ min(H,W)*U[0.02,0.15], angle ~ U[0,pi),
    colour ~ U[0,1]^3, painted opaque with a one-pixel anti-aliased rim (coverage from the
    first-order signed distance to the boundary)."""
    g = rng(seed)
    img = _lowpass_field(g, H, W, sigma=max(H, W) / 32.0)
    L = float(min(H, W))
    img = img.astype(np.float32)
    for _ in range(n_ellipses):
        cx, cy = g.uniform(0, W), g.uniform(0, H)
        ax, by = L * g.uniform(0.02, 0.15), L * g.uniform(0.02, 0.15)
        phi = g.uniform(0, math.pi)
        col = g.uniform(0, 1, size=3).astype(np.float32)
        r = max(ax, by) + 2.0
        x0, x1 = max(int(math.floor(cx - r)), 0), min(int(math.ceil(cx + r)), W - 1)
        y0, y1 = max(int(math.floor(cy - r)), 0), min(int(math.ceil(cy + r)), H - 1)
        if x0 > x1 or y0 > y1:
            continue
        dx = (np.arange(x0, x1 + 1, dtype=np.float32) - np.float32(cx))[None, :]
        dy = (np.arange(y0, y1 + 1, dtype=np.float32) - np.float32(cy))[:, None]
        c, s = np.float32(math.cos(phi)), np.float32(math.sin(phi))
        lx = (c * dx + s * dy) * np.float32(1.0 / ax)
        ly = (c * dy - s * dx) * np.float32(1.0 / by)
        f = np.sqrt(lx * lx + ly * ly)
        gx = c * lx * np.float32(1.0 / ax) - s * ly * np.float32(1.0 / by)
        gy = s * lx * np.float32(1.0 / ax) + c * ly * np.float32(1.0 / by)
        grad = np.sqrt(gx * gx + gy * gy) / np.maximum(f, np.float32(1e-12))
        cov = np.clip(np.float32(0.5) - (f - np.float32(1.0)) / np.maximum(grad, np.float32(1e-12)),
                      0.0, 1.0)
        sub = img[:, y0:y1 + 1, x0:x1 + 1]
        sub += (col[:, None, None] - sub) * cov
    return np.clip(img, 0.0, 1.0).astype(np.float32)


# --------------------------------------------------------------------------------------------
# Bitmap atlases (values in [0,1]): soft disk, star polygons, tapered cubic Bezier strokes
# --------------------------------------------------------------------------------------------
def soft_disk(size: int = 32, radius: float = 10.0, edge_sigma: float = 2.0) -> np.ndarray:
    """Disk of `radius` px centred in a size x size bitmap with a Gaussian edge of std `edge_sigma`."""
    from scipy.special import erfc
    c = (size - 1) / 2.0
    ys, xs = np.mgrid[0:size, 0:size].astype(np.float64)
    rho = np.hypot(xs - c, ys - c)
    return (0.5 * erfc((rho - radius) / (edge_sigma * math.sqrt(2.0)))).astype(np.float32)


def _supersample_grid(size: int, ss: int):
    o = (np.arange(ss) + 0.5) / ss - 0.5
    base = np.arange(size, dtype=np.float64)
    xs = (base[None, :, None, None] + o[None, None, None, :])
    ys = (base[:, None, None, None] + o[None, None, :, None])
    xs = np.broadcast_to(xs, (size, size, ss, ss))
    ys = np.broadcast_to(ys, (size, size, ss, ss))
    return xs, ys


def _star(g: np.random.Generator, size: int) -> np.ndarray:
    ss = max(2, 512 // size)  # 8x8 samples per texel at 64 px, 4x4 at 128 px
    k = int(g.integers(5, 10))
    R = 28.0 * size / 64.0
    ratio = g.uniform(0.35, 0.6)
    phase = g.uniform(0, 2 * math.pi)
    c = (size - 1) / 2.0
    ang = phase + np.arange(2 * k) * math.pi / k
    rad = np.where(np.arange(2 * k) % 2 == 0, R, R * ratio)
    px = c + rad * np.cos(ang)
    py = c + rad * np.sin(ang)
    xs, ys = _supersample_grid(size, ss)
    inside = np.zeros(xs.shape, dtype=bool)
    n = len(px)
    for i in range(n):  # even-odd crossing test
        xa, ya, xb, yb = px[i], py[i], px[(i + 1) % n], py[(i + 1) % n]
        cond = (ya > ys) != (yb > ys)
        xint = xa + (ys - ya) * (xb - xa) / (yb - ya + 1e-300)
        inside ^= cond & (xs < xint)
    return inside.mean(axis=(2, 3)).astype(np.float32)


def _stroke(g: np.random.Generator, size: int, ss: int = 4) -> np.ndarray:
    m = 0.15 * size
    P = g.uniform(m, size - 1 - m, size=(4, 2))
    w0 = g.uniform(3.0, 8.0) * size / 64.0
    t = np.linspace(0.0, 1.0, 96)
    b = ((1 - t) ** 3)[:, None] * P[0] + (3 * (1 - t) ** 2 * t)[:, None] * P[1] \
        + (3 * (1 - t) * t ** 2)[:, None] * P[2] + (t ** 3)[:, None] * P[3]
    half = 0.5 * w0 * (1.0 - 0.75 * np.abs(2.0 * t - 1.0) ** 2)  # tapers toward both ends
    n = size * ss
    coord = (np.arange(n) + 0.5) / ss - 0.5          # supersample positions in pixel units
    inside = np.zeros((n, n), dtype=bool)
    for j in range(len(t)):
        r = half[j]
        lo_x = max(int(np.floor((b[j, 0] - r + 0.5) * ss)), 0)
        hi_x = min(int(np.ceil((b[j, 0] + r + 0.5) * ss)) + 1, n)
        lo_y = max(int(np.floor((b[j, 1] - r + 0.5) * ss)), 0)
        hi_y = min(int(np.ceil((b[j, 1] + r + 0.5) * ss)) + 1, n)
        dx = coord[lo_x:hi_x][None, :] - b[j, 0]
        dy = coord[lo_y:hi_y][:, None] - b[j, 1]
        inside[lo_y:hi_y, lo_x:hi_x] |= dx * dx + dy * dy <= r * r
    return inside.reshape(size, ss, size, ss).mean(axis=(1, 3)).astype(np.float32)


@functools.lru_cache(maxsize=8)
def _stars_strokes(n_each: int, size: int, seed: int) -> np.ndarray:
    g = rng(seed)
    out = []
    for _ in range(n_each):
        out.append(_star(g, size))
    for _ in range(n_each):
        out.append(_stroke(g, size))
    return np.stack(out).astype(np.float32)


def stars_strokes_atlas(n_bitmaps: int, size: int, seed: int) -> np.ndarray:
    """[n_bitmaps, size, size] float32: first half star polygons (5-9 points, outer radius
    28/64 of the size, inner ratio U[0.35,0.6]), second half tapered cubic Bezier strokes
    (width 3-8 px at 64 px, scaled with size). Coverage by supersampling."""
    assert n_bitmaps % 2 == 0
    return _stars_strokes(n_bitmaps // 2, size, seed).copy()


# --------------------------------------------------------------------------------------------
# Initial parameters
# --------------------------------------------------------------------------------------------
def init_params(N: int, H: int, W: int, log_s_mean: float, log_s_std: float, n_bitmaps: int,
                seed: int):
    """Returns (params [N,8] float32, atlas_idx [N] int32).

    x ~ U[0,W), y ~ U[0,H), log_s ~ N(log_s_mean, log_s_std), theta ~ U[0, 2 pi),
    nu ~ N(0,1), colour logits = logit(u) with u ~ U[0,1]^3 clipped to [1e-3, 1-1e-3],
    atlas index ~ U{0..n_bitmaps-1}."""
    g = rng(seed)
    p = np.empty((N, 8), dtype=np.float64)
    p[:, 0] = g.uniform(0, W, size=N)
    p[:, 1] = g.uniform(0, H, size=N)
    p[:, 2] = g.normal(log_s_mean, log_s_std, size=N)
    p[:, 3] = g.uniform(0, 2 * math.pi, size=N)
    p[:, 4] = g.normal(0.0, 1.0, size=N)
    u = np.clip(g.uniform(0, 1, size=(N, 3)), 1e-3, 1 - 1e-3)
    p[:, 5:8] = np.log(u / (1 - u))
    idx = g.integers(0, n_bitmaps, size=N).astype(np.int32)
    return p.astype(np.float32), idx


# --------------------------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    H: int
    W: int
    N: int
    n_ellipses: int
    atlas: str          # "disk32" | "ss64x16" | "ss128x64"
    log_s_mean: float
    log_s_std: float
    atlas_dtype: str    # "f32" | "bf16"
    tile: int
    adam_steps: int
    config_id: int


WORKLOADS = {
    "c0": Workload("c0", 128, 128, 64, 8, "disk32", math.log(8.0), 0.3, "f32", 16, 100, 0),
    "c1": Workload("c1", 512, 512, 4096, 64, "ss64x16", math.log(12.0), 0.5, "f32", 16, 500, 1),
    "c2": Workload("c2", 2048, 2048, 65536, 512, "ss128x64", math.log(10.0), 0.6, "bf16", 16, 0, 2),
    "c4": Workload("c4", 256, 256, 1024, 8, "ss64x16", math.log(12.0), 0.5, "f32", 16, 500, 4),
}


def make_atlas(kind: str) -> np.ndarray:
    """Atlas as float32 [B, Hb, Wb] (a bf16 workload stores these values rounded to bf16)."""
    if kind == "disk32":
        return soft_disk(32)[None]
    if kind == "ss64x16":
        return stars_strokes_atlas(16, 64, seed=7001)
    if kind == "ss128x64":
        return stars_strokes_atlas(64, 128, seed=7002)
    raise ValueError(kind)


def make_workload(name: str, item: int = 0):
    """Returns dict with target [3,H,W] f32, atlas [B,Hb,Wb] f32 (bf16-rounded values when the
    workload stores bf16), atlas_bf16 bits or None, params [N,8] f32, idx [N] i32."""
    w = WORKLOADS[name]
    seed = 1000 * w.config_id + item
    target = target_image(w.H, w.W, w.n_ellipses, seed)
    atlas = make_atlas(w.atlas)
    bits = None
    if w.atlas_dtype == "bf16":
        bits = f32_to_bf16_bits(atlas)
        atlas = bf16_bits_to_f32(bits)
    params, idx = init_params(w.N, w.H, w.W, w.log_s_mean, w.log_s_std, atlas.shape[0],
                              seed + 500)
    return dict(workload=w, target=target, atlas=atlas, atlas_bf16=bits, params=params, idx=idx)


# Batched workload: 64 independent fits of uneven size and primitive count sharing one atlas.
BATCH_SIZES = (256, 384, 512, 768, 1024)


def make_batch(n_images: int = 64, seed: int = 3000):
    g = rng(seed)
    atlas = make_atlas("ss64x16")
    items = []
    for k in range(n_images):
        S = int(BATCH_SIZES[int(g.integers(0, len(BATCH_SIZES)))])
        N = int(round(math.exp(g.uniform(math.log(512), math.log(16384)))))
        target = target_image(S, S, 8, seed + 1 + k)
        params, idx = init_params(N, S, S, math.log(12.0), 0.5, atlas.shape[0], seed + 10001 + k)
        items.append(dict(H=S, W=S, N=N, target=target, params=params, idx=idx))
    return atlas, items


# --------------------------------------------------------------------------------------------
# Learned-initialiser data: many 256x256 targets and slot-template initial parameters, drawn on
# the GPU with torch generators (same recipe as target_image / init_params; different random
# streams, so the values are not those of the NumPy generators).
# --------------------------------------------------------------------------------------------
SLOT_GRID = 32        # 32 x 32 cells, one per slot
SLOT_BLOCK = 8        # slots are numbered block by block: 8 x 8 cells per block, blocks row-major
SLOT_ATLAS_SEED = 4242


def slot_cells(grid: int = SLOT_GRID, block: int = SLOT_BLOCK):
    """(row, column) of the grid cell of every slot: slot i lies in block i // block^2 (blocks
    in row-major order over the grid), at position i % block^2 of that block (row-major inside
    it). block = 1 numbers the cells row-major."""
    if grid % block:
        raise ValueError("the block size must divide the grid")
    i = np.arange(grid * grid)
    b, j = i // (block * block), i % (block * block)
    bpr = grid // block
    return (b // bpr) * block + j // block, (b % bpr) * block + j % block


def slot_atlas_index(n_slots: int, n_bitmaps: int) -> np.ndarray:
    """Fixed atlas index per slot, the same for every target (so that slot i means the same
    kind of primitive across fits)."""
    return rng(SLOT_ATLAS_SEED).integers(0, n_bitmaps, size=n_slots).astype(np.int32)


def target_images_torch(n: int, H: int, W: int, n_ellipses: int, seed: int, device):
    """[n, 3, H, W] float32 targets on `device`: periodic Gaussian low-pass of white noise
    (sigma = max(H, W) / 32 px), min-max normalised per channel, then `n_ellipses` opaque
    ellipses with anti-aliased rims (centre uniform, semi-axes min(H,W) U[0.02, 0.15], angle
    U[0, pi), colour uniform), clipped to [0, 1]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    noise = torch.randn(n, 3, H, W, generator=g, device=device, dtype=torch.float32)
    fy = torch.fft.fftfreq(H, device=device)[:, None]
    fx = torch.fft.rfftfreq(W, device=device)[None, :]
    sigma = max(H, W) / 32.0
    resp = torch.exp(-2.0 * math.pi ** 2 * sigma ** 2 * (fx ** 2 + fy ** 2))
    f = torch.fft.irfft2(torch.fft.rfft2(noise) * resp, s=(H, W))
    lo = f.amin(dim=(2, 3), keepdim=True)
    hi = f.amax(dim=(2, 3), keepdim=True)
    img = (f - lo) / torch.clamp(hi - lo, min=1e-12)
    L = float(min(H, W))
    u = torch.rand(n, n_ellipses, 8, generator=g, device=device)
    cx, cy = u[..., 0] * W, u[..., 1] * H
    ax = L * (0.02 + 0.13 * u[..., 2])
    by = L * (0.02 + 0.13 * u[..., 3])
    phi = math.pi * u[..., 4]
    col = u[..., 5:8]
    ys = torch.arange(H, device=device, dtype=torch.float32)[None, :, None]
    xs = torch.arange(W, device=device, dtype=torch.float32)[None, None, :]
    for e in range(n_ellipses):
        c, s = torch.cos(phi[:, e])[:, None, None], torch.sin(phi[:, e])[:, None, None]
        dx = xs - cx[:, e][:, None, None]
        dy = ys - cy[:, e][:, None, None]
        iax, iby = (1.0 / ax[:, e])[:, None, None], (1.0 / by[:, e])[:, None, None]
        lx = (c * dx + s * dy) * iax
        ly = (c * dy - s * dx) * iby
        r = torch.sqrt(lx * lx + ly * ly)
        gx = c * lx * iax - s * ly * iby
        gy = s * lx * iax + c * ly * iby
        grad = torch.sqrt(gx * gx + gy * gy) / torch.clamp(r, min=1e-12)
        cov = torch.clamp(0.5 - (r - 1.0) / torch.clamp(grad, min=1e-12), 0.0, 1.0)[:, None]
        img = img + (col[:, e][:, :, None, None] - img) * cov
    return torch.clamp(img, 0.0, 1.0).contiguous()


def slot_init_params_torch(n: int, H: int, W: int, log_s_mean: float, log_s_std: float,
                           seed: int, device, grid: int = SLOT_GRID, block: int = SLOT_BLOCK):
    """[n, grid*grid, 8] float32 initial parameters from the slot template: slot i starts at a
    uniform point of its grid cell (slot_cells: stratified, so positions are still uniform over
    the image);
    log_s ~ N(log_s_mean, log_s_std), theta ~ U[0, 2 pi), nu ~ N(0, 1), colour logits of
    U[1e-3, 1 - 1e-3]. The atlas index of slot i is slot_atlas_index()[i]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    S = grid * grid
    rows, cols = slot_cells(grid, block)
    gx = torch.tensor(cols, device=device, dtype=torch.float32)
    gy = torch.tensor(rows, device=device, dtype=torch.float32)
    u = torch.rand(n, S, 6, generator=g, device=device)
    z = torch.randn(n, S, 2, generator=g, device=device)
    p = torch.empty(n, S, 8, device=device)
    p[..., 0] = (gx + u[..., 0]) * (W / grid)
    p[..., 1] = (gy + u[..., 1]) * (H / grid)
    p[..., 2] = log_s_mean + log_s_std * z[..., 0]
    p[..., 3] = 2.0 * math.pi * u[..., 2]
    p[..., 4] = z[..., 1]
    cu = torch.clamp(u[..., 3:6], 1e-3, 1 - 1e-3)
    p[..., 5:8] = torch.log(cu / (1 - cu))
    return p
