"""FP64 CPU oracle for the DiffBMP rasteriser (Sec. 3.1, Supp. Sec. S1, Supp. Alg. 3).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg
are the only callers. It shares no code with the GPU path (no kernels, headers, tables or
helpers); the two meet only through the seeded input generators.

The C file `diffbmp_oracle.c` holds the per-pixel plain definition; this module loads it with
ctypes and adds the plain optimiser pieces (MSE loss, Adam) in NumPy float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "diffbmp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (generic x86-64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i = ctypes.c_int
        d = ctypes.c_double
        lib.oracle_render.argtypes = [i, P, P, P, i, i, i, i, i, P, i, d, i, i, i, i, P, P, i]
        lib.oracle_render.restype = i
        lib.oracle_render_backward.argtypes = [i, P, P, P, i, i, i, i, i, P, i, d, i, i, i, i,
                                               P, P, P, i]
        lib.oracle_render_backward.restype = i
        lib.oracle_pixel_trace.argtypes = [i, P, P, P, i, i, i, d, i, i, i, P, P, P, P]
        lib.oracle_pixel_trace.restype = i
        lib.oracle_support_pairs.argtypes = [i, P, P, i, i, i, i, i, i, i, i]
        lib.oracle_support_pairs.restype = ctypes.c_longlong
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = i
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _prep(params, idx, atlas):
    params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 8)
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1)
    atlas = np.ascontiguousarray(atlas, dtype=np.float64)
    if atlas.ndim == 2:
        atlas = atlas[None]
    assert params.shape[0] == idx.shape[0]
    return params, idx, atlas


def _bg(bg, H, W):
    bg = np.ascontiguousarray(np.asarray(bg, dtype=np.float64))
    if bg.size == 3:
        return bg.reshape(3), 0
    assert bg.shape == (3, H, W)
    return bg, 1


def render(params, idx, atlas, H, W, bg=(1.0, 1.0, 1.0), alpha_max=1.0, crop=None,
           threads=0):
    """Returns (image [3,h,w], alpha [h,w]) in float64 for crop=(x0,y0,w,h) (default: full)."""
    lib = _load()
    params, idx, atlas = _prep(params, idx, atlas)
    bgv, per = _bg(bg, H, W)
    x0, y0, w, h = crop if crop is not None else (0, 0, W, H)
    img = np.zeros((3, h, w))
    alp = np.zeros((h, w))
    B, Hb, Wb = atlas.shape
    rc = lib.oracle_render(params.shape[0], _ptr(params), _ptr(idx), _ptr(atlas), B, Hb, Wb, H, W,
                           _ptr(bgv), per, float(alpha_max), x0, y0, w, h, _ptr(img), _ptr(alp),
                           int(threads))
    if rc != 0:
        raise ValueError("oracle_render: invalid arguments (rc=%d)" % rc)
    return img, alp


def render_backward(params, idx, atlas, H, W, gI, gA=None, bg=(1.0, 1.0, 1.0), alpha_max=1.0,
                    crop=None, threads=0):
    """Returns dL/dparams [N,8] float64 for the crop's pixels given gI [3,h,w], gA [h,w]."""
    lib = _load()
    params, idx, atlas = _prep(params, idx, atlas)
    bgv, per = _bg(bg, H, W)
    x0, y0, w, h = crop if crop is not None else (0, 0, W, H)
    gI = np.ascontiguousarray(gI, dtype=np.float64).reshape(3, h, w)
    if gA is not None:
        gA = np.ascontiguousarray(gA, dtype=np.float64).reshape(h, w)
    out = np.zeros_like(params)
    B, Hb, Wb = atlas.shape
    rc = lib.oracle_render_backward(params.shape[0], _ptr(params), _ptr(idx), _ptr(atlas), B, Hb,
                                    Wb, H, W, _ptr(bgv), per, float(alpha_max), x0, y0, w, h,
                                    _ptr(gI), _ptr(gA), _ptr(out), int(threads))
    if rc != 0:
        raise ValueError("oracle_render_backward: failed (rc=%d)" % rc)
    return out


def pixel_trace(params, idx, atlas, px, py, alpha_max=1.0):
    """Front-to-back list of the layers touching pixel (px,py): (ks, alphas, Ts, T_N)."""
    lib = _load()
    params, idx, atlas = _prep(params, idx, atlas)
    N = params.shape[0]
    ks = np.zeros(max(N, 1), dtype=np.int32)
    al = np.zeros(max(N, 1))
    Ts = np.zeros(max(N, 1))
    tf = np.zeros(1)
    B, Hb, Wb = atlas.shape
    n = lib.oracle_pixel_trace(N, _ptr(params), _ptr(idx), _ptr(atlas), B, Hb, Wb,
                               float(alpha_max), int(px), int(py), N, _ptr(ks), _ptr(al), _ptr(Ts),
                               _ptr(tf))
    if n < 0:
        raise ValueError("oracle_pixel_trace: invalid arguments")
    return ks[:n].copy(), al[:n].copy(), Ts[:n].copy(), float(tf[0])


def threads():
    return int(_load().oracle_threads())


def support_pairs_bruteforce(params, Hb, Wb, H, W, crop=None, threads=0):
    """Exact count of (pixel, primitive) pairs inside the bitmap support, by testing every
    pixel against every primitive."""
    lib = _load()
    params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 8)
    x0, y0, w, h = crop if crop is not None else (0, 0, W, H)
    return int(lib.oracle_support_pairs(params.shape[0], _ptr(params), None, 0, Hb, Wb, x0, y0,
                                        w, h, int(threads)))


# ------------------------------------------------------------------------------------------
# Plain optimiser pieces (float64): mean-squared error over the 3HW values and Adam.
# ------------------------------------------------------------------------------------------
def mse(image, target):
    """Loss = mean over all 3HW values of (I - target)^2; returns (loss, dL/dI)."""
    d = np.asarray(image, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def psnr(image, target):
    d = np.asarray(image, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(10.0 * np.log10(1.0 / np.mean(d * d)))


class Adam:
    """Adam (Kingma & Ba 2015, Algorithm 1) with bias correction, on a float64 array."""

    def __init__(self, shape, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(shape)
        self.v = np.zeros(shape)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * grad
        self.v = self.b2 * self.v + (1.0 - self.b2) * grad * grad
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)
