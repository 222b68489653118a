"""ctypes binding of the optimisation aids (include/dbmp_aids.h) and of the layer export
(include/dbmp_export.h). Argument marshalling only: each function forwards to the C function of
the same name in libdiffbmp.so; tensors are passed as device pointers. A few helpers at the end
allocate the outputs with PyTorch and draw the random inputs the calls take.
"""
from __future__ import annotations

import ctypes
import os

from . import capi
from .capi import DbmpError, ptr

HEADER_AIDS = os.path.join(os.path.dirname(capi.HERE), "include", "dbmp_aids.h")
HEADER_EXPORT = os.path.join(os.path.dirname(capi.HERE), "include", "dbmp_export.h")

_lib = None


def _atlas_code(a):
    import torch
    return {torch.bfloat16: capi.DBMP_BF16, torch.float16: capi.DBMP_F16}.get(a.dtype,
                                                                              capi.DBMP_F32)


def load():
    global _lib
    if _lib is not None:
        return _lib
    lib = capi.load()
    P, I, LL, F, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_float, \
        ctypes.c_double
    U64 = ctypes.c_ulonglong
    sig = {
        "dbmp_blur_atlas": ([P, P, I, I, I, I, F, F, P], I),
        "dbmp_sa_init_workspace_bytes": ([I, I], LL),
        "dbmp_sa_init": ([P, P, I, I, I, D, P, P, P, I, D, D, D, D, P, LL, P, P], I),
        "dbmp_noise_canvas": ([P, U64, U64, I, I, P], I),
        "dbmp_constraint_loss": ([P, P, P, P, P, I, I, F, P, P, P], I),
        "dbmp_reinit_transparent": ([P, P, P, P, P, I, D, P], I),
        "dbmp_export_boxes": ([P, P, I, I, I, I, I, D, P, P, P], I),
        "dbmp_export_layers": ([P, P, P, I, P, I, I, I, I, I, I, D, F, P, P, I, I, P, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _chk(rc, name):
    if rc != capi.DBMP_OK:
        raise DbmpError(rc, name)
    return rc


def dbmp_blur_atlas(stream, atlas, B, Hb, Wb, atlas_dtype, sigma, truncate, out):
    return _chk(load().dbmp_blur_atlas(stream, ptr(atlas), int(B), int(Hb), int(Wb),
                                       int(atlas_dtype), float(sigma), float(truncate), ptr(out)),
                "dbmp_blur_atlas")


def dbmp_sa_init_workspace_bytes(H, W):
    n = int(load().dbmp_sa_init_workspace_bytes(int(H), int(W)))
    if n < 0:
        raise DbmpError(capi.DBMP_EINVAL, "dbmp_sa_init_workspace_bytes")
    return n


def dbmp_sa_init(stream, target, H, W, win, base, u_pos, u_theta, z_col, N, s_min, s_max,
                 nu_init, sigma_c, workspace, workspace_bytes, nlv_out, params_out):
    return _chk(load().dbmp_sa_init(stream, ptr(target), int(H), int(W), int(win), float(base),
                                    ptr(u_pos), ptr(u_theta), ptr(z_col), int(N), float(s_min),
                                    float(s_max), float(nu_init), float(sigma_c), ptr(workspace),
                                    int(workspace_bytes), ptr(nlv_out), ptr(params_out)),
                "dbmp_sa_init")


def dbmp_noise_canvas(stream, seed, iteration, H, W, bg_out):
    return _chk(load().dbmp_noise_canvas(stream, int(seed), int(iteration), int(H), int(W),
                                         ptr(bg_out)), "dbmp_noise_canvas")


def dbmp_constraint_loss(stream, image, alpha, target, target_alpha, H, W, lam, dL_dimage,
                         dL_dalpha, loss):
    return _chk(load().dbmp_constraint_loss(stream, ptr(image), ptr(alpha), ptr(target),
                                            ptr(target_alpha), int(H), int(W), float(lam),
                                            ptr(dL_dimage), ptr(dL_dalpha), ptr(loss)),
                "dbmp_constraint_loss")


def dbmp_reinit_transparent(stream, params, m, v, proposal, N, threshold, count):
    return _chk(load().dbmp_reinit_transparent(stream, ptr(params), ptr(m), ptr(v),
                                               ptr(proposal), int(N), float(threshold),
                                               ptr(count)), "dbmp_reinit_transparent")


def dbmp_export_boxes(stream, params, N, Hb, Wb, H, W, rho, boxes, offsets, max_wh):
    return _chk(load().dbmp_export_boxes(stream, ptr(params), int(N), int(Hb), int(Wb), int(H),
                                         int(W), float(rho), ptr(boxes), ptr(offsets),
                                         ptr(max_wh)), "dbmp_export_boxes")


def dbmp_export_layers(stream, params, atlas_idx, N, atlas, B, Hb, Wb, atlas_dtype, H, W, rho,
                       alpha_max, boxes, offsets, max_w, max_h, alpha_out, colour_out):
    return _chk(load().dbmp_export_layers(stream, ptr(params), ptr(atlas_idx), int(N), ptr(atlas),
                                          int(B), int(Hb), int(Wb), int(atlas_dtype), int(H),
                                          int(W), float(rho), float(alpha_max), ptr(boxes),
                                          ptr(offsets), int(max_w), int(max_h), ptr(alpha_out),
                                          ptr(colour_out)), "dbmp_export_layers")


# ------------------------------------------------------------------------------------------
# Helpers: outputs allocated with PyTorch, random inputs drawn on the device
# ------------------------------------------------------------------------------------------
def blur_atlas(atlas, sigma=1.0, truncate=3.0):
    """Blurred copy of a [B, Hb, Wb] float32, bfloat16 or float16 device atlas (soft
    rasterisation)."""
    import torch
    a = atlas if atlas.dim() == 3 else atlas[None]
    a = a.contiguous()
    code = _atlas_code(a)
    out = torch.empty_like(a)
    dbmp_blur_atlas(capi.stream_handle(), a, a.shape[0], a.shape[1], a.shape[2], code, sigma,
                    truncate, out)
    return out


def sa_init(target, N, s_min, s_max, nu_init=-2.0, sigma_c=0.02, win=7, base=0.1,
            generator=None, draws=None):
    """Structure-aware initial parameters [N, 8] for a [3, H, W] device target; returns
    (params, nlv, draws). draws = (u_pos, u_theta, z_col): device float32 random inputs (drawn
    with `generator` when not given)."""
    import torch
    dev = target.device
    _, H, W = target.shape
    if draws is None:
        u = torch.rand(N, device=dev, generator=generator)
        ut = torch.rand(N, device=dev, generator=generator)
        z = torch.randn(N, 3, device=dev, generator=generator)
        draws = (u, ut, z)
    nbytes = dbmp_sa_init_workspace_bytes(H, W)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    nlv = torch.empty(H, W, device=dev)
    params = torch.empty(N, 8, device=dev)
    dbmp_sa_init(capi.stream_handle(), target.contiguous(), H, W, win, base, draws[0], draws[1],
                 draws[2], N, s_min, s_max, nu_init, sigma_c, ws, nbytes, nlv, params)
    return params, nlv, draws


def export_layers(params, atlas_idx, atlas, H, W, rho=2.0, alpha_max=1.0):
    """Every primitive's layer at export scale rho: (boxes [N, 4] int32 = x0, y0, w, h,
    offsets [N + 1] int64, alpha (packed float32, layer i at offsets[i] .. offsets[i + 1], row-major
    over its box), colours [N, 3]). Synchronises once, to size the alpha buffer."""
    import torch
    dev = params.device
    a = atlas if atlas.dim() == 3 else atlas[None]
    code = _atlas_code(a)
    N = params.shape[0]
    B, Hb, Wb = a.shape
    boxes = torch.empty(max(N, 1), 4, dtype=torch.int32, device=dev)
    offsets = torch.empty(N + 1, dtype=torch.int64, device=dev)
    max_wh = torch.empty(2, dtype=torch.int32, device=dev)
    st = capi.stream_handle()
    dbmp_export_boxes(st, params, N, Hb, Wb, H, W, rho, boxes, offsets, max_wh)
    total = int(offsets[N].item())
    mw, mh = (int(v) for v in max_wh.cpu())
    alpha = torch.empty(max(total, 1), device=dev)
    colours = torch.empty(max(N, 1), 3, device=dev)
    dbmp_export_layers(st, params, atlas_idx, N, a.contiguous(), B, Hb, Wb, code, H, W, rho,
                       alpha_max, boxes, offsets, mw, mh, alpha, colours)
    return boxes[:N], offsets, alpha[:total], colours[:N]

