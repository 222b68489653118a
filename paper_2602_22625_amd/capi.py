"""ctypes binding of libdiffbmp.so (include/diffbmp.h). Argument marshalling only: every
function here forwards to the C function of the same name; tensors are passed as device
pointers, streams as raw hipStream_t handles. There is no fallback: if the library is missing
the import of a function raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiffbmp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "diffbmp.h")

DBMP_OK, DBMP_EINVAL, DBMP_ENOMEM, DBMP_EHIP, DBMP_EOVERFLOW, DBMP_ESTATE, DBMP_ENONFINITE = \
    0, -1, -2, -3, -4, -5, -6
DBMP_F32, DBMP_BF16, DBMP_F16 = 0, 1, 2
DBMP_SCHED_GRID, DBMP_SCHED_SORTED, DBMP_SCHED_PERSISTENT = 0, 1, 2
DBMP_ATLAS_GLOBAL, DBMP_ATLAS_LDS = 0, 1
DBMP_ATLAS_LDS_MAX_BYTES = 32768
DBMP_NOALLOC_SCRATCH_MB = 64  # include/diffbmp.h
STATUS_NAMES = {0: "DBMP_OK", -1: "DBMP_EINVAL", -2: "DBMP_ENOMEM", -3: "DBMP_EHIP",
                -4: "DBMP_EOVERFLOW", -5: "DBMP_ESTATE", -6: "DBMP_ENONFINITE"}


class DbmpError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


class ImageDesc(ctypes.Structure):
    """dbmp_image_desc"""
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("N", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("prim_offset", ctypes.c_int64),
                ("pixel_offset", ctypes.c_int64)]


_lib = None


def load():
    """Loads libdiffbmp.so. torch is imported first so that the library binds to the HIP
    runtime torch already loaded (both carry the soname libamdhip64.so.7)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdiffbmp.so is not built: run `python -m paper_2602_22625_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, LL, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_float
    sig = {
        "dbmp_create": ([ctypes.POINTER(P), I, LL], I),
        "dbmp_destroy": ([P], I),
        "dbmp_reserve": ([P, LL], I),
        "dbmp_set_schedule": ([P, I, I, I], I),
        "dbmp_set_atlas_placement": ([P, I], I),
        "dbmp_time_next_launch": ([P, I, P, P], I),
        "dbmp_set_atlas": ([P, P, P, I, I, I, I], I),
        "dbmp_render": ([P, P, P, P, I, P, I, I, I, I, I, I, P, I, F, I, P, P], I),
        "dbmp_render_backward": ([P, P, P, P, P], I),
        "dbmp_render_mse": ([P, P, P, P, I, P, I, I, I, I, I, I, P, I, F, I, P, P, P, I], I),
        "dbmp_render_batched_mse": ([P, P, I, P, P, P, P, I, I, I, I, P, F, I, P, P, P, I], I),
        "dbmp_fit_step": ([P, P, P, P, I, I, I, P, I, F, I, P, P, P, P, P, P, F, F, F, F], I),
        "dbmp_fit_step_batched": ([P, P, I, P, P, P, P, F, I, P, P, P, P, P, P, F, F, F, F], I),
        "dbmp_render_backward_mse": ([P, P, P, P, P, I], I),
        "dbmp_mse_loss": ([P, P, P], I),
        "dbmp_render_batched": ([P, P, I, P, P, P, P, I, I, I, I, P, F, I, P, P], I),
        "dbmp_check": ([P, P], I),
        "dbmp_longest_list": ([P, P], LL),
        "dbmp_support_pairs": ([P, P, I], LL),
        "dbmp_last_error": ([P], ctypes.c_char_p),
        "dbmp_workspace_epoch": ([P], LL),
        "dbmp_workspace_bytes": ([P], LL),
        "dbmp_render_mse_noalloc": ([P, P, P, I, P, I, I, I, I, I, I, P, I, F, I, I, P, P, P, I,
                                     P, ctypes.POINTER(ctypes.c_size_t)], I),
        "dbmp_mse_grad": ([P, P, P, LL, P, P], I),
        "dbmp_adam_step": ([P, P, P, P, P, LL, F, F, F, F, P, I], I),
    }
    sig.update({
        "dbmp_cnn_conv_forward": ([P, P, I, I, I, I, P, P, I, I, P, P], I),
        "dbmp_cnn_conv_backward_data": ([P, P, I, I, I, I, P, I, P, P], I),
        "dbmp_cnn_conv_backward_weight": ([P, P, P, I, I, I, I, I, P, P], I),
        "dbmp_cnn_linear_forward": ([P, P, I, I, P, P, I, I, P, P], I),
        "dbmp_cnn_linear_backward_data": ([P, P, I, I, P, I, P, P], I),
        "dbmp_cnn_linear_backward_weight": ([P, P, P, I, I, I, P, P], I),
        "dbmp_cnn_cast_weights": ([P, P, I, I, I, P, P], I),
        "dbmp_cnn_pack_input": ([P, P, I, I, I, P], I),
        "dbmp_cnn_param_loss": ([P, P, P, P, LL, F, P, P, P, P], I),
        "dbmp_cnn_code_params": ([P, P, LL, I, I, I, F, P, P, F, I, P], I),
    })
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def ptr(x):
    """Device pointer of a tensor (or None / int passthrough)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _chk(ctx, rc):
    if rc != DBMP_OK:
        msg = load().dbmp_last_error(ctx).decode() if ctx else ""
        raise DbmpError(rc, msg)
    return rc


# ------------------------------------------------------------------------------------------
# Same-name wrappers
# ------------------------------------------------------------------------------------------
def dbmp_create(device=0, list_capacity=0):
    h = ctypes.c_void_p()
    _chk(None, load().dbmp_create(ctypes.byref(h), int(device), int(list_capacity)))
    return h.value


def dbmp_destroy(ctx):
    return _chk(None, load().dbmp_destroy(ctx))


def dbmp_reserve(ctx, list_capacity):
    return _chk(ctx, load().dbmp_reserve(ctx, int(list_capacity)))


def dbmp_set_schedule(ctx, schedule, workgroups_per_cu=4, items_per_grab=1):
    return _chk(ctx, load().dbmp_set_schedule(ctx, int(schedule), int(workgroups_per_cu),
                                              int(items_per_grab)))


def dbmp_set_atlas_placement(ctx, placement):
    return _chk(ctx, load().dbmp_set_atlas_placement(ctx, int(placement)))


def dbmp_time_next_launch(ctx, stage, start_event, stop_event):
    """start_event / stop_event: raw hipEvent_t handles (torch.cuda.Event.cuda_event) or None."""
    return _chk(ctx, load().dbmp_time_next_launch(ctx, int(stage), start_event, stop_event))


def dbmp_set_atlas(ctx, stream, atlas, B, Hb, Wb, atlas_dtype):
    return _chk(ctx, load().dbmp_set_atlas(ctx, stream, ptr(atlas), int(B), int(Hb), int(Wb),
                                           int(atlas_dtype)))


def dbmp_render(ctx, stream, params, atlas_idx, N, atlas, B, Hb, Wb, atlas_dtype, H, W, bg,
                bg_per_pixel, alpha_max, tile, image, alpha):
    return _chk(ctx, load().dbmp_render(ctx, stream, ptr(params), ptr(atlas_idx), int(N),
                                        ptr(atlas), int(B), int(Hb), int(Wb), int(atlas_dtype),
                                        int(H), int(W), ptr(bg), int(bg_per_pixel),
                                        float(alpha_max), int(tile), ptr(image), ptr(alpha)))


def dbmp_render_mse(ctx, stream, params, atlas_idx, N, atlas, B, Hb, Wb, atlas_dtype, H, W, bg,
                    bg_per_pixel, alpha_max, tile, target, image, dL_dparams, accumulate):
    return _chk(ctx, load().dbmp_render_mse(ctx, stream, ptr(params), ptr(atlas_idx), int(N),
                                            ptr(atlas), int(B), int(Hb), int(Wb),
                                            int(atlas_dtype), int(H), int(W), ptr(bg),
                                            int(bg_per_pixel), float(alpha_max), int(tile),
                                            ptr(target), ptr(image), ptr(dL_dparams),
                                            int(accumulate)))


def dbmp_render_mse_noalloc(stream, params, atlas_idx, N, atlas, B, Hb, Wb, atlas_dtype, H, W,
                            bg, bg_per_pixel, alpha_max, tile, list_capacity, target, image,
                            dL_dparams, accumulate, status):
    """Returns the scratch bytes the call used; raises DbmpError (with the bytes the sizes need
    when the static scratch is too small)."""
    need = ctypes.c_size_t(0)
    rc = load().dbmp_render_mse_noalloc(stream, ptr(params), ptr(atlas_idx), int(N), ptr(atlas),
                                        int(B), int(Hb), int(Wb), int(atlas_dtype), int(H),
                                        int(W), ptr(bg), int(bg_per_pixel), float(alpha_max),
                                        int(tile), int(list_capacity), ptr(target), ptr(image),
                                        ptr(dL_dparams), int(accumulate), ptr(status),
                                        ctypes.byref(need))
    if rc != DBMP_OK:
        raise DbmpError(rc, "dbmp_render_mse_noalloc: these sizes need %d scratch bytes"
                        % need.value)
    return need.value


def dbmp_render_batched_mse(ctx, stream, descs, params, atlas_idx, atlas, B, Hb, Wb,
                            atlas_dtype, bg, alpha_max, tile, target, image, dL_dparams,
                            accumulate):
    arr = (ImageDesc * len(descs))(*descs)
    return _chk(ctx, load().dbmp_render_batched_mse(ctx, stream, len(descs), arr,
                                                    ptr(params), ptr(atlas_idx), ptr(atlas),
                                                    int(B), int(Hb), int(Wb), int(atlas_dtype),
                                                    ptr(bg), float(alpha_max), int(tile),
                                                    ptr(target), ptr(image), ptr(dL_dparams),
                                                    int(accumulate)))


def dbmp_fit_step(ctx, stream, params, atlas_idx, N, H, W, bg, bg_per_pixel, alpha_max, tile,
                  target, image, grad, m, v, state, lr, beta1, beta2, eps):
    return _chk(ctx, load().dbmp_fit_step(ctx, stream, ptr(params), ptr(atlas_idx), int(N),
                                          int(H), int(W), ptr(bg), int(bg_per_pixel),
                                          float(alpha_max), int(tile), ptr(target), ptr(image),
                                          ptr(grad), ptr(m), ptr(v), ptr(state), float(lr),
                                          float(beta1), float(beta2), float(eps)))


def dbmp_fit_step_batched(ctx, stream, descs, params, atlas_idx, bg, alpha_max, tile, target,
                          image, grad, m, v, state, lr, beta1, beta2, eps):
    arr = (ImageDesc * len(descs))(*descs)
    return _chk(ctx, load().dbmp_fit_step_batched(ctx, stream, len(descs), arr, ptr(params),
                                                  ptr(atlas_idx), ptr(bg), float(alpha_max),
                                                  int(tile), ptr(target), ptr(image), ptr(grad),
                                                  ptr(m), ptr(v), ptr(state), float(lr),
                                                  float(beta1), float(beta2), float(eps)))


def dbmp_render_backward(ctx, stream, dL_dimage, dL_dalpha, dL_dparams):
    return _chk(ctx, load().dbmp_render_backward(ctx, stream, ptr(dL_dimage), ptr(dL_dalpha),
                                                 ptr(dL_dparams)))


def dbmp_render_backward_mse(ctx, stream, target, dL_dalpha, dL_dparams, accumulate=0):
    return _chk(ctx, load().dbmp_render_backward_mse(ctx, stream, ptr(target), ptr(dL_dalpha),
                                                     ptr(dL_dparams), int(accumulate)))


def dbmp_mse_loss(ctx, stream, out):
    return _chk(ctx, load().dbmp_mse_loss(ctx, stream, ptr(out)))


def dbmp_render_batched(ctx, stream, descs, params, atlas_idx, atlas, B, Hb, Wb, atlas_dtype,
                        bg, alpha_max, tile, image, alpha):
    arr = (ImageDesc * len(descs))(*descs)
    return _chk(ctx, load().dbmp_render_batched(ctx, stream, len(descs), arr, ptr(params),
                                                ptr(atlas_idx), ptr(atlas), int(B), int(Hb),
                                                int(Wb), int(atlas_dtype), ptr(bg),
                                                float(alpha_max), int(tile), ptr(image),
                                                ptr(alpha)))


def dbmp_check(ctx, stream):
    """Returns the status code (does not raise)."""
    return load().dbmp_check(ctx, stream)


def dbmp_longest_list(ctx, stream):
    return int(load().dbmp_longest_list(ctx, stream))


def dbmp_support_pairs(ctx, stream, reset=0):
    return int(load().dbmp_support_pairs(ctx, stream, int(reset)))


def dbmp_last_error(ctx):
    return load().dbmp_last_error(ctx).decode()


def dbmp_workspace_epoch(ctx):
    return int(load().dbmp_workspace_epoch(ctx))


def dbmp_workspace_bytes(ctx):
    return int(load().dbmp_workspace_bytes(ctx))


def dbmp_mse_grad(stream, image, target, n, grad, loss):
    return _chk(None, load().dbmp_mse_grad(stream, ptr(image), ptr(target), int(n), ptr(grad),
                                           ptr(loss)))


def dbmp_adam_step(stream, params, grad, m, v, n, lr, beta1, beta2, eps, step, zero_grad=0):
    return _chk(None, load().dbmp_adam_step(stream, ptr(params), ptr(grad), ptr(m), ptr(v),
                                            int(n), float(lr), float(beta1), float(beta2),
                                            float(eps), ptr(step), int(zero_grad)))


# ------------------------------------------------------------------------------------------
# Initialiser layers (include/dbmp_cnn.h): bf16 tensors are torch.bfloat16 (or int16 views)
# ------------------------------------------------------------------------------------------
HEADER_CNN = os.path.join(os.path.dirname(HERE), "include", "dbmp_cnn.h")


def _cnn(rc, name):
    if rc != 0:
        raise DbmpError(rc, name)
    return rc


def dbmp_cnn_conv_forward(stream, x, B, H, W, Cin, w, bias, Cout, relu, y, y32=None):
    return _cnn(load().dbmp_cnn_conv_forward(stream, ptr(x), B, H, W, Cin, ptr(w), ptr(bias),
                                             Cout, int(relu), ptr(y), ptr(y32)),
                "dbmp_cnn_conv_forward")


def dbmp_cnn_conv_backward_data(stream, dz, B, H, W, Cin, wt, Cout, mask, dx):
    return _cnn(load().dbmp_cnn_conv_backward_data(stream, ptr(dz), B, H, W, Cin, ptr(wt), Cout,
                                                   ptr(mask), ptr(dx)),
                "dbmp_cnn_conv_backward_data")


def dbmp_cnn_conv_backward_weight(stream, x, dz, B, H, W, Cin, Cout, dw, db):
    return _cnn(load().dbmp_cnn_conv_backward_weight(stream, ptr(x), ptr(dz), B, H, W, Cin, Cout,
                                                     ptr(dw), ptr(db)),
                "dbmp_cnn_conv_backward_weight")


def dbmp_cnn_linear_forward(stream, x, B, K, w, bias, N, relu, y, y32=None):
    return _cnn(load().dbmp_cnn_linear_forward(stream, ptr(x), B, K, ptr(w), ptr(bias), N,
                                               int(relu), ptr(y), ptr(y32)),
                "dbmp_cnn_linear_forward")


def dbmp_cnn_linear_backward_data(stream, dz, B, N, wt, K, mask, dx):
    return _cnn(load().dbmp_cnn_linear_backward_data(stream, ptr(dz), B, N, ptr(wt), K,
                                                     ptr(mask), ptr(dx)),
                "dbmp_cnn_linear_backward_data")


def dbmp_cnn_linear_backward_weight(stream, x, dz, B, K, N, dw, db):
    return _cnn(load().dbmp_cnn_linear_backward_weight(stream, ptr(x), ptr(dz), B, K, N,
                                                       ptr(dw), ptr(db)),
                "dbmp_cnn_linear_backward_weight")


def dbmp_cnn_cast_weights(stream, w, R, T, C, wb, wt):
    return _cnn(load().dbmp_cnn_cast_weights(stream, ptr(w), R, T, C, ptr(wb), ptr(wt)),
                "dbmp_cnn_cast_weights")


def dbmp_cnn_pack_input(stream, img, B, H, W, x):
    return _cnn(load().dbmp_cnn_pack_input(stream, ptr(img), B, H, W, ptr(x)),
                "dbmp_cnn_pack_input")


def _host8(v):
    if v is None:
        return None
    arr = (ctypes.c_float * 8)(*[float(x) for x in v])
    return ctypes.cast(arr, ctypes.c_void_p), arr


def dbmp_cnn_param_loss(stream, pred, target, weights8, n, scale, dpred, loss, extra=None,
                        extra_scale8=None):
    xs = _host8(extra_scale8)
    return _cnn(load().dbmp_cnn_param_loss(stream, ptr(pred), ptr(target), ptr(weights8), int(n),
                                           float(scale), ptr(extra), xs[0] if xs else None,
                                           ptr(dpred), ptr(loss)),
                "dbmp_cnn_param_loss")


def dbmp_cnn_code_params(stream, src, n_rows, slots, grid, block, cell, scale8, bias8, clip,
                         decode, out):
    sc, bi = _host8(scale8), _host8(bias8)
    return _cnn(load().dbmp_cnn_code_params(stream, ptr(src), int(n_rows), int(slots), int(grid),
                                            int(block), float(cell), sc[0], bi[0], float(clip),
                                            int(decode), ptr(out)),
                "dbmp_cnn_code_params")
