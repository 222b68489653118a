"""The C-ABI library loads on a host without a GPU, exports every function include/diffbmp.h
declares, and rejects bad arguments on the host before touching the device."""
import ctypes
import re

import pytest

from paper_2602_22625_amd import capi


def header_functions(path=None):
    src = open(path or capi.HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dbmp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for n in ["dbmp_create", "dbmp_destroy", "dbmp_render", "dbmp_render_backward",
              "dbmp_render_batched", "dbmp_check", "dbmp_last_error", "dbmp_mse_grad",
              "dbmp_adam_step", "dbmp_reserve", "dbmp_longest_list",
              "dbmp_render_backward_mse", "dbmp_mse_loss", "dbmp_support_pairs",
              "dbmp_set_atlas", "dbmp_render_mse", "dbmp_render_batched_mse",
              "dbmp_set_schedule", "dbmp_time_next_launch"]:
        assert n in names


def test_header_atlas_dtypes_match_the_binding():
    """The atlas element types of diffbmp.h, float16 selecting the reduced-precision raster."""
    import re
    text = open(capi.HEADER).read()
    m = re.search(r"typedef enum \{([^}]*)\} dbmp_dtype;", text)
    vals = dict((k.strip(), int(v)) for k, v in (e.split("=") for e in m.group(1).split(",")))
    assert vals == {"DBMP_F32": capi.DBMP_F32, "DBMP_BF16": capi.DBMP_BF16,
                    "DBMP_F16": capi.DBMP_F16}


def test_library_exports_every_declared_symbol():
    lib = capi.load()
    for n in header_functions() + header_functions(capi.HEADER_CNN):
        assert hasattr(lib, n), n
        assert callable(getattr(capi, n)), n  # the binding has a function of the same name


def test_initialiser_header_declares_its_layers():
    names = header_functions(capi.HEADER_CNN)
    assert names == sorted([
        "dbmp_cnn_conv_forward", "dbmp_cnn_conv_backward_data", "dbmp_cnn_conv_backward_weight",
        "dbmp_cnn_linear_forward", "dbmp_cnn_linear_backward_data",
        "dbmp_cnn_linear_backward_weight", "dbmp_cnn_cast_weights", "dbmp_cnn_pack_input",
        "dbmp_cnn_param_loss", "dbmp_cnn_code_params"])


def test_initialiser_host_argument_checks():
    lib = capi.load()
    # odd sizes, channel counts not a multiple of 8, missing buffers: rejected before launch
    assert lib.dbmp_cnn_conv_forward(None, None, 1, 8, 8, 8, None, None, 8, 1, None, None) == -1
    assert lib.dbmp_cnn_conv_forward(None, 16, 1, 7, 8, 8, 16, None, 8, 1, 16, None) == -1
    assert lib.dbmp_cnn_conv_forward(None, 16, 1, 8, 8, 3, 16, None, 8, 1, 16, None) == -1
    assert lib.dbmp_cnn_conv_backward_data(None, 16, 1, 8, 8, 8, 16, 4, None, 16) == -1
    assert lib.dbmp_cnn_linear_forward(None, 16, 2, 12, 16, None, 4, 0, 16, None) == -1
    assert lib.dbmp_cnn_param_loss(None, 16, 16, 16, 12, 1.0, None, None, 16, None) == -1
    assert lib.dbmp_cnn_param_loss(None, 16, 16, None, 16, 1.0, None, None, 16, None) == -1
    s8 = (ctypes.c_float * 8)(*([1.0] * 8))
    z8 = (ctypes.c_float * 8)(*([0.0] * 8))
    assert lib.dbmp_cnn_code_params(None, 16, 4, 16, 4, 1, ctypes.c_float(8.0),
                                    ctypes.cast(z8, ctypes.c_void_p),
                                    ctypes.cast(s8, ctypes.c_void_p), ctypes.c_float(4.0), 1,
                                    16) == -1
    assert lib.dbmp_cnn_code_params(None, 16, 4, 16, 4, 1, ctypes.c_float(8.0),
                                    ctypes.cast(s8, ctypes.c_void_p),
                                    ctypes.cast(s8, ctypes.c_void_p), ctypes.c_float(0.0), 1,
                                    16) == -1
    # the block size must divide the grid
    assert lib.dbmp_cnn_code_params(None, 16, 4, 16, 4, 3, ctypes.c_float(8.0),
                                    ctypes.cast(s8, ctypes.c_void_p),
                                    ctypes.cast(s8, ctypes.c_void_p), ctypes.c_float(4.0), 1,
                                    16) == -1
    assert lib.dbmp_cnn_cast_weights(None, None, 1, 1, 1, None, None) == -1


def test_host_argument_checks_need_no_device():
    lib = capi.load()
    assert lib.dbmp_render(None, None, None, None, 0, None, 1, 2, 2, 0, 4, 4, None, 0, 1.0, 16,
                           None, None) == capi.DBMP_EINVAL
    assert lib.dbmp_render_backward(None, None, None, None, None) == capi.DBMP_EINVAL
    assert lib.dbmp_mse_grad(None, None, None, -1, None, None) == capi.DBMP_EINVAL
    assert lib.dbmp_mse_grad(None, None, None, 0, None, None) == capi.DBMP_OK
    assert lib.dbmp_adam_step(None, None, None, None, None, 4, 1e-2, 0.9, 0.999, 1e-8,
                              None, 0) == capi.DBMP_EINVAL
    assert lib.dbmp_check(None, None) == capi.DBMP_EINVAL
    assert lib.dbmp_reserve(None, 10) == capi.DBMP_EINVAL
    assert lib.dbmp_destroy(None) == capi.DBMP_EINVAL
    assert lib.dbmp_last_error(None) == b"null context"
    assert lib.dbmp_render_backward_mse(None, None, None, None, None, 0) == capi.DBMP_EINVAL
    assert lib.dbmp_set_atlas(None, None, None, 1, 2, 2, 0) == capi.DBMP_EINVAL
    assert lib.dbmp_mse_loss(None, None, None) == capi.DBMP_EINVAL
    assert lib.dbmp_longest_list(None, None) == -1
    assert lib.dbmp_workspace_epoch(None) == -1
    assert lib.dbmp_workspace_bytes(None) == -1
    assert lib.dbmp_set_schedule(None, 1, 4, 1) == capi.DBMP_EINVAL
    assert lib.dbmp_set_atlas_placement(None, 1) == capi.DBMP_EINVAL
    assert lib.dbmp_fit_step(None, None, None, None, 0, 4, 4, None, 0, 1.0, 16, None, None,
                             None, None, None, None, 1e-2, 0.9, 0.999, 1e-8) == capi.DBMP_EINVAL
    assert lib.dbmp_fit_step_batched(None, None, 1, None, None, None, None, 1.0, 16, None, None,
                                     None, None, None, None, 1e-2, 0.9, 0.999,
                                     1e-8) == capi.DBMP_EINVAL
    assert lib.dbmp_time_next_launch(None, 1, None, None) == capi.DBMP_EINVAL
    assert lib.dbmp_render_mse(None, None, None, None, 0, None, 1, 2, 2, 0, 4, 4, None, 0, 1.0,
                               16, None, None, None, 0) == capi.DBMP_EINVAL
    assert lib.dbmp_render_batched_mse(None, None, 1, None, None, None, None, 1, 2, 2, 0, None,
                                       1.0, 16, None, None, None, 0) == capi.DBMP_EINVAL
    h = ctypes.c_void_p()
    assert lib.dbmp_create(ctypes.byref(h), 0, -5) == capi.DBMP_EINVAL


def test_noalloc_host_checks_need_no_device():
    """dbmp_render_mse_noalloc checks its arguments and its scratch need before any HIP call:
    bad arguments give DBMP_EINVAL, sizes beyond the static scratch DBMP_ENOMEM with the bytes
    they need reported (dummy non-null pointers are never dereferenced on the host)."""
    lib = capi.load()
    need = ctypes.c_size_t(0)
    fake = ctypes.c_void_p(16)
    args = [None, fake, fake, 64, fake, 1, 32, 32, 0, 128, 128, fake, 0, 1.0, 16, 64, fake,
            fake, fake, 0, fake, ctypes.byref(need)]
    bad = list(args)
    bad[16] = None  # no target
    assert lib.dbmp_render_mse_noalloc(*bad) == capi.DBMP_EINVAL
    bad = list(args)
    bad[14] = 12    # tile size
    assert lib.dbmp_render_mse_noalloc(*bad) == capi.DBMP_EINVAL
    bad = list(args)
    bad[15] = 0     # list capacity
    assert lib.dbmp_render_mse_noalloc(*bad) == capi.DBMP_EINVAL
    bad = list(args)
    bad[8] = 3      # atlas dtype: DBMP_F32, DBMP_BF16 and DBMP_F16 only
    assert lib.dbmp_render_mse_noalloc(*bad) == capi.DBMP_EINVAL
    big = list(args)
    big[9] = big[10] = 4096  # 4096 x 4096: 128 MiB of per-pixel state alone
    assert lib.dbmp_render_mse_noalloc(*big) == capi.DBMP_ENOMEM
    assert need.value > capi.DBMP_NOALLOC_SCRATCH_MB << 20
    assert need.value >= 8 * 4096 * 4096

