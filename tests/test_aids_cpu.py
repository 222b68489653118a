"""The optimisation-aid and export entry points (include/dbmp_aids.h, include/dbmp_export.h)
are exported by the library, bound under the same names, and reject bad arguments on the host
before touching a device."""
import ctypes

from paper_2602_22625_amd import aids, capi
from test_capi_cpu import header_functions


def test_aids_and_export_symbols():
    lib = aids.load()
    names = header_functions(aids.HEADER_AIDS) + header_functions(aids.HEADER_EXPORT)
    assert set(names) >= {"dbmp_blur_atlas", "dbmp_sa_init", "dbmp_sa_init_workspace_bytes",
                          "dbmp_noise_canvas", "dbmp_constraint_loss", "dbmp_reinit_transparent",
                          "dbmp_export_boxes", "dbmp_export_layers"}
    for n in names:
        assert hasattr(lib, n), n
        assert callable(getattr(aids, n)), n


def test_aids_host_checks():
    lib = aids.load()
    E = capi.DBMP_EINVAL
    f = ctypes.c_void_p(256)
    assert lib.dbmp_blur_atlas(None, None, 1, 8, 8, 0, 1.0, 3.0, f) == E
    assert lib.dbmp_blur_atlas(None, f, 1, 8, 8, 0, 0.0, 3.0, ctypes.c_void_p(1 << 20)) == E
    assert lib.dbmp_blur_atlas(None, f, 1, 8, 8, 0, 1.0, 3.0, f) == E  # out overlaps atlas
    assert lib.dbmp_blur_atlas(None, f, 1, 8, 2000, 0, 1.0, 3.0, ctypes.c_void_p(1 << 30)) == E
    assert lib.dbmp_sa_init_workspace_bytes(0, 5) == -1
    assert lib.dbmp_sa_init_workspace_bytes(512, 512) >= 16 * 512 * 512
    ws = lib.dbmp_sa_init_workspace_bytes(16, 16)
    args = [None, f, 16, 16, 7, 0.1, f, f, f, 4, 2.0, 20.0, -2.0, 0.02, f, ws, f, f]
    for k, v in [(4, 8), (4, 17), (5, 1.5), (10, 0.0), (11, 1.0), (15, ws - 1), (1, None)]:
        bad = list(args)
        bad[k] = v
        assert lib.dbmp_sa_init(*bad) == E, k
    assert lib.dbmp_noise_canvas(None, 1, 2, 0, 4, f) == E
    assert lib.dbmp_constraint_loss(None, f, f, f, f, 4, 4, -1.0, f, f, None) == E
    assert lib.dbmp_reinit_transparent(None, f, None, None, f, 4, 1.0, None) == E
    assert lib.dbmp_reinit_transparent(None, None, None, None, None, 0, 0.3, None) == capi.DBMP_OK
    assert lib.dbmp_export_boxes(None, f, 4, 32, 32, 16, 16, 0.0, f, f, f) == E
    assert lib.dbmp_export_boxes(None, f, 4, 32, 32, 16, 16, 2.0, f, None, f) == E
    assert lib.dbmp_export_layers(None, f, f, 4, f, 1, 32, 32, 0, 16, 16, 2.0, 1.0, f, f, 33, 8,
                                  f, f) == E  # max_w past the export canvas
    assert lib.dbmp_export_layers(None, f, f, 4, f, 1, 32, 32, 5, 16, 16, 2.0, 1.0, f, f, 8, 8,
                                  f, f) == E
