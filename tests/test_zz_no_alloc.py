"""dbmp_render_mse_noalloc (no context, nothing allocated: the workspace is a static device
array) against the context entry point dbmp_render_mse on the same inputs, called through the C
ABI: two calls in a row, the second smaller, then an overflowing call and a good one after it
(the status words and the tile counters are cleared by each call)."""
import numpy as np
import pytest
import torch

from paper_2602_22625_amd import capi, synth

pytestmark = pytest.mark.gpu

BLOCKS = {"xy": [0, 1], "log_s": [2], "theta": [3], "nu": [4], "colour": [5, 6, 7]}


def _inputs(name, bf16=False):
    d = synth.make_workload(name)
    w = d["workload"]
    dev = "cuda"
    p = torch.tensor(d["params"], device=dev)
    idx = torch.tensor(d["idx"], device=dev)
    if bf16 == "f16":  # the reduced-precision raster
        a = torch.tensor(d["atlas"].astype(np.float16), device=dev)
    elif bf16:
        a = torch.tensor(synth.f32_to_bf16_bits(d["atlas"]).view(np.int16),
                         device=dev).view(torch.bfloat16)
    else:
        a = torch.tensor(d["atlas"], device=dev)
    t = torch.tensor(d["target"], device=dev)
    return w.H, w.W, p, idx, a, t


def _noalloc(H, W, p, idx, a, t, tile, cap, accumulate=0, grad=None):
    N = p.shape[0]
    B, Hb, Wb = a.shape
    code = {torch.bfloat16: capi.DBMP_BF16, torch.float16: capi.DBMP_F16}.get(a.dtype,
                                                                            capi.DBMP_F32)
    bg = torch.ones(3, device="cuda")
    img = torch.empty(3, H, W, device="cuda")
    g = grad if grad is not None else torch.empty(N, 8, device="cuda")
    status = torch.full((4,), 7, dtype=torch.int32, device="cuda")  # the call clears it
    used = capi.dbmp_render_mse_noalloc(capi.stream_handle(), p, idx, N, a, B, Hb, Wb, code,
                                        H, W, bg, 0, 1.0, tile, cap, t, img, g, accumulate,
                                        status)
    torch.cuda.synchronize()
    return img, g, status.cpu().numpy(), used


def _context(H, W, p, idx, a, t, tile):
    from paper_2602_22625_amd.render import Renderer
    R = Renderer(check=True)
    img, g = R.render_mse(p, idx, a, H, W, t, None, 1.0, tile)
    torch.cuda.synchronize()
    return img, g


def _assert_same(img_n, g_n, img_c, g_c):
    a, b = img_n.cpu().numpy().astype(np.float64), img_c.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(a - b)) / np.max(np.abs(b)) <= 1e-5
    gn, gc = g_n.cpu().numpy().astype(np.float64), g_c.cpu().numpy().astype(np.float64)
    for k, cols in BLOCKS.items():
        x, y = gn[:, cols], gc[:, cols]
        assert np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-30) <= 1e-4, k
        assert np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30) <= 1e-4, k


def test_noalloc_matches_render_mse_on_two_calls_second_smaller():
    # 512x512 / 4,096 fp32, then 128x128 / 64 bf16, then 128x128 fp16 (each call smaller than
    # the first)
    cases = [("c1", 16, False), ("c0", 8, True), ("c0", 16, "f16")]
    for name, tile, bf16 in cases:
        H, W, p, idx, a, t = _inputs(name, bf16)
        print("noalloc case", name, tile, a.dtype, flush=True)
        img_n, g_n, status, used = _noalloc(H, W, p, idx, a, t, tile, cap=256)
        assert np.all(status == 0), status
        assert 0 < used <= capi.DBMP_NOALLOC_SCRATCH_MB << 20
        img_c, g_c = _context(H, W, p, idx, a, t, tile)
        assert torch.equal(img_n, img_c)  # the same kernels: the image bit for bit
        _assert_same(img_n, g_n, img_c, g_c)


def test_noalloc_accumulates_and_reports_overflow():
    H, W, p, idx, a, t = _inputs("c0")
    img_c, g_c = _context(H, W, p, idx, a, t, 16)
    # accumulate: each call adds its gradient to what the buffer holds (two calls: twice it)
    acc = torch.zeros(p.shape[0], 8, device="cuda")
    for _ in range(2):
        _, acc, status, _ = _noalloc(H, W, p, idx, a, t, 16, cap=64, accumulate=1, grad=acc)
        assert np.all(status == 0)
    _assert_same(img_c, acc, img_c, 2 * g_c)
    # a list capacity below the longest list (1, rounded up to 32, against lists of about 150
    # primitives on the 512x512 workload's 32x32 tiles): reported in status[0], and the tiles
    # whose list did not fit are skipped, nothing read past a list
    H1, W1, p1, idx1, a1, t1 = _inputs("c1")
    _, _, status, _ = _noalloc(H1, W1, p1, idx1, a1, t1, 32, cap=1)
    assert status[0] != 0 and status[1] == 0 and status[2] == 0
    # the next call starts from cleared counters and status
    img_n, g_n, status, _ = _noalloc(H, W, p, idx, a, t, 16, cap=64)
    assert np.all(status == 0)
    assert torch.equal(img_n, img_c)
    _assert_same(img_n, g_n, img_c, g_c)


def test_noalloc_refuses_sizes_beyond_its_scratch():
    H, W, p, idx, a, t = _inputs("c0")
    N = p.shape[0]
    big_H = big_W = 4096  # 8 H W bytes of per-pixel state alone exceed the scratch
    img = torch.empty(1, device="cuda")
    status = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(capi.DbmpError) as e:
        capi.dbmp_render_mse_noalloc(capi.stream_handle(), p, idx, N, a, *a.shape,
                                     capi.DBMP_F32, big_H, big_W, torch.ones(3, device="cuda"),
                                     0, 1.0, 16, 64, img, img, torch.empty(N, 8, device="cuda"),
                                     0, status)
    assert e.value.code == capi.DBMP_ENOMEM
    torch.cuda.synchronize()
