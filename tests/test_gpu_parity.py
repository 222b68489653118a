"""GPU parity: the HIP rasteriser (through the C ABI) against the FP64 CPU oracle.

Tolerances (fixed by the requirement on this path):
  images     max|I_gpu - I_ref| / max|I_ref|                          <= 1e-5
  gradients  per parameter block {xy, log_s, theta, nu, colour}:
             max|g_gpu - g_ref| / max|g_ref|  and  ||g_gpu - g_ref||_2 / ||g_ref||_2  <= 1e-4
The gradient gate is a reading of "1e-4 relative" for a vector: every component is measured
against the largest of its block, not against itself. A component far below its block's largest
(a primitive whose pixels nearly cancel) is only bounded in that sense: its float32 sum is a
cancelling sum of per-pixel terms accumulated with atomics in no fixed order, so its own
relative error can be large while its absolute error stays at the block's rounding level.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_22625_amd import synth

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5
GRAD_TOL = 1e-4
BLOCKS = {"xy": [0, 1], "log_s": [2], "theta": [3], "nu": [4], "colour": [5, 6, 7]}


def img_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    return float(np.max(np.abs(gpu - ref)) / max(np.max(np.abs(ref)), 1e-12))


def grad_errs(gpu, ref):
    out = {}
    for k, cols in BLOCKS.items():
        a = np.asarray(gpu, dtype=np.float64)[:, cols]
        b = ref[:, cols]
        inf = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)
        l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        out[k] = (float(inf), float(l2))
    return out


def assert_grads(gpu, ref, tol=GRAD_TOL):
    errs = grad_errs(gpu, ref)
    bad = {k: v for k, v in errs.items() if v[0] > tol or v[1] > tol}
    assert not bad, errs


@pytest.fixture(scope="module")
def R():
    from paper_2602_22625_amd.render import Renderer
    return Renderer()


def to_dev(d, atlas_bf16=False):
    dev = torch.device("cuda")
    p = torch.tensor(d["params"], device=dev)
    idx = torch.tensor(d["idx"], device=dev)
    if atlas_bf16:
        a = torch.tensor(d["atlas_bf16"].view(np.int16), device=dev).view(torch.bfloat16)
    else:
        a = torch.tensor(d["atlas"], device=dev)
    return p, idx, a


def gpu_render(R, p, idx, a, H, W, bg, alpha_max=1.0, tile=16):
    bg_t = torch.tensor(np.asarray(bg, dtype=np.float32), device="cuda")
    img, alp = R.render(p, idx, a, H, W, bg_t, alpha_max, tile)
    torch.cuda.synchronize()
    return img, alp, bg_t


def gpu_grad(R, gI, gA, N):
    gI_t = torch.tensor(gI, dtype=torch.float32, device="cuda")
    gA_t = None if gA is None else torch.tensor(gA, dtype=torch.float32, device="cuda")
    out = R.backward(gI_t, gA_t, n_params=N)
    R.check()
    return out.cpu().numpy()


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_c0_forward_backward(R, tile):
    d = synth.make_workload("c0")
    H = W = 128
    p, idx, a = to_dev(d)
    img, alp, _ = gpu_render(R, p, idx, a, H, W, (1, 1, 1), tile=tile)
    ref, refA = oracle.render(d["params"], d["idx"], d["atlas"], H, W)
    assert img_err(img.cpu(), ref) <= IMG_TOL
    assert img_err(alp.cpu(), refA) <= IMG_TOL
    g = np.random.default_rng(1).standard_normal((3, H, W))
    gA = np.random.default_rng(2).standard_normal((H, W))
    gref = oracle.render_backward(d["params"], d["idx"], d["atlas"], H, W, g, gA)
    assert_grads(gpu_grad(R, g, gA, 64), gref)


def test_images_bitwise_identical_across_tile_sizes(R):
    d = synth.make_workload("c1")
    p, idx, a = to_dev(d)
    outs = []
    for tile in (8, 16, 32, 0):  # 0: the library's choice
        img, alp, _ = gpu_render(R, p, idx, a, 512, 512, (1, 1, 1), tile=tile)
        outs.append((img.cpu().numpy().copy(), alp.cpu().numpy().copy()))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_c1_crop_forward_backward(R):
    """Full 512x512 / 4096-primitive GPU render; oracle on a 160x144 window (many tiles, ragged
    window edges) with the loss gradient restricted to that window."""
    d = synth.make_workload("c1")
    H = W = 512
    p, idx, a = to_dev(d)
    img, alp, _ = gpu_render(R, p, idx, a, H, W, (1, 1, 1))
    crop = (203, 77, 160, 144)
    x0, y0, w, h = crop
    ref, refA = oracle.render(d["params"], d["idx"], d["atlas"], H, W, crop=crop)
    assert img_err(img.cpu().numpy()[:, y0:y0 + h, x0:x0 + w], ref) <= IMG_TOL
    assert img_err(alp.cpu().numpy()[y0:y0 + h, x0:x0 + w], refA) <= IMG_TOL
    rng = np.random.default_rng(3)
    g = rng.standard_normal((3, h, w))
    gA = rng.standard_normal((h, w))
    gref = oracle.render_backward(d["params"], d["idx"], d["atlas"], H, W, g, gA, crop=crop)
    G = np.zeros((3, H, W)); G[:, y0:y0 + h, x0:x0 + w] = g
    GA = np.zeros((H, W)); GA[y0:y0 + h, x0:x0 + w] = gA
    ggpu = gpu_grad(R, G, GA, d["params"].shape[0])
    touched = np.abs(gref).sum(axis=1) > 0
    assert touched.sum() > 100
    assert_grads(ggpu, gref)
    assert np.all(ggpu[~touched] == 0.0)  # primitives outside the window get exactly zero


def test_ragged_bf16_per_pixel_background(R):
    """A canvas that is not a multiple of the tile, bf16 atlas, per-pixel background,
    alpha_max < 1."""
    g = np.random.default_rng(5)
    H, W, N = 77, 101, 300
    atlas = synth.make_atlas("ss64x16")
    bits = synth.f32_to_bf16_bits(atlas)
    atl = synth.bf16_bits_to_f32(bits)
    params, idx = synth.init_params(N, H, W, math.log(9.0), 0.5, atlas.shape[0], 77)
    bg = g.uniform(0, 1, (3, H, W)).astype(np.float32)
    d = dict(params=params, idx=idx, atlas=atl, atlas_bf16=bits)
    p, i_t, a = to_dev(d, atlas_bf16=True)
    for tile in (8, 16, 32):
        img, alp, _ = gpu_render(R, p, i_t, a, H, W, bg, alpha_max=0.8, tile=tile)
        ref, refA = oracle.render(params, idx, atl, H, W, bg=bg, alpha_max=0.8)
        assert img_err(img.cpu(), ref) <= IMG_TOL
        assert img_err(alp.cpu(), refA) <= IMG_TOL
        gI = g.standard_normal((3, H, W))
        gref = oracle.render_backward(params, idx, atl, H, W, gI, None, bg=bg, alpha_max=0.8)
        assert_grads(gpu_grad(R, gI, None, N), gref)


def test_c2_full_size_sampled_windows(R):
    """2048x2048, 65,536 primitives, bf16 atlas, 16x16 tiles: the oracle checks two windows of
    the full-size GPU render, and the gradient of a window-restricted loss. Runs on the module's
    renderer after the smaller canvases, so every workspace buffer grows here, after other tests
    have allocated and freed device memory in this process (the tile counters of the larger
    canvas must start at zero even when the allocator returns recycled memory)."""
    d = synth.make_workload("c2")
    H = W = 2048
    p, idx, a = to_dev(d, atlas_bf16=True)
    img, alp, _ = gpu_render(R, p, idx, a, H, W, (1, 1, 1), tile=16)
    imgn, alpn = img.cpu().numpy(), alp.cpu().numpy()
    for crop in [(1000, 1000, 40, 40), (2017, 3, 31, 29)]:
        x0, y0, w, h = crop
        ref, refA = oracle.render(d["params"], d["idx"], d["atlas"], H, W, crop=crop)
        assert img_err(imgn[:, y0:y0 + h, x0:x0 + w], ref) <= IMG_TOL
        assert img_err(alpn[y0:y0 + h, x0:x0 + w], refA) <= IMG_TOL
    crop = (1000, 1000, 40, 40)
    x0, y0, w, h = crop
    rng = np.random.default_rng(8)
    g = rng.standard_normal((3, h, w))
    G = np.zeros((3, H, W), dtype=np.float32); G[:, y0:y0 + h, x0:x0 + w] = g
    gref = oracle.render_backward(d["params"], d["idx"], d["atlas"], H, W, g, None, crop=crop)
    ggpu = gpu_grad(R, G, None, d["params"].shape[0])
    assert_grads(ggpu, gref)


# ------------------------------------------------------------------------------------------
# Edge cases
# ------------------------------------------------------------------------------------------
def test_no_primitives_gives_background(R):
    a = torch.tensor(synth.soft_disk(32)[None], device="cuda")
    p = torch.zeros(0, 8, device="cuda")
    idx = torch.zeros(0, dtype=torch.int32, device="cuda")
    img, alp, _ = gpu_render(R, p, idx, a, 37, 45, (0.25, 0.5, 0.75))
    assert torch.all(img[0] == 0.25) and torch.all(img[1] == 0.5) and torch.all(img[2] == 0.75)
    assert torch.all(alp == 0)
    out = R.backward(torch.ones(3, 37, 45, device="cuda"), None, n_params=0)
    assert out.numel() == 0


def test_off_canvas_and_zero_opacity_primitives(R):
    d = synth.make_workload("c0")
    params = d["params"].copy()
    params[3, 0] = -500.0        # far off canvas
    params[7, 4] = -1000.0       # sigmoid(nu) == 0
    p = torch.tensor(params, device="cuda")
    idx = torch.tensor(d["idx"], device="cuda")
    a = torch.tensor(d["atlas"], device="cuda")
    img, alp, _ = gpu_render(R, p, idx, a, 128, 128, (1, 1, 1))
    ref, _ = oracle.render(params, d["idx"], d["atlas"], 128, 128)
    assert img_err(img.cpu(), ref) <= IMG_TOL
    g = np.random.default_rng(4).standard_normal((3, 128, 128))
    gg = gpu_grad(R, g, None, 64)
    assert np.all(gg[3] == 0) and np.all(gg[7] == 0)
    gref = oracle.render_backward(params, d["idx"], d["atlas"], 128, 128, g, None)
    assert_grads(gg, gref)


def test_fully_opaque_layers_and_deep_stacks(R):
    """alpha = 1 exactly (alpha_max = 1, sigmoid(nu) rounds to 1, solid texels) and 400 layers
    over one region, so transmittance reaches 0 and drops below every threshold."""
    H = W = 48
    g = np.random.default_rng(9)
    solid = np.ones((1, 16, 16), dtype=np.float32)
    disk = synth.soft_disk(32)[::2, ::2][None].astype(np.float32)
    atlas = np.concatenate([solid, disk, np.zeros_like(solid)]).astype(np.float32)
    N = 400
    params = np.zeros((N, 8), dtype=np.float32)
    params[:, 0] = g.uniform(16, 32, N)
    params[:, 1] = g.uniform(16, 32, N)
    params[:, 2] = np.log(g.uniform(6, 12, N))
    params[:, 3] = g.uniform(0, 2 * np.pi, N)
    params[:, 4] = g.normal(1.0, 2.0, N)
    params[:, 5:] = g.normal(0, 1, (N, 3))
    params[::37, 4] = 40.0   # opaque layers (alpha == 1 on the solid bitmap)
    idx = g.integers(0, 2, N).astype(np.int32)
    idx[::37] = 0
    idx[5] = 2               # an all-zero bitmap
    d = dict(params=params, idx=idx, atlas=atlas)
    p, i_t, a = to_dev(d)
    img, alp, _ = gpu_render(R, p, i_t, a, H, W, (0.3, 0.2, 0.1))
    ref, refA = oracle.render(params, idx, atlas, H, W, bg=(0.3, 0.2, 0.1))
    assert img_err(img.cpu(), ref) <= IMG_TOL
    gI = g.standard_normal((3, H, W))
    gA = g.standard_normal((H, W))
    gref = oracle.render_backward(params, idx, atlas, H, W, gI, gA, bg=(0.3, 0.2, 0.1))
    gg = gpu_grad(R, gI, gA, N)
    assert np.all(np.isfinite(gg))
    assert_grads(gg, gref)


def test_long_tile_lists_all_sort_paths(R):
    """Tile lists of > 64 and > 2048 entries (register, LDS and global-memory sort paths)."""
    H = W = 64
    g = np.random.default_rng(10)
    atlas = synth.soft_disk(32)[None]
    N = 3000
    params = np.zeros((N, 8), dtype=np.float32)
    params[:, 0] = g.uniform(0, 64, N)
    params[:, 1] = g.uniform(0, 64, N)
    params[:, 2] = np.log(g.uniform(8, 30, N))
    params[:, 3] = g.uniform(0, 6.28, N)
    params[:, 4] = g.normal(-4, 1, N)
    params[:, 5:] = g.normal(0, 1, (N, 3))
    idx = np.zeros(N, dtype=np.int32)
    d = dict(params=params, idx=idx, atlas=atlas)
    p, i_t, a = to_dev(d)
    ref, _ = oracle.render(params, idx, atlas, H, W)
    from paper_2602_22625_amd.render import Renderer
    for tile in (8, 32):
        Rl = Renderer()
        img, _, _ = gpu_render(Rl, p, i_t, a, H, W, (1, 1, 1), tile=tile)
        assert img_err(img.cpu(), ref) <= IMG_TOL
    assert Rl.longest_list() > 2048  # at tile 32 the whole canvas is 4 tiles of ~3000 entries


def test_device_errors_are_flagged(R):
    from paper_2602_22625_amd import capi
    d = synth.make_workload("c0")
    p, idx, a = to_dev(d)
    bad = idx.clone()
    bad[5] = 7  # atlas has one bitmap
    with pytest.raises(capi.DbmpError) as e:
        gpu_render(R, p, bad, a, 128, 128, (1, 1, 1))
    assert e.value.code == capi.DBMP_EINVAL
    pn = p.clone()
    pn[3, 2] = float("nan")
    with pytest.raises(capi.DbmpError) as e:
        gpu_render(R, pn, idx, a, 128, 128, (1, 1, 1))
    assert e.value.code == capi.DBMP_ENONFINITE
    # host-side argument checks
    bg = torch.ones(3, device="cuda")
    with pytest.raises(capi.DbmpError):
        R.render(p, idx, a, 128, 128, bg, 1.5, 16)
    with pytest.raises(capi.DbmpError):
        R.render(p, idx, a, 128, 128, bg, 1.0, 12)


def test_list_overflow_is_reported_then_grown():
    from paper_2602_22625_amd import capi
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c1")
    p, idx, a = to_dev(d)
    small = Renderer(list_capacity=8, check=False)
    bg = torch.ones(3, device="cuda")
    small.render(p, idx, a, 512, 512, bg, 1.0, 16)
    assert capi.dbmp_check(small.ctx, capi.stream_handle()) == capi.DBMP_EOVERFLOW
    need = small.longest_list()
    assert need > 8
    capi.dbmp_reserve(small.ctx, need)
    img, _ = small.render(p, idx, a, 512, 512, bg, 1.0, 16)
    small.check()
    big = Renderer()
    img2, _ = big.render(p, idx, a, 512, 512, bg, 1.0, 16)
    torch.cuda.synchronize()
    assert torch.equal(img, img2)


def test_workspace_bytes_cover_the_per_primitive_and_per_pixel_state():
    """dbmp_workspace_bytes reports the library's own device memory: at least the records
    (160 B per primitive), the per-pixel (K, T_K) and the padded atlas of the last render, and it
    only grows (with the workspace epoch) when a larger canvas needs more."""
    from paper_2602_22625_amd import capi
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c0")
    p, idx, a = to_dev(d)
    R0 = Renderer()
    assert R0.workspace_bytes() >= 0
    bg = torch.ones(3, device="cuda")
    R0.render(p, idx, a, 128, 128, bg, 1.0, 16)
    R0.check()
    b1, e1 = R0.workspace_bytes(), capi.dbmp_workspace_epoch(R0.ctx)
    padded = (32 + 2) * (32 + 2) * 4
    assert b1 >= 160 * 64 + 8 * 128 * 128 + padded
    assert b1 < 4 * (160 * 64 + 8 * 128 * 128 + padded) + (1 << 20)
    R0.render(p, idx, a, 128, 128, bg, 1.0, 16)  # same size: nothing grows
    assert R0.workspace_bytes() == b1 and capi.dbmp_workspace_epoch(R0.ctx) == e1
    R0.render(p, idx, a, 512, 512, bg, 1.0, 16)
    R0.check()
    assert R0.workspace_bytes() >= b1 + 8 * (512 * 512 - 128 * 128)
    assert capi.dbmp_workspace_epoch(R0.ctx) > e1


# (schedule, workgroups per CU, items per grab)
SCHEDULES = [(0, 4, 1), (1, 4, 1), (2, 1, 1), (2, 8, 16), (2, 4, 0)]


@pytest.mark.parametrize("sched", SCHEDULES)
def test_batched_equals_single(R, sched):
    """Every image of a batch (uneven sizes, an empty image, gaps between primitive ranges) is
    bitwise the single-image render, under every launch schedule."""
    from paper_2602_22625_amd.render import Renderer
    g = np.random.default_rng(12)
    atlas = synth.make_atlas("ss64x16")
    sizes = [(64, 80, 150), (200, 120, 900), (33, 47, 40), (128, 128, 0), (96, 96, 500)]
    descs, ps, ids, po, xo = [], [], [], 0, 0
    for k, (H, W, N) in enumerate(sizes):
        pr, ix = synth.init_params(N, H, W, math.log(10.0), 0.5, 16, 900 + k)
        descs.append((H, W, N, po, xo))
        ps.append(pr); ids.append(ix)
        po += N + 3   # gaps between images' primitive ranges are allowed
        ps.append(np.zeros((3, 8), np.float32)); ids.append(np.zeros(3, np.int32))
        xo += H * W + 5
    P = torch.tensor(np.concatenate(ps), device="cuda")
    I = torch.tensor(np.concatenate(ids), device="cuda")
    A = torch.tensor(atlas, device="cuda")
    bgs = torch.tensor(g.uniform(0, 1, (len(sizes), 3)).astype(np.float32), device="cuda")
    Rb = Renderer()
    Rb.set_schedule(*sched)
    img, alp = Rb.render_batched(descs, P, I, A, bgs, 1.0, 16)
    torch.cuda.synchronize()
    for k, (H, W, N, p0, x0) in enumerate(descs):
        si, sa = R.render(P[p0:p0 + N].contiguous(), I[p0:p0 + N].contiguous(), A, H, W,
                          bgs[k].contiguous(), 1.0, 16)
        torch.cuda.synchronize()
        bi = img[3 * x0:3 * x0 + 3 * H * W].view(3, H, W)
        assert torch.equal(bi, si), k
        assert torch.equal(alp[x0:x0 + H * W].view(H, W), sa), k


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("tile", [8, 32])
def test_batched_mse_backward_matches_oracle(sched, tile):
    """Batched forward + MSE backward (each image's loss a mean over its own 3HW values) against
    the oracle image by image, under every launch schedule; per-image losses from
    dbmp_mse_loss."""
    from paper_2602_22625_amd.render import Renderer
    atlas = synth.make_atlas("ss64x16")
    sizes = [(72, 56, 120), (40, 104, 60), (16, 16, 0), (88, 64, 200)]
    descs, ps, ids, tg, po, xo = [], [], [], [], 0, 0
    for k, (H, W, N) in enumerate(sizes):
        pr, ix = synth.init_params(N, H, W, math.log(9.0), 0.5, 16, 700 + k)
        descs.append((H, W, N, po, xo))
        ps.append(pr); ids.append(ix)
        tg.append(synth.target_image(H, W, 4, 800 + k).reshape(-1))
        po += N
        xo += H * W
    P = torch.tensor(np.concatenate(ps), device="cuda")
    I = torch.tensor(np.concatenate(ids), device="cuda")
    A = torch.tensor(atlas, device="cuda")
    T = torch.tensor(np.concatenate(tg), device="cuda")
    bgs = torch.ones(len(sizes), 3, device="cuda")
    Rb = Renderer()
    Rb.set_schedule(*sched)
    img, _ = Rb.render_batched(descs, P, I, A, bgs, 1.0, tile)
    out = Rb.backward_mse(T, None, n_params=po)
    loss = torch.zeros(len(sizes), device="cuda")
    Rb.mse_loss(loss)
    Rb.check()
    out = out.cpu().numpy()
    loss = loss.cpu().numpy()
    for k, (H, W, N, p0, x0) in enumerate(descs):
        if N == 0:
            continue
        ref, _ = oracle.render(ps[k], ids[k], atlas, H, W)
        t = tg[k].reshape(3, H, W)
        sse = float(np.sum((ref - t) ** 2))
        assert abs(loss[k] - sse) <= 1e-5 * sse, (k, loss[k], sse)
        _, gI = oracle.mse(ref, t)
        gref = oracle.render_backward(ps[k], ids[k], atlas, H, W, gI)
        assert_grads(out[p0:p0 + N], gref)


def test_longest_first_order_from_binning_and_from_its_own_kernel():
    """The longest-list-first tile order is computed by an extra binning workgroup from the
    previous forward's lengths up to 4,096 tiles and by a kernel of its own beyond: images equal
    the grid order's bitwise on both paths (4,096 and 4,225 tiles) and on a small canvas, over
    repeated forwards (the first with no previous lengths) and fused steps."""
    from paper_2602_22625_amd import capi
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c1")
    p, idx, a = to_dev(d)
    t = torch.tensor(d["target"], device="cuda")
    for S, tile in [(512, 8), (520, 8), (128, 16)]:
        R0, R1 = Renderer(), Renderer()
        R1.set_schedule(capi.DBMP_SCHED_SORTED)
        tS = torch.nn.functional.pad(t, (0, max(0, S - 512), 0, max(0, S - 512)))[:, :S, :S]
        tS = tS.contiguous()
        for k in range(3):
            q = p + 0.25 * k
            i0, a0 = R0.render(q, idx, a, S, S, None, 1.0, tile)
            i1, a1 = R1.render(q, idx, a, S, S, None, 1.0, tile)
            torch.cuda.synchronize()
            assert torch.equal(i0, i1) and torch.equal(a0, a1), (S, tile, k)
            f0, g0 = R0.render_mse(q, idx, a, S, S, tS, None, 1.0, tile)
            f1, g1 = R1.render_mse(q, idx, a, S, S, tS, None, 1.0, tile)
            R0.check()
            R1.check()
            assert torch.equal(f0, f1), (S, tile, k)
            a0_, a1_ = g0.cpu().numpy().astype(np.float64), g1.cpu().numpy().astype(np.float64)
            scale = np.abs(a0_).max(axis=0) + 1e-30  # per column: atomics in another order
            assert np.all(np.abs(a0_ - a1_) <= 1e-5 * scale), (S, tile, k)


def test_pipelined_and_single_cell_walks_agree():
    """A one-tile-per-workgroup launch of at most 16 waves per compute unit runs the walks that
    keep a second cell in flight; a larger one runs them one cell at a time. The same 512 x 512
    image (4,096 waves at 8 x 8, 16 x 16 and 32 x 32 tiles) rendered alone and as the first
    image of a batch with a 1024 x 1024 canvas: images bitwise equal, fused-step gradients
    within 1e-5 per column (atomics in another order), for the float32, bfloat16 and float16
    atlases (the last the reduced-precision build)."""
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c1")
    dev = torch.device("cuda")
    t = torch.tensor(d["target"], device=dev)
    N = d["params"].shape[0]
    for bf16 in (False, True, "f16"):
        p, idx, a = to_dev(d)
        if bf16:
            a = a.to(torch.float16 if bf16 == "f16" else torch.bfloat16)
        P2 = torch.cat([p, p]).contiguous()
        I2 = torch.cat([idx, idx]).contiguous()
        bg = torch.ones(2, 3, device=dev)
        descs = [(512, 512, N, 0, 0), (1024, 1024, N, N, 512 * 512)]
        T2 = torch.zeros(3 * (512 * 512 + 1024 * 1024), device=dev)
        T2[:3 * 512 * 512] = t.reshape(-1)
        for tile in (8, 16, 32):
            R1, R2 = Renderer(), Renderer()
            i1, a1 = R1.render(p, idx, a, 512, 512, torch.ones(3, device=dev), 1.0, tile)
            i2, a2 = R2.render_batched(descs, P2, I2, a, bg, 1.0, tile)
            torch.cuda.synchronize()
            R1.check()
            R2.check()
            assert torch.equal(i1.reshape(-1), i2[:3 * 512 * 512]), (bf16, tile)
            assert torch.equal(a1.reshape(-1), a2[:512 * 512]), (bf16, tile)
            f1, g1 = R1.render_mse(p, idx, a, 512, 512, t, torch.ones(3, device=dev), 1.0, tile)
            f2, g2 = R2.render_batched_mse(descs, P2, I2, a, bg, T2, 1.0, tile)
            R1.check()
            R2.check()
            assert torch.equal(f1.reshape(-1), f2[:3 * 512 * 512]), (bf16, tile)
            x1 = g1.cpu().numpy().astype(np.float64)
            x2 = g2[:N].cpu().numpy().astype(np.float64)
            scale = np.abs(x1).max(axis=0) + 1e-30
            assert np.all(np.abs(x1 - x2) <= 1e-5 * scale), (bf16, tile)


def _long_and_deep_scenes():
    """The scenes of the deep-stack and long-list tests: 400 layers with opaque ones over a 48 x 48
    canvas, and 3,000 primitives over 64 x 64 (lists beyond the LDS sort capacity)."""
    g = np.random.default_rng(9)
    solid = np.ones((1, 16, 16), dtype=np.float32)
    disk = synth.soft_disk(32)[::2, ::2][None].astype(np.float32)
    atlas = np.concatenate([solid, disk, np.zeros_like(solid)]).astype(np.float32)
    N = 400
    deep = np.zeros((N, 8), dtype=np.float32)
    deep[:, 0] = g.uniform(16, 32, N)
    deep[:, 1] = g.uniform(16, 32, N)
    deep[:, 2] = np.log(g.uniform(6, 12, N))
    deep[:, 3] = g.uniform(0, 2 * np.pi, N)
    deep[:, 4] = g.normal(1.0, 2.0, N)
    deep[:, 5:] = g.normal(0, 1, (N, 3))
    deep[::37, 4] = 40.0
    idx = g.integers(0, 2, N).astype(np.int32)
    idx[::37] = 0
    idx[5] = 2
    yield "deep", 48, deep, idx, atlas, (0.3, 0.2, 0.1)
    g = np.random.default_rng(10)
    N = 3000
    lng = np.zeros((N, 8), dtype=np.float32)
    lng[:, 0] = g.uniform(0, 64, N)
    lng[:, 1] = g.uniform(0, 64, N)
    lng[:, 2] = np.log(g.uniform(8, 30, N))
    lng[:, 3] = g.uniform(0, 6.28, N)
    lng[:, 4] = g.normal(-4, 1, N)
    lng[:, 5:] = g.normal(0, 1, (N, 3))
    yield "long", 64, lng, np.zeros(N, dtype=np.int32), synth.soft_disk(32)[None], (1, 1, 1)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("tile", [8, 32])
def test_walk_builds_agree_on_deep_and_long_lists(tile, dtype):
    """The deep-stack and long-list scenes rendered alone (a launch of few waves: the pipelined
    walks) and as the first image of a batch with a 1024 x 1024 canvas (the one-cell walks), over
    several batches of staged records and the LDS and global-memory sort paths: images bitwise
    equal; the backward with dL/dI and dL/dA on the first image only, within 1e-5 of each
    column's scale. dtype f16: the reduced-precision build."""
    from paper_2602_22625_amd.render import Renderer
    dev = torch.device("cuda")
    for name, S, params, idx, atlas, bg in _long_and_deep_scenes():
        N = params.shape[0]
        p = torch.tensor(params, device=dev)
        i_t = torch.tensor(idx, device=dev)
        a = torch.tensor(atlas, device=dev)
        if dtype == "f16":
            a = a.to(torch.float16)
        bg1 = torch.tensor(np.asarray(bg, dtype=np.float32), device=dev)
        R1, R2 = Renderer(), Renderer()
        i1, a1 = R1.render(p, i_t, a, S, S, bg1, 1.0, tile)
        descs = [(S, S, N, 0, 0), (1024, 1024, N, N, S * S)]
        P2 = torch.cat([p, p]).contiguous()
        I2 = torch.cat([i_t, i_t]).contiguous()
        i2, a2 = R2.render_batched(descs, P2, I2, a, torch.stack([bg1, bg1]).contiguous(), 1.0,
                                   tile)
        torch.cuda.synchronize()
        R1.check()
        R2.check()
        assert torch.equal(i1.reshape(-1), i2[:3 * S * S]), (name, tile)
        assert torch.equal(a1.reshape(-1), a2[:S * S]), (name, tile)
        g = np.random.default_rng(11)
        gI = g.standard_normal((3, S, S)).astype(np.float32)
        gA = g.standard_normal((S, S)).astype(np.float32)
        gI2 = torch.zeros(3 * (S * S + 1024 * 1024), device=dev)
        gI2[:3 * S * S] = torch.tensor(gI.reshape(-1), device=dev)
        gA2 = torch.zeros(S * S + 1024 * 1024, device=dev)
        gA2[:S * S] = torch.tensor(gA.reshape(-1), device=dev)
        g1 = R1.backward(torch.tensor(gI, device=dev), torch.tensor(gA, device=dev), n_params=N)
        g2 = R2.backward(gI2, gA2, n_params=2 * N)
        R1.check()
        R2.check()
        x1 = g1.cpu().numpy().astype(np.float64)
        x2 = g2[:N].cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(x1)) and np.all(np.isfinite(x2))
        scale = np.abs(x1).max(axis=0) + 1e-30
        assert np.all(np.abs(x1 - x2) <= 1e-5 * scale), (name, tile)


def test_autograd_function_matches_oracle(R):
    from paper_2602_22625_amd.render import render
    d = synth.make_workload("c0")
    p = torch.tensor(d["params"], device="cuda", requires_grad=True)
    idx = torch.tensor(d["idx"], device="cuda")
    a = torch.tensor(d["atlas"], device="cuda")
    tgt = torch.tensor(d["target"], device="cuda")
    img, alp = render(p, R, idx, a, 128, 128)
    loss = ((img - tgt) ** 2).mean() + 0.5 * alp.mean()
    loss.backward()
    ref, refA = oracle.render(d["params"], d["idx"], d["atlas"], 128, 128)
    _, gI = oracle.mse(ref, d["target"])
    gA = np.full((128, 128), 0.5 / (128 * 128))
    gref = oracle.render_backward(d["params"], d["idx"], d["atlas"], 128, 128, gI, gA)
    assert_grads(p.grad.cpu().numpy(), gref)


def _one_bitmap_c1():
    """The 512 x 512 / 4,096-primitive workload drawing every primitive from one 64 x 64 bitmap
    (a padded atlas of 17.9 KB in float32, 9.0 KB in float16)."""
    d = synth.make_workload("c1")
    return d["params"], np.zeros_like(d["idx"]), d["atlas"][:1].copy(), d["target"]


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_atlas_in_lds_equals_global(dtype):
    """dbmp_set_atlas_placement(DBMP_ATLAS_LDS): launches of the pipelined build stage the padded
    atlas in LDS and sample it there. Against the default placement on the same inputs: images
    and alpha bitwise equal, gradients (dL/dI and dL/dA) and fused-step gradients within 1e-5
    of each column's scale; at 128^2 (the 64-primitive workload) and on the 512^2 canvas with
    one bitmap; and with the full 16-bitmap atlas (279 KB: too large, so the launch reads
    device memory) also bitwise."""
    from paper_2602_22625_amd import capi
    from paper_2602_22625_amd.render import Renderer
    dev = torch.device("cuda")
    d0 = synth.make_workload("c0")
    d1 = synth.make_workload("c1")
    cases = [(128, d0["params"], d0["idx"], d0["atlas"], d0["target"]),
             (512,) + _one_bitmap_c1(),
             (512, d1["params"], d1["idx"], d1["atlas"], d1["target"])]
    for S, params, idx, atlas, target in cases:
        p = torch.tensor(params, device=dev)
        i_t = torch.tensor(idx, device=dev)
        a = torch.tensor(atlas, device=dev)
        if dtype == "f16":
            a = a.to(torch.float16)
        t = torch.tensor(target, device=dev)
        bg = torch.ones(3, device=dev)
        rng = np.random.default_rng(S)
        gI = torch.tensor(rng.standard_normal((3, S, S)), dtype=torch.float32, device=dev)
        gA = torch.tensor(rng.standard_normal((S, S)), dtype=torch.float32, device=dev)
        outs = []
        for place in (capi.DBMP_ATLAS_GLOBAL, capi.DBMP_ATLAS_LDS):
            R = Renderer()
            R.set_atlas_placement(place)
            img, alp = R.render(p, i_t, a, S, S, bg, 1.0, 16)
            g = R.backward(gI, gA, n_params=params.shape[0])
            f, gf = R.render_mse(p, i_t, a, S, S, t, bg, 1.0, 16)
            R.check()
            outs.append([x.cpu().numpy().copy() for x in (img, alp, g, f, gf)])
        (i0, a0, g0, f0, h0), (i1, a1, g1, f1, h1) = outs
        assert np.array_equal(i0, i1) and np.array_equal(a0, a1) and np.array_equal(f0, f1), S
        for x0, x1 in ((g0, g1), (h0, h1)):
            scale = np.abs(x0).max(axis=0) + 1e-30
            assert np.all(np.abs(x0.astype(np.float64) - x1) <= 1e-5 * scale), S


def test_stored_atlas_equals_per_call_atlas():
    """dbmp_set_atlas once + renders with atlas=NULL == renders given the atlas (bitwise)."""
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c1")
    p, idx, a = to_dev(d)
    R1, R2 = Renderer(), Renderer()
    R2.set_atlas(a)
    for k in range(3):
        q = p + 0.37 * k
        i1, a1 = R1.render(q, idx, a, 512, 512, None, 1.0, 16)
        i2, a2 = R2.render(q, idx, None, 512, 512, None, 1.0, 16)
        torch.cuda.synchronize()
        assert torch.equal(i1, i2) and torch.equal(a1, a2)


@pytest.mark.parametrize("check", ["windows", "fd"])
def test_c2_full_size_in_fresh_process(check):
    """The 2048x2048 / 65,536-primitive checks (oracle windows and window gradient; finite
    differences and peak memory), each in a fresh interpreter: tests/c2_full_size.py."""
    script = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_full_size.py")
    r = subprocess.run([sys.executable, "-u", script, check], capture_output=True, text=True,
                       timeout=600)
    print(r.stdout[-4000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]


def test_backward_after_the_caller_dropped_the_forward_outputs():
    """The MSE backward reads the forward's image and background. A caller that drops the
    returned image (and passed no background, so the Renderer made one) must still get the
    right gradient: the Renderer keeps those buffers alive until the next forward. New
    allocations filled with NaN would take the memory of freed buffers."""
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c0")
    p, idx, a = to_dev(d)
    t = torch.tensor(d["target"], device="cuda")
    R2 = Renderer()
    R2.render(p, idx, a, 128, 128)  # outputs dropped
    junk = [torch.full((3, 128, 128), float("nan"), device="cuda") for _ in range(8)]
    junk += [torch.full((3,), float("nan"), device="cuda") for _ in range(8)]
    g = R2.backward_mse(t, None, n_params=p.shape[0])
    R2.check()
    ref, _ = oracle.render(d["params"], d["idx"], d["atlas"], 128, 128)
    _, gI = oracle.mse(ref, d["target"])
    gref = oracle.render_backward(d["params"], d["idx"], d["atlas"], 128, 128, gI)
    assert_grads(g.cpu().numpy(), gref)
    del junk
