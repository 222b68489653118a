"""GPU parity of the reduced-precision raster (float16 atlas: texel pairs blended in packed fp16,
compositing and gradients in float32) against the FP64 CPU oracle, which samples the same
fp16-rounded texels exactly.

Stated tolerance (derived from the fp16 arithmetic of the blend, unit roundoff u = 2^-11, texels
in [0, 1]): the weights are rounded toward zero to fp16 (each off by less than 2u, and
|dM/dU'|, |dM/dV'| <= 1, so at most 4u of M) and the blend rounds four packed results (at most
8u of M after propagation), so |M_gpu - M| <= 12u per sample and |alpha_gpu - alpha| <= 12u k_a
<= 12u. Compositing is exact up to float32 rounding in the perturbed alphas, and
dI/dalpha_j = T_j (c_j - G_j) with colours and background in [0, 1], so per pixel
    |I_gpu - I| <= 12u * sum_j T_j (1 + 10%, for the second-order terms) + 1e-5,
with T_j the transmittance in front of each layer over the pixel (from the oracle's pixel
trace). Gradients carry the same relative perturbation of M, M_U and M_V through products of
float32 factors; no per-element bound short of re-running the arithmetic exists, so the gate is
the float32 path's, scaled: per parameter block, max|g - g_ref| / max|g_ref| <= 3e-2 and
||g - g_ref||_2 / ||g_ref||_2 <= 1e-2. The angle's gradient sums the same per-pixel moments as
the log-scale's (dal (M_U U_c + M_V V_c) against dal (M_U r V_c - M_V U_c / r)), but over a
nearly symmetric bitmap (the 128 x 128 workload's disk) they cancel to a small remainder, and a
perturbation of M_U, M_V of fp16 size is measured against that remainder; so the angle's errors
are measured against the larger of the two blocks (max-norm and 2-norm alike). And the outcome:
a 100-step fit reaches the PSNR of the FP64 oracle's fit within 0.1 dB.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_22625_amd import capi, synth

pytestmark = pytest.mark.gpu

U16 = 2.0 ** -11
M_ERR = 12 * U16
BLOCKS = {"xy": [0, 1], "log_s": [2], "theta": [3], "nu": [4], "colour": [5, 6, 7]}


def f16(atlas):
    """The fp16 atlas (device) and the values it holds, exactly, as float64 for the oracle."""
    h = np.asarray(atlas, dtype=np.float32).astype(np.float16)
    return torch.tensor(h, device="cuda"), h.astype(np.float64)


def assert_image_within_bound(img, ref, params, idx, atlas64, crop, n_probe=400, seed=0,
                              alpha_max=1.0):
    """Every sampled pixel of the window within the blend bound (module docstring); the whole
    window within the bound at the largest transmittance sum among the samples, doubled."""
    x0, y0, w, h = crop
    diff = np.abs(np.asarray(img, dtype=np.float64) - ref)
    err = diff.max(axis=0) if diff.ndim == 3 else diff  # [h, w]
    g = np.random.default_rng(seed)
    ys = g.integers(0, h, n_probe)
    xs = g.integers(0, w, n_probe)
    worst = 0.0
    smax = 0.0
    for y, x in zip(ys, xs):
        _, _, Ts, _ = oracle.pixel_trace(params, idx, atlas64, x0 + x, y0 + y, alpha_max)
        S = float(np.sum(Ts))
        smax = max(smax, S)
        bound = 1.1 * M_ERR * S + 1e-5
        assert err[y, x] <= bound, (x0 + x, y0 + y, err[y, x], bound)
        worst = max(worst, err[y, x] / bound)
    assert err.max() <= 2.0 * (1.1 * M_ERR * smax + 1e-5), (err.max(), smax)
    return worst


def assert_grads_f16(gpu, ref, inf_tol=3e-2, l2_tol=1e-2):
    gpu = np.asarray(gpu, dtype=np.float64)
    errs = {}
    for k, cols in BLOCKS.items():
        a, b = gpu[:, cols], ref[:, cols]
        s = ref[:, [2, 3]] if k == "theta" else b  # the moments' scale (module docstring)
        errs[k] = (float(np.max(np.abs(a - b)) / max(np.max(np.abs(s)), 1e-30)),
                   float(np.linalg.norm(a - b) / max(np.max(np.linalg.norm(s, axis=0)), 1e-30)))
    bad = {k: v for k, v in errs.items() if v[0] > inf_tol or v[1] > l2_tol}
    assert not bad, errs
    return errs


@pytest.fixture(scope="module")
def R():
    from paper_2602_22625_amd.render import Renderer
    return Renderer()


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_f16_c0_forward_backward(R, tile):
    d = synth.make_workload("c0")
    H = W = 128
    a, a64 = f16(d["atlas"])
    p = torch.tensor(d["params"], device="cuda")
    idx = torch.tensor(d["idx"], device="cuda")
    img, alp = R.render(p, idx, a, H, W, torch.ones(3, device="cuda"), 1.0, tile)
    R.check()
    ref, refA = oracle.render(d["params"], d["idx"], a64, H, W)
    assert_image_within_bound(img.cpu().numpy(), ref, d["params"], d["idx"], a64,
                              (0, 0, W, H))
    # A = 1 - T_N: |dA/dalpha_j| <= T_j as well, so the same bound holds
    assert_image_within_bound(alp.cpu().numpy(), refA, d["params"], d["idx"], a64,
                              (0, 0, W, H), seed=1)
    rng = np.random.default_rng(1)
    g = rng.standard_normal((3, H, W))
    gA = rng.standard_normal((H, W))
    gref = oracle.render_backward(d["params"], d["idx"], a64, H, W, g, gA)
    out = R.backward(torch.tensor(g, dtype=torch.float32, device="cuda"),
                     torch.tensor(gA, dtype=torch.float32, device="cuda"), n_params=64)
    R.check()
    assert_grads_f16(out.cpu().numpy(), gref)


def test_f16_ragged_per_pixel_background(R):
    """A canvas that is not a multiple of the tile, per-pixel background, alpha_max < 1, at
    T = 8, 16, 32: image and alpha within the bound, gradients of dL/dI within the tolerance."""
    g = np.random.default_rng(5)
    H, W, N = 77, 101, 300
    a, a64 = f16(synth.make_atlas("ss64x16"))
    params, idx = synth.init_params(N, H, W, np.log(9.0), 0.5, a64.shape[0], 77)
    bg = g.uniform(0, 1, (3, H, W)).astype(np.float32)
    p = torch.tensor(params, device="cuda")
    i_t = torch.tensor(idx, device="cuda")
    bg_t = torch.tensor(bg, device="cuda")
    ref, refA = oracle.render(params, idx, a64, H, W, bg=bg, alpha_max=0.8)
    gI = g.standard_normal((3, H, W))
    gref = oracle.render_backward(params, idx, a64, H, W, gI, None, bg=bg, alpha_max=0.8)
    for tile in (8, 16, 32):
        img, alp = R.render(p, i_t, a, H, W, bg_t, 0.8, tile)
        R.check()
        assert_image_within_bound(img.cpu().numpy(), ref, params, idx, a64, (0, 0, W, H),
                                  n_probe=150, seed=tile, alpha_max=0.8)
        assert_image_within_bound(alp.cpu().numpy(), refA, params, idx, a64, (0, 0, W, H),
                                  n_probe=150, seed=tile + 1, alpha_max=0.8)
        out = R.backward(torch.tensor(gI, dtype=torch.float32, device="cuda"), None, n_params=N)
        R.check()
        assert_grads_f16(out.cpu().numpy(), gref)


def test_f16_c1_window(R):
    """512 x 512, 4,096 primitives: the whole canvas on the GPU, the oracle on a 160 x 144
    window with the loss gradient restricted to it."""
    d = synth.make_workload("c1")
    H = W = 512
    a, a64 = f16(d["atlas"])
    p = torch.tensor(d["params"], device="cuda")
    idx = torch.tensor(d["idx"], device="cuda")
    img, _ = R.render(p, idx, a, H, W, torch.ones(3, device="cuda"), 1.0, 16)
    R.check()
    crop = (203, 77, 160, 144)
    x0, y0, w, h = crop
    ref, _ = oracle.render(d["params"], d["idx"], a64, H, W, crop=crop)
    assert_image_within_bound(img.cpu().numpy()[:, y0:y0 + h, x0:x0 + w], ref, d["params"],
                              d["idx"], a64, crop)
    g = np.random.default_rng(3).standard_normal((3, h, w))
    gref = oracle.render_backward(d["params"], d["idx"], a64, H, W, g, crop=crop)
    G = np.zeros((3, H, W), dtype=np.float32)
    G[:, y0:y0 + h, x0:x0 + w] = g
    out = R.backward(torch.tensor(G, device="cuda"), None, n_params=d["params"].shape[0])
    R.check()
    ggpu = out.cpu().numpy()
    touched = np.abs(gref).sum(axis=1) > 0
    assert_grads_f16(ggpu, gref)
    assert np.all(ggpu[~touched] == 0.0)


def test_f16_fit_step_on_its_pipelined_build():
    """dbmp_fit_step at 512 x 512 (tiles dealt longest first: the pipelined build, ten stored
    visits), from a captured graph, against the oracle over the whole canvas: image within the
    blend bound, MSE gradient within the stated tolerance (the oracle forms dL/dI from its own
    image, the GPU from its own)."""
    from paper_2602_22625_amd.fit import Fitter
    d = synth.make_workload("c1")
    H = W = 512
    a, a64 = f16(d["atlas"])
    p = torch.tensor(d["params"], device="cuda")
    idx = torch.tensor(d["idx"], device="cuda")
    t = torch.tensor(d["target"], device="cuda")
    f = Fitter(p, idx, a, t, tile=16, lr=1e-2)
    f.set_launch(16, capi.DBMP_SCHED_SORTED)
    f.capture(1)
    f.step()
    f.check()
    img = f.image.cpu().numpy().astype(np.float64)
    ref, _ = oracle.render(d["params"], d["idx"], a64, H, W)
    assert_image_within_bound(img, ref, d["params"], d["idx"], a64, (0, 0, W, H))
    loss, gI = oracle.mse(ref, d["target"])
    gref = oracle.render_backward(d["params"], d["idx"], a64, H, W, gI)
    assert_grads_f16(f.grad.cpu().numpy(), gref)
    assert abs(f.loss() - loss) / loss < 1e-3


@pytest.mark.parametrize("grow", [0.0, 0.7])
def test_f16_2048_fit_step_on_windows(grow):
    """The 2048 x 2048 / 65,536-primitive fit step with an fp16 atlas (16 x 16 tiles in grid
    order: the one-cell build with seven stored visits), as the bfloat16 benchmark test does it:
    the target equals the library's own image outside two windows, so the MSE gradient is that
    of the windows, which the oracle evaluates pixel by pixel."""
    from paper_2602_22625_amd.fit import Fitter
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c2")
    H = W = 2048
    params = d["params"].copy()
    params[:, 2] += grow
    a, a64 = f16(d["atlas"])
    p = torch.tensor(params, device="cuda")
    idx = torch.tensor(d["idx"], device="cuda")
    full = torch.tensor(d["target"], device="cuda")
    img0, _ = Renderer().render(p, idx, a, H, W, with_alpha=False)
    target = img0.clone()
    windows = [(1000, 1000, 48, 48), (96, 1900, 40, 48)]
    for x0, y0, w, h in windows:
        target[:, y0:y0 + h, x0:x0 + w] = full[:, y0:y0 + h, x0:x0 + w]
    f = Fitter(p, idx, a, target.contiguous(), tile=16, lr=1e-2)
    f.set_launch(16, capi.DBMP_SCHED_GRID)
    f.capture(1)
    f.step()
    f.check()
    assert torch.equal(f.image, img0)
    img = f.image.cpu().numpy().astype(np.float64)
    g_ref = np.zeros((params.shape[0], 8))
    scale = 2.0 / (3.0 * H * W)
    for k, (x0, y0, w, h) in enumerate(windows):
        crop = (x0, y0, w, h)
        ref, _ = oracle.render(params, d["idx"], a64, H, W, crop=crop)
        win = img[:, y0:y0 + h, x0:x0 + w]
        assert_image_within_bound(win, ref, params, d["idx"], a64, crop, n_probe=100, seed=k)
        gI = scale * (ref - d["target"][:, y0:y0 + h, x0:x0 + w].astype(np.float64))
        g_ref += oracle.render_backward(params, d["idx"], a64, H, W, gI, crop=crop)
    assert_grads_f16(f.grad.cpu().numpy(), g_ref)


def test_f16_fit_100_steps_reaches_the_oracle_psnr():
    """128 x 128, 64 primitives: 100 Adam steps (lr 1e-2) through the fp16 fit step against 100
    steps of the FP64 oracle on the same fp16 texels: final PSNR within 0.1 dB."""
    from paper_2602_22625_amd.fit import Fitter
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c0")
    H = W = 128
    a, a64 = f16(d["atlas"])
    p = torch.tensor(d["params"], device="cuda")
    idx = torch.tensor(d["idx"], device="cuda")
    t = torch.tensor(d["target"], device="cuda")
    f = Fitter(p, idx, a, t, tile=16, lr=1e-2)
    f.capture(10)
    for _ in range(10):
        f.step()
    f.flush()
    f.check()
    theta = d["params"].astype(np.float64)
    opt = oracle.Adam(theta.shape, lr=1e-2)
    for _ in range(100):
        img, _ = oracle.render(theta, d["idx"], a64, H, W)
        _, gI = oracle.mse(img, d["target"])
        theta = opt.step(theta, oracle.render_backward(theta, d["idx"], a64, H, W, gI))
    psnr_ref = oracle.psnr(oracle.render(theta, d["idx"], a64, H, W)[0], d["target"])
    img, _ = Renderer().render(f.params, idx, a, H, W)
    psnr_gpu = oracle.psnr(img.cpu().numpy(), d["target"])
    assert abs(psnr_gpu - psnr_ref) <= 0.1, (psnr_gpu, psnr_ref)
