"""GPU parity of the initialiser's MFMA layers against the FP64 layer oracle.

Inputs are dyadic rationals with few significant bits (exact in bfloat16), chosen so that every
product is exact in float32 and every sum stays below 2^17 times the coarsest grid: the float32
accumulation is then exact in any order. So the float32 outputs must EQUAL the oracle, and the
bf16 outputs must equal the oracle's value rounded to nearest even: any indexing, layout or
tap mistake changes bits.
"""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as co
from paper_2602_22625_amd import capi, synth

pytestmark = pytest.mark.gpu


def dyadic(g, shape, num, den):
    return (g.integers(-num, num + 1, size=shape) / den).astype(np.float32)


def bf(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda").to(torch.bfloat16)


def bf16_round(a):
    return synth.bf16_bits_to_f32(synth.f32_to_bf16_bits(np.asarray(a, np.float32)))


def st():
    return capi.stream_handle()


@pytest.mark.parametrize("shape", [(2, 16, 12, 8, 24), (3, 8, 8, 16, 72), (1, 34, 18, 32, 8)])
def test_conv_forward_exact(shape):
    B, H, W, Ci, Co = shape
    g = np.random.default_rng(sum(shape))
    x = dyadic(g, (B, H, W, Ci), 4, 4)
    w = dyadic(g, (Co, 3, 3, Ci), 4, 8)
    b = dyadic(g, (Co,), 8, 16)
    ref = co.conv_forward(x, w, b)
    y = torch.empty(B, H // 2, W // 2, Co, device="cuda", dtype=torch.bfloat16)
    y32 = torch.empty(B, H // 2, W // 2, Co, device="cuda")
    wb = bf(w)
    capi.dbmp_cnn_conv_forward(st(), bf(x), B, H, W, Ci, wb, torch.tensor(b, device="cuda"), Co,
                               0, y, y32)
    torch.cuda.synchronize()
    assert np.array_equal(y32.cpu().numpy(), ref.astype(np.float32))
    assert np.array_equal(y.float().cpu().numpy(), bf16_round(ref))
    yr = torch.empty_like(y)
    capi.dbmp_cnn_conv_forward(st(), bf(x), B, H, W, Ci, wb, torch.tensor(b, device="cuda"), Co,
                               1, yr, None)
    torch.cuda.synchronize()
    assert np.array_equal(yr.float().cpu().numpy(), bf16_round(np.maximum(ref, 0)))


def test_first_layer_packs_three_channels():
    g = np.random.default_rng(5)
    img = dyadic(g, (2, 3, 20, 14), 4, 4)
    x = torch.empty(2, 20, 14, 8, device="cuda", dtype=torch.bfloat16)
    capi.dbmp_cnn_pack_input(st(), torch.tensor(img, device="cuda"), 2, 20, 14, x)
    torch.cuda.synchronize()
    xn = x.float().cpu().numpy()
    assert np.array_equal(xn[..., :3], img.transpose(0, 2, 3, 1))
    assert np.all(xn[..., 3:] == 0)


@pytest.mark.parametrize("shape", [(2, 16, 12, 8, 24), (3, 8, 8, 16, 72), (2, 32, 32, 32, 64)])
def test_conv_backward_data_exact(shape):
    B, H, W, Ci, Co = shape
    g = np.random.default_rng(10 + sum(shape))
    w = dyadic(g, (Co, 3, 3, Ci), 4, 8)
    dz = dyadic(g, (B, H // 2, W // 2, Co), 4, 16)
    mask = dyadic(g, (B, H, W, Ci), 2, 2)
    wt = torch.empty(Ci, 3, 3, Co, device="cuda", dtype=torch.bfloat16)
    capi.dbmp_cnn_cast_weights(st(), torch.tensor(w, device="cuda"), Co, 9, Ci, None, wt)
    dx = torch.empty(B, H, W, Ci, device="cuda", dtype=torch.bfloat16)
    for m in (None, mask):
        capi.dbmp_cnn_conv_backward_data(st(), bf(dz), B, H, W, Ci, wt, Co,
                                         None if m is None else bf(m), dx)
        torch.cuda.synchronize()
        ref = co.conv_backward_data(dz, w, H, W, mask=m)
        assert np.array_equal(dx.float().cpu().numpy(), bf16_round(ref))


@pytest.mark.parametrize("shape", [(2, 16, 12, 8, 24), (4, 64, 64, 8, 32), (2, 16, 16, 64, 128)])
def test_conv_backward_weight_exact(shape):
    """(4, 64, 64, ...) has 4,096 output pixels per channel: the product is split along K and
    the partial sums are added with float atomics."""
    B, H, W, Ci, Co = shape
    g = np.random.default_rng(20 + sum(shape))
    x = dyadic(g, (B, H, W, Ci), 4, 4)
    dz = dyadic(g, (B, H // 2, W // 2, Co), 4, 16)
    dw = torch.full((Co, 3, 3, Ci), 0.5, device="cuda")  # the gradient is ADDED
    db = torch.full((Co,), -0.25, device="cuda")
    capi.dbmp_cnn_conv_backward_weight(st(), bf(x), bf(dz), B, H, W, Ci, Co, dw, db)
    torch.cuda.synchronize()
    rw, rb = co.conv_backward_weight(x, dz)
    assert np.array_equal(dw.cpu().numpy(), (rw + 0.5).astype(np.float32))
    assert np.array_equal(db.cpu().numpy(), (rb - 0.25).astype(np.float32))


@pytest.mark.parametrize("dims", [(4, 64, 40), (64, 4096, 64), (64, 64, 8192), (3, 24, 5)])
def test_linear_forward_and_gradients_exact(dims):
    B, K, N = dims
    g = np.random.default_rng(30 + sum(dims))
    x = dyadic(g, (B, K), 4, 4)
    w = dyadic(g, (N, K), 4, 8)
    b = dyadic(g, (N,), 8, 16)
    dz = dyadic(g, (B, N), 4, 16)
    wb = torch.empty(N, K, device="cuda", dtype=torch.bfloat16)
    wt = torch.empty(K, N, device="cuda", dtype=torch.bfloat16)
    capi.dbmp_cnn_cast_weights(st(), torch.tensor(w, device="cuda"), N, 1, K, wb, wt)
    y = torch.empty(B, N, device="cuda", dtype=torch.bfloat16)
    y32 = torch.empty(B, N, device="cuda")
    capi.dbmp_cnn_linear_forward(st(), bf(x), B, K, wb, torch.tensor(b, device="cuda"), N, 1,
                                 y, y32)
    torch.cuda.synchronize()
    ref = co.linear_forward(x, w, b, relu=True)
    assert np.array_equal(y32.cpu().numpy(), ref.astype(np.float32))
    assert np.array_equal(y.float().cpu().numpy(), bf16_round(ref))
    if N % 8 == 0:
        dx = torch.empty(B, K, device="cuda", dtype=torch.bfloat16)
        capi.dbmp_cnn_linear_backward_data(st(), bf(dz), B, N, wt, K, bf(x), dx)
        torch.cuda.synchronize()
        assert np.array_equal(dx.float().cpu().numpy(),
                              bf16_round(co.linear_backward_data(dz, w, mask=x)))
    dw = torch.zeros(N, K, device="cuda")
    db = torch.zeros(N, device="cuda")
    capi.dbmp_cnn_linear_backward_weight(st(), bf(x), bf(dz), B, K, N, dw, db)
    torch.cuda.synchronize()
    rw, rb = co.linear_backward_weight(x, dz)
    assert np.array_equal(dw.cpu().numpy(), rw.astype(np.float32))
    assert np.array_equal(db.cpu().numpy(), rb.astype(np.float32))


def test_cast_weights_layouts():
    g = np.random.default_rng(40)
    w = g.standard_normal((24, 9, 16)).astype(np.float32)
    wb = torch.empty(24, 9, 16, device="cuda", dtype=torch.bfloat16)
    wt = torch.empty(16, 9, 24, device="cuda", dtype=torch.bfloat16)
    capi.dbmp_cnn_cast_weights(st(), torch.tensor(w, device="cuda"), 24, 9, 16, wb, wt)
    torch.cuda.synchronize()
    r = bf16_round(w)
    assert np.array_equal(wb.float().cpu().numpy(), r)
    assert np.array_equal(wt.float().cpu().numpy(), r.transpose(2, 1, 0))


def test_param_loss_matches_oracle():
    g = np.random.default_rng(50)
    p = g.standard_normal((300, 8)).astype(np.float32)
    t = g.standard_normal((300, 8)).astype(np.float32)
    w = np.array([1, 1, 0.5, 0.1, 1, 2, 2, 2], np.float32)
    dp = torch.empty(300, 8, device="cuda", dtype=torch.bfloat16)
    loss = torch.zeros(1, device="cuda")
    capi.dbmp_cnn_param_loss(st(), torch.tensor(p, device="cuda"), torch.tensor(t, device="cuda"),
                             torch.tensor(w, device="cuda"), p.size, 0.125, dp, loss)
    torch.cuda.synchronize()
    L, G = co.param_loss(p, t, w, 0.125)
    assert abs(loss.item() - L) <= 1e-5 * abs(L)
    # dpred is stored in bf16: within half an ulp of bf16 (2^-9 relative) plus the float32
    # rounding of the sine
    assert np.allclose(dp.float().cpu().numpy(), G, rtol=2 ** -8, atol=1e-6)


def test_param_loss_added_gradient_and_no_target():
    g = np.random.default_rng(51)
    p = g.standard_normal((64, 8)).astype(np.float32)
    t = g.standard_normal((64, 8)).astype(np.float32)
    x = g.standard_normal((64, 8)).astype(np.float32)
    w = np.ones(8, np.float32)
    xs = [0.5, 1, 2, 4, 0.25, 1, 1, 3]
    dp = torch.empty(64, 8, device="cuda", dtype=torch.bfloat16)
    P, X = torch.tensor(p, device="cuda"), torch.tensor(x, device="cuda")
    capi.dbmp_cnn_param_loss(st(), P, torch.tensor(t, device="cuda"),
                             torch.tensor(w, device="cuda"), p.size, 0.5, dp, None, X, xs)
    torch.cuda.synchronize()
    _, G = co.param_loss(p, t, w, 0.5)
    assert np.allclose(dp.float().cpu().numpy(), G + x * np.array(xs), rtol=2 ** -8, atol=1e-6)
    capi.dbmp_cnn_param_loss(st(), P, None, None, p.size, 0.5, dp, None, X, xs)
    torch.cuda.synchronize()
    assert np.allclose(dp.float().cpu().numpy(), x * np.array(xs), rtol=2 ** -8, atol=0)


@pytest.mark.parametrize("block", [1, 8])
def test_code_params_matches_oracle(block):
    g = np.random.default_rng(52)
    s8 = [8, 8, 0.5, 1, 2, 2, 2, 2]
    b8 = [0, 0, 2.48, 0, 0, 0, 0, 0]
    t = g.uniform(-6, 6, (3 * 1024, 8)).astype(np.float32)
    T = torch.tensor(t, device="cuda")
    out = torch.empty_like(T)
    capi.dbmp_cnn_code_params(st(), T, t.shape[0], 1024, 32, block, 8.0, s8, b8, 4.0, 1, out)
    torch.cuda.synchronize()
    ref = co.code_params(t, 1024, 32, block, 8.0, s8, b8, 4.0, True)
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-6, atol=1e-5)
    back = torch.empty_like(T)
    capi.dbmp_cnn_code_params(st(), out, t.shape[0], 1024, 32, block, 8.0, s8, b8, 4.0, 0, back)
    torch.cuda.synchronize()
    ref2 = co.code_params(ref, 1024, 32, block, 8.0, s8, b8, 4.0, False)
    assert np.allclose(back.cpu().numpy(), ref2, rtol=1e-5, atol=1e-5)
