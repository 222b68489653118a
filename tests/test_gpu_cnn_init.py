"""The learned initialiser end to end on the GPU: the network's gradients through all eight
layers against an FP64 chain of the layer oracle, and what the trained network gains over the
random start it replaces."""
import math

import numpy as np
import pytest
import torch

from oracle import cnn_oracle as co
from paper_2602_22625_amd import synth

pytestmark = pytest.mark.gpu


def bf16r(a):
    return synth.bf16_bits_to_f32(synth.f32_to_bf16_bits(np.asarray(a, np.float32))).astype(
        np.float64)


def test_network_gradients_match_fp64_layer_chain():
    """Forward, loss and backward of the whole network (B = 2) against the same chain composed
    from the FP64 layer oracle, with activations and gradients rounded to bf16 where the GPU
    stores them: each layer's weight and bias gradient within 1e-2 (relative L2; rounding ties
    that the float32 accumulation breaks differently flip single bf16 values)."""
    from paper_2602_22625_amd import cnn_init as ci
    torch.manual_seed(0)
    net = ci.InitNet(seed=3)
    img = synth.target_images_torch(2, 256, 256, 8, 77, "cuda")
    init = synth.slot_init_params_torch(2, 256, 256, ci.LOG_S_MEAN, ci.LOG_S_STD, 5, "cuda")
    codes = ci.encode(init)
    net.forward(img)
    net.loss_and_grad(codes)
    net.backward()
    torch.cuda.synchronize()
    W = [bf16r(w.cpu().numpy()) for w in net.w]
    Bs = [b.cpu().numpy().astype(np.float64) for b in net.b]
    B = 2
    x = np.zeros((B, 256, 256, 8))
    x[..., :3] = bf16r(img.permute(0, 2, 3, 1).cpu().numpy())
    xs = [x]
    a = x
    for l, (ci_, co_) in enumerate(ci.CONV):
        a = bf16r(co.conv_forward(a, W[l].reshape(co_, 3, 3, ci_), Bs[l], relu=True))
        xs.append(a)
    L = len(ci.CONV)
    a6 = a.reshape(B, -1)
    h = bf16r(co.linear_forward(a6, W[L][:, 0, :], Bs[L], relu=True))
    out = co.linear_forward(h, W[L + 1][:, 0, :], Bs[L + 1]).astype(np.float32)
    _, G = co.param_loss(out.reshape(-1, 8), codes.cpu().numpy().reshape(-1, 8),
                         np.array(ci.LOSS_W), 1.0 / (B * ci.SLOTS))
    dout = bf16r(G.reshape(B, -1))
    ref_w, ref_b = [None] * (L + 2), [None] * (L + 2)
    ref_w[L + 1], ref_b[L + 1] = co.linear_backward_weight(h, dout)
    dh = bf16r(co.linear_backward_data(dout, W[L + 1][:, 0, :], mask=h))
    ref_w[L], ref_b[L] = co.linear_backward_weight(a6, dh)
    d = bf16r(co.linear_backward_data(dh, W[L][:, 0, :], mask=a6)).reshape(a.shape)
    for l in range(L - 1, -1, -1):
        ci_, co_ = ci.CONV[l]
        ref_w[l], ref_b[l] = co.conv_backward_weight(xs[l], d)
        if l > 0:
            s = xs[l].shape[1]
            d = bf16r(co.conv_backward_data(d, W[l].reshape(co_, 3, 3, ci_), s, s, mask=xs[l]))
    for l in range(L + 2):
        gw = net.gw[l].cpu().numpy().reshape(ref_w[l].shape)
        gb = net.gb[l].cpu().numpy()
        ew = np.linalg.norm(gw - ref_w[l]) / max(np.linalg.norm(ref_w[l]), 1e-30)
        eb = np.linalg.norm(gb - ref_b[l]) / max(np.linalg.norm(ref_b[l]), 1e-30)
        assert ew < 1e-2 and eb < 1e-2, (l, ew, eb)


def test_learned_start_gains_over_random_start():
    """A small version of the whole procedure: 512 (target, 100-step fit) pairs, a short
    training, 8 held-out targets. The trained network's start must beat the random start it
    replaces (initial PSNR), and the learned arm must reach at least the plain arm's final
    PSNR bar on most targets within its step budget."""
    from paper_2602_22625_amd import cnn_init as ci
    tg, fitted = ci.generate_pairs(512, steps=100, batch=256, seed=1)
    net = ci.InitNet(seed=0)
    ci.train(net, tg, fitted, epochs=12, batch=64, lr=2e-3)
    res = ci.evaluate(net, n_targets=8, plain_steps=100, learned_steps=50, seed=10 ** 7)
    print({k: v for k, v in res.items() if k != "rows"})
    assert res["median_psnr_cnn_start"] > res["median_psnr_random_start"] + 1.0
    assert sum(r["reached"] for r in res["rows"]) >= 6
