"""Pins of the FP64 layer oracle (CPU): against the convolution and autograd of PyTorch in
float64 (an independent implementation), against brute-force loops on tiny inputs, and
against closed forms."""
import math

import numpy as np
import torch
import torch.nn.functional as F

from oracle import cnn_oracle as co


def _torch_conv(x, w, b=None):
    # NHWC / [O][3][3][I] -> NCHW / OIHW
    xt = torch.tensor(x, dtype=torch.float64).permute(0, 3, 1, 2)
    wt = torch.tensor(w, dtype=torch.float64).permute(0, 3, 1, 2)
    bt = None if b is None else torch.tensor(b, dtype=torch.float64)
    return xt, wt, bt


def test_conv_forward_matches_torch_and_brute_force():
    g = np.random.default_rng(0)
    x = g.standard_normal((2, 10, 6, 5))
    w = g.standard_normal((7, 3, 3, 5))
    b = g.standard_normal(7)
    y = co.conv_forward(x, w, b)
    xt, wt, bt = _torch_conv(x, w, b)
    ref = F.conv2d(xt, wt, bt, stride=2, padding=1).permute(0, 2, 3, 1).numpy()
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-12)
    # brute force at a few outputs
    for (bb, oy, ox, o) in [(0, 0, 0, 0), (1, 4, 2, 6), (0, 2, 1, 3)]:
        s = b[o]
        for ky in range(3):
            for kx in range(3):
                iy, ix = 2 * oy + ky - 1, 2 * ox + kx - 1
                if 0 <= iy < 10 and 0 <= ix < 6:
                    s += np.dot(w[o, ky, kx], x[bb, iy, ix])
        assert abs(y[bb, oy, ox, o] - s) < 1e-12
    assert np.all(co.conv_forward(x, w, b, relu=True) == np.maximum(y, 0))


def test_conv_identity_tap_is_strided_subsample():
    """A filter that is 1 at the centre tap and channel-diagonal copies x[2oy, 2ox]."""
    g = np.random.default_rng(1)
    x = g.standard_normal((1, 8, 8, 3))
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, 1, 1, c] = 1.0
    assert np.array_equal(co.conv_forward(x, w), x[:, ::2, ::2, :])


def test_conv_gradients_match_autograd():
    g = np.random.default_rng(2)
    x = g.standard_normal((2, 8, 12, 4))
    w = g.standard_normal((6, 3, 3, 4))
    b = g.standard_normal(6)
    dz = g.standard_normal((2, 4, 6, 6))
    xt, wt, bt = _torch_conv(x, w, b)
    xt.requires_grad_(True); wt.requires_grad_(True); bt.requires_grad_(True)
    y = F.conv2d(xt, wt, bt, stride=2, padding=1)
    (y * torch.tensor(dz).permute(0, 3, 1, 2)).sum().backward()
    dx = co.conv_backward_data(dz, w, 8, 12)
    dw, db = co.conv_backward_weight(x, dz)
    assert np.allclose(dx, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(dw, wt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)
    mask = g.standard_normal((2, 8, 12, 4))
    assert np.array_equal(co.conv_backward_data(dz, w, 8, 12, mask=mask), dx * (mask > 0))


def test_linear_and_gradients_match_autograd():
    g = np.random.default_rng(3)
    x = g.standard_normal((5, 16))
    w = g.standard_normal((9, 16))
    b = g.standard_normal(9)
    dz = g.standard_normal((5, 9))
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    y = F.linear(xt, wt, bt)
    (y * torch.tensor(dz)).sum().backward()
    assert np.allclose(co.linear_forward(x, w, b), y.detach().numpy(), rtol=1e-13, atol=1e-12)
    assert np.allclose(co.linear_backward_data(dz, w), xt.grad.numpy(), rtol=1e-12)
    dw, db = co.linear_backward_weight(x, dz)
    assert np.allclose(dw, wt.grad.numpy(), rtol=1e-12) and np.allclose(db, bt.grad.numpy())


def test_param_loss_gradient_and_angle_periodicity():
    g = np.random.default_rng(4)
    p = g.standard_normal((6, 8))
    t = g.standard_normal((6, 8))
    w = np.array([1, 1, 0.5, 0.1, 1, 2, 2, 2.0])
    L, G = co.param_loss(p, t, w, 0.25)
    h = 1e-6
    for (i, q) in [(0, 0), (3, 3), (5, 7), (2, 3)]:
        pp, pm = p.copy(), p.copy()
        pp[i, q] += h
        pm[i, q] -= h
        fd = (co.param_loss(pp, t, w, 0.25)[0] - co.param_loss(pm, t, w, 0.25)[0]) / (2 * h)
        assert abs(fd - G[i, q]) < 1e-7
    p2 = p.copy()
    p2[:, 3] += 2 * math.pi  # a full turn of the angle costs nothing
    assert abs(co.param_loss(p2, t, w, 0.25)[0] - L) < 1e-12


def test_code_params_round_trip_and_cell_centres():
    g = np.random.default_rng(5)
    s8 = [8, 8, 0.5, 1, 2, 2, 2, 2]
    b8 = [0, 0, 2.5, 0, 0, 0, 0, 0]
    t = g.uniform(-3, 3, (2 * 16, 8))
    p = co.code_params(t, 16, 4, 1, 8.0, s8, b8, 4.0, True)
    assert np.allclose(co.code_params(p, 16, 4, 1, 8.0, s8, b8, 4.0, False), t, atol=1e-12)
    # a zero code sits at the slot's cell centre with the mean scale (cells row-major)
    z = co.code_params(np.zeros((16, 8)), 16, 4, 1, 8.0, s8, b8, 4.0, True)
    assert z[5, 0] == (5 % 4 + 0.5) * 8 and z[5, 1] == (5 // 4 + 0.5) * 8 and z[5, 2] == 2.5
    # clipping applies to every column but the angle
    big = np.full((1, 8), 10.0)
    c = co.code_params(big, 16, 4, 1, 8.0, s8, b8, 4.0, True)
    assert c[0, 3] == 10.0 and c[0, 4] == 8.0


def test_code_params_block_order():
    """Slots numbered 2 x 2 cells at a time on a 4 x 4 grid: slot 5 is the second cell (row 0,
    column 1) of block 1 (the top-right block), i.e. cell (row 0, column 3); slot 13 is the
    second cell of block 3 (bottom right): cell (2, 3). Every cell holds exactly one slot, and
    the order is the one the slot template's generator lays out."""
    s8 = [8, 8, 0.5, 1, 2, 2, 2, 2]
    b8 = [0] * 8
    z = co.code_params(np.zeros((16, 8)), 16, 4, 2, 8.0, s8, b8, 4.0, True)
    assert (z[5, 0], z[5, 1]) == (3.5 * 8, 0.5 * 8)
    assert (z[13, 0], z[13, 1]) == (3.5 * 8, 2.5 * 8)
    cells = {(int(x // 8), int(y // 8)) for x, y in z[:, :2]}
    assert len(cells) == 16
    from paper_2602_22625_amd import synth
    for grid, block in [(4, 2), (32, 8), (32, 1)]:
        rows, cols = synth.slot_cells(grid, block)
        zz = co.code_params(np.zeros((grid * grid, 8)), grid * grid, grid, block, 1.0, s8, b8,
                            4.0, True)
        assert np.array_equal(zz[:, 0] - 0.5, cols) and np.array_equal(zz[:, 1] - 0.5, rows)
