"""GPU parity of the layer export (include/dbmp_export.h) against the FP64 oracle
(oracle/aids.py): each layer's alpha over its box equals the oracle's at the same export pixels,
every non-zero oracle alpha lies inside the box, and at scale 1 the layers composite to the
rasteriser's own image."""
import math

import numpy as np
import pytest
import torch

from oracle import aids as oaids
from paper_2602_22625_amd import aids, synth

pytestmark = pytest.mark.gpu


def _check_layers(params, idx, atlas_f64, H, W, rho, boxes, offsets, alpha, colours, amax=1.0):
    layers = oaids.export_layers(params, idx, atlas_f64, H, W, rho, amax)
    boxes = boxes.cpu().numpy()
    offsets = offsets.cpu().numpy()
    alpha = alpha.cpu().numpy().astype(np.float64)
    colours = colours.cpu().numpy().astype(np.float64)
    HH, WW = int(round(H * rho)), int(round(W * rho))
    nonempty = 0
    for k, ((ox, oy, ow, oh), oa, ocol) in enumerate(layers):
        x0, y0, w, h = (int(v) for v in boxes[k])
        assert offsets[k + 1] - offsets[k] == w * h
        assert 0 <= x0 and x0 + w <= WW and 0 <= y0 and y0 + h <= HH
        assert np.max(np.abs(colours[k] - ocol)) <= 1e-6
        if ow:  # the box holds every non-zero alpha of the oracle
            nonempty += 1
            assert x0 <= ox and ox + ow <= x0 + w and y0 <= oy and oy + oh <= y0 + h, k
        if w == 0:
            assert ow == 0
            continue
        Y, X = np.meshgrid(np.arange(y0, y0 + h), np.arange(x0, x0 + w), indexing="ij")
        ref = oaids.export_alpha(params[k], atlas_f64[int(idx[k])], X, Y, rho, amax)
        got = alpha[offsets[k]:offsets[k + 1]].reshape(h, w)
        scale = amax / (1 + math.exp(-params[k, 4]))
        assert np.max(np.abs(got - ref)) <= 1e-5 * scale, k
    return nonempty


@pytest.mark.parametrize("rho", [1.0, 2.0, 4.0])
def test_export_layers_match_oracle_c0(rho):
    d = synth.make_workload("c0")
    p = torch.tensor(d["params"], device="cuda")
    idx = torch.tensor(d["idx"], device="cuda")
    a = torch.tensor(d["atlas"], device="cuda")
    boxes, offsets, alpha, colours = aids.export_layers(p, idx, a, 128, 128, rho)
    torch.cuda.synchronize()
    n = _check_layers(d["params"].astype(np.float64), d["idx"], d["atlas"].astype(np.float64),
                      128, 128, rho, boxes, offsets, alpha, colours)
    assert n > 40


def test_export_layers_bf16_ragged_alpha_max():
    """A 77 x 101 canvas, 300 primitives (some off canvas), the 128x128 bf16 bitmaps, alpha_max
    0.7, scale 2."""
    bits = synth.f32_to_bf16_bits(synth.make_atlas("ss128x64")[:8])
    atl = synth.bf16_bits_to_f32(bits)
    params, idx = synth.init_params(300, 77, 101, math.log(9.0), 0.5, 8, 41)
    params[:5, 0] = -60.0  # far off canvas: empty layers
    a = torch.tensor(bits.view(np.int16), device="cuda").view(torch.bfloat16)
    boxes, offsets, alpha, colours = aids.export_layers(
        torch.tensor(params, device="cuda"), torch.tensor(idx, device="cuda"), a, 77, 101, 2.0,
        0.7)
    torch.cuda.synchronize()
    assert np.all(boxes[:5].cpu().numpy()[:, 2:] == 0)
    _check_layers(params.astype(np.float64), idx, atl.astype(np.float64), 77, 101, 2.0, boxes,
                  offsets, alpha, colours, 0.7)


def test_layers_at_scale_one_composite_to_the_render():
    from paper_2602_22625_amd.render import Renderer
    d = synth.make_workload("c1")
    H = W = 512
    p = torch.tensor(d["params"], device="cuda")
    idx = torch.tensor(d["idx"], device="cuda")
    a = torch.tensor(d["atlas"], device="cuda")
    boxes, offsets, alpha, colours = aids.export_layers(p, idx, a, H, W, 1.0)
    img, alp = Renderer().render(p, idx, a, H, W, torch.zeros(3, device="cuda"))
    torch.cuda.synchronize()
    T = torch.ones(H, W, device="cuda", dtype=torch.float64)
    C = torch.zeros(3, H, W, device="cuda", dtype=torch.float64)
    bx = boxes.cpu().numpy()
    off = offsets.cpu().numpy()
    for k in range(p.shape[0]):  # front to back (index order), Eqs. (4)-(5)
        x0, y0, w, h = (int(v) for v in bx[k])
        if w == 0:
            continue
        la = alpha[off[k]:off[k + 1]].view(h, w).double()
        Tk = T[y0:y0 + h, x0:x0 + w]
        C[:, y0:y0 + h, x0:x0 + w] += Tk * la * colours[k].double()[:, None, None]
        T[y0:y0 + h, x0:x0 + w] = Tk * (1 - la)
    assert (C.float() - img).abs().max().item() <= 1e-5 * img.abs().max().item()
    assert ((1 - T).float() - alp).abs().max().item() <= 1e-5
