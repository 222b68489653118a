"""Full-size checks on the 2048 x 2048 workload (65,536 primitives, bf16 atlas, 16 x 16 tiles),
run by test_gpu_parity in a fresh interpreter: `python tests/c2_full_size.py windows|fd`.
Exit status 0 means the check passed; a failed assertion exits non-zero with its traceback.

windows  the oracle checks two windows of the full-size GPU render (one of them ragged at the
         canvas corner), and the gradient of a loss restricted to one window (Sec. 3.1.1-3.1.2,
         Supp. Eqs. S4-S5), at the parity tolerances of the other GPU tests.
fd       gradients of the MSE loss from the autograd Function against central differences of
         fp32 renders on 32 parameters (4 per column), and the peak memory of a fit step.
"""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2602_22625_amd import synth  # noqa: E402
from paper_2602_22625_amd.render import Renderer, render  # noqa: E402

H = W = 2048
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


def to_dev(d):
    dev = torch.device("cuda")
    p = torch.tensor(d["params"], device=dev)
    idx = torch.tensor(d["idx"], device=dev)
    a = torch.tensor(d["atlas_bf16"].view(np.int16), device=dev).view(torch.bfloat16)
    return p, idx, a


def check_windows():
    d = synth.make_workload("c2")
    p, idx, a = to_dev(d)
    R = Renderer()
    bg = torch.ones(3, device="cuda")
    img, alp = R.render(p, idx, a, H, W, bg, 1.0, 16)
    torch.cuda.synchronize()
    imgn, alpn = img.cpu().numpy(), alp.cpu().numpy()
    for crop in [(1000, 1000, 40, 40), (2017, 3, 31, 29)]:
        x0, y0, w, h = crop
        ref, refA = oracle.render(d["params"], d["idx"], d["atlas"], H, W, crop=crop)
        e1 = img_err(imgn[:, y0:y0 + h, x0:x0 + w], ref)
        e2 = img_err(alpn[y0:y0 + h, x0:x0 + w], refA)
        print("window", crop, "image err %.3g alpha err %.3g" % (e1, e2), flush=True)
        assert e1 <= IMG_TOL and e2 <= IMG_TOL
    x0, y0, w, h = 1000, 1000, 40, 40
    g = np.random.default_rng(8).standard_normal((3, h, w))
    G = np.zeros((3, H, W), dtype=np.float32)
    G[:, y0:y0 + h, x0:x0 + w] = g
    gref = oracle.render_backward(d["params"], d["idx"], d["atlas"], H, W, g, None,
                                  crop=(x0, y0, w, h))
    out = R.backward(torch.tensor(G, device="cuda"), None, n_params=d["params"].shape[0])
    R.check()
    errs = grad_errs(out.cpu().numpy(), gref)
    print("window gradient errors", errs, flush=True)
    assert all(v[0] <= GRAD_TOL and v[1] <= GRAD_TOL for v in errs.values()), errs


def check_fd():
    """Steps: 1e-4 px for x, y; 1e-5 for log s and theta; 1e-2 for the logits. The image is
    piecewise bilinear in the geometric parameters with a kink at every texel boundary, and
    here a pixel spans about 7.6 texels: a step of 1e-2 px moves 15 % of the footprint's
    samples across a kink, where a central difference no longer estimates the derivative. The
    small geometric steps keep crossings below 0.2 % while the fp32 image differences stay
    ~1e3 ulp. Gate: 1e-2 relative per parameter (the floor of an fp32 difference check). The
    loss difference is formed in float64 as mean((I+ - I-)(I+ + I- - 2t))."""
    d = synth.make_workload("c2")
    dev = torch.device("cuda")
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    p0, idx, a = to_dev(d)
    tgt = torch.tensor(d["target"], device=dev)
    R = Renderer()
    p = p0.clone().requires_grad_(True)
    img, _ = render(p, R, idx, a, H, W)
    loss = ((img - tgt) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    ws = R.workspace_bytes()
    peak = torch.cuda.max_memory_allocated() - base + ws
    print("peak memory of forward + backward: %.3f GB (library workspace %.3f GB)"
          % (peak / 1e9, ws / 1e9), flush=True)
    # O(HW + N + pairs): inputs, target, image, alpha and this loss's autograd temporaries (torch's
    # allocator, about 0.38 GB: several 50 MB image-sized tensors) and the library's records,
    # lists, per-pixel (K, T_K) and padded atlas (about 0.08 GB). A per-layer cache would need
    # gigabytes here.
    assert peak < 0.6e9, peak
    g = p.grad.detach().cpu().numpy().astype(np.float64)
    R.check()

    steps = [1e-4, 1e-4, 1e-5, 1e-5, 1e-2, 1e-2, 1e-2, 1e-2]
    rng = np.random.default_rng(2602)
    picks = []
    for q in range(8):
        col = np.abs(g[:, q])
        cand = np.nonzero(col >= 0.05 * np.percentile(col, 99))[0]
        picks += [(int(i), q) for i in rng.choice(cand, 4, replace=False)]
    two_t = 2.0 * tgt
    fd = []
    with torch.no_grad():
        for i, q in picks:
            h = steps[q]
            pp = p0.clone()
            pp[i, q] += h
            Ip = R.render(pp, idx, a, H, W, None, 1.0, 16, with_alpha=False)[0].clone()
            pm = p0.clone()
            pm[i, q] -= h
            Im = R.render(pm, idx, a, H, W, None, 1.0, 16, with_alpha=False)[0]
            dL = ((Ip - Im).double() * (Ip + Im - two_t).double()).sum() / (3.0 * H * W)
            # the step actually taken: x + h rounds to a multiple of the fp32 ulp
            fd.append(float(dL) / (float(pp[i, q]) - float(pm[i, q])))
    fd = np.array(fd)
    an = np.array([g[i, q] for i, q in picks])
    rel = np.abs(fd - an) / np.maximum(np.abs(an), 1e-30)
    print("FD relative errors per column:",
          [np.round(rel[4 * q:4 * q + 4], 5).tolist() for q in range(8)], flush=True)
    assert np.all(rel < 1e-2), list(zip(picks, an, fd, rel))


CHECKS = {"windows": check_windows, "fd": check_fd}

if __name__ == "__main__":
    name = sys.argv[1] if len(sys.argv) > 1 else ""
    if name not in CHECKS:
        sys.exit("usage: c2_full_size.py windows|fd")
    print("c2 full-size check:", name, flush=True)
    assert torch.cuda.is_available(), "needs a GPU"
    CHECKS[name]()
    print("c2 full-size check passed:", name, flush=True)
