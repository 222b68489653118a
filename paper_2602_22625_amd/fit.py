"""Plain fitting loop: render -> MSE gradient -> backward -> Adam, all in the library's kernels,
optionally captured once into a HIP graph and replayed per step (Supp. Table S1 loss/optimiser,
flat learning rate).

The pair buffer is sized from the first (checked) step with headroom; replays are asynchronous,
and `check()` polls the device flags (overflow, invalid input) every `check_every` steps. On
overflow the buffer is grown, the graph is captured again and the steps since the last good
check are repeated from a saved copy of the state.
"""
from __future__ import annotations

import torch

from . import capi
from .render import Renderer


class Fitter:
    def __init__(self, params, atlas_idx, atlas, target, bg=None, alpha_max=1.0, tile=16,
                 lr=1e-2, betas=(0.9, 0.999), eps=1e-8, renderer=None, headroom=2.0):
        dev = params.device
        self.H, self.W = int(target.shape[1]), int(target.shape[2])
        self.params = params.detach().clone().contiguous()
        self.N = self.params.shape[0]
        self.atlas_idx = atlas_idx
        self.atlas = atlas
        self.target = target.contiguous()
        self.bg = bg if bg is not None else torch.ones(3, device=dev, dtype=torch.float32)
        self.alpha_max, self.tile = alpha_max, tile
        self.lr, self.betas, self.eps = lr, betas, eps
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = torch.zeros(2, dtype=torch.int32, device=dev)  # [steps, scratch]
        self.grad = torch.zeros_like(self.params)
        self.image = torch.empty(3, self.H, self.W, device=dev, dtype=torch.float32)
        self.gimage = torch.empty_like(self.image)
        self.loss_buf = torch.zeros(3, device=dev, dtype=torch.float32)  # [sum sq, scratch x2]
        self.R = renderer if renderer is not None else Renderer(device=dev.index, check=False)
        self.headroom = headroom
        self.graph = None
        self._sized = False

    # one Adam iteration, enqueued on the current stream
    def _enqueue(self):
        st = capi.stream_handle()
        self.R.render(self.params, self.atlas_idx, self.atlas, self.H, self.W, self.bg,
                      self.alpha_max, self.tile, image=self.image, with_alpha=False)
        capi.dbmp_mse_grad(st, self.image, self.target, self.image.numel(), self.gimage,
                           self.loss_buf)
        self.R.backward(self.gimage, None, out=self.grad)
        capi.dbmp_adam_step(st, self.params, self.grad, self.m, self.v, self.params.numel(),
                            self.lr, self.betas[0], self.betas[1], self.eps, self.step_count)

    def _size(self):
        """Render once synchronously and size the pair buffer with headroom."""
        self.R.render(self.params, self.atlas_idx, self.atlas, self.H, self.W, self.bg,
                      self.alpha_max, self.tile, image=self.image, with_alpha=False)
        rc = capi.dbmp_check(self.R.ctx, capi.stream_handle())
        need = self.R.pair_count()
        capi.dbmp_reserve(self.R.ctx, int(need * self.headroom) + 4096)
        if rc not in (capi.DBMP_OK, capi.DBMP_EOVERFLOW):
            raise capi.DbmpError(rc, capi.dbmp_last_error(self.R.ctx))
        self._sized = True

    def step(self):
        if not self._sized:
            self._size()
        if self.graph is not None:
            self.graph.replay()
        else:
            self._enqueue()

    def _state(self):
        return [self.params, self.m, self.v, self.step_count]

    def snapshot(self):
        return [t.clone() for t in self._state()]

    def restore(self, snap):
        for t, c in zip(self._state(), snap):
            t.copy_(c)

    def capture(self):
        """Capture one Adam iteration into a HIP graph. A warm-up step runs first on a side
        stream (first launches of every kernel, no workspace growth inside the capture); its
        effect on the optimiser state is undone, so capturing does not alter the trajectory."""
        if not self._sized:
            self._size()
        snap = self.snapshot()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._enqueue()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.restore(snap)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._enqueue()
        self.graph = g

    def run(self, steps, check_every=50):
        """`steps` Adam iterations; every `check_every` steps the device flags are polled. On a
        full pair buffer the steps since the last good poll are redone with a larger buffer."""
        done = 0
        snap = self.snapshot()
        while done < steps:
            k = min(check_every, steps - done)
            for _ in range(k):
                self.step()
            rc = capi.dbmp_check(self.R.ctx, capi.stream_handle())
            if rc == capi.DBMP_EOVERFLOW:
                self.restore(snap)
                need = self.R.pair_count()
                capi.dbmp_reserve(self.R.ctx, int(need * self.headroom) + 4096)
                if self.graph is not None:
                    self.graph = None
                    self.capture()
                continue
            if rc != capi.DBMP_OK:
                raise capi.DbmpError(rc, capi.dbmp_last_error(self.R.ctx))
            done += k
            snap = self.snapshot()
        return self

    def check(self):
        """Synchronise and raise on device-side errors (overflow included)."""
        rc = capi.dbmp_check(self.R.ctx, capi.stream_handle())
        if rc != capi.DBMP_OK:
            raise capi.DbmpError(rc, capi.dbmp_last_error(self.R.ctx))

    def loss(self):
        """MSE of the last rendered image (synchronises)."""
        return float(self.loss_buf[0].item()) / self.image.numel()

    def psnr(self):
        import math
        return 10.0 * math.log10(1.0 / max(self.loss(), 1e-30))
