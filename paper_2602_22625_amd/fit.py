"""Plain fitting loop: render -> MSE gradient -> backward -> Adam, all in the library's kernels,
optionally captured once into a HIP graph and replayed per step (Supp. Table S1 loss/optimiser,
flat learning rate).

The per-tile list capacity is sized from the first (checked) step with headroom; replays are
asynchronous, and `run()` polls the device flags (overflow, invalid input) every `check_every`
steps. On overflow the capacity is raised, the graph is captured again and the steps since the
last good poll are repeated from a saved copy of the state.
"""
from __future__ import annotations

import torch

from . import capi
from .render import Renderer


class Fitter:
    def __init__(self, params, atlas_idx, atlas, target, bg=None, alpha_max=1.0, tile=16,
                 lr=1e-2, betas=(0.9, 0.999), eps=1e-8, renderer=None, headroom=2.0,
                 accumulate=True):
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
        self.loss_buf = torch.zeros(1, device=dev, dtype=torch.float32)
        self.R = renderer if renderer is not None else Renderer(device=dev.index, check=False)
        self.headroom = headroom
        self.accumulate = accumulate  # backward adds into grad, Adam zeroes it (no clear kernel)
        self.graph = None
        self._sized = False

    # One Adam iteration, enqueued on the current stream: forward (the atlas was stored once),
    # backward with the MSE gradient formed inside the kernel and accumulated into a gradient
    # buffer that Adam zeroes after reading: four kernels per step.
    def _enqueue(self):
        st = capi.stream_handle()
        self.R.render(self.params, self.atlas_idx, None, self.H, self.W, self.bg,
                      self.alpha_max, self.tile, image=self.image, with_alpha=False)
        self.R.backward_mse(self.target, None, out=self.grad, accumulate=self.accumulate)
        capi.dbmp_adam_step(st, self.params, self.grad, self.m, self.v, self.params.numel(),
                            self.lr, self.betas[0], self.betas[1], self.eps, self.step_count,
                            zero_grad=1 if self.accumulate else 0)

    def _size(self):
        """Store the atlas, render once synchronously and size the tile lists with headroom."""
        self.R.set_atlas(self.atlas)
        self.R.render(self.params, self.atlas_idx, None, self.H, self.W, self.bg,
                      self.alpha_max, self.tile, image=self.image, with_alpha=False)
        rc = capi.dbmp_check(self.R.ctx, capi.stream_handle())
        need = self.R.longest_list()
        capi.dbmp_reserve(self.R.ctx, int(need * self.headroom) + 1)
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
        return [self.params, self.m, self.v, self.step_count, self.grad]

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
                need = self.R.longest_list()
                capi.dbmp_reserve(self.R.ctx, int(need * max(self.headroom, 1.25)) + 1)
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
        """MSE of the image of the last step (before its Adam update; synchronises)."""
        self.R.mse_loss(self.loss_buf)
        return float(self.loss_buf[0].item()) / self.image.numel()

    def psnr(self):
        import math
        return 10.0 * math.log10(1.0 / max(self.loss(), 1e-30))
