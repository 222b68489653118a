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
                 accumulate=True, fused=True, adam_in_binning=True):
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
        # [updates applied, scratch counter, gradient pending, unused]
        self.step_count = torch.zeros(4, dtype=torch.int32, device=dev)
        self.grad = torch.zeros_like(self.params)
        self.image = torch.empty(3, self.H, self.W, device=dev, dtype=torch.float32)
        self.loss_buf = torch.zeros(1, device=dev, dtype=torch.float32)
        self.R = renderer if renderer is not None else Renderer(device=dev.index, check=False)
        self.headroom = headroom
        self.accumulate = accumulate  # backward adds into grad, Adam zeroes it (no clear kernel)
        self.fused = fused  # forward and MSE backward in one launch (dbmp_render_mse)
        # the binning applies the previous step's Adam update (dbmp_fit_step): two launches per
        # step; the last gradient stays pending until flush()
        self.adam_in_binning = fused and accumulate and adam_in_binning
        self.graph = None
        self._graph_steps = 1
        self._graph_epoch = -1
        self._hold = None
        self._sized = False

    # One Adam iteration, enqueued on the current stream. dbmp_fit_step: binning (with the
    # pending Adam update) and the fused forward + MSE backward. Otherwise: forward (the atlas was
    # stored once), the MSE backward (fused into the forward or a launch of its own) accumulating
    # into a gradient buffer, and Adam, which zeroes it.
    def _render(self):
        self.R.render(self.params, self.atlas_idx, None, self.H, self.W, self.bg,
                      self.alpha_max, self.tile, image=self.image, with_alpha=False)

    def _render_mse(self):
        self.R.render_mse(self.params, self.atlas_idx, None, self.H, self.W, self.target,
                          self.bg, self.alpha_max, self.tile, image=self.image, out=self.grad,
                          accumulate=self.accumulate)

    def _fit_step(self, st):
        capi.dbmp_fit_step(self.R.ctx, st, self.params, self.atlas_idx, self.N, self.H, self.W,
                           self.bg, 0 if self.bg.numel() == 3 else 1, self.alpha_max, self.tile,
                           self.target, self.image, self.grad, self.m, self.v, self.step_count,
                           self.lr, self.betas[0], self.betas[1], self.eps)
        self.R._fwd_buffers = (self.image, self.bg)
        self.R._fwd_shape = (self.N, self.H * self.W)

    def flush(self):
        """Apply the Adam update of a gradient left pending by the last step (synchronises)."""
        if self.adam_in_binning and int(self.step_count[2].item()):
            capi.dbmp_adam_step(capi.stream_handle(), self.params, self.grad, self.m, self.v,
                                self.params.numel(), self.lr, self.betas[0], self.betas[1],
                                self.eps, self.step_count, zero_grad=1)
            self.step_count[2] = 0
        return self

    def _held_step(self):
        if self._hold is not None:
            self.params.copy_(self._hold)
        self._enqueue()

    def _enqueue(self):
        st = capi.stream_handle()
        if self.adam_in_binning:
            self._fit_step(st)
            return
        if self.fused:
            self._render_mse()
        else:
            self._render()
            self.R.backward_mse(self.target, None, out=self.grad, accumulate=self.accumulate)
        capi.dbmp_adam_step(st, self.params, self.grad, self.m, self.v, self.params.numel(),
                            self.lr, self.betas[0], self.betas[1], self.eps, self.step_count,
                            zero_grad=1 if self.accumulate else 0)

    def _size(self):
        """Store the atlas, render once synchronously and size the tile lists with headroom."""
        self.R.set_atlas(self.atlas)
        self._render()
        rc = capi.dbmp_check(self.R.ctx, capi.stream_handle())
        need = self.R.longest_list()
        capi.dbmp_reserve(self.R.ctx, int(need * self.headroom) + 1)
        if rc not in (capi.DBMP_OK, capi.DBMP_EOVERFLOW):
            raise capi.DbmpError(rc, capi.dbmp_last_error(self.R.ctx))
        self._sized = True

    def step(self):
        """One replay of the captured graph (graph_steps Adam iterations), else one eager
        iteration."""
        if not self._sized:
            self._size()
        if self.graph is not None and \
                capi.dbmp_workspace_epoch(self.R.ctx) != self._graph_epoch:
            # the context's workspace was reallocated since the capture (another caller of the
            # same renderer needed more room): the graph's addresses are stale
            self.graph = None
            self.capture(self._graph_steps, self._hold)
        if self.graph is not None:
            self.graph.replay()
        else:
            self._enqueue()

    @property
    def graph_steps(self):
        """Adam iterations per step() call."""
        return self._graph_steps if self.graph is not None else 1

    def _state(self):
        return [self.params, self.m, self.v, self.step_count, self.grad]

    def snapshot(self):
        return [t.clone() for t in self._state()]

    def restore(self, snap):
        for t, c in zip(self._state(), snap):
            t.copy_(c)

    def capture(self, steps_per_graph=1, hold=None):
        """Capture `steps_per_graph` Adam iterations into one HIP graph (replayed by step()):
        several iterations per replay spread the host's replay cost, the optimiser state being
        on the device. A warm-up step runs first on a side stream (first launches of every
        kernel, no workspace growth inside the capture); its effect on the optimiser state is
        undone, so capturing does not alter the trajectory.
        hold: a device tensor of parameters; every captured iteration first copies it into the
        fit's parameters (one device copy), so that each step starts from the same primitives:
        a measurement of the step at a fixed state, which the number of steps cannot move."""
        if steps_per_graph < 1:
            raise ValueError("steps_per_graph must be >= 1")
        if not self._sized:
            self._size()
        self._hold = hold
        snap = self.snapshot()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._held_step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.restore(snap)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(steps_per_graph):
                self._held_step()
        self.graph = g
        self._graph_steps = steps_per_graph
        self._graph_epoch = capi.dbmp_workspace_epoch(self.R.ctx)

    def run(self, steps, check_every=50):
        """`steps` Adam iterations; every `check_every` steps the device flags are polled. On a
        full pair buffer the steps since the last good poll are redone with a larger buffer."""
        done = 0
        snap = self.snapshot()
        while done < steps:
            k = min(check_every, steps - done)
            gs = self.graph_steps
            for _ in range(k // gs):
                self.step()
            for _ in range(k % gs):  # the remainder eagerly
                self._enqueue()
            rc = capi.dbmp_check(self.R.ctx, capi.stream_handle())
            if rc == capi.DBMP_EOVERFLOW:
                self.restore(snap)
                need = self.R.longest_list()
                capi.dbmp_reserve(self.R.ctx, int(need * max(self.headroom, 1.25)) + 1)
                if self.graph is not None:
                    self.graph = None
                    self.capture(gs, self._hold)
                continue
            if rc != capi.DBMP_OK:
                raise capi.DbmpError(rc, capi.dbmp_last_error(self.R.ctx))
            done += k
            snap = self.snapshot()
        return self.flush()

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

    def set_launch(self, tile, schedule, workgroups_per_cu=4, items_per_grab=1):
        """Tile size and launch schedule; drops a captured graph and re-sizes the lists."""
        self.tile = tile
        self.R.set_schedule(schedule, workgroups_per_cu, items_per_grab)
        self.graph = None
        self._sized = False

    def autotune(self, tuner, key, steps=3, cands=None, force=False):
        """Choose tile size and schedule with `tuner` (an autotune.Autotuner): each candidate
        runs `steps` timed eager steps after a sizing step; the optimiser state is restored
        afterwards, so tuning leaves the trajectory unchanged. Returns the chosen cfg."""
        snap = self.snapshot()

        def measure(cfg):
            self.set_launch(*cfg)
            self.step()  # sizing and first launches, untimed
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                self.step()
            e1.record(st)
            self.check()
            self.restore(snap)
            return e0.elapsed_time(e1) * 1e-3 / steps

        best = tuner.tune(key, measure, cands, force)
        self.restore(snap)
        self.set_launch(*best)
        return best


class BatchFitter(Fitter):
    """Many independent fits advanced together: one batched forward (all images' tiles in one
    launch per stage), one MSE backward, one Adam over all parameters, captured as one graph
    per step. fits: list of (params [N_i, 8], atlas_idx [N_i], target [3, H_i, W_i]) on the
    device; images share the atlas, alpha_max and the tile size. bg: [n_images, 3] or None
    (white)."""

    def __init__(self, fits, atlas, bg=None, alpha_max=1.0, tile=16, lr=1e-2,
                 betas=(0.9, 0.999), eps=1e-8, renderer=None, headroom=2.0, fused=True,
                 adam_in_binning=True):
        dev = fits[0][0].device
        self.descs = []
        prim, pix = 0, 0
        for p, _, t in fits:
            H, W = int(t.shape[1]), int(t.shape[2])
            self.descs.append((H, W, int(p.shape[0]), prim, pix))
            prim += int(p.shape[0])
            pix += H * W
        self.n_images = len(fits)
        self.params = torch.cat([p.detach().float() for p, _, _ in fits]).contiguous()
        self.N = self.params.shape[0]
        self.atlas_idx = torch.cat([i for _, i, _ in fits]).contiguous()
        self.atlas = atlas
        self.target = torch.cat([t.reshape(-1) for _, _, t in fits]).contiguous()
        self.bg = bg if bg is not None else torch.ones(self.n_images, 3, device=dev)
        self.alpha_max, self.tile = alpha_max, tile
        self.lr, self.betas, self.eps = lr, betas, eps
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = torch.zeros(4, dtype=torch.int32, device=dev)
        self.grad = torch.zeros_like(self.params)
        self.image = torch.empty(3 * pix, device=dev, dtype=torch.float32)
        self.loss_buf = torch.zeros(self.n_images, device=dev, dtype=torch.float32)
        self.R = renderer if renderer is not None else Renderer(device=dev.index, check=False)
        self.headroom = headroom
        self.accumulate = True
        self.fused = fused
        self.adam_in_binning = fused and adam_in_binning
        self.graph = None
        self._graph_steps = 1
        self._graph_epoch = -1
        self._hold = None
        self._sized = False

    def _render(self):
        self.R.render_batched(self.descs, self.params, self.atlas_idx, None, self.bg,
                              self.alpha_max, self.tile, image=self.image, with_alpha=False)

    def _fit_step(self, st):
        capi.dbmp_fit_step_batched(self.R.ctx, st, self._cdescs(), self.params, self.atlas_idx,
                                   self.bg, self.alpha_max, self.tile, self.target, self.image,
                                   self.grad, self.m, self.v, self.step_count, self.lr,
                                   self.betas[0], self.betas[1], self.eps)
        self.R._fwd_buffers = (self.image, self.bg)
        self.R._fwd_shape = (self.N, self.image.numel() // 3)

    def _cdescs(self):
        return [capi.ImageDesc(int(h), int(w), int(n), 0, int(po), int(xo))
                for (h, w, n, po, xo) in self.descs]

    def _render_mse(self):
        self.R.render_batched_mse(self.descs, self.params, self.atlas_idx, None, self.bg,
                                  self.target, self.alpha_max, self.tile, image=self.image,
                                  out=self.grad, accumulate=True)

    def shapes(self):
        return [(h, w, n) for (h, w, n, _, _) in self.descs]

    def losses(self):
        """Per-image MSE of the last step's images (synchronises)."""
        self.R.mse_loss(self.loss_buf)
        sse = self.loss_buf.double().cpu()
        return [float(sse[i]) / (3 * h * w) for i, (h, w, _, _, _) in enumerate(self.descs)]

    def loss(self):
        return sum(self.losses()) / self.n_images

    def psnrs(self):
        import math
        return [10.0 * math.log10(1.0 / max(l, 1e-30)) for l in self.losses()]

    def image_of(self, i):
        h, w, _, _, po = self.descs[i]
        return self.image[3 * po:3 * (po + h * w)].view(3, h, w)

    def params_of(self, i):
        _, _, n, pr, _ = self.descs[i]
        return self.params[pr:pr + n]
