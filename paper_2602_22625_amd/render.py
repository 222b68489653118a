"""PyTorch-facing layer over the C ABI: a Renderer (owns one dbmp context) and RenderFn, the
torch.autograd.Function whose backward is dbmp_render_backward.

PyTorch supplies device memory and the stream only; every step of the forward and backward runs
in the library's HIP kernels. The forward keeps no per-layer state: the context holds the tile
lists and O(1) values per pixel, and the backward recomputes transmittance per tile.
"""
from __future__ import annotations

import torch

from . import capi


def _dtype_code(atlas: torch.Tensor) -> int:
    if atlas.dtype == torch.float32:
        return capi.DBMP_F32
    if atlas.dtype == torch.bfloat16:
        return capi.DBMP_BF16
    if atlas.dtype == torch.float16:  # the reduced-precision raster
        return capi.DBMP_F16
    raise TypeError("atlas must be float32, bfloat16 or float16, got %s" % atlas.dtype)


def _need(t, name, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def _check_rows(t, rows, name):
    """t must be a [rows, 8] gradient or parameter table."""
    if t.dim() != 2 or t.shape[1] != 8 or t.shape[0] != rows:
        raise ValueError("%s must have shape (%d, 8), got %s" % (name, rows, tuple(t.shape)))


def _check_numel(t, n, name):
    if t.numel() != n:
        raise ValueError("%s must hold %d values (the forward's layout), got %d"
                         % (name, n, t.numel()))


def _batch_layout(descs):
    """(parameter rows, pixels) a batched call reads and writes."""
    rows = max(int(d[3]) + int(d[2]) for d in descs)
    npix = max(int(d[4]) + int(d[0]) * int(d[1]) for d in descs)
    return rows, npix


def check_backward_args(fwd, dL_dimage=None, dL_dalpha=None, out=None, target=None,
                        n_params=None):
    """Host-side size checks of a backward against the forward it differentiates. fwd =
    (rows, npix) of that forward: the kernels read 3 * npix image values (dL/dI or the MSE
    target), npix alpha values, and add into rows x 8 gradients. Pure shape logic (no device)."""
    if fwd is None:
        raise RuntimeError("no forward has run on this renderer")
    rows, npix = fwd
    if n_params is not None and int(n_params) != rows:
        raise ValueError("n_params=%d but the forward read %d parameter rows" % (n_params, rows))
    if dL_dimage is not None:
        _check_numel(dL_dimage, 3 * npix, "dL_dimage")
    if target is not None:
        _check_numel(target, 3 * npix, "target")
    if dL_dalpha is not None:
        _check_numel(dL_dalpha, npix, "dL_dalpha")
    if out is not None:
        _check_rows(out, rows, "out")


def check_batch_args(descs, params, atlas_idx, image=None, alpha=None, target=None, out=None):
    """Host-side size checks of a batched call: every image's primitive rows and pixels must lie
    inside the buffers given. Pure shape logic (no device)."""
    if not descs:
        raise ValueError("need at least one image descriptor")
    rows, npix = _batch_layout(descs)
    if params.dim() != 2 or params.shape[1] != 8 or params.shape[0] < rows:
        raise ValueError("params must be [>= %d, 8], got %s" % (rows, tuple(params.shape)))
    if atlas_idx.numel() < rows:
        raise ValueError("atlas_idx must hold >= %d values, got %d" % (rows, atlas_idx.numel()))
    if image is not None:
        _check_numel(image, 3 * npix, "image")
    if alpha is not None:
        _check_numel(alpha, npix, "alpha")
    if target is not None:
        _check_numel(target, 3 * npix, "target")
    if out is not None:
        _check_rows(out, rows, "out")
    return rows, npix


class Renderer:
    """One dbmp context. `check=True` synchronises after each forward to detect a tile list
    that did not fit, grows the capacity and renders again; `check=False` keeps every call
    asynchronous (for graph capture) and leaves overflow to an explicit `check()`."""

    def __init__(self, device=None, list_capacity: int = 0, check: bool = True):
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        self.ctx = capi.dbmp_create(dev.index, list_capacity)
        self.check_each = check
        self.generation = 0
        # device buffers the context's saved forward state points to (the backward reads the
        # image and the background): held until the next forward so they cannot be freed and
        # reused while a backward may still read them
        self._fwd_buffers = ()
        # (parameter rows, pixels) of the last forward: what a backward may read and write
        self._fwd_shape = None

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                capi.dbmp_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    def set_schedule(self, schedule, workgroups_per_cu=4, items_per_grab=1):
        """Launch schedule of the raster kernels (capi.DBMP_SCHED_*); results do not depend on
        it."""
        capi.dbmp_set_schedule(self.ctx, schedule, workgroups_per_cu, items_per_grab)

    def set_atlas_placement(self, placement):
        """Where the raster kernels read texels (capi.DBMP_ATLAS_GLOBAL or DBMP_ATLAS_LDS);
        results do not depend on it."""
        capi.dbmp_set_atlas_placement(self.ctx, placement)

    # -- atlas -------------------------------------------------------------------------------
    def set_atlas(self, atlas):
        """Pads and stores the bitmaps once; later renders may pass atlas=None."""
        if atlas.dim() == 2:
            atlas = atlas[None]
        _need(atlas, "atlas")
        B, Hb, Wb = atlas.shape
        capi.dbmp_set_atlas(self.ctx, capi.stream_handle(), atlas, B, Hb, Wb, _dtype_code(atlas))

    # -- forward -----------------------------------------------------------------------------
    def render(self, params, atlas_idx, atlas, H, W, bg=None, alpha_max=1.0, tile=16,
               image=None, alpha=None, with_alpha=True):
        """atlas=None renders with the atlas stored by set_atlas (or the previous render)."""
        _need(params, "params", torch.float32)
        N = params.shape[0]
        if params.dim() != 2 or params.shape[1] != 8:
            raise ValueError("params must be [N, 8]")
        _need(atlas_idx, "atlas_idx", torch.int32, (N,))
        if atlas is None:
            B = Hb = Wb = 0
            dcode = 0
        else:
            if atlas.dim() == 2:
                atlas = atlas[None]
            _need(atlas, "atlas")
            B, Hb, Wb = atlas.shape
            dcode = _dtype_code(atlas)
        if bg is None:
            bg = torch.ones(3, device=params.device, dtype=torch.float32)
        _need(bg, "bg", torch.float32)
        if bg.numel() == 3:
            bg_pp = 0
        elif tuple(bg.shape) == (3, H, W):
            bg_pp = 1
        else:
            raise ValueError("bg must have 3 values or shape [3, H, W]")
        if image is None:
            image = torch.empty(3, H, W, device=params.device, dtype=torch.float32)
        _need(image, "image", torch.float32, (3, H, W))
        if alpha is None and with_alpha:
            alpha = torch.empty(H, W, device=params.device, dtype=torch.float32)
        if alpha is not None:
            _need(alpha, "alpha", torch.float32, (H, W))
        st = capi.stream_handle()
        args = (self.ctx, st, params, atlas_idx, N, atlas, B, Hb, Wb, dcode, H, W,
                bg, bg_pp, alpha_max, tile, image, alpha)
        self._fwd_buffers = (image, alpha, bg)
        self._fwd_shape = (N, H * W)
        capi.dbmp_render(*args)
        if self.check_each:
            rc = capi.dbmp_check(self.ctx, st)
            if rc == capi.DBMP_EOVERFLOW:
                need = capi.dbmp_longest_list(self.ctx, st)
                capi.dbmp_reserve(self.ctx, int(need * 1.25) + 16)
                capi.dbmp_render(*args)
                rc = capi.dbmp_check(self.ctx, st)
            if rc != capi.DBMP_OK:
                raise capi.DbmpError(rc, capi.dbmp_last_error(self.ctx))
        self.generation += 1
        return image, alpha

    def render_batched(self, descs, params, atlas_idx, atlas, bg, alpha_max=1.0, tile=16,
                       image=None, alpha=None, with_alpha=True):
        """descs: list of (H, W, N, prim_offset, pixel_offset). bg: [n_images, 3]. atlas=None
        renders with the stored atlas."""
        _need(params, "params", torch.float32)
        _need(atlas_idx, "atlas_idx", torch.int32)
        _need(bg, "bg", torch.float32, (len(descs), 3))
        if atlas is None:
            B = Hb = Wb = 0
            dcode = 0
        else:
            _need(atlas, "atlas")
            B, Hb, Wb = atlas.shape
            dcode = _dtype_code(atlas)
        rows, npix = check_batch_args(descs, params, atlas_idx, image, alpha)
        if image is None:
            image = torch.empty(3 * npix, device=params.device, dtype=torch.float32)
        if alpha is None and with_alpha:
            alpha = torch.empty(npix, device=params.device, dtype=torch.float32)
        _need(image, "image", torch.float32)
        if alpha is not None:
            _need(alpha, "alpha", torch.float32)
        cd = [capi.ImageDesc(int(h), int(w), int(n), 0, int(po), int(xo))
              for (h, w, n, po, xo) in descs]
        st = capi.stream_handle()
        args = (self.ctx, st, cd, params, atlas_idx, atlas, B, Hb, Wb, dcode, bg,
                alpha_max, tile, image, alpha)
        self._fwd_buffers = (image, alpha, bg)
        self._fwd_shape = (rows, npix)
        capi.dbmp_render_batched(*args)
        if self.check_each:
            rc = capi.dbmp_check(self.ctx, st)
            if rc == capi.DBMP_EOVERFLOW:
                need = capi.dbmp_longest_list(self.ctx, st)
                capi.dbmp_reserve(self.ctx, int(need * 1.25) + 16)
                capi.dbmp_render_batched(*args)
                rc = capi.dbmp_check(self.ctx, st)
            if rc != capi.DBMP_OK:
                raise capi.DbmpError(rc, capi.dbmp_last_error(self.ctx))
        self.generation += 1
        return image, alpha

    # -- fused fit step: forward + MSE backward ----------------------------------------------
    def render_mse(self, params, atlas_idx, atlas, H, W, target, bg=None, alpha_max=1.0,
                   tile=16, image=None, out=None, accumulate=False):
        """Forward and the MSE backward in one launch per stage (dbmp_render_mse): returns
        (image, dL/dparams). With check=True an overflowing list is grown and the step redone
        when the gradient is overwritten; an accumulating caller gets the error and restores its
        own state (Fitter.run does)."""
        _need(params, "params", torch.float32)
        N = params.shape[0]
        _need(atlas_idx, "atlas_idx", torch.int32, (N,))
        _need(target, "target", torch.float32, (3, H, W))
        if atlas is None:
            B = Hb = Wb = 0
            dcode = 0
        else:
            if atlas.dim() == 2:
                atlas = atlas[None]
            _need(atlas, "atlas")
            B, Hb, Wb = atlas.shape
            dcode = _dtype_code(atlas)
        if bg is None:
            bg = torch.ones(3, device=params.device, dtype=torch.float32)
        _need(bg, "bg", torch.float32)
        bg_pp = 0 if bg.numel() == 3 else 1
        if bg_pp and tuple(bg.shape) != (3, H, W):
            raise ValueError("bg must have 3 values or shape [3, H, W]")
        if image is None:
            image = torch.empty(3, H, W, device=params.device, dtype=torch.float32)
        _need(image, "image", torch.float32, (3, H, W))
        if out is None:
            out = torch.zeros(N, 8, device=params.device, dtype=torch.float32)
        _need(out, "out", torch.float32)
        _check_rows(out, N, "out")
        st = capi.stream_handle()
        args = (self.ctx, st, params, atlas_idx, N, atlas, B, Hb, Wb, dcode, H, W, bg, bg_pp,
                alpha_max, tile, target, image, out, 1 if accumulate else 0)
        self._fwd_buffers = (image, bg)
        self._fwd_shape = (N, H * W)
        capi.dbmp_render_mse(*args)
        if self.check_each:
            rc = capi.dbmp_check(self.ctx, st)
            if rc == capi.DBMP_EOVERFLOW and not accumulate:
                need = capi.dbmp_longest_list(self.ctx, st)
                capi.dbmp_reserve(self.ctx, int(need * 1.25) + 16)
                capi.dbmp_render_mse(*args)
                rc = capi.dbmp_check(self.ctx, st)
            if rc != capi.DBMP_OK:
                raise capi.DbmpError(rc, capi.dbmp_last_error(self.ctx))
        self.generation += 1
        return image, out

    def render_batched_mse(self, descs, params, atlas_idx, atlas, bg, target, alpha_max=1.0,
                           tile=16, image=None, out=None, accumulate=False):
        """dbmp_render_batched_mse; target laid out like the batched image."""
        _need(params, "params", torch.float32)
        _need(atlas_idx, "atlas_idx", torch.int32)
        _need(bg, "bg", torch.float32, (len(descs), 3))
        _need(target, "target", torch.float32)
        if atlas is None:
            B = Hb = Wb = 0
            dcode = 0
        else:
            _need(atlas, "atlas")
            B, Hb, Wb = atlas.shape
            dcode = _dtype_code(atlas)
        rows, npix = check_batch_args(descs, params, atlas_idx, image, None, target, out)
        if image is None:
            image = torch.empty(3 * npix, device=params.device, dtype=torch.float32)
        if out is None:
            out = torch.zeros(rows, 8, device=params.device, dtype=torch.float32)
        _need(image, "image", torch.float32)
        _need(out, "out", torch.float32)
        cd = [capi.ImageDesc(int(h), int(w), int(n), 0, int(po), int(xo))
              for (h, w, n, po, xo) in descs]
        st = capi.stream_handle()
        args = (self.ctx, st, cd, params, atlas_idx, atlas, B, Hb, Wb, dcode, bg, alpha_max,
                tile, target, image, out, 1 if accumulate else 0)
        self._fwd_buffers = (image, bg)
        self._fwd_shape = (rows, npix)
        capi.dbmp_render_batched_mse(*args)
        if self.check_each:
            rc = capi.dbmp_check(self.ctx, st)
            if rc == capi.DBMP_EOVERFLOW and not accumulate:
                need = capi.dbmp_longest_list(self.ctx, st)
                capi.dbmp_reserve(self.ctx, int(need * 1.25) + 16)
                capi.dbmp_render_batched_mse(*args)
                rc = capi.dbmp_check(self.ctx, st)
            if rc != capi.DBMP_OK:
                raise capi.DbmpError(rc, capi.dbmp_last_error(self.ctx))
        self.generation += 1
        return image, out

    # -- backward ----------------------------------------------------------------------------
    def backward(self, dL_dimage, dL_dalpha=None, n_params=None, out=None):
        _need(dL_dimage, "dL_dimage", torch.float32)
        if dL_dalpha is not None:
            _need(dL_dalpha, "dL_dalpha", torch.float32)
        if n_params is None and out is None:
            raise ValueError("give n_params or out")
        check_backward_args(self._fwd_shape, dL_dimage=dL_dimage, dL_dalpha=dL_dalpha, out=out,
                            n_params=n_params)
        if out is None:
            out = torch.empty(n_params, 8, device=dL_dimage.device, dtype=torch.float32)
        _need(out, "out", torch.float32)
        capi.dbmp_render_backward(self.ctx, capi.stream_handle(), dL_dimage, dL_dalpha, out)
        return out

    def backward_mse(self, target, dL_dalpha=None, n_params=None, out=None, accumulate=False):
        """Backward of L = mean((I - target)^2) (+ any dL/dA) for the last forward; the gradient
        of the loss w.r.t. the image is formed inside the kernel. accumulate=True adds into out."""
        _need(target, "target", torch.float32)
        if dL_dalpha is not None:
            _need(dL_dalpha, "dL_dalpha", torch.float32)
        if n_params is None and out is None:
            raise ValueError("give n_params or out")
        check_backward_args(self._fwd_shape, target=target, dL_dalpha=dL_dalpha, out=out,
                            n_params=n_params)
        if out is None:
            out = torch.empty(n_params, 8, device=target.device, dtype=torch.float32)
        _need(out, "out", torch.float32)
        capi.dbmp_render_backward_mse(self.ctx, capi.stream_handle(), target, dL_dalpha, out,
                                      1 if accumulate else 0)
        return out

    def mse_loss(self, out):
        """Per-image sum of squared errors of the last backward_mse into out (device)."""
        capi.dbmp_mse_loss(self.ctx, capi.stream_handle(), out)
        return out

    def check(self):
        rc = capi.dbmp_check(self.ctx, capi.stream_handle())
        if rc != capi.DBMP_OK:
            raise capi.DbmpError(rc, capi.dbmp_last_error(self.ctx))

    def longest_list(self):
        return capi.dbmp_longest_list(self.ctx, capi.stream_handle())

    def workspace_bytes(self):
        """Device bytes the library's own workspace holds (not counted by torch's allocator)."""
        return capi.dbmp_workspace_bytes(self.ctx)


class RenderFn(torch.autograd.Function):
    """(image, alpha) = RenderFn.apply(params, renderer, atlas_idx, atlas, H, W, bg, alpha_max,
    tile). Differentiable in params only. The backward re-runs the forward on the renderer if
    another forward has used it since (its saved per-tile state belongs to the last one)."""

    @staticmethod
    def forward(fctx, params, renderer, atlas_idx, atlas, H, W, bg, alpha_max, tile):
        fctx.set_materialize_grads(False)
        p = params.detach()
        image, alpha = renderer.render(p, atlas_idx, atlas, H, W, bg, alpha_max, tile)
        fctx.renderer = renderer
        fctx.generation = renderer.generation
        fctx.cfg = (H, W, alpha_max, tile)
        fctx.save_for_backward(p, atlas_idx, atlas, bg)
        return image, alpha

    @staticmethod
    def backward(fctx, g_image, g_alpha):
        p, atlas_idx, atlas, bg = fctx.saved_tensors
        r = fctx.renderer
        H, W, alpha_max, tile = fctx.cfg
        if r.generation != fctx.generation:
            r.render(p, atlas_idx, atlas, H, W, bg, alpha_max, tile)
        if g_image is None:
            g_image = torch.zeros(3, H, W, device=p.device, dtype=torch.float32)
        d = r.backward(g_image.contiguous(), None if g_alpha is None else g_alpha.contiguous(),
                       n_params=p.shape[0])
        return d, None, None, None, None, None, None, None, None


def render(params, renderer, atlas_idx, atlas, H, W, bg=None, alpha_max=1.0, tile=16):
    if bg is None:
        bg = torch.ones(3, device=params.device, dtype=torch.float32)
    return RenderFn.apply(params, renderer, atlas_idx, atlas, H, W, bg, alpha_max, tile)
