"""Masked fine-tuning of the kept Gaussians (Sec. 4.2.1-4.2.2).

After pruning by the spatial-temporal variation score and filtering with the
keyframe masks, the remaining Gaussians are optimised against the training
views for a number of iterations, each frame using the mask of its window, so
that the Gaussians the masks keep absorb what was dropped.  A step renders one
view through the library's forward, takes the adjoint of
L = 1/2 sum (I - I*)^2 through the library's backward and updates every
parameter tensor with the library's Adam kernel.  Only Gaussians processed by
some step ever receive a gradient, so the others keep their values.
"""
from __future__ import annotations

import ctypes
from typing import Callable, Dict, Optional, Sequence, Tuple

import torch

from . import _lib
from .render import Context, GaussianModel, _ptr, _stream

# per-tensor learning rates (a common choice for Gaussian splatting models)
DEFAULT_LR = {"mean": 1.6e-4, "log_scale": 5e-3, "q_left": 1e-3, "q_right": 1e-3, "opacity_logit": 5e-2,
              "sh": 2.5e-3}


class Adam:
    """Adam over the model's parameter tensors, updated in place on the device."""

    def __init__(self, ctx: Context, model: GaussianModel, lr: Optional[Dict[str, float]] = None,
                 betas: Tuple[float, float] = (0.9, 0.999), eps: float = 1e-15):
        self.ctx, self.model = ctx, model
        self.lr = dict(DEFAULT_LR if lr is None else lr)
        self.betas, self.eps = betas, eps
        self.m = {k: torch.zeros_like(getattr(model, k)) for k in GaussianModel.FIELDS}
        self.v = {k: torch.zeros_like(getattr(model, k)) for k in GaussianModel.FIELDS}
        self.t = 0

    def step(self, grads: Dict[str, torch.Tensor]):
        self.t += 1
        for k in GaussianModel.FIELDS:
            p = getattr(self.model, k)
            _lib.check(self.ctx.lib.fdgs_adam_step(
                self.ctx.handle, _ptr(p), _ptr(grads[k]), _ptr(self.m[k]), _ptr(self.v[k]),
                ctypes.c_int64(p.numel()), ctypes.c_float(self.lr[k]), ctypes.c_float(self.betas[0]),
                ctypes.c_float(self.betas[1]), ctypes.c_float(self.eps), int(self.t), _stream(self.ctx.device)))


class MaskedFineTuner:
    """views: sequence of (camera, t, target image [3, H, W] device tensor).
    mask_of(t) returns (idx, n_idx) device tensors of the frame's window, or
    None to process every Gaussian."""

    def __init__(self, ctx: Context, model: GaussianModel, views: Sequence,
                 mask_of: Optional[Callable] = None, cfg: Optional[_lib.RenderCfg] = None,
                 lr: Optional[Dict[str, float]] = None):
        self.ctx, self.model, self.views = ctx, model, list(views)
        self.mask_of = mask_of
        self.cfg = cfg if cfg is not None else _lib.default_cfg()
        self.opt = Adam(ctx, model, lr)
        self.grads = {k: torch.zeros_like(getattr(model, k)) for k in GaussianModel.FIELDS}

    def loss(self, k: int) -> float:
        cam, t, target = self.views[k % len(self.views)]
        kw = {}
        if self.mask_of is not None:
            idx, n_idx = self.mask_of(t)
            kw = dict(idx=idx, n_idx=n_idx)
        rgb, _, _ = self.ctx.render(self.model, cam, t, self.cfg, **kw)
        return 0.5 * float(((rgb - target) ** 2).sum())

    def step(self, k: int) -> float:
        """One iteration on view k (mod the number of views); returns the loss before the update."""
        cam, t, target = self.views[k % len(self.views)]
        kw = {}
        if self.mask_of is not None:
            idx, n_idx = self.mask_of(t)
            kw = dict(idx=idx, n_idx=n_idx)
        rgb, _, state = self.ctx.render(self.model, cam, t, self.cfg, keep_state=True, **kw)
        diff = rgb - target
        for g in self.grads.values():
            g.zero_()
        self.ctx.backward(state, diff, self.model, self.grads)
        self.ctx.release(state)
        self.opt.step(self.grads)
        return 0.5 * float((diff * diff).sum())
