"""Multi-view training step: V views rendered in one global tile space, the
per-view L1 photometric gradient, one backward that accumulates every view's
gradients into one set, and an Adam step, all enqueued on one stream with
fixed buffers so that the whole step can be captured in one HIP graph.

    tr = MultiViewTrainer(gs, poses, targets)   # gs is updated in place
    tr.step()                                    # eager
    tr.capture(); tr.replay()                    # one graph launch per step

The loss is the mean absolute error of each view (Sec. "Preliminary of 3D
Gaussian Splatting": attributes are fitted by gradient descent on a
photometric loss between rendered and reference images), summed over the
views: dL/dC = sign(C - C*) / (3 H_v W_v) on the pixels of view v.  The
gradient is the library's backward (sgs_render_bwd) and the update the
library's Adam (sgs_adam_step); torch only supplies memory, the stream and
the elementwise sign.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _abi
from ._abi import check, load
from .raster import CameraBatch, GaussianSet, Renderer, _ptr, _stream

# learning rates per attribute (the 3DGS defaults the paper builds on; the
# appendix sets the skew's to 1e-4)
DEFAULT_LR = {"mean": 1.6e-4, "log_scale": 5e-3, "quat": 1e-3, "skew": 1e-4, "opa_logit": 5e-2,
              "sh": 2.5e-3, "opa2_logit": 5e-2, "opa_dir": 1e-4}


class Adam:
    """Adam over the parameter tensors of a GaussianSet (one library call,
    two launches per step; moments and the step count live on the device)."""

    def __init__(self, gs: GaussianSet, lr: dict | None = None, betas=(0.9, 0.999), eps: float = 1e-15):
        self.gs = gs
        self.lr = {**DEFAULT_LR, **(lr or {})}
        self.betas = betas
        self.eps = eps
        dev = gs.mean.device
        self.names = [f for f in GaussianSet.FIELDS if getattr(gs, f) is not None]
        self.m1 = {f: torch.zeros_like(getattr(gs, f)) for f in self.names}
        self.m2 = {f: torch.zeros_like(getattr(gs, f)) for f in self.names}
        self.state = torch.zeros(4, dtype=torch.float32, device=dev)
        self._groups = None
        self._grads = None

    def step(self, grads: dict, stream=None) -> None:
        if self._groups is None or self._grads is not grads:
            arr = (_abi.AdamGroup * len(self.names))()
            for k, f in enumerate(self.names):
                p, g = getattr(self.gs, f), grads[f]
                assert g is not None and g.shape == p.shape and g.is_contiguous()
                arr[k] = _abi.AdamGroup(_ptr(p), _ptr(g), _ptr(self.m1[f]), _ptr(self.m2[f]), p.numel(),
                                        float(self.lr[f]), 0)
            self._groups, self._grads = arr, grads
        check("sgs_adam_step", load().sgs_adam_step(self._groups, len(self.names), _ptr(self.state),
                                                     float(self.betas[0]), float(self.betas[1]),
                                                     float(self.eps), _stream(stream)))


def l1_weights(cams: CameraBatch, device) -> torch.Tensor:
    """Per-pixel weight 1 / (3 H_v W_v) of the views' mean absolute errors."""
    w = torch.empty(cams.total_pixels, dtype=torch.float32, device=device)
    for v in range(cams.n_views):
        c = cams.view(v)
        w[c.pix_base:c.pix_base + c.width * c.height] = 1.0 / (3.0 * c.width * c.height)
    return w


class MultiViewTrainer:
    """Training steps over a fixed set of views of one scene."""

    def __init__(self, gs: GaussianSet, poses, targets: torch.Tensor, opt: _abi.Options | None = None,
                 lr: dict | None = None, headroom: float = 1.5):
        self.gs = gs
        self.opt = opt if opt is not None else _abi.default_options()
        self.cams = CameraBatch.from_poses(poses, self.opt, gs.mean.device)
        assert targets.shape == (3, self.cams.total_pixels)
        self.targets = targets.contiguous()
        self.R = Renderer(gs, self.cams, self.opt, headroom=headroom)
        self.w = l1_weights(self.cams, gs.mean.device)
        self.adam = Adam(gs, lr)
        self.dL = torch.empty_like(self.targets)
        self.graph = None

    def step(self, stream=None) -> torch.Tensor:
        """Forward of all views, L1 gradient, backward, Adam; returns the
        rendered planes (valid until the next step)."""
        out = self.R.forward(stream)
        torch.sub(out, self.targets, out=self.dL)
        self.dL.sign_().mul_(self.w)
        grads = self.R.backward(self.dL, stream)
        self.adam.step(grads, stream)
        return out

    def loss(self) -> float:
        """Sum over views of the mean absolute error of the last forward (host sync)."""
        return float(((self.R.out_rgb - self.targets).abs() * self.w).sum())

    def capture(self):
        """Captures one step into a HIP graph (after one eager warm-up step on
        a side stream, which also allocates the backward's buffers)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self) -> None:
        self.graph.replay()

    def overflowed(self) -> bool:
        return self.R.overflowed()
