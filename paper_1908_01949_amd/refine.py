"""torch.autograd view of the differentiated refinement (argument marshalling only).

``Refinement`` owns a refinement setup on a ``rknscan.Context`` whose outputs are
device pointers; ``residuals(seeds)`` returns the inlier residuals r = D - d of every
seed as a tensor whose backward runs the library's adjoint sweep. Every number is
computed by the HIP kernels behind ``rkn_residuals_fwd`` and ``rkn_adjoint_bwd``:
the forward records checkpoints of the propagation and the adjoint of that
forward is the only backward the library holds, so a backward must follow the last
forward of its ``Refinement`` (this is checked).
"""
from __future__ import annotations

import numpy as np
import torch

from . import rknscan as rk


class Refinement:
    """Seeds grouped by event (non-decreasing ``seed_event``), their inlier sets fixed
    by the classification rule at ``seeds5``; checkpoints every ``ckpt_every`` steps."""

    def __init__(self, context: rk.Context, params: rk.rkn_scan_params, seed_event, seeds5,
                 ckpt_every: int = 64):
        if not getattr(context, "stream", None):
            raise ValueError("create the Context on a torch stream, e.g. rknscan.Context(0, "
                             "torch.cuda.Stream().cuda_stream): its work is ordered with torch's "
                             "through that stream")
        self._stream = torch.cuda.ExternalStream(context.stream)
        params.ptr_flags = rk.RKN_PTR_DEVICE
        self.context = context
        se = np.ascontiguousarray(seed_event, np.int32)
        s5 = np.ascontiguousarray(np.asarray(seeds5, np.float64).reshape(-1, 5))
        rk.rkn_refine_setup(context.ctx, params, se, s5, ckpt_every)
        self.n = se.size
        self.H = max(getattr(context, "max_hits", 0), 1)
        self._token = 0

    def _enter(self):
        cur = torch.cuda.current_stream()
        self._stream.wait_stream(cur)
        return cur

    def _leave(self, cur):
        cur.wait_stream(self._stream)

    def residuals(self, seeds: torch.Tensor) -> torch.Tensor:
        """[n][H] FP32 inlier residuals (NaN outside the inlier set and past an event's
        hits); differentiable with respect to ``seeds`` ([n][5] FP64 on the device)."""
        return RknResiduals.apply(seeds, self)

    def phi(self, seeds: torch.Tensor) -> torch.Tensor:
        """Phi = sum of squared inlier residuals per seed, FP64 (not differentiable)."""
        resid = torch.empty((self.n, self.H), dtype=torch.float32, device=seeds.device)
        out = torch.empty(self.n, dtype=torch.float64, device=seeds.device)
        s = seeds.detach().contiguous()
        cur = self._enter()
        rk.rkn_residuals_fwd(self.context.ctx, s, resid, out)
        self._leave(cur)
        self._token += 1
        return out

    def gauss_newton(self, iters: int = 10, scale=(1.0, 100.0, 100.0, 100.0, 100.0), device="cuda"):
        """Gauss-Newton from the setup seeds: (refined seeds [n][5], Phi [n][iters+1])."""
        seeds = torch.empty((self.n, 5), dtype=torch.float64, device=device)
        phi = torch.empty((self.n, iters + 1), dtype=torch.float64, device=device)
        cur = self._enter()
        rk.rkn_gn_refine(self.context.ctx, iters, np.asarray(scale, np.float64), seeds, phi)
        self._leave(cur)
        self._token += 1
        return seeds, phi


class RknResiduals(torch.autograd.Function):
    @staticmethod
    def forward(ctx, seeds: torch.Tensor, ref: Refinement):
        if seeds.dtype != torch.float64 or seeds.shape != (ref.n, 5) or not seeds.is_cuda:
            raise ValueError(f"seeds must be a [{ref.n}][5] float64 device tensor")
        resid = torch.empty((ref.n, ref.H), dtype=torch.float32, device=seeds.device)
        s = seeds.detach().contiguous()
        cur = ref._enter()
        rk.rkn_residuals_fwd(ref.context.ctx, s, resid, None)
        ref._leave(cur)
        ref._token += 1
        ctx.ref = ref
        ctx.token = ref._token
        return resid

    @staticmethod
    def backward(ctx, grad_resid: torch.Tensor):
        ref = ctx.ref
        if ref._token != ctx.token:
            raise RuntimeError("the adjoint needs the checkpoints of the last forward pass of this "
                               "Refinement; run the forward again before backward")
        # entries outside the inlier set (NaN residuals) are never read by the adjoint
        g = grad_resid.detach().to(torch.float32).contiguous()
        d_seed = torch.empty((ref.n, 5), dtype=torch.float64, device=grad_resid.device)
        cur = ref._enter()
        rk.rkn_adjoint_bwd(ref.context.ctx, g, d_seed, None, None)
        ref._leave(cur)
        return d_seed, None
