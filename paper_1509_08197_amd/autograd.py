"""Differentiable tree aggregation (eq. C) over the hand-written adjoint.

``tree_aggregate(cost, sigma, forest, wgt=None, save_up=True)`` returns
agg(v,x) = sum_u exp(-W(v,u)/sigma) cost(u,x) and back-propagates to the cost
volume, to sigma and (if ``wgt`` is given) to the per-pixel edge weights.  The
tree topology is fixed (it comes from integer keys), so the weights and sigma
are differentiated with the topology held constant.  The weights are loaded
into the forest only while the forward and the backward of this call run (the
forest keeps its own weights otherwise), so several calls on one forest with
different weights each get their own gradients.  With ``save_up`` the
forward keeps the leaf-to-root sums U as the backward's checkpoint; without
it the backward recomputes them from the cost.
"""

from __future__ import annotations

from typing import Optional

import torch

from . import hdp


class TreeAggregate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cost, sigma, wgt, forest, save_up):
        s = float(sigma)
        with _weights(forest, wgt):
            if save_up:
                agg, up = hdp.aggregate(forest, cost.detach().contiguous(), s, keep_up=True,
                                        ws=forest_ws(forest))
            else:
                agg = hdp.aggregate(forest, cost.detach().contiguous(), s, ws=forest_ws(forest))
                up = None
        ctx.forest = forest
        ctx.sigma = s
        ctx.has_w = wgt is not None
        w_saved = wgt.detach().contiguous() if wgt is not None else torch.empty(0)
        ctx.save_for_backward(cost.detach(), agg, up if up is not None else torch.empty(0),
                              w_saved)
        ctx.save_up = save_up
        return agg

    @staticmethod
    def backward(ctx, g):
        cost, agg, up, w_saved = ctx.saved_tensors
        need_c, need_s, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        # the adjoint reads the weights from the forest: load this call's weights
        # (another call may have used other weights since), then restore
        with _weights(ctx.forest, w_saved if ctx.has_w else None):
            gc, gw, gs = hdp.aggregate_backward(
                ctx.forest, cost, agg, g.contiguous(), ctx.sigma,
                up=up if ctx.save_up else None, want_w=bool(need_w and ctx.has_w),
                want_sigma=bool(need_s), ws=forest_ws(ctx.forest))
        return (gc if need_c else None, gs.reshape(()) if gs is not None else None,
                gw if (need_w and ctx.has_w) else None, None, None)


class _weights:
    """Load per-pixel edge weights into the forest for the duration of a block and
    put the forest's own weights back afterwards (no-op for wgt None)."""

    def __init__(self, forest, wgt):
        self.forest, self.wgt, self.saved = forest, wgt, None

    def __enter__(self):
        if self.wgt is not None:
            self.saved = self.forest.array("wgt").clone()
            hdp.set_weights(self.forest, self.wgt.detach().contiguous())

    def __exit__(self, *exc):
        if self.saved is not None:
            hdp.set_weights(self.forest, self.saved)
        return False


_ws = {}


def forest_ws(forest):
    """Aggregation workspace reused by the autograd path (one per device)."""
    dev = forest.buf.device
    if dev not in _ws:
        _ws[dev] = hdp.Workspace()
    return _ws[dev]


def tree_aggregate(cost: torch.Tensor, sigma, forest: "hdp.Forest",
                   wgt: Optional[torch.Tensor] = None, save_up: bool = True) -> torch.Tensor:
    if not torch.is_tensor(sigma):
        sigma = torch.tensor(float(sigma), dtype=torch.float32, device=cost.device)
    return TreeAggregate.apply(cost, sigma, wgt, forest, save_up)
