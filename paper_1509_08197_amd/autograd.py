"""Differentiable tree aggregation (eq. C) over the hand-written adjoint.

``tree_aggregate(cost, sigma, forest, wgt=None, save_up=True)`` returns
agg(v,x) = sum_u exp(-W(v,u)/sigma) cost(u,x) and back-propagates to the cost
volume, to sigma and (if ``wgt`` is given) to the per-pixel edge weights.  The
tree topology is fixed (it comes from integer keys), so the weights and sigma
are differentiated with the topology held constant.  With ``save_up`` the
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
        if wgt is not None:
            hdp.set_weights(forest, wgt.detach().contiguous())
        s = float(sigma)
        if save_up:
            agg, up = hdp.aggregate(forest, cost.detach().contiguous(), s, keep_up=True,
                                    ws=forest_ws(forest))
        else:
            agg, up = hdp.aggregate(forest, cost.detach().contiguous(), s, ws=forest_ws(forest)), None
        ctx.forest = forest
        ctx.sigma = s
        ctx.has_w = wgt is not None
        ctx.save_for_backward(cost.detach(), agg, up if up is not None else torch.empty(0))
        ctx.save_up = save_up
        return agg

    @staticmethod
    def backward(ctx, g):
        cost, agg, up = ctx.saved_tensors
        need_c, need_s, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gc, gw, gs = hdp.aggregate_backward(
            ctx.forest, cost, agg, g.contiguous(), ctx.sigma, up=up if ctx.save_up else None,
            want_w=bool(need_w and ctx.has_w), want_sigma=bool(need_s), ws=forest_ws(ctx.forest))
        return (gc if need_c else None, gs.reshape(()) if gs is not None else None,
                gw if (need_w and ctx.has_w) else None, None, None)


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
