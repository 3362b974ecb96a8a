"""torch.autograd.Function for the Sinkhorn divergence (Def. 2.3) and its gradient (Sec. 4.2.2).

The backward pass is libshot's hand-written adjoint of Alg. 1 (balanced, or
unbalanced with a finite tau),
reached through ``shot_sinkhorn_divergence_grad``: mode "unrolled" is the exact
reverse-mode derivative of the T-iteration computation, with the forward
iterates recomputed from sqrt(T)-spaced checkpoints instead of stored;
mode "envelope" is the potential-based gradient.  With ``eager=True`` (default)
the gradient is produced in the same library call as S; with ``eager=False``
the forward computes S only and the backward recomputes everything.
"""

import math

import torch


class SinkhornDivergenceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p, q, plan, eps, T, mode, checkpoint_every, grid_of_pair, eager, tau):
        if q.requires_grad:
            raise NotImplementedError("gradients with respect to q are not provided; detach q")
        ctx.plan = plan
        ctx.args = (eps, T, mode, checkpoint_every, grid_of_pair, tau)
        ctx.eager = bool(eager) and p.requires_grad
        pd, qd = p.detach().contiguous(), q.detach().contiguous()
        if ctx.eager:
            S, g, info = plan.divergence_grad(pd, qd, eps, T=T, mode=mode, checkpoint_every=checkpoint_every,
                                              grid_of_pair=grid_of_pair, tau=tau)
            ctx.save_for_backward(g)
        else:
            S, info = plan.divergence(pd, qd, eps, tau, T=T, grid_of_pair=grid_of_pair)
            ctx.save_for_backward(pd, qd)
        ctx.info = info
        return torch.as_tensor(S, dtype=torch.float64, device=p.device)

    @staticmethod
    def backward(ctx, gS):
        plan = ctx.plan
        eps, T, mode, ck, goi, tau = ctx.args
        if ctx.eager:
            (g,) = ctx.saved_tensors
        else:
            pd, qd = ctx.saved_tensors
            _, g, _ = plan.divergence_grad(pd, qd, eps, T=T, mode=mode, checkpoint_every=ck, grid_of_pair=goi,
                                           tau=tau)
        # per-pair scaling of the per-pair gradient blocks
        goi_l = goi if goi is not None else [0] * gS.numel()
        sizes = [plan.field_size(k) for k in goi_l]
        scale = torch.repeat_interleave(gS.to(g.dtype), torch.as_tensor(sizes, device=g.device))
        grad_p = (g.reshape(-1) * scale).reshape(g.shape)
        return grad_p, None, None, None, None, None, None, None, None, None


def sinkhorn_divergence(p, q, plan, eps, T=100, mode="unrolled", checkpoint_every=0, grid_of_pair=None,
                        eager=True, tau=math.inf):
    """Differentiable S(p, q) per pair (float64 tensor of shape (npairs,)); gradient flows to p."""
    return SinkhornDivergenceFn.apply(p, q, plan, eps, T, mode, checkpoint_every, grid_of_pair, eager, tau)
