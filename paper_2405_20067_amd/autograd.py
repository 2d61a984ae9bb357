"""torch.autograd layer over libngd: the mixture's colour as a differentiable
function of its parameters, with the library's hand-written backward.

Raw parameters and their activations (torch ops, so autograd carries the
chain rule through them):

    Sec. 3.1  factor L: diagonal entries exp(x), strictly-lower entries
              2 sigmoid(x) - 1 (the lower triangle of L; the text's "i < j"
              is read as the strictly-lower entries i > j of a lower factor)
    Sec. 4.1  brightness alpha = exp(a), colour c = sigmoid(c_raw)
    mean      used as it is

`NgdMixtureEval` takes the activated values.  Its forward loads them into a
library mixture (ngd_mixture_update: float64 inversion on the device),
rebuilds the cull for the queries (ngd_cull_build) and evaluates
(ngd_eval); its backward calls ngd_eval_backward, which returns the
gradients with respect to the activated mean, factor, weight and colour.
`NgdL2Loss` wraps the library's squared-error losses the same way.  All
arithmetic runs in the library's kernels on torch's current stream.
"""

from __future__ import annotations

import torch

from . import ngd

__all__ = ["diag_mask", "activate_factor", "raw_factor", "activate", "Evaluator",
           "NgdMixtureEval", "NgdComposedEval", "NgdL2Loss", "mixture_eval", "GaussianMixture"]


def diag_mask(n: int, device=None) -> torch.Tensor:
    """Boolean mask of the diagonal entries of a packed lower factor (entry
    i(i+1)/2 + j holds (i, j), j <= i)."""
    r, c = torch.tril_indices(n, n, device=device)
    return r == c


def activate_factor(raw: torch.Tensor, n: int) -> torch.Tensor:
    """Sec. 3.1: exp on the diagonal, 2 sigmoid - 1 on the strictly-lower
    entries; `raw` is (K, n(n+1)/2) packed by rows."""
    d = diag_mask(n, raw.device)
    # exp only where it is taken: a large strictly-lower raw value would
    # otherwise give exp = inf and a NaN gradient through the unused branch
    return torch.where(d, torch.exp(torch.where(d, raw, torch.zeros_like(raw))),
                       2.0 * torch.sigmoid(raw) - 1.0)


def raw_factor(factor: torch.Tensor, n: int, margin: float = 1e-6) -> torch.Tensor:
    """Inverse of activate_factor for a factor with a positive diagonal.
    Strictly-lower entries are clamped into (-1, 1) by `margin` first (the
    activation's range)."""
    d = diag_mask(n, factor.device)
    off = factor.clamp(-1.0 + margin, 1.0 - margin)
    return torch.where(d, torch.log(factor.clamp_min(torch.finfo(factor.dtype).tiny)),
                       torch.log1p(off) - torch.log1p(-off))


def activate(raw_mean, raw_fac, raw_weight, raw_colour):
    """(mean, L, alpha, c) from raw parameters (Sec. 3.1, Sec. 4.1)."""
    n = raw_mean.shape[1]
    return (raw_mean, activate_factor(raw_fac, n), torch.exp(raw_weight),
            torch.sigmoid(raw_colour))


class Evaluator:
    """What one differentiable evaluation needs besides the parameters: the
    projection vectors and cull parameters (`proj` None: dense, no cull),
    the forward's precision, and the library handles, reused from call to
    call (the mixture handle is recreated when the number of Gaussians
    changes; the cull is rebuilt in place).

    One Evaluator serves one live graph at a time: a second forward before
    the first one's backward updates the same handles, and that backward
    then raises instead of returning gradients of other parameters."""

    def __init__(self, n: int, proj=None, params: ngd.CullParams | None = None,
                 precision: int = ngd.FP32):
        self.n = int(n)
        self.proj = proj
        self.params = params if params is not None or proj is None else ngd.default_params()
        self.precision = precision
        self.mix: ngd.Mixture | None = None
        self.cull = ngd.Cull() if proj is not None else None

    def mixture(self, k: int) -> ngd.Mixture:
        if self.mix is None or self.mix.k != k:
            self.mix = ngd.Mixture(self.n, k)
        return self.mix


def _f32(t: torch.Tensor) -> torch.Tensor:
    return t.detach().to(torch.float32).contiguous()


class NgdMixtureEval(torch.autograd.Function):
    """f(x) = sum over each query's culled candidates of
    G_i(x - m_i) alpha_i c_i (Sec. 4.1, Eq. 8), (q, 3) float32, from
    activated parameters mean (K, n), factor (K, n(n+1)/2), weight (K,),
    colour (K, 3) and queries (q, n).  No gradient for the queries."""

    @staticmethod
    def forward(ctx, mean, factor, weight, colour, queries, ev: Evaluator):
        k = mean.shape[0]
        mix = ev.mixture(k)
        x = _f32(queries)
        mix.update(_f32(mean), _f32(factor), _f32(weight), _f32(colour))
        if ev.cull is not None:
            ev.cull.build(mix, x, ev.proj, ev.params)
        f = ngd.eval_mixture(mix, ev.cull, x, precision=ev.precision)
        ctx.ev, ctx.mix, ctx.version = ev, mix, mix.info()[2]
        ctx.save_for_backward(x)
        return f

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_f):
        (x,) = ctx.saved_tensors
        ev, mix = ctx.ev, ctx.mix
        if ev.mix is not mix or mix.info()[2] != ctx.version:
            raise RuntimeError("NgdMixtureEval: the Evaluator was used for another forward "
                               "before this backward; use one Evaluator per live graph")
        gm, gf, gw, gc = ngd.eval_backward(mix, ev.cull, x, _f32(grad_f),
                                           precision=ev.precision)
        return gm, gf, gw, gc, None, None


class NgdComposedEval(torch.autograd.Function):
    """f(x) like NgdMixtureEval for a mixture of kp parents and kc children
    given relative to their parents (Sec. 3.3, Eq. 6-7), composed inside the
    library (ngd_mixture_update_composed; backward
    ngd_eval_backward_composed): mean (kp, n) and factor (kp, n(n+1)/2) of
    the parents, weight (k,) and colour (k, 3) of all, parent (kc,) int32
    non-decreasing, rel_factor U (kc, n(n+1)/2), rel_mean m_u (kc, n).
    Gradients flow to every float argument."""

    @staticmethod
    def forward(ctx, mean, factor, weight, colour, parent, rel_factor, rel_mean, queries,
                ev: Evaluator):
        k = weight.shape[0]
        mix = ev.mixture(k)
        x = _f32(queries)
        mix.update_composed(mean.shape[0], _f32(mean), _f32(factor), _f32(weight), _f32(colour),
                            parent.detach().to(torch.int32).contiguous(), _f32(rel_factor),
                            _f32(rel_mean))
        if ev.cull is not None:
            ev.cull.build(mix, x, ev.proj, ev.params)
        f = ngd.eval_mixture(mix, ev.cull, x, precision=ev.precision)
        ctx.ev, ctx.mix, ctx.version = ev, mix, mix.info()[2]
        ctx.save_for_backward(x)
        return f

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_f):
        (x,) = ctx.saved_tensors
        ev, mix = ctx.ev, ctx.mix
        if ev.mix is not mix or mix.info()[2] != ctx.version:
            raise RuntimeError("NgdComposedEval: the Evaluator was used for another forward "
                               "before this backward; use one Evaluator per live graph")
        gm, gf, gw, gc, gu, gmu = ngd.eval_backward_composed(mix, ev.cull, x, _f32(grad_f),
                                                            precision=ev.precision)
        return gm, gf, gw, gc, None, gu, gmu, None, None


class NgdL2Loss(torch.autograd.Function):
    """Mean squared error of f (q, 3) against target, or with eps > 0 the
    relative one of Sec. 4.1 (weights 1/(|f| + eps)^2 held constant), as a
    one-element tensor; the library returns its gradient with the value."""

    @staticmethod
    def forward(ctx, f, target, eps: float = 0.0):
        if eps > 0.0:
            loss, grad = ngd.rel_l2_loss(_f32(f), _f32(target), eps=eps)
        else:
            loss, grad = ngd.l2_loss(_f32(f), _f32(target))
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_loss):
        (grad,) = ctx.saved_tensors
        return grad * grad_loss.reshape(()), None, None


def mixture_eval(raw_mean, raw_fac, raw_weight, raw_colour, queries, ev: Evaluator):
    """The colours at the queries from raw parameters: activations in torch,
    then NgdMixtureEval."""
    return NgdMixtureEval.apply(*activate(raw_mean, raw_fac, raw_weight, raw_colour),
                                queries, ev)


class GaussianMixture(torch.nn.Module):
    """A mixture of K Gaussians in n dimensions with raw parameters as
    nn.Parameters; forward(queries) gives the (q, 3) colours through the
    library, differentiable in every parameter."""

    def __init__(self, mean, factor, weight, colour, proj=None, params=None,
                 precision: int = ngd.FP32):
        super().__init__()
        n = mean.shape[1]
        f32 = lambda t: t.detach().to(torch.float32).clone()
        self.mean = torch.nn.Parameter(f32(mean))
        self.factor_raw = torch.nn.Parameter(raw_factor(f32(factor), n))
        self.weight_raw = torch.nn.Parameter(torch.log(f32(weight)))
        self.colour_raw = torch.nn.Parameter(torch.logit(f32(colour).clamp(1e-6, 1 - 1e-6)))
        self.ev = Evaluator(n, proj, params, precision)

    def activated(self):
        return activate(self.mean, self.factor_raw, self.weight_raw, self.colour_raw)

    def forward(self, queries):
        return mixture_eval(self.mean, self.factor_raw, self.weight_raw, self.colour_raw,
                            queries, self.ev)
