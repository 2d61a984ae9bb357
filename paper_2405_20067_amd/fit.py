"""Fitting loop on the culled path, with optimisation-controlled refinement.

Each step runs the library's path unchanged (ngd_mixture_update,
ngd_cull_build, ngd_eval, the loss, ngd_eval_backward); torch holds the raw
parameters, applies the activations of Sec. 4.1 (brightness alpha = exp(a),
colour c = sigmoid(c_raw); mean and factor L are used as they are) and the
parent-child composition of Sec. 3.3, takes the chain rule from the
library's gradients with respect to the activated parameters, and steps
Adam.

Refinement (Sec. 3.3, Eq. 6-7): from the second phase on, every parent
carries one child defined in the parent's frame by a relative factor U
(lower triangular) and offset m_u:

    L_child = L_parent U,    m_child = L_parent m_u + m_parent,

so that the child follows every update of its parent.  A new child spans its
parent (U = I, m_u = 0 up to a small random perturbation) with a negligible
brightness.  At the end of each phase the children whose brightness exceeds
the threshold t are materialised: they become parents (with their absolute
parameters, so the represented function does not change), and their slot,
like every new parent, gets a fresh default child.
"""

from __future__ import annotations

import math

import torch

from . import ngd

__all__ = ["compose_child", "pack", "unpack", "Fit"]


def _tril(n: int, device):
    """Row-major lower-triangle indices: entry e of a packed factor is
    (i, j) with e = i(i+1)/2 + j, j <= i."""
    return torch.tril_indices(n, n, device=device)


def unpack(packed: torch.Tensor, n: int) -> torch.Tensor:
    """(K, n(n+1)/2) packed lower factors to (K, n, n) matrices."""
    r, c = _tril(n, packed.device)
    full = packed.new_zeros((packed.shape[0], n, n))
    full[:, r, c] = packed
    return full


def pack(full: torch.Tensor) -> torch.Tensor:
    """(K, n, n) lower-triangular matrices to (K, n(n+1)/2) packed factors."""
    n = full.shape[-1]
    r, c = _tril(n, full.device)
    return full[:, r, c]


def compose_child(l_parent, m_parent, u, m_u):
    """The child's absolute factor and mean from its relative parameters
    (Sec. 3.3, Eq. 6-7): L_c = L_p U, m_c = L_p m_u + m_p."""
    n = m_parent.shape[1]
    lp = unpack(l_parent, n)
    lc = torch.bmm(lp, unpack(u, n).contiguous())   # lower x lower is lower
    mc = torch.bmm(lp, m_u.unsqueeze(-1).contiguous()).squeeze(-1) + m_parent
    return pack(lc), mc


class Fit:
    """Adam on raw parameters of a mixture, children from the second phase.

    mean (K, n), factor (K, n(n+1)/2), weight (K,) > 0, colour (K, 3) in
    (0, 1): the initial mixture (activated values), any device tensors.
    """

    def __init__(self, mean, factor, weight, colour, *, lr=1e-3, lr_alpha=None,
                 threshold=0.01, phase=300, max_k=524288, child_alpha=1e-4, child_jitter=1e-2,
                 loss="l2", eps=0.01, precision=ngd.FP32, cull_params=None, seed=0):
        dev = mean.device
        self.n = mean.shape[1]
        self.lr, self.threshold, self.phase = lr, threshold, phase
        self.lr_alpha = lr if lr_alpha is None else lr_alpha
        self.max_k, self.child_alpha, self.child_jitter = max_k, child_alpha, child_jitter
        self.loss_kind, self.eps, self.precision = loss, eps, precision
        self.params = cull_params if cull_params is not None else ngd.default_params()
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        f32 = dict(dtype=torch.float32, device=dev)
        self.mean = mean.detach().to(**f32).clone().requires_grad_(True)
        self.factor = factor.detach().to(**f32).clone().requires_grad_(True)
        self.a = torch.log(weight.detach().to(**f32)).requires_grad_(True)
        self.c = torch.logit(colour.detach().to(**f32).clamp(1e-4, 1 - 1e-4)).requires_grad_(True)
        self.child = None   # (u, m_u, a, c) once the second phase starts
        self.steps = 0
        self._mix = None
        self._cull = ngd.Cull()
        self._new_optimizer()

    # -- parameters ------------------------------------------------------
    def _leaves(self):
        out = [self.mean, self.factor, self.a, self.c]
        if self.child is not None:
            out += list(self.child)
        return out

    def _new_optimizer(self):
        # moments restart whenever the parameter set changes (refinement);
        # the log-brightnesses have a learning rate of their own
        leaves = self._leaves()
        alpha = [self.a] + ([self.child[2]] if self.child is not None else [])
        rest = [t for t in leaves if all(t is not b for b in alpha)]
        self.opt = torch.optim.Adam([dict(params=rest, lr=self.lr),
                                     dict(params=alpha, lr=self.lr_alpha)])

    @property
    def k(self) -> int:
        return self.mean.shape[0] * (2 if self.child is not None else 1)

    def _default_children(self, count: int):
        n, dev = self.n, self.mean.device
        tri = n * (n + 1) // 2
        eye = pack(torch.eye(n, device=dev).expand(count, n, n).contiguous())
        j = self.child_jitter
        rnd = lambda *s: torch.randn(*s, generator=self.gen, device=dev)
        u = eye + j * rnd(count, tri)
        m_u = j * rnd(count, n)
        a = math.log(self.child_alpha) + 0.1 * rnd(count)
        c = rnd(count, 3)
        return [t.contiguous() for t in (u, m_u, a, c)]

    def add_children(self):
        """Every parent gets a default child (the start of the second phase)."""
        with torch.no_grad():
            self.child = tuple(t.requires_grad_(True)
                               for t in self._default_children(self.mean.shape[0]))
        self._new_optimizer()

    def absolute(self):
        """The activated mixture (parents, then children), in the graph."""
        w = torch.exp(self.a)
        col = torch.sigmoid(self.c)
        if self.child is None:
            return self.mean, self.factor, w, col
        u, m_u, a_c, c_c = self.child
        lc, mc = compose_child(self.factor, self.mean, u, m_u)
        return (torch.cat([self.mean, mc]), torch.cat([self.factor, lc]),
                torch.cat([w, torch.exp(a_c)]), torch.cat([col, torch.sigmoid(c_c)]))

    # -- one step --------------------------------------------------------
    def _mixture(self, mean, factor, weight, colour):
        k = mean.shape[0]
        if self._mix is None or self._mix.k != k:
            self._mix = ngd.Mixture(self.n, k)
        self._mix.update(mean.detach().contiguous(), factor.detach().contiguous(),
                         weight.detach().contiguous(), colour.detach().contiguous())
        return self._mix

    def evaluate(self, queries, proj):
        """The current mixture's values at the queries (no gradient)."""
        with torch.no_grad():
            mix = self._mixture(*self.absolute())
            self._cull.build(mix, queries, proj, self.params)
            return ngd.eval_mixture(mix, self._cull, queries, precision=self.precision)

    def step(self, queries, target, proj):
        """One Adam step on the loss of the mixture against target at the
        queries; returns the loss (a device tensor of one float)."""
        mean, factor, weight, colour = self.absolute()
        mix = self._mixture(mean, factor, weight, colour)
        self._cull.build(mix, queries, proj, self.params)
        f = ngd.eval_mixture(mix, self._cull, queries, precision=self.precision)
        if self.loss_kind == "rel":
            loss, g = ngd.rel_l2_loss(f, target, eps=self.eps)
        else:
            loss, g = ngd.l2_loss(f, target)
        grads = ngd.eval_backward(mix, self._cull, queries, g, precision=self.precision)
        self.opt.zero_grad(set_to_none=True)
        torch.autograd.backward([mean, factor, weight, colour], list(grads))
        self.opt.step()
        self.steps += 1
        if self.steps % self.phase == 0:
            if self.child is None:
                self.add_children()
            else:
                self.refine()
        return loss

    # -- refinement --------------------------------------------------------
    def refine(self) -> int:
        """Materialise the children brighter than the threshold; returns how
        many became parents (at most what max_k leaves room for)."""
        if self.child is None:
            return 0
        with torch.no_grad():
            u, m_u, a_c, c_c = self.child
            kp = self.mean.shape[0]
            room = max(0, self.max_k // 2 - kp)
            sel = torch.nonzero(torch.exp(a_c) > self.threshold).flatten()[:room]
            count = int(sel.numel())
            if count == 0:
                return 0
            lc, mc = compose_child(self.factor[sel], self.mean[sel], u[sel], m_u[sel])
            new_parent = [torch.cat([self.mean, mc]), torch.cat([self.factor, lc]),
                          torch.cat([self.a, a_c[sel]]), torch.cat([self.c, c_c[sel]])]
            self.mean, self.factor, self.a, self.c = (t.contiguous().requires_grad_(True)
                                                      for t in new_parent)
            # fresh children: the materialised slots and every new parent
            fresh = self._default_children(count * 2)
            kids = []
            for old, new in zip((u, m_u, a_c, c_c), fresh):
                old = old.detach().clone()
                old[sel] = new[:count]
                kids.append(torch.cat([old, new[count:]]).contiguous().requires_grad_(True))
            self.child = tuple(kids)
        self._new_optimizer()
        return count
