"""Fitting loop on the culled path, with optimisation-controlled refinement.

Each step is one differentiable evaluation through the torch.autograd layer
(`NgdMixtureEval`: ngd_mixture_update, ngd_cull_build, ngd_eval; its
backward ngd_eval_backward; with children, by default `NgdComposedEval`,
which has the library compose them: ngd_mixture_update_composed and
ngd_eval_backward_composed), the library's loss (`NgdL2Loss`), and an Adam
step on raw parameters.  The activations are torch ops, so autograd chains
the library's gradients through them:

    Sec. 3.1  factor L: exp on the diagonal, 2 sigmoid - 1 strictly below it
    Sec. 4.1  brightness alpha = exp(a), colour c = sigmoid(c_raw)

so every factor the library receives has a positive diagonal.

Refinement (Sec. 3.3, Eq. 6-7): from the second phase on, every parent
carries one child defined in the parent's frame by a relative factor U
(lower triangular, the same activations as L) and offset m_u:

    L_child = L_parent U,    m_child = L_parent m_u + m_parent,

so that the child follows every update of its parent.  A new child spans its
parent (raw U = 0, i.e. U = I, and m_u = 0, up to a small random
perturbation) with a negligible brightness.  At the end of each phase the
children whose brightness exceeds the threshold t are materialised: they
become parents (with their absolute parameters, so the represented function
does not change), and their slot, like every new parent, gets a fresh
default child.

`state_dict` / `load_state_dict` (and `save` / `load`, plain tensors through
torch.save) carry the raw parameters, the children, Adam's moments, the step
count and the random generator, so that a run resumed from a checkpoint
takes the same steps as one that was not interrupted.
"""

from __future__ import annotations

import math

import torch

from . import ngd
from .autograd import (Evaluator, NgdComposedEval, NgdL2Loss, NgdMixtureEval, activate_factor,
                       raw_factor)

__all__ = ["compose_child", "pack", "unpack", "absolute_params", "Fit"]


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


def absolute_params(n, mean, factor_raw, a, c, child=None):
    """(mean, L, alpha, colour) of the whole mixture, parents then children,
    from raw parameters: the activations of Sec. 3.1 / 4.1 and, for the
    children (raw u, m_u, a, c), the composition of Eq. 6-7."""
    lp = activate_factor(factor_raw, n)
    w = torch.exp(a)
    col = torch.sigmoid(c)
    if child is None:
        return mean, lp, w, col
    u, m_u, a_c, c_c = child
    lc, mc = compose_child(lp, mean, activate_factor(u, n), m_u)
    return (torch.cat([mean, mc]), torch.cat([lp, lc]),
            torch.cat([w, torch.exp(a_c)]), torch.cat([col, torch.sigmoid(c_c)]))


class Fit:
    """Adam on raw parameters of a mixture, children from the second phase.

    mean (K, n), factor (K, n(n+1)/2) with a positive diagonal and
    strictly-lower entries in (-1, 1), weight (K,) > 0, colour (K, 3) in
    (0, 1): the initial mixture (activated values), any device tensors.
    """

    def __init__(self, mean, factor, weight, colour, *, lr=1e-3, lr_alpha=None, lr_child=None,
                 threshold=0.01, phase=300, max_k=524288, child_alpha=1e-4, child_jitter=1e-2,
                 loss="l2", eps=0.01, precision=ngd.FP32, cull_params=None, seed=0,
                 compose="kernel", adam_eps=1e-15):
        dev = mean.device
        self.n = mean.shape[1]
        self.lr, self.threshold, self.phase = lr, threshold, phase
        self.lr_alpha = lr if lr_alpha is None else lr_alpha
        self.lr_child = lr if lr_child is None else lr_child
        self.max_k, self.child_alpha, self.child_jitter = max_k, child_alpha, child_jitter
        self.adam_eps = adam_eps
        self.loss_kind, self.eps, self.precision = loss, eps, precision
        if compose not in ("kernel", "torch"):
            raise ValueError(f"compose must be 'kernel' or 'torch', got {compose!r}")
        self.compose = compose
        self.params = cull_params if cull_params is not None else ngd.default_params()
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        f32 = dict(dtype=torch.float32, device=dev)
        self.mean = mean.detach().to(**f32).clone().requires_grad_(True)
        self.factor = raw_factor(factor.detach().to(**f32), self.n).requires_grad_(True)
        self.a = torch.log(weight.detach().to(**f32)).requires_grad_(True)
        self.c = torch.logit(colour.detach().to(**f32).clamp(1e-4, 1 - 1e-4)).requires_grad_(True)
        self.child = None   # raw (u, m_u, a, c) once the second phase starts
        self.steps = 0
        # one entry per refinement: (step, children materialised, the
        # children's largest brightness, how many exceeded a tenth of t)
        self.refine_log: list[tuple[int, int, float, int]] = []
        self.ev = Evaluator(self.n, None, self.params, precision)
        self.ev.cull = ngd.Cull()
        self._new_optimizer()

    # -- parameters ------------------------------------------------------
    def _leaves(self):
        out = [self.mean, self.factor, self.a, self.c]
        if self.child is not None:
            out += list(self.child)
        return out

    def _new_optimizer(self):
        # moments restart whenever the parameter set changes (refinement);
        # the log-brightnesses have a learning rate of their own, and so do
        # the children's relative factor, offset and colour (their steps are
        # in units of the parent's frame).  Adam's epsilon is far below the
        # usual 1e-8: a mean loss over millions of queries gives a dim child
        # gradients of order 1e-10, which an epsilon of 1e-8 would swamp, so
        # that the child could never move or brighten.
        groups = [dict(params=[self.mean, self.factor, self.c], lr=self.lr),
                  dict(params=[self.a], lr=self.lr_alpha)]
        if self.child is not None:
            u, m_u, a_c, c_c = self.child
            groups += [dict(params=[u, m_u, c_c], lr=self.lr_child),
                       dict(params=[a_c], lr=self.lr_alpha)]
        self.opt = torch.optim.Adam(groups, eps=self.adam_eps)

    @property
    def k(self) -> int:
        return self.mean.shape[0] * (2 if self.child is not None else 1)

    def _default_children(self, count: int):
        n, dev = self.n, self.mean.device
        tri = n * (n + 1) // 2
        j = self.child_jitter
        rnd = lambda *s: torch.randn(*s, generator=self.gen, device=dev)
        u = j * rnd(count, tri)            # raw U near 0: U near the identity
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
        return absolute_params(self.n, self.mean, self.factor, self.a, self.c, self.child)

    # -- one step --------------------------------------------------------
    def _forward(self, queries):
        """The mixture's values at the queries, in the graph: with children
        and compose="kernel" the library composes them (NgdComposedEval),
        otherwise torch does (absolute parameters into NgdMixtureEval)."""
        if self.child is None or self.compose == "torch":
            return NgdMixtureEval.apply(*self.absolute(), queries, self.ev)
        u, m_u, a_c, c_c = self.child
        kp = self.mean.shape[0]
        parent = torch.arange(kp, dtype=torch.int32, device=self.mean.device)
        weight = torch.cat([torch.exp(self.a), torch.exp(a_c)])
        colour = torch.cat([torch.sigmoid(self.c), torch.sigmoid(c_c)])
        return NgdComposedEval.apply(self.mean, activate_factor(self.factor, self.n), weight,
                                     colour, parent, activate_factor(u, self.n), m_u, queries,
                                     self.ev)

    def evaluate(self, queries, proj):
        """The current mixture's values at the queries (no gradient)."""
        self.ev.proj = proj
        with torch.no_grad():
            return self._forward(queries)

    def step(self, queries, target, proj):
        """One Adam step on the loss of the mixture against target at the
        queries; returns the loss (a device tensor of one float).  At each
        phase end the loss is read back (one synchronisation per phase) and
        a non-finite loss raises."""
        self.ev.proj = proj
        f = self._forward(queries)
        loss = NgdL2Loss.apply(f, target, self.eps if self.loss_kind == "rel" else 0.0)
        self.opt.zero_grad(set_to_none=True)
        loss.backward()
        self.opt.step()
        self.steps += 1
        if self.steps % self.phase == 0:
            if not math.isfinite(float(loss.detach()[0])):
                raise FloatingPointError(f"fit: non-finite loss at step {self.steps}")
            if self.child is None:
                self.add_children()
            else:
                self.refine()
        return loss.detach()

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
            bright = torch.exp(a_c)
            sel = torch.nonzero(bright > self.threshold).flatten()[:room]
            count = int(sel.numel())
            self.refine_log.append((self.steps, count, float(bright.max()),
                                    int((bright > 0.1 * self.threshold).sum())))
            if count == 0:
                return 0
            lp = activate_factor(self.factor[sel], self.n)
            lc, mc = compose_child(lp, self.mean[sel], activate_factor(u[sel], self.n),
                                   m_u[sel])
            # the new parents' raw factors (positive diagonal: L_p,ii U_ii > 0)
            new_parent = [torch.cat([self.mean, mc]),
                          torch.cat([self.factor, raw_factor(lc, self.n)]),
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

    # -- checkpoints -------------------------------------------------------
    def state_dict(self) -> dict:
        """Raw parameters, children, Adam's state, step count and generator
        state, as plain tensors and numbers."""
        names = ["mean", "factor", "a", "c"]
        st = {f"param.{k}": getattr(self, k).detach().clone() for k in names}
        if self.child is not None:
            for k, t in zip(("u", "m_u", "a", "c"), self.child):
                st[f"child.{k}"] = t.detach().clone()
        opt = self.opt.state_dict()
        for i, leaf in enumerate(self._leaves()):
            s = self.opt.state.get(leaf, {})
            for key, v in s.items():
                st[f"adam.{i}.{key}"] = v.detach().clone() if torch.is_tensor(v) else \
                    torch.tensor(v)
        st["adam.groups"] = torch.tensor([len(g["params"]) for g in opt["param_groups"]])
        st["steps"] = torch.tensor(self.steps)
        st["gen"] = self.gen.get_state()
        return st

    def load_state_dict(self, st: dict):
        """Restores what state_dict saved (tensors moved to this fit's
        device); the hyper-parameters are the constructor's."""
        dev = self.mean.device
        get = lambda k: st[k].to(dev)
        with torch.no_grad():
            self.mean, self.factor, self.a, self.c = (
                get(f"param.{k}").clone().requires_grad_(True) for k in ("mean", "factor", "a",
                                                                          "c"))
            if "child.u" in st:
                self.child = tuple(get(f"child.{k}").clone().requires_grad_(True)
                                   for k in ("u", "m_u", "a", "c"))
            else:
                self.child = None
        self._new_optimizer()
        for i, leaf in enumerate(self._leaves()):
            s = {key.split(".", 2)[2]: v for key, v in st.items()
                 if key.startswith(f"adam.{i}.")}
            if s:
                self.opt.state[leaf] = {key: (v.to(dev) if key != "step" else v.clone())
                                        for key, v in s.items()}
        self.steps = int(st["steps"])
        self.gen.set_state(st["gen"])

    def save(self, path: str):
        torch.save(self.state_dict(), path)

    def load(self, path: str):
        self.load_state_dict(torch.load(path, map_location="cpu", weights_only=True))
