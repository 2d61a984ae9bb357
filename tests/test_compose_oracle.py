"""Pins of the oracle's parent-child composition (Sec. 3.3, Eq. 6-7) and of
its chain rule, on the CPU.

compose: a child's Gaussian at x = m_p + L_p (m_u + U z) is exp(-|z|^2 / 2)
exactly (the closed form of a Gaussian at m + L z, with L = L_p U and
m = L_p m_u + m_p), for parents and children of either diagonal sign.
compose_grad: central finite differences of the loss sum(g * f) through
compose and the float64 forward, for every parent and relative parameter,
with several children per parent."""

import numpy as np
import pytest

import oracle


def _lower(rng, k, n, lo=0.5, hi=1.5):
    a = np.tril(rng.standard_normal((k, n, n))) * 0.3
    a[:, np.arange(n), np.arange(n)] = rng.uniform(lo, hi, (k, n)) * rng.choice([-1, 1], (k, n))
    r, c = np.tril_indices(n)
    return a[:, r, c]


def _family(n, kp, parent, seed):
    rng = np.random.default_rng(seed)
    kc = len(parent)
    mean_p = rng.uniform(0, 1, (kp, n))
    factor_p = _lower(rng, kp, n, 0.05, 0.2)
    rel_factor = _lower(rng, kc, n, 0.5, 1.5)
    rel_mean = rng.standard_normal((kc, n)) * 0.7
    return mean_p, factor_p, np.asarray(parent), rel_factor, rel_mean


@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_composed_child_closed_form(n):
    mean_p, factor_p, parent, rel_factor, rel_mean = _family(n, 3, [0, 0, 1, 2, 2], seed=n)
    m, L = oracle.compose(mean_p, factor_p, parent, rel_factor, rel_mean)
    assert m.shape == (8, n) and L.shape == (8, n * (n + 1) // 2)
    np.testing.assert_array_equal(m[:3], mean_p)
    np.testing.assert_array_equal(L[:3], factor_p)
    rng = np.random.default_rng(100 + n)
    r, c = np.tril_indices(n)
    for j, p in enumerate(parent):
        lp = np.zeros((n, n))
        lp[r, c] = factor_p[p]
        u = np.zeros((n, n))
        u[r, c] = rel_factor[j]
        z = rng.standard_normal(n)
        x = mean_p[p] + lp @ (rel_mean[j] + u @ z)
        got = oracle.gaussian(m[3 + j], L[3 + j], x)
        assert got == pytest.approx(np.exp(-0.5 * z @ z), rel=1e-10)
        # the mean is the image of the child's offset
        np.testing.assert_allclose(m[3 + j], mean_p[p] + lp @ rel_mean[j], rtol=0, atol=1e-14)


def test_compose_grad_matches_finite_differences():
    n, kp = 3, 3
    parent = [0, 0, 1, 2]
    mean_p, factor_p, parent, rel_factor, rel_mean = _family(n, kp, parent, seed=7)
    k = kp + len(parent)
    rng = np.random.default_rng(8)
    weight = rng.uniform(0.2, 1.0, k)
    colour = rng.uniform(0.0, 1.0, (k, 3))
    m0, L0 = oracle.compose(mean_p, factor_p, parent, rel_factor, rel_mean)
    # queries around every Gaussian so that each contributes
    x = np.concatenate([m0 + 0.05 * rng.standard_normal((k, n)) for _ in range(6)])
    g = rng.standard_normal((x.shape[0], 3))

    def loss(mp, fp, rf, rm):
        m, L = oracle.compose(mp, fp, parent, rf, rm)
        return float((oracle.eval_mixture(m, L, weight, colour, x) * g).sum())

    gm_abs, gl_abs, _, _ = oracle.grad(m0, L0, weight, colour, x, g)
    want = oracle.compose_grad(factor_p, parent, rel_factor, rel_mean, gm_abs, gl_abs)
    params = [mean_p, factor_p, rel_factor, rel_mean]
    for which, (p0, w) in enumerate(zip(params, want)):
        fd = np.zeros_like(p0)
        for idx in np.ndindex(p0.shape):
            h = 1e-6 * max(abs(p0[idx]), 1e-2)
            up = [q.copy() for q in params]
            dn = [q.copy() for q in params]
            up[which][idx] += h
            dn[which][idx] -= h
            fd[idx] = (loss(*up) - loss(*dn)) / (2 * h)
        scale = np.abs(fd).max()
        assert np.abs(w - fd).max() <= 1e-6 * scale, which
