"""The activations of the autograd layer and their chain rule, on the CPU.

Sec. 3.1 parameterises the factor through exp on its diagonal and
2 sigmoid - 1 below it; Sec. 4.1 takes alpha = exp(a) and c = sigmoid(c_raw).
The GPU autograd tests compare the library's raw-parameter gradients with
the oracle's float64 gradient chained through these maps (`chain` below).
Here that chain is pinned to central finite differences of the oracle's
forward sum taken in raw-parameter space, and the torch activation code
(which the product path runs on the device) is checked against the same
float64 maps and their derivatives.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2405_20067_amd import inputs
from paper_2405_20067_amd.autograd import activate, activate_factor, diag_mask, raw_factor


def np_activate(raw_mean, raw_fac, raw_w, raw_c):
    """The Sec. 3.1 / Sec. 4.1 maps in float64 numpy."""
    n = raw_mean.shape[1]
    d = np.diag_indices(n)
    r, c = np.tril_indices(n)
    diag = r == c
    lf = np.where(diag, np.exp(np.where(diag, raw_fac, 0.0)), 2.0 / (1.0 + np.exp(-raw_fac)) - 1.0)
    del d
    return raw_mean, lf, np.exp(raw_w), 1.0 / (1.0 + np.exp(-raw_c))


def chain(raw, grads):
    """Gradients with respect to the raw parameters from those with respect
    to the activated ones: d exp = exp, d(2 sigmoid - 1) = 2 s (1 - s),
    d sigmoid = s (1 - s)."""
    raw_mean, raw_fac, raw_w, raw_c = raw
    gm, gl, ga, gc = grads
    n = raw_mean.shape[1]
    r, c = np.tril_indices(n)
    diag = r == c
    s_off = 1.0 / (1.0 + np.exp(-raw_fac))
    dl = np.where(diag, np.exp(np.where(diag, raw_fac, 0.0)), 2.0 * s_off * (1.0 - s_off))
    s_c = 1.0 / (1.0 + np.exp(-raw_c))
    return gm, gl * dl, ga * np.exp(raw_w), gc * s_c * (1.0 - s_c)


def raw_case(n, k, q, seed):
    mix = inputs.gen_mixture(n, k, "cube", (2.0, 6.0), 0.5, seed=seed)
    rng = np.random.default_rng(seed + 100)
    raw_fac = raw_factor(torch.from_numpy(mix["factor"].astype(np.float64)), n).numpy()
    raw_fac = raw_fac + 0.3 * rng.standard_normal(raw_fac.shape)   # off-diagonals away from 0
    raw = (mix["mean"].astype(np.float64), raw_fac,
           np.log(mix["weight"].astype(np.float64)) + 0.1 * rng.standard_normal(k),
           rng.standard_normal((k, 3)))
    x = inputs.gen_near_queries([mix], q, seed=seed + 1).astype(np.float64)
    g = rng.standard_normal((q, 3))
    return raw, x, g


def objective(raw, x, g):
    """sum_q g(q) . f(q) of the activated mixture, by the oracle."""
    return float(np.sum(g * oracle.eval_mixture(*np_activate(*raw), x)))


@pytest.mark.parametrize("n", [1, 2, 3])
def test_raw_chain_matches_central_differences(n):
    raw, x, g = raw_case(n, 3, 40, seed=10 + n)
    got = chain(raw, oracle.grad(*np_activate(*raw), x, g))
    for which, gr in enumerate(got):
        base = raw[which]
        for idx in np.ndindex(base.shape):
            h = 1e-6 * max(abs(base[idx]), 1e-2)
            plus = [a.copy() for a in raw]
            minus = [a.copy() for a in raw]
            plus[which][idx] += h
            minus[which][idx] -= h
            fd = (objective(plus, x, g) - objective(minus, x, g)) / (2 * h)
            scale = max(np.abs(gr).max(), 1e-12)
            assert abs(fd - gr[idx]) <= 1e-6 * scale + 1e-9 * abs(fd), (which, idx, fd, gr[idx])


def test_torch_activations_match_the_maps():
    raw, _, _ = raw_case(4, 7, 1, seed=3)
    t = [torch.from_numpy(a).requires_grad_(True) for a in raw]
    act = activate(*t)
    want = np_activate(*raw)
    for a, b in zip(act, want):
        np.testing.assert_allclose(a.detach().numpy(), b, rtol=1e-15, atol=0)
    # torch's chain rule through the maps equals `chain`
    rng = np.random.default_rng(0)
    ups = [rng.standard_normal(a.shape) for a in want]
    torch.autograd.backward(list(act), [torch.from_numpy(u) for u in ups])
    for a, b in zip([x.grad.numpy() for x in t], chain(raw, ups)):
        np.testing.assert_allclose(a, b, rtol=1e-14, atol=0)


def test_factor_activation_properties():
    n = 5
    d = diag_mask(n)
    assert int(d.sum()) == n
    # entry i(i+1)/2 + i is (i, i)
    assert [int(i) for i in torch.nonzero(d).flatten()] == [i * (i + 1) // 2 + i for i in range(n)]
    raw = torch.linspace(-30.0, 30.0, 2 * 15, dtype=torch.float64).reshape(2, 15)
    lf = activate_factor(raw, n)
    assert bool((lf[:, d] > 0).all())
    assert bool((lf[:, ~d].abs() <= 1).all())
    # raw -> factor -> raw round trip where the maps are well conditioned
    raw = torch.from_numpy(np.random.default_rng(1).uniform(-4, 4, (6, 15)))
    np.testing.assert_allclose(raw_factor(activate_factor(raw, n), n).numpy(), raw.numpy(),
                               rtol=0, atol=1e-10)
    # a strictly-lower raw entry large enough to overflow exp leaves no NaN gradient
    big = torch.zeros((1, 15), dtype=torch.float32)
    big[0, 1] = 500.0
    big.requires_grad_(True)
    activate_factor(big, n).sum().backward()
    assert bool(torch.isfinite(big.grad).all())
