"""Pin of the oracle's conditioning (the paper's global conditioning,
Sec. 3.2) on the CPU: the conditioned p-D mixture, evaluated by the float64
oracle's direct sum at x_p, equals the N-D mixture evaluated at (x_p, x_c)
-- the Schur-complement identity, checked against the N-D forward (forward
substitution, a different route from the explicit inverses).  Also: factors
of either diagonal sign, p = 1 and p = n - 1, and a point far from every
Gaussian (weights underflow to zero together with the N-D values)."""

import numpy as np
import pytest

import oracle
from paper_2405_20067_amd import inputs


@pytest.mark.parametrize("n,p", [(2, 1), (4, 3), (6, 3), (10, 3), (10, 1), (10, 9)])
def test_conditioned_mixture_equals_the_slice(n, p):
    layout = {4: "cube", 6: "pos3+dir3", 10: "pos3+nrm3+view3+rough1"}.get(n, "cube")
    mix = inputs.gen_mixture(n, 40, layout, (2.0, 8.0), 1.0, seed=n + p)
    rng = np.random.default_rng(p)
    flip = np.where(rng.random((40, n)) < 0.3, -1.0, 1.0)
    r, c = np.tril_indices(n)
    factor = mix["factor"].astype(np.float64) * flip[:, c]
    xc = mix["mean"][3, p:].astype(np.float64) + 0.05 * rng.standard_normal(n - p)
    cm, cf, cw, cc = oracle.condition(mix["mean"], factor, mix["weight"], mix["colour"], p, xc)
    assert cf.shape == (40, p * (p + 1) // 2)
    xp = mix["mean"][:, :p].astype(np.float64)[:25] + 0.1 * rng.standard_normal((25, p))
    full = np.concatenate([xp, np.repeat(xc[None], 25, 0)], 1)
    want = oracle.eval_mixture(mix["mean"], factor, mix["weight"], mix["colour"], full)
    got = oracle.eval_mixture(cm, cf, cw, cc, xp)
    assert np.abs(want).max() > 1e-3
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12 * np.abs(want).max())
    # every conditioned factor has a positive diagonal (a Cholesky factor)
    rp, cp = np.tril_indices(p)
    assert np.all(cf[:, rp == cp] > 0)
