"""The parent-child composition of the refinement (Sec. 3.3, Eq. 6-7), on the
CPU: the relative child parameters are pinned against the definition of the
child's covariance, V_c = (L_p U)(L_p U)^T with mean L_p m_u + m_p, by brute
force through an explicit inverse and the float64 oracle's Gaussian."""

import numpy as np
import pytest

import oracle
from paper_2405_20067_amd import inputs

torch = pytest.importorskip("torch")


def _lower(rng, k, n, scale=1.0):
    a = np.tril(rng.standard_normal((k, n, n))) * scale
    a[:, np.arange(n), np.arange(n)] = rng.uniform(0.3, 1.5, (k, n)) * rng.choice([-1, 1], (k, n))
    return a


@pytest.mark.parametrize("n", [1, 3, 6, 10])
def test_pack_roundtrip_matches_the_library_layout(n):
    from paper_2405_20067_amd.fit import pack, unpack
    rng = np.random.default_rng(n)
    full = _lower(rng, 5, n)
    packed = pack(torch.from_numpy(full))
    # packed entry e = i(i+1)/2 + j holds L_ij (row-major lower triangle)
    for i in range(n):
        for j in range(i + 1):
            np.testing.assert_array_equal(packed[:, i * (i + 1) // 2 + j].numpy(), full[:, i, j])
    np.testing.assert_array_equal(unpack(packed, n).numpy(), full)


def test_identity_child_is_its_parent():
    from paper_2405_20067_amd.fit import compose_child, pack
    n, k = 4, 7
    mix = inputs.gen_mixture(n, k, seed=3)
    lp = torch.from_numpy(mix["factor"]).double()
    mp = torch.from_numpy(mix["mean"]).double()
    eye = pack(torch.eye(n, dtype=torch.float64).expand(k, n, n).contiguous())
    lc, mc = compose_child(lp, mp, eye, torch.zeros(k, n, dtype=torch.float64))
    np.testing.assert_array_equal(lc.numpy(), lp.numpy())
    np.testing.assert_array_equal(mc.numpy(), mp.numpy())


@pytest.mark.parametrize("n", [2, 3, 6])
def test_child_gaussian_matches_its_definition(n):
    """G_child(x) from the composed (L_c, m_c) through the oracle equals
    exp(-1/2 (x - m_c)^T V_c^-1 (x - m_c)) with V_c = L_p U U^T L_p^T built
    and inverted explicitly (a wrong product order or a transposed U fails)."""
    from paper_2405_20067_amd.fit import compose_child, pack
    rng = np.random.default_rng(10 + n)
    k = 6
    lp, u = _lower(rng, k, n), _lower(rng, k, n, 0.3)
    mp, mu = rng.standard_normal((k, n)), rng.standard_normal((k, n)) * 0.5
    lc, mc = compose_child(pack(torch.from_numpy(lp)), torch.from_numpy(mp),
                           pack(torch.from_numpy(u)), torch.from_numpy(mu))
    lc, mc = lc.numpy(), mc.numpy()
    for i in range(k):
        a = lp[i] @ u[i]
        v = a @ a.T
        m = lp[i] @ mu[i] + mp[i]
        for _ in range(5):
            x = m + rng.standard_normal(n) * 0.7
            d = x - m
            want = np.exp(-0.5 * d @ np.linalg.inv(v) @ d)
            got = oracle.gaussian(mc[i], lc[i], x)
            assert got == pytest.approx(want, rel=1e-9, abs=1e-300)
