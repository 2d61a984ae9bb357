"""Conditioning inside the library (ngd_mixture_condition, the paper's global
conditioning, Sec. 3.2) against the float64 oracle: the conditioned
parameters (mean, covariance from the factor, weight), and the conditioned
3-D mixture evaluated through the library (cull and forward) against the
N-D oracle on the slice (x_p, x_c).  Also the image-order tiling on a
G-buffer and the argument checks."""

import numpy as np
import pytest

import oracle
from gpu_helpers import dev, host, normwise
from paper_2405_20067_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _cov(fac, p):
    r, c = np.tril_indices(p)
    L = np.zeros((fac.shape[0], p, p))
    L[:, r, c] = fac
    return L @ np.transpose(L, (0, 2, 1))


@pytest.mark.parametrize("n,p", [(10, 3), (6, 3), (4, 1)])
def test_condition_matches_the_oracle(torch_cuda, n, p):
    from paper_2405_20067_amd import ngd
    x = inputs.gen_gbuffer(64, 64) if n == 10 else None
    if n == 10:
        mix = inputs.gen_mixture_on(x, 3000, (10.0, 200.0), 5.0, jitter=0.02, seed=5)
        xc = x[1000, p:]
    else:
        layout = {6: "pos3+dir3", 4: "cube"}[n]
        mix = inputs.gen_mixture(n, 3000, layout, (5.0, 50.0), 2.0, seed=n)
        xc = mix["mean"][7, p:]
    xc = np.ascontiguousarray(xc, np.float32)
    m = ngd.Mixture(n, 3000)
    m.update(dev(mix["mean"]), dev(mix["factor"]), dev(mix["weight"]), dev(mix["colour"]))
    cm, cf, cw, cc = [host(t) for t in m.condition(p, xc)]
    om, of, ow, oc = oracle.condition(mix["mean"], mix["factor"], mix["weight"], mix["colour"],
                                      p, xc)
    live = ow > 1e-30 * ow.max()        # weights that are not underflowed to 0
    assert live.sum() > 10
    np.testing.assert_allclose(cm[live], om[live], rtol=0, atol=2e-5 * np.abs(om).max())
    cov_g, cov_o = _cov(cf.astype(np.float64), p), _cov(of, p)
    scale = np.abs(cov_o).reshape(3000, -1).max(1)[:, None, None]
    assert np.all(np.abs(cov_g - cov_o) <= 1e-4 * scale)
    assert normwise(cw, ow) <= 1e-5
    np.testing.assert_array_equal(cc, mix["colour"])
    # the conditioned mixture through the library, on the slice x_c
    q = 4096
    rng = np.random.default_rng(3)
    xp = (om[rng.choice(np.nonzero(live)[0], q)] + 0.02 * rng.standard_normal((q, p))
          ).astype(np.float32)
    m3 = ngd.Mixture(p, 3000)
    m3.update(*[dev(a) for a in (cm, cf, cw, cc)])
    m3.validate()
    xpd = dev(xp)
    c3 = ngd.Cull().build(m3, xpd, inputs.gen_projections(p, 16, seed=9))
    f3 = host(ngd.eval_mixture(m3, c3, xpd))
    full = np.concatenate([xp.astype(np.float64), np.repeat(xc[None].astype(np.float64), q, 0)],
                          1)
    fo = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], full)
    assert np.abs(fo).max() > 1e-3
    assert normwise(f3, fo) <= 1e-4


def test_condition_rejects_bad_arguments(torch_cuda):
    from paper_2405_20067_amd import ngd
    mix = inputs.gen_mixture(4, 10, seed=1)
    m = ngd.Mixture(4, 10)
    m.update(dev(mix["mean"]), dev(mix["factor"]), dev(mix["weight"]), dev(mix["colour"]))
    for p, xc in ((0, [0.1] * 4), (4, []), (2, [0.1, float("nan")])):
        with pytest.raises(ngd.NgdError) as ei:
            m.condition(p, xc)
        assert ei.value.code == ngd.E_INVAL


def test_image_tiles_on_a_gbuffer(torch_cuda):
    """The given-order tiling on a G-buffer laid out in 16 x 16 pixel tiles:
    bit-exact against the CPU cull, and the culled forward against the
    float64 oracle on sampled pixels."""
    from paper_2405_20067_amd import ngd
    x = inputs.gen_gbuffer(96, 96)
    mix = inputs.gen_mixture_on(x, 4000, (10.0, 200.0), 5.0, jitter=0.02, seed=7)
    proj = inputs.gen_projections(10, 16, seed=8)
    m = ngd.Mixture(10, 4000)
    m.update(dev(mix["mean"]), dev(mix["factor"]), dev(mix["weight"]), dev(mix["colour"]))
    p = ngd.default_params()
    p.tiling = 2
    xd = dev(x)
    c = ngd.Cull().build(m, xd, proj, p)
    got = c.export()
    want = oracle.cull(mix["mean"], mix["factor"], x, proj, tau=1e-4, tile=256, tiling=2)
    for key in ("perm", "gperm", "tile_off", "cand", "g_off", "g_tiles", "tile_lo", "tile_hi"):
        np.testing.assert_array_equal(got[key], want[key], err_msg=key)
    f = host(ngd.eval_mixture(m, c, xd))
    idx = np.random.default_rng(1).choice(x.shape[0], 1024, replace=False)
    fo = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x[idx])
    assert np.abs(fo).max() > 1e-3
    assert normwise(f[idx], fo) <= 1e-4
