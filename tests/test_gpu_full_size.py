"""Parity at the full sizes of the named workloads, in the launch
configuration the benchmark times (same inputs, same cull parameters).

The oracle cannot sum every pair at these sizes, so it computes sampled
outputs one by one: the full float64 sum over all K Gaussians at sampled
queries, and the float64 gradient of sampled Gaussians, both over their
candidate tiles' queries (the arithmetic error, bar 1e-4) and over all
queries (the left-out pairs' terms within the cull's bound).
The cull is compared with the CPU re-implementation over its whole output.
"""

import numpy as np
import pytest

import oracle
from gpu_helpers import (dev, host, normwise, omitted_pairs_grad_bound,
                         queries_of_gaussians)
from paper_2405_20067_amd import inputs

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _workload(name):
    w = inputs.WORKLOADS[name]
    mix = inputs.workload_mixture(w)
    tgt = (inputs.workload_mixture(w, k=w.k_target, seed=inputs.SEED_TARGET)
           if w.k_target else None)
    x = inputs.gen_workload_queries(w, mixtures=[m for m in (mix, tgt) if m is not None])
    proj = inputs.gen_projections(w.n, 16, inputs.SEED_PROJ)
    return w, mix, x, proj


@pytest.mark.parametrize("name", ["6d-culled", "10d-fwdbwd"])
def test_full_size_cull_forward_backward(torch_cuda, name):
    from paper_2405_20067_amd import ngd
    w, mix, x, proj = _workload(name)
    print(f"[{name}] n={w.n} k={w.k} q={w.q}", flush=True)
    m = ngd.Mixture(w.n, w.k)
    m.update(dev(mix["mean"]), dev(mix["factor"]), dev(mix["weight"]), dev(mix["colour"]))
    m.validate()
    xd = dev(x)
    c = ngd.Cull().build(m, xd, proj, ngd.default_params())
    f = host(ngd.eval_mixture(m, c, xd))
    g = inputs.gen_grad_out(w.q, seed=31, scale=1.0 / w.q)
    grads = [host(t) for t in ngd.eval_backward(m, c, xd, dev(g))]

    # the whole cull, bit for bit
    got = c.export()
    want = oracle.cull(mix["mean"], mix["factor"], x, proj, tau=1e-4, tile=256,
                       key_proj=16, key_bits=2)
    assert got["total"] == want["total"]
    for key in ("perm", "gperm", "tile_off", "cand", "g_off", "g_tiles"):
        np.testing.assert_array_equal(got[key], want[key], err_msg=key)

    rng = np.random.default_rng(7)
    # forward: sampled queries against the full sum over all K
    qs = rng.choice(w.q, 192, replace=False)
    fo = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x[qs])
    assert normwise(f[qs], fo) <= TOL_FP32
    # the matrix-core forward on the same cull: the same sampled bar, and
    # against the float32 forward within the skip certificate
    fm = host(ngd.eval_mixture(m, c, xd, precision=ngd.BF16_MFMA))
    assert normwise(fm[qs], fo) <= TOL_FP32
    ac = mix["weight"].astype(np.float64)[:, None] * np.abs(mix["colour"])
    slack = 1e-4 * 2.0 ** -20 * ac.sum(0)
    assert np.all(np.abs(fm.astype(np.float64) - f) <= slack + 1e-6 * np.abs(f).max())
    gm = [host(t) for t in ngd.eval_backward(m, c, xd, dev(g), precision=ngd.BF16_MFMA)]
    _check_sampled_backward(mix, x, g, grads, gm, got, w, rng)


def _check_sampled_backward(mix, x, g, grads, gm, exported, w, rng, nsel=24):
    """Sampled Gaussians (the ones with the largest gradients among a random
    subset, so the comparison is not of zeros): both precisions' gradients
    against the float64 gradient over the queries of their candidate tiles at
    1e-4, and against the full float64 gradient over all queries within 1e-4
    plus the bound on the left-out pairs' terms."""
    pool = rng.choice(w.k, 4096, replace=False)
    mag = np.abs(grads[2][pool])
    sel = pool[np.argsort(-mag)[:nsel]]
    qoff, qidx = queries_of_gaussians(exported, sel, w.q, 256)
    part = oracle.grad_lists(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x, g,
                             sel, qoff, qidx)
    full = oracle.grad(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x, g, sel=sel)
    bounds = omitted_pairs_grad_bound(mix, g, sel, 1e-4)
    for name_o, a, am, b, f, bd in zip(("mean", "factor", "weight", "colour"), grads, gm, part,
                                       full, bounds):
        e32, e16 = normwise(a[sel], b), normwise(am[sel], b)
        ef = normwise(a[sel], f)
        print(f"  d{name_o}: fp32 {e32:.2e}, bf16 {e16:.2e} vs candidate pairs; "
              f"fp32 {ef:.2e} vs all pairs", flush=True)
        assert e32 <= TOL_FP32, name_o
        assert e16 <= TOL_FP32, name_o
        lim = TOL_FP32 * np.abs(f).max() + bd.reshape(len(sel), -1)
        assert np.all(np.abs(a[sel] - f).reshape(len(sel), -1) <= lim), name_o
        assert np.all(np.abs(am[sel] - f).reshape(len(sel), -1) <= lim), name_o


def test_full_size_4m_queries_both_precisions(torch_cuda):
    """2^22 queries (the matrix-core comparison workload): sampled colours
    of both forwards against the float64 oracle over all K Gaussians."""
    from paper_2405_20067_amd import ngd
    w, mix, x, proj = _workload("10d-4m")
    print(f"[10d-4m] n={w.n} k={w.k} q={w.q}", flush=True)
    m = ngd.Mixture(w.n, w.k)
    m.update(dev(mix["mean"]), dev(mix["factor"]), dev(mix["weight"]), dev(mix["colour"]))
    xd = dev(x)
    c = ngd.Cull().build(m, xd, proj, ngd.default_params())
    ff = host(ngd.eval_mixture(m, c, xd, precision=ngd.FP32))
    fm = host(ngd.eval_mixture(m, c, xd, precision=ngd.BF16_MFMA))
    rng = np.random.default_rng(11)
    qs = rng.choice(w.q, 128, replace=False)
    fo = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x[qs])
    assert normwise(ff[qs], fo) <= TOL_FP32
    assert normwise(fm[qs], fo) <= TOL_FP32
    ac = mix["weight"].astype(np.float64)[:, None] * np.abs(mix["colour"])
    slack = 1e-4 * 2.0 ** -20 * ac.sum(0)
    assert np.all(np.abs(fm.astype(np.float64) - ff) <= slack + 1e-6 * np.abs(ff).max())
    # the backward of both precisions on the same cull
    g = inputs.gen_grad_out(w.q, seed=37, scale=1.0 / w.q)
    gd = dev(g)
    gm = [host(t) for t in ngd.eval_backward(m, c, xd, gd, precision=ngd.BF16_MFMA)]
    ngd.eval_mixture(m, c, xd, precision=ngd.FP32)
    grads = [host(t) for t in ngd.eval_backward(m, c, xd, gd, precision=ngd.FP32)]
    _check_sampled_backward(mix, x, g, grads, gm, c.export(), w, rng)
