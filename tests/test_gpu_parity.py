"""Parity of the HIP path (through the C-ABI) against the float64 CPU oracle.

Bars: integer outputs of the cull (permutations, offsets, candidate and
transposed lists) bit-exact against the CPU cull; float32 values within the
1e-4 normwise relative error of the target (max |x - x_ref| / max |x_ref|
per output tensor), against the full oracle sum (culled pairs included) and
against the oracle restricted to the same candidate pairs.
"""

import numpy as np
import pytest

import oracle
from gpu_helpers import (case, dev, host, normwise, omitted_pairs_grad_bound, per_gaussian_csr,
                         per_query_csr)
from paper_2405_20067_amd import inputs

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _mixture(torch_cuda, mix):
    from paper_2405_20067_amd import ngd
    m = ngd.Mixture(mix["mean"].shape[1], mix["mean"].shape[0])
    m.update(dev(mix["mean"]), dev(mix["factor"]), dev(mix["weight"]), dev(mix["colour"]))
    return m


def _params(tile=256, tau=1e-4, n_proj=16, key_proj=16, key_bits=2, tiling=0):
    from paper_2405_20067_amd import ngd
    p = ngd.default_params()
    p.tile, p.tau, p.n_proj, p.key_proj, p.key_bits = tile, tau, n_proj, key_proj, key_bits
    p.tiling = tiling
    return p


CULL_CASES = [
    dict(n=4, k=300, q=3000, tile=256),
    dict(n=6, k=777, q=5000, tile=100),
    dict(n=10, k=1500, q=4100, tile=256),
    dict(n=3, k=64, q=70, tile=1),
    dict(n=10, k=65, q=257, tile=64),
    dict(n=2, k=130, q=1000, tile=1024, key_bits=3, key_proj=10, tiling=1),
    dict(n=10, k=1500, q=4100, tile=256, tiling=1),
    dict(n=6, k=5000, q=70000, tile=256),
    # long lists: tiles with several forward items (more than 512 candidates)
    # and, where marked, Gaussians with several backward items (more than 32
    # tiles)
    dict(n=4, k=3000, q=20000, tile=256, long=2),
    dict(n=6, k=2500, q=9000, tile=512, long=1),
    dict(n=10, k=3000, q=9000, tile=256, sdiag=(3.0, 30.0), long=2),
    # few, large tiles: most pairs are candidates (over 3000 of the 4096
    # Gaussians per tile), more in each 64-chunk round of the list build than
    # a wave stages at once
    dict(n=4, k=4096, q=1500, tile=256, sdiag=(8.0, 12.0)),
    # other culling thresholds: 3 sigma (kappa^2 = 9) and a tight one
    dict(n=6, k=2000, q=9000, tile=256, tau=0.011108996538242306),
    dict(n=10, k=1500, q=4100, tile=64, tau=1e-6),
    # queries in their given order (tiles laid out by the caller)
    dict(n=10, k=1500, q=4100, tile=256, tiling=2),
    dict(n=3, k=500, q=1000, tile=100, tiling=2),
]


def _case(cfg):
    return case(cfg["n"], cfg["k"], cfg["q"], seed=cfg["n"] * 7 + cfg["k"], sdiag=cfg.get("sdiag"))


def _ids(c):
    fmt = lambda v: "-".join(f"{x:g}" for x in v) if isinstance(v, tuple) else v
    return "-".join(f"{k}{fmt(v)}" for k, v in c.items())


@pytest.mark.parametrize("cfg", CULL_CASES, ids=_ids)
def test_cull_bit_exact(torch_cuda, cfg):
    from paper_2405_20067_amd import ngd
    n, k, q = cfg["n"], cfg["k"], cfg["q"]
    key_bits = cfg.get("key_bits", 2)
    key_proj = cfg.get("key_proj", 16)
    tiling = cfg.get("tiling", 0)
    mix, x, proj = _case(cfg)
    m = _mixture(torch_cuda, mix)
    xd = dev(x)
    tau = cfg.get("tau", 1e-4)
    c = ngd.Cull().build(m, xd, proj, _params(tile=cfg["tile"], tau=tau, key_bits=key_bits,
                                               key_proj=key_proj, tiling=tiling))
    got = c.export()
    want = oracle.cull(mix["mean"], mix["factor"], x, proj, tau=tau, tile=cfg["tile"],
                       key_proj=key_proj, key_bits=key_bits, tiling=tiling)
    assert got["ntiles"] == want["ntiles"]
    assert got["total"] == want["total"]
    for key in ("perm", "gperm", "tile_off", "cand", "g_off", "g_tiles", "tile_lo", "tile_hi"):
        np.testing.assert_array_equal(got[key], want[key], err_msg=key)
    lens = np.diff(want["tile_off"])
    assert got["max_per_tile"] == (lens.max() if lens.size else 0)


@pytest.mark.parametrize("cfg", [c for c in CULL_CASES if c["tile"] > 1], ids=_ids)
def test_culled_forward_matches_oracle(torch_cuda, cfg):
    from paper_2405_20067_amd import ngd
    n, k, q = cfg["n"], cfg["k"], cfg["q"]
    mix, x, proj = _case(cfg)
    m = _mixture(torch_cuda, mix)
    xd = dev(x)
    tau = cfg.get("tau", 1e-4)
    c = ngd.Cull().build(m, xd, proj, _params(tile=cfg["tile"], tau=tau,
                                               tiling=cfg.get("tiling", 0)))
    f = host(ngd.eval_mixture(m, c, xd))
    full = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x)
    if tau <= 1e-4:   # a looser threshold is bounded by the check below only
        assert normwise(f, full) <= TOL_FP32
    # arithmetic error alone: the oracle over exactly the candidate pairs
    exp = c.export()
    qoff, gidx = per_query_csr(exp, q, cfg["tile"])
    restricted = oracle.eval_lists(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x,
                                   qoff, gidx)
    assert normwise(f, restricted) <= TOL_FP32
    # cull error alone is bounded by tau * sum over culled pairs of alpha c
    ac = mix["weight"].astype(np.float64)[:, None] * mix["colour"]
    bound = tau * (ac.sum(0)[None, :] - np.add.reduceat(ac[gidx], qoff[:-1], axis=0)
                    * (np.diff(qoff) > 0)[:, None])
    # (float64 summation order differs between the two sums: allow its rounding)
    assert np.all(np.abs(full - restricted) <= bound + 1e-12 * np.abs(full) + 1e-300)


def test_dense_forward_4d_full_size(torch_cuda):
    """The 4-D workload at its full size: K=256, 65,536 uniform queries."""
    from paper_2405_20067_amd import ngd
    w = inputs.WORKLOADS["4d-dense"]
    mix = inputs.workload_mixture(w)
    x = inputs.gen_workload_queries(w)
    m = _mixture(torch_cuda, mix)
    f = host(ngd.eval_mixture(m, None, dev(x)))
    want = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x)
    assert normwise(f, want) <= TOL_FP32
    big = np.abs(want) > 1e-3 * np.abs(want).max()
    assert np.max(np.abs(f - want)[big] / np.abs(want)[big]) < 1e-3


@pytest.mark.parametrize("cfg", [dict(n=4, k=200, q=2000), dict(n=6, k=400, q=3000),
                                 dict(n=10, k=600, q=2600)], ids=_ids)
def test_dense_backward_matches_oracle(torch_cuda, cfg):
    from paper_2405_20067_amd import ngd
    n, k, q = cfg["n"], cfg["k"], cfg["q"]
    mix, x, _ = case(n, k, q, seed=3 * n + 1)
    g = inputs.gen_grad_out(q, seed=n)
    m = _mixture(torch_cuda, mix)
    got = [host(t) for t in ngd.eval_backward(m, None, dev(x), dev(g))]
    want = oracle.grad(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x, g)
    for name, a, b in zip(("mean", "factor", "weight", "colour"), got, want):
        assert normwise(a, b) <= TOL_FP32, name


@pytest.mark.parametrize("cfg", [c for c in CULL_CASES if c["tile"] > 1 and c["n"] > 2], ids=_ids)
def test_culled_backward_matches_oracle(torch_cuda, cfg):
    """The backward of the culled forward is the gradient of the sum over the
    candidate pairs: compared with the oracle's gradient over exactly those
    pairs (the arithmetic error, bar 1e-4).  Against the full oracle the
    difference also holds the left-out pairs' gradient terms, which the cull's
    guarantee bounds per Gaussian (omitted_pairs_grad_bound)."""
    from paper_2405_20067_amd import ngd
    n, k, q = cfg["n"], cfg["k"], cfg["q"]
    mix, x, proj = _case(cfg)
    g = inputs.gen_grad_out(q, seed=k)
    m = _mixture(torch_cuda, mix)
    xd = dev(x)
    tau = cfg.get("tau", 1e-4)
    c = ngd.Cull().build(m, xd, proj, _params(tile=cfg["tile"], tau=tau,
                                              tiling=cfg.get("tiling", 0)))
    exp = c.export()
    if cfg.get("long", 0) >= 1:   # the long-list cases really exercise multiple items
        assert np.diff(exp["tile_off"]).max() > 512
    if cfg.get("long", 0) >= 2:
        assert np.diff(exp["g_off"]).max() > 32
    got = [host(t) for t in ngd.eval_backward(m, c, xd, dev(g))]
    sel, qoff, qidx = per_gaussian_csr(exp, q, cfg["tile"])
    part = oracle.grad_lists(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x, g,
                             sel, qoff, qidx)
    full = oracle.grad(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x, g)
    bounds = omitted_pairs_grad_bound(mix, g, np.arange(k), tau)
    for name, a, b, f, bd in zip(("mean", "factor", "weight", "colour"), got, part, full,
                                 bounds):
        want = np.zeros_like(f)
        want[sel] = b
        assert normwise(a, want) <= TOL_FP32, name
        bd = bd.reshape(k, -1)
        assert np.all(np.abs(a - f).reshape(k, -1) <=
                      TOL_FP32 * np.abs(f).max() + bd), name


def test_repeat_runs_are_bitwise_identical(torch_cuda):
    from paper_2405_20067_amd import ngd
    mix, x, proj = case(10, 2000, 6000, seed=5)
    g = inputs.gen_grad_out(6000, seed=5)
    m = _mixture(torch_cuda, mix)
    xd, gd = dev(x), dev(g)
    runs = []
    for _ in range(2):
        c = ngd.Cull().build(m, xd, proj, _params())
        f = host(ngd.eval_mixture(m, c, xd))
        grads = [host(t) for t in ngd.eval_backward(m, c, xd, gd)]
        runs.append([f] + grads)
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)


def test_rebuild_in_place_and_stale_detection(torch_cuda):
    from paper_2405_20067_amd import ngd
    mix, x, proj = case(6, 300, 1500, seed=9)
    m = _mixture(torch_cuda, mix)
    xd = dev(x)
    c = ngd.Cull().build(m, xd, proj, _params())
    h0 = c.handle.value
    f0 = host(ngd.eval_mixture(m, c, xd))
    # a new parameter upload makes the cull stale
    m.update(dev(mix["mean"]), dev(mix["factor"]), dev(mix["weight"]), dev(mix["colour"]))
    with pytest.raises(ngd.NgdError) as ei:
        ngd.eval_mixture(m, c, xd)
    assert ei.value.code == ngd.E_STALE
    # another query buffer is stale too
    c.build(m, xd, proj, _params())
    assert c.handle.value == h0
    with pytest.raises(ngd.NgdError) as ei:
        ngd.eval_mixture(m, c, dev(x))
    assert ei.value.code == ngd.E_STALE
    np.testing.assert_array_equal(host(ngd.eval_mixture(m, c, xd)), f0)
    # a smaller rebuild in the same handle
    c.build(m, xd[:700], proj, _params())
    f1 = host(ngd.eval_mixture(m, c, xd[:700]))
    want = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x[:700])
    assert normwise(f1, want) <= TOL_FP32


def test_rebuild_growing_and_shrinking_lists(torch_cuda):
    """The list kernels are launched before the host knows the list sizes,
    into the buffers as they are: a rebuild whose lists outgrow them must
    build them again after the buffers grow, and one that fits must leave
    no stale entries.  Each build's lists equal the CPU cull's bit for bit."""
    from paper_2405_20067_amd import ngd
    mix, x, proj = case(6, 2000, 9000, seed=12)
    m = _mixture(torch_cuda, mix)
    c = ngd.Cull()
    for qn in (300, 9000, 9000, 2500, 9000):
        xs = np.ascontiguousarray(x[:qn])
        xd = dev(xs)
        c.build(m, xd, proj, _params())
        got = c.export()
        want = oracle.cull(mix["mean"], mix["factor"], xs, proj, tau=1e-4, tile=256,
                           key_proj=16, key_bits=2)
        assert got["total"] == want["total"], qn
        for key in ("tile_off", "cand", "g_off", "g_tiles"):
            np.testing.assert_array_equal(got[key], want[key], err_msg=f"{key} q={qn}")
        f = host(ngd.eval_mixture(m, c, xd))
        full = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], xs)
        assert normwise(f, full) <= TOL_FP32, qn


def test_destroy_returns_all_device_memory(torch_cuda):
    """Every workspace a cull allocates (the front's, the lists', the
    backward's and the matrix-core forward's) is freed by ngd_cull_destroy:
    repeated build / evaluate / backward / destroy cycles leave the device's
    free memory where it was."""
    from paper_2405_20067_amd import ngd
    mix, x, proj = case(10, 1 << 15, 1 << 17, seed=33)
    m = _mixture(torch_cuda, mix)
    xd = dev(x)
    g = dev(inputs.gen_grad_out(x.shape[0], seed=4))

    def cycle():
        c = ngd.Cull().build(m, xd, proj, _params())
        for prec in (ngd.FP32, ngd.BF16_MFMA):
            ngd.eval_mixture(m, c, xd, precision=prec)
            ngd.eval_backward(m, c, xd, g, precision=prec)
        torch_cuda.cuda.synchronize()
        assert c.stats()["total"] > 2 * 10 ** 5   # lists of a megabyte and more
        c.close()

    cycle()   # the first cycle may leave driver-side caches warm
    torch_cuda.cuda.synchronize()
    free0 = torch_cuda.cuda.mem_get_info()[0]
    for _ in range(6):
        cycle()
    torch_cuda.cuda.synchronize()
    free1 = torch_cuda.cuda.mem_get_info()[0]
    assert free1 >= free0 - (16 << 20), (free0 - free1) / 2 ** 20


def test_validate_flags_singular_factor(torch_cuda):
    from paper_2405_20067_amd import ngd
    mix, _, _ = case(4, 50, 10, seed=2)
    m = _mixture(torch_cuda, mix)
    m.validate()
    bad = mix["factor"].copy()
    bad[7, 2] = 0.0          # L_11 of Gaussian 7
    m.update(dev(mix["mean"]), dev(bad), dev(mix["weight"]), dev(mix["colour"]))
    with pytest.raises(ngd.NgdError) as ei:
        m.validate()
    assert ei.value.code == ngd.E_SINGULAR
    nanw = mix["weight"].copy()
    nanw[3] = np.nan
    m.update(dev(mix["mean"]), dev(mix["factor"]), dev(nanw), dev(mix["colour"]))
    with pytest.raises(ngd.NgdError):
        m.validate()


def test_edge_cases(torch_cuda):
    from paper_2405_20067_amd import ngd
    import torch
    mix, x, proj = case(4, 40, 300, seed=4)
    m = _mixture(torch_cuda, mix)
    # no queries
    empty = torch.empty((0, 4), dtype=torch.float32, device="cuda")
    c = ngd.Cull().build(m, empty, proj, _params())
    assert c.stats() == dict(total=0, max_per_tile=0, ntiles=0)
    assert ngd.eval_mixture(m, c, empty).shape == (0, 3)
    gm, gf, gw, gc = ngd.eval_backward(m, c, empty, torch.empty((0, 3), device="cuda"))
    assert float(gm.abs().max()) == 0.0 and float(gw.abs().max()) == 0.0
    # one query (the one where the mixture is largest, so f is not ~0)
    all_f = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x)
    i = int(np.argmax(all_f.sum(1)))
    xd1 = dev(x[i:i + 1])
    c1 = ngd.Cull().build(m, xd1, proj, _params())
    f1 = host(ngd.eval_mixture(m, c1, xd1))
    assert normwise(f1, all_f[i:i + 1]) <= TOL_FP32
    # queries far from every Gaussian: everything culled, f = 0, grads = 0
    far = dev(x + np.float32(50.0))
    cf = ngd.Cull().build(m, far, proj, _params())
    assert cf.stats()["total"] == 0
    assert float(ngd.eval_mixture(m, cf, far).abs().max()) == 0.0
    grads = ngd.eval_backward(m, cf, far, dev(inputs.gen_grad_out(300)))
    assert all(float(t.abs().max()) == 0.0 for t in grads)
    # no Gaussians
    m0 = ngd.Mixture(4, 0)
    z = torch.empty((0,), dtype=torch.float32, device="cuda")
    m0.update(z, z, z, z)
    xd = dev(x)
    c0 = ngd.Cull().build(m0, xd, proj, _params())
    assert float(ngd.eval_mixture(m0, c0, xd).abs().max()) == 0.0
    assert float(ngd.eval_mixture(m0, None, xd).abs().max()) == 0.0


def test_rel_l2_loss(torch_cuda):
    """The relative loss against the float64 oracle: predictions of both
    signs and of magnitudes from 1e-3 to 1e3, sizes across one and many
    reduction chunks."""
    from paper_2405_20067_amd import ngd
    rng = np.random.default_rng(1)
    for q in (1, 1000, 300001):
        mag = 10.0 ** rng.uniform(-3, 3, (q, 3))
        f = (mag * rng.choice([-1.0, 1.0], (q, 3))).astype(np.float32)
        t = (f * rng.uniform(0.5, 1.5, (q, 3)) + rng.standard_normal((q, 3))).astype(np.float32)
        for eps in (0.01, 1.0):
            loss, grad = ngd.rel_l2_loss(dev(f), dev(t), eps=eps)
            want_loss, want_grad = oracle.rel_l2(f, t, eps=np.float32(eps))
            assert float(host(loss)[0]) == pytest.approx(want_loss, rel=1e-5)
            np.testing.assert_allclose(host(grad), want_grad, rtol=1e-5, atol=0)


def test_l2_loss(torch_cuda):
    from paper_2405_20067_amd import ngd
    rng = np.random.default_rng(0)
    for q in (1, 1000, 300001):
        f = rng.standard_normal((q, 3)).astype(np.float32)
        t = rng.standard_normal((q, 3)).astype(np.float32)
        loss, grad = ngd.l2_loss(dev(f), dev(t))
        d = f.astype(np.float64) - t
        assert float(host(loss)[0]) == pytest.approx(np.mean(d * d), rel=1e-6)
        np.testing.assert_allclose(host(grad), 2 * d / d.size, rtol=1e-6, atol=0)


@pytest.mark.parametrize("n", [4, 10])
def test_mixed_sign_diagonals(torch_cuda, n):
    """Factors with negative and mixed-sign diagonals (the library accepts
    any nonzero diagonal).  Flipping the sign of column j of L leaves V = L L^T,
    hence every value and the cull, unchanged, and flips the factor
    gradient's column: the culled lists must equal those of the unflipped
    mixture and of the CPU cull, and the forwards and backwards of both
    precisions must match the oracle on the flipped parameters at 1e-4."""
    from paper_2405_20067_amd import ngd
    k, q = 1200, 4100
    mix, x, proj = case(n, k, q, seed=41 + n)
    rng = np.random.default_rng(n)
    flip = np.where(rng.random((k, n)) < 0.5, -1.0, 1.0).astype(np.float32)
    flip[0] = -1.0                       # one Gaussian with every diagonal negative
    r, cidx = np.tril_indices(n)
    mixf = dict(mix, factor=np.ascontiguousarray(mix["factor"] * flip[:, cidx]))
    assert (mixf["factor"][:, r == cidx] < 0).any() and (mixf["factor"][:, r == cidx] > 0).any()
    g = inputs.gen_grad_out(q, seed=3)
    xd = dev(x)
    m0, m1 = _mixture(torch_cuda, mix), _mixture(torch_cuda, mixf)
    m1.validate()
    c0 = ngd.Cull().build(m0, xd, proj, _params())
    c1 = ngd.Cull().build(m1, xd, proj, _params())
    e0, e1 = c0.export(), c1.export()
    want = oracle.cull(mixf["mean"], mixf["factor"], x, proj, tau=1e-4, tile=256,
                       key_proj=16, key_bits=2)
    for key in ("perm", "gperm", "tile_off", "cand", "g_off", "g_tiles"):
        np.testing.assert_array_equal(e1[key], e0[key], err_msg=key)
        np.testing.assert_array_equal(e1[key], want[key], err_msg=key)
    fo = oracle.eval_mixture(mixf["mean"], mixf["factor"], mixf["weight"], mixf["colour"], x)
    sel, qoff, qidx = per_gaussian_csr(e1, q, 256)
    part = oracle.grad_lists(mixf["mean"], mixf["factor"], mixf["weight"], mixf["colour"], x, g,
                             sel, qoff, qidx)
    for prec in (ngd.FP32, ngd.BF16_MFMA):
        f = host(ngd.eval_mixture(m1, c1, xd, precision=prec))
        assert normwise(f, fo) <= TOL_FP32, prec
        got = [host(t) for t in ngd.eval_backward(m1, c1, xd, dev(g), precision=prec)]
        for name, a, b in zip(("mean", "factor", "weight", "colour"), got, part):
            want_g = np.zeros_like(a, dtype=np.float64)
            want_g[sel] = b
            assert normwise(a, want_g) <= TOL_FP32, (prec, name)


@pytest.mark.parametrize("n", [4, 10])
def test_pairs_at_the_skip_threshold_are_kept(torch_cuda, n):
    """Pairs just inside the forward's skip threshold must be evaluated.
    Correlated Gaussians (V_ii well above L_ii^2), far apart; each tile of
    128 queries (given order) holds 64 queries at a Gaussian's mean, which
    keep it a candidate, and 64 at its extreme point along one axis,
    x - m = r V e_i / sqrt(V_ii): Mahalanobis distance r, and the same
    distance r from the mean in that coordinate alone, in sigma_i.  With
    r = 6.5 and 6.75, below the threshold sqrt(2 ln(1/tau) + 40 ln 2) = 6.79
    (tau = 1e-4), the value exp(-r^2 / 2) exceeds what the skip may drop,
    tau 2^-20, so every precision must return it: a query box or a
    per-coordinate bound narrower than r sigma_i would lose it."""
    from paper_2405_20067_amd import ngd
    rng = np.random.default_rng(90 + n)
    k, tile, tau = 4, 128, 1e-4
    r_, c_ = np.tril_indices(n)
    fac = np.where(r_ == c_, rng.uniform(0.5, 1.5, (k, r_.size)),
                   rng.uniform(-1.0, 1.0, (k, r_.size)))
    L = np.zeros((k, n, n))
    L[:, r_, c_] = fac
    V = L @ L.transpose(0, 2, 1)
    assert (np.einsum("kii->ki", V) > 1.5 * np.einsum("kii->ki", L) ** 2).any()
    mean = np.zeros((k, n))
    mean[:, 0] = 1000.0 * np.arange(k)
    xs = []
    for g in range(k):
        sd = np.sqrt(np.diag(V[g]))
        for i in range(n):
            for sgn in (-1.0, 1.0):
                for rad in (6.5, 6.75):
                    centre = mean[g] + 1e-3 * sd * rng.standard_normal((64, n))
                    edge = mean[g] + sgn * rad * V[g][:, i] / sd[i]
                    probe = edge + 1e-6 * sd * rng.standard_normal((64, n))
                    xs += [centre, probe]
    x = np.ascontiguousarray(np.concatenate(xs), dtype=np.float32)
    q = x.shape[0]
    mix = dict(mean=mean.astype(np.float32), factor=fac.astype(np.float32),
               weight=np.ones(k, np.float32),
               colour=np.tile(np.float32([0.5, 0.7, 0.9]), (k, 1)))
    proj = inputs.gen_projections(n, 16, seed=7)
    m = _mixture(torch_cuda, mix)
    xd = dev(x)
    c = ngd.Cull().build(m, xd, proj, _params(tile=tile, tau=tau, tiling=2))
    exp = c.export()
    assert np.all(np.diff(exp["tile_off"]) == 1)   # each tile: its own Gaussian only
    qoff, gidx = per_query_csr(exp, q, tile)
    want = oracle.eval_lists(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x,
                             qoff, gidx)
    probes = np.concatenate([np.arange(t * tile + 64, (t + 1) * tile) for t in range(q // tile)])
    colour = mix["colour"][0].astype(np.float64)
    g_val = want[probes] / colour
    assert g_val.min() > 1.25 * tau * 2.0 ** -20    # above what the skip may drop
    for prec in (ngd.FP32, ngd.BF16_MFMA):
        f = host(ngd.eval_mixture(m, c, xd, precision=prec)).astype(np.float64)
        err = np.abs(f - want)
        assert np.all(err <= 1e-4 * np.abs(want) + tau * 2.0 ** -20 * colour), (
            prec, float((err / np.maximum(np.abs(want), 1e-300)).max()))


@pytest.mark.parametrize("n", list(range(1, 13)))
def test_every_dimension_forward_and_backward(torch_cuda, n):
    """Every compiled dimension 1..12: the culled forward of both precisions
    against the float64 oracle over the same candidate pairs, and the
    backward against the oracle's gradient over the candidate queries of
    each Gaussian (small sizes; tiles of 256 with a ragged last tile)."""
    from paper_2405_20067_amd import ngd
    k, q = 300, 1500
    mix, x, proj = case(n, k, q, seed=500 + n)
    m = _mixture(torch_cuda, mix)
    xd = dev(x)
    c = ngd.Cull().build(m, xd, proj, _params())
    exp = c.export()
    qoff, gidx = per_query_csr(exp, q, 256)
    want = oracle.eval_lists(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x,
                             qoff, gidx)
    g = inputs.gen_grad_out(q, seed=6)
    sel, goff, gq = per_gaussian_csr(exp, q, 256)
    part = oracle.grad_lists(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x, g,
                             sel, goff, gq)
    for prec in (ngd.FP32, ngd.BF16_MFMA):
        f = host(ngd.eval_mixture(m, c, xd, precision=prec))
        assert normwise(f, want) <= TOL_FP32, (n, prec)
        got = [host(t) for t in ngd.eval_backward(m, c, xd, dev(g), precision=prec)]
        for name, a, b in zip(("mean", "factor", "weight", "colour"), got, part):
            want_g = np.zeros_like(a, dtype=np.float64)
            want_g[sel] = b
            assert normwise(a, want_g) <= TOL_FP32, (n, prec, name)
