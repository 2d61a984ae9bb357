"""Shared helpers of the GPU parity tests (inputs, device upload, error
measures).  Holds none of the method's arithmetic."""

import numpy as np

from paper_2405_20067_amd import inputs


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def normwise(got, want):
    """max |got - want| / max |want| (the per-output error of the bench)."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = np.abs(want).max()
    if scale == 0:
        return float(np.abs(got).max())
    return float(np.abs(got - want).max() / scale)


def case(n, k, q, layout=None, seed=1, near=0.5, sdiag=None, soff=None):
    """A seeded mixture + queries of the given size; half the queries near
    the components unless near=0."""
    layout = layout or {4: "cube", 6: "pos3+dir3", 10: "pos3+nrm3+view3+rough1"}.get(n, "cube")
    if sdiag is None:
        sdiag = (5.0, 50.0) if n <= 4 else (10.0, 200.0)
    if soff is None:
        soff = 2.0 if n <= 4 else 5.0
    mix = inputs.gen_mixture(n, k, layout, sdiag, soff, seed=seed)
    n_near = int(round(q * near)) if k > 0 else 0
    x = inputs.gen_queries(n, q - n_near, layout, seed=seed + 1)
    if n_near:
        xn = inputs.gen_near_queries([mix], n_near, seed=seed + 2)
        x = np.concatenate([x, xn])
        x = x[np.random.default_rng(seed + 3).permutation(q)]
    proj = inputs.gen_projections(n, 16, seed=seed + 4)
    return mix, np.ascontiguousarray(x, dtype=np.float32), proj


def per_query_csr(c, q, tile):
    """CSR (qoff, gidx) of each query's candidate Gaussians (caller order)."""
    pos = np.empty(q, np.int64)
    pos[c["perm"]] = np.arange(q)
    tiles = pos // tile
    counts = np.diff(c["tile_off"])[tiles]
    qoff = np.zeros(q + 1, np.int64)
    qoff[1:] = np.cumsum(counts)
    gidx = np.empty(qoff[-1], np.int32)
    for p in range(q):
        t = tiles[p]
        lst = c["cand"][c["tile_off"][t]:c["tile_off"][t + 1]]
        gidx[qoff[p]:qoff[p + 1]] = c["gperm"][lst]
    return qoff, gidx


def per_gaussian_csr(c, q, tile):
    """For every Gaussian with candidate tiles: (sel, qoff, qidx) listing the
    queries of its tiles (caller's indices), for the oracle's grad_lists."""
    sel, qoff, qidx = [], [0], []
    for s_pos in range(len(c["gperm"])):
        tiles = c["g_tiles"][c["g_off"][s_pos]:c["g_off"][s_pos + 1]]
        if tiles.size == 0:
            continue
        qs = np.concatenate([c["perm"][t * tile:min((t + 1) * tile, q)] for t in tiles])
        sel.append(c["gperm"][s_pos])
        qidx.append(qs)
        qoff.append(qoff[-1] + qs.size)
    qidx = np.concatenate(qidx) if qidx else np.zeros(0, np.int64)
    return np.array(sel, np.int64), np.array(qoff, np.int64), qidx.astype(np.int64)


def queries_of_gaussians(c, sel, q, tile):
    """(qoff, qidx): the queries of the candidate tiles of each caller
    Gaussian sel[j] (caller's indices), from an exported cull."""
    pos = np.empty(len(c["gperm"]), np.int64)
    pos[c["gperm"]] = np.arange(len(c["gperm"]))
    qoff, qidx = [0], []
    for gi in sel:
        s_pos = pos[gi]
        tiles = c["g_tiles"][c["g_off"][s_pos]:c["g_off"][s_pos + 1]]
        qs = (np.concatenate([c["perm"][t * tile:min((t + 1) * tile, q)] for t in tiles])
              if tiles.size else np.zeros(0, np.int64))
        qidx.append(qs.astype(np.int64))
        qoff.append(qoff[-1] + qs.size)
    qidx = np.concatenate(qidx) if qidx else np.zeros(0, np.int64)
    return np.array(qoff, np.int64), qidx


def omitted_pairs_grad_bound(mix, g, sel, tau):
    """Per selected Gaussian, a bound on what the pairs the culled gradient
    leaves out can add to each gradient output, from the cull's guarantee.

    A pair is left out only when the interval test of Eq. 5 rejects it (then
    by Cauchy-Schwarz, (r^T d)^2 <= sigma_r^2 M, its Mahalanobis distance is
    M >= kappa^2 = 2 ln(1/tau) at every query of the tile) or when the
    in-kernel skip certifies G < tau 2^-20 (M larger still).  For M >=
    kappa^2 >= 2: G <= tau, G sqrt(M) <= tau kappa and G M <= tau kappa^2
    (exp(-M/2) M^p decreases for M >= 2p).  The pair's terms are
    d alpha = G s, d c = alpha G g, d m = alpha G s z and d L = tril(alpha G s
    z y^T), with s = g . c, |y| = sqrt(M) and |z| = |L^-T y| <= |L^-1|_2
    sqrt(M).  Summed over every query (a superset of the ones left out),
    with a 1% margin for the float32 rounding of the interval test.
    Returns (mean, factor, weight, colour) bounds of shapes (s,), (s,),
    (s,), (s, 3), each bounding every entry of that output."""
    n = mix["mean"].shape[1]
    k2 = 2.0 * np.log(1.0 / tau)
    assert k2 >= 2.0
    kap = np.sqrt(k2)
    gsum = np.abs(np.asarray(g, np.float64)).sum(0)          # sum over queries of |g_ch|
    sel = np.asarray(sel, np.int64)
    r, cidx = np.tril_indices(n)
    L = np.zeros((sel.size, n, n))
    L[:, r, cidx] = mix["factor"][sel]
    snorm = np.linalg.norm(np.linalg.inv(L), 2, axis=(1, 2))
    alpha = mix["weight"][sel].astype(np.float64)
    ssum = np.abs(mix["colour"][sel].astype(np.float64)) @ gsum   # sum over queries of |s|
    out = (alpha * ssum * snorm * tau * kap, alpha * ssum * snorm * tau * k2, ssum * tau,
           alpha[:, None] * tau * gsum[None, :])
    return tuple(1.01 * v for v in out)
