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
