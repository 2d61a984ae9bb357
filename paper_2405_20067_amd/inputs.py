"""Seeded synthetic workloads for the N-D Gaussian mixture hot path.

This module only draws random inputs; it holds none of the method's
arithmetic (no evaluation, no culling, no gradients).  Both the GPU path's
callers and the CPU test oracle take their inputs from here.

Shapes and value distributions follow the workloads the paper fits
(Sec. 4.1: 10-D surface G-buffer queries -- position, normal, view
direction, roughness; Sec. 4.2: 6-D position + direction), at the sizes of
the named workloads below.  The paper's own scenes are not available, so
these seeded inputs stand in for them.

Factor distribution.  A workload names a lower-triangular factor with a
log-uniform diagonal "inverse scale" and normal off-diagonals.  It is read
as the factor S of the *precision* (V^-1 = S^T S): S_ii = exp(U[ln a, ln b]),
S_ij ~ N(0, sd^2) for i > j.  The mixture parameter of the paper
(Sec. 3.1, Eq. 2) is L with V = L L^T, so L = S^-1 is formed in float64
(a library inverse) and rounded once to float32.

Draw order for one mixture (numpy PCG64, fixed): means, S diagonal,
S strictly-lower entries (packed row-major), weights, colours.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "tri",
    "sample_domain",
    "gen_mixture",
    "gen_queries",
    "gen_near_queries",
    "gen_workload_queries",
    "gen_grad_out",
    "gen_projections",
    "gen_gbuffer",
    "gen_mixture_on",
    "gen_detailed_mixture",
    "SEED_MIXTURE",
    "SEED_QUERIES",
    "SEED_PROJ",
    "SEED_TARGET",
]

SEED_MIXTURE = 1
SEED_QUERIES = 2
SEED_PROJ = 3
SEED_TARGET = 4096007


def tri(n: int) -> int:
    """Number of entries in an n x n lower triangle."""
    return n * (n + 1) // 2


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # dimension N
    k: int                 # number of Gaussians
    q: int                 # number of queries
    layout: str            # domain: "cube", "pos3+dir3", "pos3+nrm3+view3+rough1"
    s_diag: tuple          # log-uniform range of the precision-factor diagonal
    s_off_sd: float        # sd of the precision-factor off-diagonals
    near_frac: float       # fraction of queries drawn near mixture components
    k_target: int = 0      # size of the hidden target mixture (0: none)
    culled: bool = True
    backward: bool = False
    description: str = ""


WORKLOADS = {
    "4d-dense": Workload(
        "4d-dense", 4, 256, 65536, "cube", (5.0, 50.0), 2.0, 0.0,
        culled=False,
        description="4-D plain mixture, K=256, 65,536 uniform queries, "
                    "FP32 forward without culling"),
    "6d-culled": Workload(
        "6d-culled", 6, 65536, 1 << 20, "pos3+dir3", (10.0, 200.0), 5.0, 0.0,
        description="6-D position+direction mixture, K=65,536, 2^20 uniform "
                    "queries, FP32 forward with 16-projection culling, tau=1e-4"),
    "10d-fwdbwd": Workload(
        "10d-fwdbwd", 10, 262144, 1 << 20, "pos3+nrm3+view3+rough1",
        (10.0, 200.0), 5.0, 0.5, k_target=4096, backward=True,
        description="10-D surface mixture (pos, normal, view, roughness), "
                    "K=262,144, 2^20 queries, culled FP32 forward + backward "
                    "of an L2 loss against a hidden K=4,096 mixture"),
    "10d-uniform": Workload(
        "10d-uniform", 10, 262144, 1 << 20, "pos3+nrm3+view3+rough1",
        (10.0, 200.0), 5.0, 0.0, k_target=4096, backward=True,
        description="the 10-D fwd+bwd workload with all 2^20 queries uniform over the "
                    "domain (none drawn near the mixtures)"),
    "10d-4m": Workload(
        "10d-4m", 10, 262144, 1 << 22, "pos3+nrm3+view3+rough1",
        (10.0, 200.0), 5.0, 0.5, k_target=4096, backward=True,
        description="10-D, K=262,144, 2^22 queries, culled forward + backward; BF16 MFMA "
                    "filter against the float32 kernel"),
}


def _unit_sphere(rng: np.random.Generator, count: int) -> np.ndarray:
    g = rng.standard_normal((count, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def sample_domain(rng: np.random.Generator, layout: str, n: int,
                  count: int) -> np.ndarray:
    """Points of the workload's domain, float64 (count x n)."""
    if layout == "cube":
        return rng.random((count, n))
    if layout == "pos3+dir3":
        assert n == 6
        pos = rng.random((count, 3))
        return np.concatenate([pos, _unit_sphere(rng, count)], axis=1)
    if layout == "pos3+nrm3+view3+rough1":
        assert n == 10
        pos = rng.random((count, 3))
        nrm = _unit_sphere(rng, count)
        view = _unit_sphere(rng, count)
        rough = rng.random((count, 1))
        return np.concatenate([pos, nrm, view, rough], axis=1)
    raise ValueError(f"unknown layout {layout!r}")


def gen_mixture(n: int, k: int, layout: str = "cube",
                s_diag=(5.0, 50.0), s_off_sd: float = 2.0,
                seed: int = SEED_MIXTURE) -> dict:
    """A seeded mixture; every array float32 and C-contiguous.

    mean   (k, n)
    factor (k, n(n+1)/2)   L packed lower, row-major: idx(i, j) = i(i+1)/2 + j
    weight (k,)            brightness alpha (already activated, > 0)
    colour (k, 3)          RGB (already activated, in [0, 1])
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mean = sample_domain(rng, layout, n, k)
    lo, hi = math.log(s_diag[0]), math.log(s_diag[1])
    s_d = np.exp(rng.uniform(lo, hi, size=(k, n)))
    n_off = tri(n) - n
    s_o = rng.standard_normal((k, n_off)) * s_off_sd
    weight = rng.uniform(0.1, 1.0, size=k)
    colour = rng.random((k, 3))

    s_full = np.zeros((k, n, n))
    ii = np.arange(n)
    s_full[:, ii, ii] = s_d
    rows, cols = np.tril_indices(n, -1)   # row-major over strictly-lower
    s_full[:, rows, cols] = s_o
    l_full = np.linalg.inv(s_full)        # input generation only
    r_all, c_all = np.tril_indices(n)
    factor = l_full[:, r_all, c_all]
    return dict(
        mean=np.ascontiguousarray(mean, dtype=np.float32),
        factor=np.ascontiguousarray(factor, dtype=np.float32),
        weight=np.ascontiguousarray(weight, dtype=np.float32),
        colour=np.ascontiguousarray(colour, dtype=np.float32),
    )


def gen_queries(n: int, q: int, layout: str = "cube",
                seed: int = SEED_QUERIES) -> np.ndarray:
    """q uniform points of the domain, float32 (q, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(sample_domain(rng, layout, n, q),
                                dtype=np.float32)


def gen_near_queries(mixtures, q: int, seed: int) -> np.ndarray:
    """q points drawn from the mixtures' own components: pick a component j
    uniformly over all components of all given mixtures, then x = m_j + L_j u
    with u ~ N(0, I).  This is how a fitted mixture sits on its data: the
    queries are where the Gaussians are."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = np.concatenate([m["mean"] for m in mixtures]).astype(np.float64)
    facs = np.concatenate([m["factor"] for m in mixtures]).astype(np.float64)
    kk, n = means.shape
    j = rng.integers(0, kk, size=q)
    u = rng.standard_normal((q, n))
    r_all, c_all = np.tril_indices(n)
    l_full = np.zeros((q, n, n))
    l_full[:, r_all, c_all] = facs[j]
    x = means[j] + np.einsum("qab,qb->qa", l_full, u)
    return np.ascontiguousarray(x, dtype=np.float32)


def gen_workload_queries(w: Workload, q: int | None = None, mixtures=(),
                         seed: int = SEED_QUERIES) -> np.ndarray:
    """The workload's queries: a fraction near_frac drawn near the given
    mixtures' components (interleaved in a seeded random order), the rest
    uniform over the domain."""
    q = w.q if q is None else q
    n_near = int(round(q * w.near_frac)) if mixtures else 0
    uni = gen_queries(w.n, q - n_near, w.layout, seed)
    if n_near == 0:
        return uni
    near = gen_near_queries(list(mixtures), n_near, seed + 7919)
    allq = np.concatenate([uni, near])
    order = np.random.Generator(np.random.PCG64(seed + 104729)).permutation(q)
    return np.ascontiguousarray(allq[order])


def gen_grad_out(q: int, seed: int = 11, scale: float = 1.0) -> np.ndarray:
    """A seeded upstream gradient dl/df, float32 (q, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal((q, 3)) * scale,
                                dtype=np.float32)


def gen_projections(n: int, n_proj: int = 16, seed: int = SEED_PROJ) -> np.ndarray:
    """n_proj random unit vectors in R^n (Sec. 3.2 samples them at random and
    fixes nothing else): standard normal draws, normalised in float64,
    rounded once to float32.  Shape (n_proj, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((n_proj, n))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return np.ascontiguousarray(g, dtype=np.float32)


def workload_mixture(w: Workload, k: int | None = None,
                     seed: int = SEED_MIXTURE) -> dict:
    return gen_mixture(w.n, w.k if k is None else k, w.layout, w.s_diag,
                       w.s_off_sd, seed)


def gen_gbuffer(width: int = 800, height: int = 800, tile: int = 16,
                constant_features=None) -> np.ndarray:
    """A synthetic 10-D G-buffer (position 3, normal 3, view direction 3,
    roughness 1), the kind of per-pixel input the paper's global
    illumination scenes evaluate its Gaussians at; float32, (height*width,
    10), laid out tile by tile (tiles of tile x tile pixels in row-major
    order of tiles, row-major pixels inside a tile), so that the cull's
    given-order tiling (tiling 2) forms the paper's 16 x 16 pixel tiles.

    The scene (no randomness): a pinhole camera at (0.5, 0.5, 1.8) looking
    down -z through the open front of the unit box [0, 1]^3, whose inside
    walls (floor, ceiling, back and side walls) and a sphere of radius 0.22
    at (0.5, 0.25, 0.45) are the visible surfaces.  Normal: the surface
    normal facing the camera; view: the unit vector from the point to the
    camera; roughness 0.2 + 0.6 (0.5 + 0.5 sin(7x) cos(5z + 3y)), a smooth
    texture.  With `constant_features` (7 values: normal, view, roughness),
    every pixel keeps its position and takes those (the case of Sec. 3.2
    where every input but the position is constant over the image)."""
    if width % tile or height % tile:
        raise ValueError("width and height must be multiples of the tile size")
    cam = np.array([0.5, 0.5, 1.8])
    v, u = np.meshgrid((np.arange(height) + 0.5) / height, (np.arange(width) + 0.5) / width,
                       indexing="ij")
    # image plane z = 1 (the box's open face), inside [0.02, 0.98]^2, so that
    # every ray enters the box and meets an inside wall or the sphere
    tgt = np.stack([0.02 + 0.96 * u, 0.98 - 0.96 * v, np.ones_like(u)], -1)
    d = tgt - cam
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    t_best = np.full(u.shape, np.inf)
    nrm = np.zeros(u.shape + (3,))
    # inside walls: planes x=0, x=1, y=0, y=1, z=0 with inward normals
    for axis, val, sgn in ((0, 0.0, 1.0), (0, 1.0, -1.0), (1, 0.0, 1.0), (1, 1.0, -1.0),
                           (2, 0.0, 1.0)):
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (val - cam[axis]) / d[..., axis]
        pt = cam + t[..., None] * d
        inside = np.all((pt >= -1e-9) & (pt <= 1 + 1e-9), axis=-1) & (t > 0)
        hit = inside & (t < t_best)
        t_best = np.where(hit, t, t_best)
        nv = np.zeros(3)
        nv[axis] = sgn
        nrm = np.where(hit[..., None], nv, nrm)
    # the sphere
    cen, rad = np.array([0.5, 0.25, 0.45]), 0.22
    oc = cam - cen
    b = np.einsum("...i,i->...", d, oc)
    disc = b * b - (oc @ oc - rad * rad)
    ts = -b - np.sqrt(np.maximum(disc, 0.0))
    hit = (disc > 0) & (ts > 0) & (ts < t_best)
    t_best = np.where(hit, ts, t_best)
    pts = cam + t_best[..., None] * d
    sn = (pts - cen) / rad
    nrm = np.where(hit[..., None], sn, nrm)
    assert np.isfinite(t_best).all()
    pos = pts
    view = cam - pos
    view /= np.linalg.norm(view, axis=-1, keepdims=True)
    rough = 0.2 + 0.6 * (0.5 + 0.5 * np.sin(7 * pos[..., 0]) * np.cos(5 * pos[..., 2] +
                                                                      3 * pos[..., 1]))
    feat = np.concatenate([pos, nrm, view, rough[..., None]], -1)
    if constant_features is not None:
        cst = np.asarray(constant_features, np.float64).ravel()
        assert cst.size == 7
        feat[..., 3:] = cst
    # tile-major layout
    th, tw = height // tile, width // tile
    feat = feat.reshape(th, tile, tw, tile, 10).transpose(0, 2, 1, 3, 4).reshape(-1, 10)
    return np.ascontiguousarray(feat, dtype=np.float32)


def gen_mixture_on(points: np.ndarray, k: int, s_diag=(10.0, 200.0), s_off_sd: float = 5.0,
                   jitter: float = 0.02, seed: int = SEED_MIXTURE) -> dict:
    """A mixture sitting on given data, as a fitted one does: the means are
    k of the points (seeded choice) moved by N(0, jitter^2) per coordinate;
    factors, brightness and colours as gen_mixture draws them."""
    n = points.shape[1]
    mix = gen_mixture(n, k, "cube", s_diag, s_off_sd, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 17))
    j = rng.integers(0, points.shape[0], size=k)
    mean = points[j].astype(np.float64) + jitter * rng.standard_normal((k, n))
    mix["mean"] = np.ascontiguousarray(mean, dtype=np.float32)
    return mix


def gen_detailed_mixture(coarse: dict, sub: int = 16, spread: float = 1.0,
                         narrow: float = 0.35, seed: int = SEED_TARGET + 1) -> dict:
    """A mixture with detail inside a coarse one: every coarse component j
    is replaced by `sub` narrower components, means m_j + spread L_j z
    (z ~ N(0, I)), factors narrow * L_j, brightness alpha_j * 4 / sub and
    colours c_j moved by N(0, 0.2^2) (clipped to [0, 1]).  A fit that starts
    from the coarse components has to add Gaussians to reach this one."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k, n = coarse["mean"].shape
    src = np.repeat(np.arange(k), sub)
    r_all, c_all = np.tril_indices(n)
    lf = np.zeros((k * sub, n, n))
    lf[:, r_all, c_all] = coarse["factor"][src]
    z = rng.standard_normal((k * sub, n))
    mean = coarse["mean"][src] + spread * np.einsum("kij,kj->ki", lf, z)
    colour = np.clip(coarse["colour"][src] + 0.2 * rng.standard_normal((k * sub, 3)), 0, 1)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(mean=f32(mean), factor=f32(narrow * coarse["factor"][src]),
                weight=f32(coarse["weight"][src] * 4.0 / sub), colour=f32(colour))
