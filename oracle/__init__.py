"""CPU oracle for the N-D Gaussian mixture hot path -- TEST INFRASTRUCTURE.

Plain float64 C code (ngd_oracle.c: the direct sum and its gradient) and a
CPU re-implementation of the tile cull (ngd_cull_ref.c), loaded with ctypes;
in numpy float64, the parent-child composition of Sec. 3.3 (Eq. 6-7) with
its chain rule, and the conditioning of Sec. 3.2 by the textbook formulas.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product path shares no code with it.

The arithmetic functions take float32 arrays (the values the GPU receives)
and promote them exactly to float64; float64 arrays are used as given (the
finite-difference pins need that).  The cull takes float32 only.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = [
    "lib",
    "eval_mixture",
    "eval_lists",
    "grad",
    "grad_lists",
    "msq_pairs",
    "gaussian",
    "cull",
    "kappa2_from_tau",
    "rel_l2",
    "threads",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libngd_oracle.so")
_lib = None

_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def lib():
    """The loaded oracle library (built on first use if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    L = ctypes.CDLL(_LIB_PATH)
    i, i64, p = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    L.ngd_oracle_threads.argtypes = []
    L.ngd_oracle_threads.restype = ctypes.c_int
    L.ngd_oracle_set_threads.argtypes = [i]
    L.ngd_oracle_set_threads.restype = ctypes.c_int
    L.ngd_oracle_gaussian.argtypes = [i, _f64p, _f64p, _f64p]
    L.ngd_oracle_gaussian.restype = ctypes.c_double
    L.ngd_oracle_eval.argtypes = [i, i64, _f64p, _f64p, _f64p, _f64p, i64, _f64p, _f64p]
    L.ngd_oracle_eval_lists.argtypes = [i, _f64p, _f64p, _f64p, _f64p, i64, _f64p,
                                        _i64p, _i32p, _f64p]
    L.ngd_oracle_grad.argtypes = [i, i64, _f64p, _f64p, _f64p, _f64p, i64, _f64p, _f64p,
                                  _i64p, i64, _f64p, _f64p, _f64p, _f64p]
    L.ngd_oracle_grad_lists.argtypes = [i, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                        _i64p, i64, _i64p, _i64p, _f64p, _f64p, _f64p,
                                        _f64p]
    L.ngd_oracle_msq_pairs.argtypes = [i, _f64p, _f64p, _f64p, i64, _i64p, _i64p, _f64p]
    for fn in ("ngd_oracle_eval", "ngd_oracle_eval_lists", "ngd_oracle_grad",
               "ngd_oracle_grad_lists", "ngd_oracle_msq_pairs"):
        getattr(L, fn).restype = ctypes.c_int
    L.ngd_cull_ref_run.argtypes = [i, i64, _f32p, _f32p, i64, _f32p, i, _f32p,
                                   ctypes.c_float, i, i, i, i]
    L.ngd_cull_ref_run.restype = p
    L.ngd_cull_ref_total.argtypes = [p]
    L.ngd_cull_ref_total.restype = i64
    L.ngd_cull_ref_ntiles.argtypes = [p]
    L.ngd_cull_ref_ntiles.restype = i64
    L.ngd_cull_ref_get.argtypes = [p, _i32p, _i32p, _i64p, _i32p, _i64p, _i32p, _f32p,
                                   _f32p, _f32p, _f32p, _u32p, _u32p, _f32p, _f32p, _f32p]
    L.ngd_cull_ref_get.restype = None
    L.ngd_cull_ref_free.argtypes = [p]
    L.ngd_cull_ref_free.restype = None
    _lib = L
    return L


def _d(a):
    """Contiguous float64 copy; float32 inputs (what the GPU receives) are
    promoted exactly, float64 inputs are kept as they are."""
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t):
    return a.ctypes.data_as(t)


def _check_mix(mean, factor, weight, colour):
    mean = _d(mean)
    k, n = mean.shape
    factor = _d(factor).reshape(k, n * (n + 1) // 2)
    weight = _d(weight).reshape(k)
    colour = _d(colour).reshape(k, 3)
    return n, k, mean, factor, weight, colour


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return lib().ngd_oracle_threads()


def set_threads(t: int) -> int:
    """Sets the OpenMP threads of later calls; returns the count in force."""
    return lib().ngd_oracle_set_threads(int(t))


def gaussian(mean, factor, x) -> float:
    """One Gaussian's value at one point (Eq. 1 with V = L L^T)."""
    mean, factor, x = _d(mean).ravel(), _d(factor).ravel(), _d(x).ravel()
    return lib().ngd_oracle_gaussian(mean.size, _p(mean, _f64p), _p(factor, _f64p),
                                     _p(x, _f64p))


def eval_mixture(mean, factor, weight, colour, queries) -> np.ndarray:
    """Direct float64 sum over all Gaussians (Eq. 8); returns (q, 3)."""
    n, k, mean, factor, weight, colour = _check_mix(mean, factor, weight, colour)
    x = _d(queries).reshape(-1, n)
    out = np.zeros((x.shape[0], 3))
    rc = lib().ngd_oracle_eval(n, k, _p(mean, _f64p), _p(factor, _f64p),
                               _p(weight, _f64p), _p(colour, _f64p), x.shape[0],
                               _p(x, _f64p), _p(out, _f64p))
    assert rc == 0
    return out


def eval_lists(mean, factor, weight, colour, queries, qoff, gidx) -> np.ndarray:
    """Sum restricted to Gaussians gidx[qoff[p]:qoff[p+1]] for query p."""
    n, k, mean, factor, weight, colour = _check_mix(mean, factor, weight, colour)
    x = _d(queries).reshape(-1, n)
    qoff = np.ascontiguousarray(qoff, dtype=np.int64)
    gidx = np.ascontiguousarray(gidx, dtype=np.int32)
    assert qoff.size == x.shape[0] + 1
    out = np.zeros((x.shape[0], 3))
    rc = lib().ngd_oracle_eval_lists(n, _p(mean, _f64p), _p(factor, _f64p),
                                     _p(weight, _f64p), _p(colour, _f64p), x.shape[0],
                                     _p(x, _f64p), _p(qoff, _i64p), _p(gidx, _i32p),
                                     _p(out, _f64p))
    assert rc == 0
    return out


def grad(mean, factor, weight, colour, queries, g, sel=None):
    """float64 gradient of l w.r.t. (mean, factor, weight, colour) of the
    Gaussians in sel (all when None), given g = dl/df of shape (q, 3)."""
    n, k, mean, factor, weight, colour = _check_mix(mean, factor, weight, colour)
    x = _d(queries).reshape(-1, n)
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(x.shape[0], 3))
    if sel is None:
        nsel, selp = k, None
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        nsel, selp = sel.size, _p(sel, _i64p)
    tri = n * (n + 1) // 2
    gm, gl = np.zeros((nsel, n)), np.zeros((nsel, tri))
    ga, gc = np.zeros(nsel), np.zeros((nsel, 3))
    rc = lib().ngd_oracle_grad(n, k, _p(mean, _f64p), _p(factor, _f64p),
                               _p(weight, _f64p), _p(colour, _f64p), x.shape[0],
                               _p(x, _f64p), _p(g, _f64p), selp, nsel, _p(gm, _f64p),
                               _p(gl, _f64p), _p(ga, _f64p), _p(gc, _f64p))
    assert rc == 0
    return gm, gl, ga, gc


def grad_lists(mean, factor, weight, colour, queries, g, sel, qoff, qidx):
    """Gradient of the Gaussians sel[s] summed over queries qidx[qoff[s]:qoff[s+1]]."""
    n, k, mean, factor, weight, colour = _check_mix(mean, factor, weight, colour)
    x = _d(queries).reshape(-1, n)
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(x.shape[0], 3))
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    qoff = np.ascontiguousarray(qoff, dtype=np.int64)
    qidx = np.ascontiguousarray(qidx, dtype=np.int64)
    nsel = sel.size
    tri = n * (n + 1) // 2
    gm, gl = np.zeros((nsel, n)), np.zeros((nsel, tri))
    ga, gc = np.zeros(nsel), np.zeros((nsel, 3))
    rc = lib().ngd_oracle_grad_lists(n, _p(mean, _f64p), _p(factor, _f64p),
                                     _p(weight, _f64p), _p(colour, _f64p), _p(x, _f64p),
                                     _p(g, _f64p), _p(sel, _i64p), nsel, _p(qoff, _i64p),
                                     _p(qidx, _i64p), _p(gm, _f64p), _p(gl, _f64p),
                                     _p(ga, _f64p), _p(gc, _f64p))
    assert rc == 0
    return gm, gl, ga, gc


def msq_pairs(mean, factor, queries, qi, gi) -> np.ndarray:
    """Squared Mahalanobis distance (x-m)^T V^-1 (x-m) of listed pairs."""
    mean = _d(mean)
    k, n = mean.shape
    factor = _d(factor).reshape(k, -1)
    x = _d(queries).reshape(-1, n)
    qi = np.ascontiguousarray(qi, dtype=np.int64)
    gi = np.ascontiguousarray(gi, dtype=np.int64)
    out = np.zeros(qi.size)
    rc = lib().ngd_oracle_msq_pairs(n, _p(mean, _f64p), _p(factor, _f64p), _p(x, _f64p),
                                    qi.size, _p(qi, _i64p), _p(gi, _i64p), _p(out, _f64p))
    assert rc == 0
    return out


def rel_l2(f, target, eps=0.01):
    """The relative squared error and its gradient, in float64.

    Sec. 4.1 trains with a relative L2 loss after Noise2Noise; its form is
    taken from there: every squared error is divided by the squared scale of
    the prediction, (|f| + eps)^2, and that scale is treated as a constant
    when differentiating.  With m = f.size:
        loss = (1/m) sum_i (f_i - t_i)^2 / (|f_i| + eps)^2
        grad_i = 2 (f_i - t_i) / (|f_i| + eps)^2 / m
    Returns (loss, grad) with grad shaped like f.
    """
    f = np.asarray(f, np.float64)
    t = np.asarray(target, np.float64)
    m = f.size
    if m == 0:
        return 0.0, np.zeros_like(f)
    scale = np.abs(f) + float(eps)
    err = f - t
    loss = float(np.sum(err * err / (scale * scale)) / m)
    grad = 2.0 * err / (scale * scale) / m
    return loss, grad


def kappa2_from_tau(tau: float) -> np.float32:
    """The squared interval half-width, in units of sigma, for which every
    culled pair has G <= tau: kappa^2 = 2 ln(1/tau), rounded to float32."""
    return np.float32(-2.0 * math.log(float(tau)))


def cull(mean, factor, queries, proj, tau=1e-4, tile=256, key_proj=16, key_bits=2, tiling=0):
    """CPU re-implementation of the tile cull (tiling 0: k-d order, 1: Morton
    key, 2: the queries' given order).  Returns a dict of arrays:
    perm, gperm, tile_off, cand, g_off, g_tiles, tile_lo, tile_hi, g_mr,
    g_thr, qkey, gkey, qlo, qhi (see ngd_cull_ref.c)."""
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    k, n = mean.shape
    factor = np.ascontiguousarray(factor, dtype=np.float32).reshape(k, n * (n + 1) // 2)
    queries = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, n)
    proj = np.ascontiguousarray(proj, dtype=np.float32).reshape(-1, n)
    q, n_proj = queries.shape[0], proj.shape[0]
    L = lib()
    h = L.ngd_cull_ref_run(n, k, _p(mean, _f32p), _p(factor, _f32p), q,
                           _p(queries, _f32p), n_proj, _p(proj, _f32p),
                           ctypes.c_float(kappa2_from_tau(tau)), tile, key_proj, key_bits,
                           tiling)
    if not h:
        raise ValueError("invalid cull arguments")
    try:
        total = L.ngd_cull_ref_total(h)
        T = L.ngd_cull_ref_ntiles(h)
        out = dict(
            perm=np.zeros(q, np.int32), gperm=np.zeros(k, np.int32),
            tile_off=np.zeros(T + 1, np.int64), cand=np.zeros(max(total, 1), np.int32),
            g_off=np.zeros(k + 1, np.int64), g_tiles=np.zeros(max(total, 1), np.int32),
            tile_lo=np.zeros((max(T, 1), n_proj), np.float32),
            tile_hi=np.zeros((max(T, 1), n_proj), np.float32),
            g_mr=np.zeros((max(k, 1), n_proj), np.float32),
            g_thr=np.zeros((max(k, 1), n_proj), np.float32),
            qkey=np.zeros(max(q, 1), np.uint32), gkey=np.zeros(max(k, 1), np.uint32),
            qlo=np.zeros(n_proj, np.float32), qhi=np.zeros(n_proj, np.float32),
            q_r=np.zeros((max(q, 1), n_proj), np.float32))
        o = out
        L.ngd_cull_ref_get(h, _p(o["perm"], _i32p), _p(o["gperm"], _i32p),
                           _p(o["tile_off"], _i64p), _p(o["cand"], _i32p),
                           _p(o["g_off"], _i64p), _p(o["g_tiles"], _i32p),
                           _p(o["tile_lo"], _f32p), _p(o["tile_hi"], _f32p),
                           _p(o["g_mr"], _f32p), _p(o["g_thr"], _f32p),
                           _p(o["qkey"], _u32p), _p(o["gkey"], _u32p),
                           _p(o["qlo"], _f32p), _p(o["qhi"], _f32p), _p(o["q_r"], _f32p))
    finally:
        L.ngd_cull_ref_free(h)
    out["cand"] = out["cand"][:total]
    out["g_tiles"] = out["g_tiles"][:total]
    out["tile_lo"] = out["tile_lo"][:T]
    out["tile_hi"] = out["tile_hi"][:T]
    out["g_mr"] = out["g_mr"][:k]
    out["g_thr"] = out["g_thr"][:k]
    out["qkey"] = out["qkey"][:q]
    out["q_r"] = out["q_r"][:q]
    out["gkey"] = out["gkey"][:k]
    out["ntiles"] = T
    out["total"] = total
    out["tile"] = tile
    out["kappa2"] = kappa2_from_tau(tau)
    return out


def _unpack(packed, n):
    r, c = np.tril_indices(n)
    full = np.zeros(packed.shape[:-1] + (n, n))
    full[..., r, c] = packed
    return full


def compose(mean_p, factor_p, parent, rel_factor, rel_mean):
    """Absolute (mean, factor) of parents then children in float64, from the
    children's parameters relative to their parents (Sec. 3.3, Eq. 6-7):
    L_c = L_p U, m_c = L_p m_u + m_p.  Factors packed lower by rows."""
    mean_p, factor_p = _d(mean_p), _d(factor_p)
    n = mean_p.shape[1]
    parent = np.asarray(parent, np.int64)
    lp = _unpack(factor_p[parent], n)
    u = _unpack(_d(rel_factor), n)
    lc = lp @ u
    mc = np.einsum("kij,kj->ki", lp, _d(rel_mean)) + mean_p[parent]
    r, c = np.tril_indices(n)
    return (np.concatenate([mean_p, mc]), np.concatenate([factor_p, lc[:, r, c]]))


def compose_grad(factor_p, parent, rel_factor, rel_mean, g_mean, g_factor):
    """Gradients with respect to (mean_p, factor_p, rel_factor, rel_mean) from
    those with respect to every Gaussian's absolute (mean, factor), parents
    then children (the derivative of the products of Eq. 6-7, restricted to
    the lower triangles)."""
    factor_p = _d(factor_p)
    kp = factor_p.shape[0]
    g_mean, g_factor = _d(g_mean), _d(g_factor)
    n = g_mean.shape[1]
    parent = np.asarray(parent, np.int64)
    lp = _unpack(factor_p[parent], n)
    u = _unpack(_d(rel_factor), n)
    mu = _d(rel_mean)
    gl = _unpack(g_factor[kp:], n)
    gm = g_mean[kp:]
    r, c = np.tril_indices(n)
    g_u = np.transpose(lp, (0, 2, 1)) @ gl
    g_mu = np.einsum("kji,kj->ki", lp, gm)
    g_lp = gl @ np.transpose(u, (0, 2, 1)) + gm[:, :, None] * mu[:, None, :]
    out_m = g_mean[:kp].copy()
    out_l = g_factor[:kp].copy()
    np.add.at(out_m, parent, gm)
    np.add.at(out_l, parent, g_lp[:, r, c])
    return out_m, out_l, g_u[:, r, c], g_mu


def condition(mean, factor, weight, colour, p, xc):
    """Every Gaussian conditioned on the values xc of its dimensions p..n-1
    (the paper's global conditioning, Sec. 3.2), by the textbook formulas in
    float64 with explicit inverses:
        mean'   = m_p + V_pc V_cc^-1 (x_c - m_c)
        cov'    = V_pp - V_pc V_cc^-1 V_cp,  factor' its Cholesky factor
        weight' = alpha exp(-(x_c - m_c)^T V_cc^-1 (x_c - m_c) / 2)
    with V = L L^T.  Returns (mean', factor' packed, weight', colour)."""
    n, k, mean, factor, weight, colour = _check_mix(mean, factor, weight, colour)
    L = _unpack(factor, n)
    V = L @ np.transpose(L, (0, 2, 1))
    xc = np.asarray(xc, np.float64).ravel()
    d = xc[None, :] - mean[:, p:]
    icc = np.linalg.inv(V[:, p:, p:])
    vpc = V[:, :p, p:]
    mu = mean[:, :p] + np.einsum("kij,kjl,kl->ki", vpc, icc, d)
    cov = V[:, :p, :p] - vpc @ icc @ np.transpose(vpc, (0, 2, 1))
    mc = np.einsum("ki,kij,kj->k", d, icc, d)
    r, c = np.tril_indices(p)
    fac = np.linalg.cholesky(cov)[:, r, c]
    return mu, fac, weight * np.exp(-0.5 * mc), colour.copy()
