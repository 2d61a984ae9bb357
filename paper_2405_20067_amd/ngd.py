"""Python binding of libngd (include/ngd.h): argument marshalling only.

Every function here converts torch tensors to device pointers and the
current HIP stream, calls the C-ABI function of the same name, and turns a
negative status into NgdError.  All arithmetic runs in the library's HIP
kernels; if libngd.so is missing this module raises instead of falling back.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "NgdError", "CullParams", "Mixture", "Cull", "lib", "LIB_PATH",
    "eval_mixture", "eval_prepare", "eval_backward", "eval_backward_composed", "eval_stats",
    "l2_loss", "l2_loss_noalloc",
    "rel_l2_loss", "FP32", "BF16_MFMA",
    "E_INVAL", "E_SINGULAR", "E_HIP", "E_NOMEM", "E_STALE",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libngd.so")
FP32 = 0
BF16_MFMA = 1
E_INVAL, E_SINGULAR, E_HIP, E_NOMEM, E_STALE = -1, -2, -3, -4, -5

_lib = None


class NgdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class CullParams(ctypes.Structure):
    _fields_ = [("n_proj", ctypes.c_int), ("tau", ctypes.c_float), ("tile", ctypes.c_int),
                ("key_proj", ctypes.c_int), ("key_bits", ctypes.c_int), ("tiling", ctypes.c_int)]

    def __repr__(self):
        return (f"CullParams(n_proj={self.n_proj}, tau={self.tau:g}, tile={self.tile}, "
                f"key_proj={self.key_proj}, key_bits={self.key_bits}, tiling={self.tiling})")


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

# (name, restype, argtypes) of every exported function
_SIGS = [
    ("ngd_last_error", ctypes.c_char_p, []),
    ("ngd_version", ctypes.c_int, []),
    ("ngd_cull_params_default", ctypes.c_int, [ctypes.POINTER(CullParams)]),
    ("ngd_set_allocator", ctypes.c_int, [ALLOC_FN, FREE_FN, ctypes.c_void_p]),
    ("ngd_mixture_create", ctypes.c_int,
     [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]),
    ("ngd_mixture_update", ctypes.c_int,
     [ctypes.c_void_p] * 5 + [ctypes.c_void_p]),
    ("ngd_mixture_validate", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("ngd_mixture_update_composed", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int64] + [ctypes.c_void_p] * 8),
    ("ngd_mixture_info", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
      ctypes.POINTER(ctypes.c_int64)]),
    ("ngd_mixture_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("ngd_cull_build", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(CullParams),
      ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("ngd_cull_stats", ctypes.c_int,
     [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 3),
    ("ngd_cull_export", ctypes.c_int, [ctypes.c_void_p] * 9),
    ("ngd_cull_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("ngd_eval", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_void_p]),
    ("ngd_eval_prepare", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
      ctypes.c_void_p]),
    ("ngd_eval_stats", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
      ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    ("ngd_eval_backward", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
      ctypes.c_int] + [ctypes.c_void_p] * 5),
    ("ngd_mixture_condition", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_float)] + [ctypes.c_void_p] * 5),
    ("ngd_eval_backward_composed", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
      ctypes.c_int] + [ctypes.c_void_p] * 7),
    ("ngd_l2_loss", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p]),
    ("ngd_l2_loss_noalloc", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p]),
    ("ngd_rel_l2_loss", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p,
      ctypes.c_void_p, ctypes.c_void_p]),
]
EXPORTED = [s[0] for s in _SIGS]


def lib():
    """The loaded libngd.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2405_20067_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise NgdError(rc, lib().ngd_last_error().decode())


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, numel=None, dtype=None):
    """Device pointer of a contiguous float32 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != (dtype or torch.float32):
        raise TypeError(f"{name} must be {dtype or torch.float32}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def default_params() -> CullParams:
    p = CullParams()
    _check(lib().ngd_cull_params_default(ctypes.byref(p)))
    return p


class Mixture:
    """A mixture handle (ngd_mixture): n dimensions, k Gaussians."""

    def __init__(self, n: int, k: int):
        h = ctypes.c_void_p()
        _check(lib().ngd_mixture_create(int(n), int(k), ctypes.byref(h)))
        self._h = h
        self.n, self.k = int(n), int(k)
        self.tri = self.n * (self.n + 1) // 2
        self.kp = -1   # parents of the last composed update (-1: plain update)

    @property
    def handle(self):
        return self._h

    def update(self, mean, factor, weight, colour, stream=None):
        k, n, t = self.k, self.n, self.tri
        _check(lib().ngd_mixture_update(self._h, _ptr(mean, "mean", k * n),
                                        _ptr(factor, "factor", k * t),
                                        _ptr(weight, "weight", k),
                                        _ptr(colour, "colour", k * 3), _stream(stream)))
        self.kp = -1

    def update_composed(self, kp, mean, factor, weight, colour, parent, rel_factor, rel_mean,
                        stream=None):
        """Parents 0..kp-1 given absolutely, children kp.. given relative to
        their parents (include/ngd.h, ngd_mixture_update_composed)."""
        import torch
        k, n, t = self.k, self.n, self.tri
        kc = k - int(kp)
        _check(lib().ngd_mixture_update_composed(
            self._h, int(kp), _ptr(mean, "mean", kp * n), _ptr(factor, "factor", kp * t),
            _ptr(weight, "weight", k), _ptr(colour, "colour", k * 3),
            _ptr(parent, "parent", kc, torch.int32), _ptr(rel_factor, "rel_factor", kc * t),
            _ptr(rel_mean, "rel_mean", kc * n), _stream(stream)))
        self.kp = int(kp)

    def condition(self, p, xc, stream=None):
        """(mean (k, p), factor (k, p(p+1)/2), weight (k,), colour (k, 3)):
        every Gaussian conditioned on the values xc of dimensions p..n-1
        (include/ngd.h, ngd_mixture_condition); the arguments of
        Mixture(p, k).update."""
        import torch
        xc = np.ascontiguousarray(np.asarray(xc, dtype=np.float32).ravel())
        if xc.size != self.n - int(p):
            raise ValueError(f"xc needs {self.n - int(p)} values, got {xc.size}")
        p = int(p)
        dev = torch.device("cuda", torch.cuda.current_device())
        e = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
        out = (e(self.k, p), e(self.k, p * (p + 1) // 2), e(self.k), e(self.k, 3))
        _check(lib().ngd_mixture_condition(
            self._h, p, xc.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            *[ctypes.c_void_p(t.data_ptr()) for t in out], _stream(stream)))
        return out

    def validate(self, stream=None):
        _check(lib().ngd_mixture_validate(self._h, _stream(stream)))

    def info(self):
        n, k, v = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ngd_mixture_info(self._h, ctypes.byref(n), ctypes.byref(k),
                                      ctypes.byref(v)))
        return n.value, k.value, v.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ngd_mixture_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cull:
    """A cull handle (ngd_cull); build() may be called again to rebuild in
    place, reusing its device memory."""

    def __init__(self):
        self._h = ctypes.c_void_p()
        self.q = 0
        self.n_proj = 0

    @property
    def handle(self):
        return self._h

    def build(self, mix: Mixture, queries, proj, params: CullParams | None = None,
              stream=None):
        params = params or default_params()
        proj = np.ascontiguousarray(proj, dtype=np.float32)
        if proj.shape != (params.n_proj, mix.n):
            raise ValueError(f"proj must be ({params.n_proj}, {mix.n}), got {proj.shape}")
        q = queries.numel() // mix.n if queries is not None else 0
        _check(lib().ngd_cull_build(mix.handle, _ptr(queries, "queries", q * mix.n), q,
                                    ctypes.byref(params),
                                    proj.ctypes.data_as(ctypes.c_void_p), _stream(stream),
                                    ctypes.byref(self._h)))
        self.q, self.n_proj, self.k, self.params = q, params.n_proj, mix.k, params
        return self

    def stats(self):
        t, m, nt = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ngd_cull_stats(self._h, ctypes.byref(t), ctypes.byref(m),
                                    ctypes.byref(nt)))
        return dict(total=t.value, max_per_tile=m.value, ntiles=nt.value)

    def export(self):
        st = self.stats()
        T, total = st["ntiles"], st["total"]
        out = dict(perm=np.zeros(max(self.q, 1), np.int32),
                   gperm=np.zeros(max(self.k, 1), np.int32),
                   tile_off=np.zeros(T + 1, np.int64),
                   cand=np.zeros(max(total, 1), np.int32),
                   g_off=np.zeros(self.k + 1, np.int64),
                   g_tiles=np.zeros(max(total, 1), np.int32),
                   tile_lo=np.zeros((max(T, 1), self.n_proj), np.float32),
                   tile_hi=np.zeros((max(T, 1), self.n_proj), np.float32))
        v = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().ngd_cull_export(self._h, v(out["perm"]), v(out["gperm"]),
                                     v(out["tile_off"]), v(out["cand"]), v(out["g_off"]),
                                     v(out["g_tiles"]), v(out["tile_lo"]), v(out["tile_hi"])))
        out["perm"] = out["perm"][:self.q]
        out["gperm"] = out["gperm"][:self.k]
        out["cand"] = out["cand"][:total]
        out["g_tiles"] = out["g_tiles"][:total]
        out["tile_lo"] = out["tile_lo"][:T]
        out["tile_hi"] = out["tile_hi"][:T]
        out.update(st)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ngd_cull_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_mixture(mix: Mixture, cull: Cull | None, queries, out=None, precision=FP32,
                 stream=None):
    """f (q x 3) for the queries; `cull` None evaluates densely."""
    import torch
    q = queries.numel() // mix.n
    if out is None:
        out = torch.empty((q, 3), dtype=torch.float32, device=queries.device)
    _check(lib().ngd_eval(mix.handle, cull.handle if cull is not None else None,
                          _ptr(queries, "queries", q * mix.n), q, int(precision),
                          _ptr(out, "out", q * 3), _stream(stream)))
    return out


def eval_prepare(mix: Mixture, cull: Cull, queries, precision=FP32, stream=None):
    """Builds what a forward of `precision` derives once per cull build
    (ngd_eval does it itself when it is missing)."""
    q = queries.numel() // mix.n
    _check(lib().ngd_eval_prepare(mix.handle, cull.handle, _ptr(queries, "queries", q * mix.n),
                                  q, int(precision), _stream(stream)))


def eval_stats(mix: Mixture, cull: Cull, queries, precision=FP32, stream=None):
    """Work counters of the culled forward of `precision`: dict(examined,
    filtered, pass1, pass2, kept), counted in (64-query group, candidate)
    pairs; `filtered` are those the first filter did not skip (the
    matrix-core one with BF16_MFMA, the per-coordinate box test with FP32)."""
    q = queries.numel() // mix.n
    counts = (ctypes.c_int64 * 5)()
    _check(lib().ngd_eval_stats(mix.handle, cull.handle, _ptr(queries, "queries", q * mix.n),
                                q, int(precision), counts, _stream(stream)))
    return dict(examined=counts[0], filtered=counts[1], pass1=counts[2], pass2=counts[3],
                kept=counts[4])


def eval_backward(mix: Mixture, cull: Cull | None, queries, grad_out, grads=None,
                  precision=FP32, stream=None):
    """(g_mean, g_factor, g_weight, g_colour) for upstream gradient grad_out."""
    import torch
    q = queries.numel() // mix.n
    dev = queries.device
    if grads is None:
        grads = (torch.empty((mix.k, mix.n), dtype=torch.float32, device=dev),
                 torch.empty((mix.k, mix.tri), dtype=torch.float32, device=dev),
                 torch.empty((mix.k,), dtype=torch.float32, device=dev),
                 torch.empty((mix.k, 3), dtype=torch.float32, device=dev))
    gm, gf, gw, gc = grads
    _check(lib().ngd_eval_backward(mix.handle, cull.handle if cull is not None else None,
                                   _ptr(queries, "queries", q * mix.n), q,
                                   _ptr(grad_out, "grad_out", q * 3), int(precision),
                                   _ptr(gm, "g_mean", mix.k * mix.n),
                                   _ptr(gf, "g_factor", mix.k * mix.tri),
                                   _ptr(gw, "g_weight", mix.k),
                                   _ptr(gc, "g_colour", mix.k * 3), _stream(stream)))
    return grads


def eval_backward_composed(mix: Mixture, cull: Cull | None, queries, grad_out, precision=FP32,
                           stream=None):
    """(g_mean (kp, n), g_factor (kp, tri), g_weight (k,), g_colour (k, 3),
    g_rel_factor (kc, tri), g_rel_mean (kc, n)) of a composed mixture."""
    import torch
    q = queries.numel() // mix.n
    dev = queries.device
    # after a plain update (kp < 0) the library refuses the call itself
    kp = max(mix.kp, 0)
    kc = mix.k - kp if mix.kp >= 0 else 0
    e = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
    out = (e(kp, mix.n), e(kp, mix.tri), e(mix.k), e(mix.k, 3), e(kc, mix.tri), e(kc, mix.n))
    _check(lib().ngd_eval_backward_composed(
        mix.handle, cull.handle if cull is not None else None,
        _ptr(queries, "queries", q * mix.n), q, _ptr(grad_out, "grad_out", q * 3),
        int(precision), *[ctypes.c_void_p(t.data_ptr()) for t in out], _stream(stream)))
    return out


def rel_l2_loss(f, target, eps=0.01, loss=None, grad=None, stream=None):
    """(loss, grad): relative squared error over q x 3, weights 1/(|f| + eps)^2
    held constant (include/ngd.h, ngd_rel_l2_loss)."""
    import torch
    q = f.numel() // 3
    if loss is None:
        loss = torch.empty((1,), dtype=torch.float32, device=f.device)
    if grad is None:
        grad = torch.empty_like(f)
    _check(lib().ngd_rel_l2_loss(_ptr(f, "f", q * 3), _ptr(target, "target", q * 3), q,
                                 float(eps), _ptr(loss, "loss", 1),
                                 _ptr(grad, "grad", q * 3), _stream(stream)))
    return loss, grad


def l2_loss(f, target, loss=None, grad=None, stream=None):
    """(loss, grad): mean squared error over q x 3 and its gradient."""
    import torch
    q = f.numel() // 3
    if loss is None:
        loss = torch.empty((1,), dtype=torch.float32, device=f.device)
    if grad is None:
        grad = torch.empty_like(f)
    _check(lib().ngd_l2_loss(_ptr(f, "f", q * 3), _ptr(target, "target", q * 3), q,
                             _ptr(loss, "loss", 1), _ptr(grad, "grad", q * 3),
                             _stream(stream)))
    return loss, grad


def l2_loss_noalloc(f, target, loss, grad, stream=None):
    """ngd_l2_loss_noalloc: the mean squared error and its gradient into the
    caller's `loss` (1) and `grad` (q x 3), with no allocation anywhere."""
    q = f.numel() // 3
    _check(lib().ngd_l2_loss_noalloc(_ptr(f, "f", q * 3), _ptr(target, "target", q * 3), q,
                                     _ptr(loss, "loss", 1), _ptr(grad, "grad", q * 3),
                                     _stream(stream)))
    return loss, grad
