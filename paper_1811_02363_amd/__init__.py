"""MI355X (gfx950) fast high-dimensional bilateral and nonlocal-means filtering.

Python binding of ``libfhd.so`` (C ABI in ``include/fhd.h``).  This module only
marshals arguments: every step of the filter runs in the library's HIP
kernels and host code.  PyTorch supplies device memory and the current HIP
stream.  Importing works without a GPU; calling a filter needs the built
library and a GPU and fails loudly otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import torch

__all__ = [
    "FHDError", "Params", "Info", "load", "lib_path", "symbols",
    "filter", "filter_centers", "filter_centers_noalloc", "filter_backward", "saved_buffer", "FilterFunction", "filter_autograd",
    "pack_batch", "filter_batch", "filter_batch_backward",
    "cluster", "pinv", "bruteforce", "nlm_guide", "scale_guide", "ScaleGuide", "approx_error",
    "filter_volume", "bruteforce_volume", "timing_enable", "timing_read", "timing_units",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libfhd.so")

FHD_OK, FHD_EINVAL, FHD_ENOMEM, FHD_EHIP, FHD_ENUMERIC, FHD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
_STATUS = {0: "FHD_OK", -1: "FHD_EINVAL", -2: "FHD_ENOMEM", -3: "FHD_EHIP",
           -4: "FHD_ENUMERIC", -5: "FHD_EUNSUPPORTED"}
SPATIAL = {"gaussian": 0, "box": 1, "young": 2}
CONTRACT = {"fp32": 0, "bf16": 1, "fp16": 2}
COEF = {"lsq": 0, "hard": 1, "exact": 2}

# Every entry point declared in include/fhd.h.
symbols = [
    "fhd_default_params", "fhd_create", "fhd_destroy", "fhd_set_stream", "fhd_last_error",
    "fhd_workspace_size", "fhd_saved_size", "fhd_saved_size_batch", "fhd_set_workspace", "fhd_cluster", "fhd_pinv",
    "fhd_filter_centers", "fhd_filter_centers_noalloc", "fhd_filter", "fhd_filter_backward", "fhd_filter_batch",
    "fhd_filter_batch_backward", "fhd_bruteforce", "fhd_nlm_guide", "fhd_scale_guide",
    "fhd_approx_error", "fhd_exact_ls", "fhd_last_k_eff", "fhd_filter_volume", "fhd_bruteforce_volume",
    "fhd_timing_enable", "fhd_timing_read", "fhd_timing_units",
]
STAGES = ("cluster", "weights", "row", "col", "brute", "lloyd")


class FHDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("sigma_s", ctypes.c_float), ("radius", ctypes.c_int), ("sigma_r", ctypes.c_float),
        ("K", ctypes.c_int), ("spatial", ctypes.c_int), ("contract", ctypes.c_int),
        ("coef", ctypes.c_int), ("kmeans_max_iter", ctypes.c_int), ("pinv_rtol", ctypes.c_double),
        ("strict", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("K_eff", ctypes.c_int), ("pinv_rank", ctypes.c_int), ("kmeans_rounds", ctypes.c_int),
        ("kmeans_splits", ctypes.c_int), ("E_K", ctypes.c_double), ("cond_A", ctypes.c_double),
        ("pinv_norm", ctypes.c_double), ("ms_cluster", ctypes.c_float),
        ("ms_solve", ctypes.c_float), ("ms_filter", ctypes.c_float),
        ("den_min", ctypes.c_float), ("den_nonpos", ctypes.c_longlong),
        ("den_small", ctypes.c_longlong), ("nonfinite", ctypes.c_longlong),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_lock = threading.Lock()
_ctxs = {}


def load():
    """Load ``libfhd.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(lib_path):
            raise FHDError(FHD_EUNSUPPORTED,
                           f"{lib_path} is missing: build it with `python -m paper_1811_02363_amd.build`")
        lib = ctypes.CDLL(lib_path)
        P, V, I, F, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
        pp = P(Params)
        pi = P(Info)
        sig = {
            "fhd_default_params": (None, [pp]),
            "fhd_create": (I, [P(V), I, V]),
            "fhd_destroy": (I, [V]),
            "fhd_set_stream": (I, [V, V]),
            "fhd_last_error": (ctypes.c_char_p, [V]),
            "fhd_workspace_size": (I, [pp, I, I, I, I, P(ctypes.c_size_t)]),
            "fhd_set_workspace": (I, [V, V, ctypes.c_size_t]),
            "fhd_saved_size": (I, [pp, I, I, I, I, P(ctypes.c_size_t)]),
            "fhd_saved_size_batch": (I, [pp, I, V, V, I, I, P(ctypes.c_size_t)]),
            "fhd_cluster": (I, [V, V, I, I, I, I, I, V, V, P(I), pi]),
            "fhd_pinv": (I, [V, I, I, D, D, V, V, P(I), P(D)]),
            "fhd_filter_centers": (I, [V, V, I, V, I, I, I, V, I, V, pp, V, V, pi, V, ctypes.c_size_t]),
            "fhd_filter_centers_noalloc": (I, [V, V, I, V, I, I, I, V, I, V, pp, V, V]),
            "fhd_filter": (I, [V, V, I, V, I, I, I, pp, V, V, V, pi, V, ctypes.c_size_t]),
            "fhd_filter_backward": (I, [V, V, I, V, I, I, I, V, I, pp, V, V, V, V, V, P(D), P(D), V, V,
                                        ctypes.c_size_t]),
            "fhd_filter_batch": (I, [V, I, V, V, V, V, I, V, I, pp, V, V, V, V, pi, V, ctypes.c_size_t]),
            "fhd_filter_batch_backward": (I, [V, I, V, V, V, V, I, V, I, V, V, pp, V, V, V, V, V,
                                              P(D), P(D), V, ctypes.c_size_t]),
            "fhd_bruteforce": (I, [V, V, I, V, I, I, I, pp, V, V]),
            "fhd_nlm_guide": (I, [V, V, I, I, I, I, I, V, V]),
            "fhd_scale_guide": (I, [V, V, I, ctypes.c_longlong, V, V]),
            "fhd_approx_error": (I, [V, V, I, I, I, V, I, pp, V, P(D)]),
            "fhd_exact_ls": (I, [V, V, I, I, I, V, I, pp, V, V, V]),
            "fhd_last_k_eff": (I, [V]),
            "fhd_filter_volume": (I, [V, V, I, V, I, I, I, I, pp, V, V, V, pi]),
            "fhd_bruteforce_volume": (I, [V, V, I, V, I, I, I, I, pp, V, V]),
            "fhd_timing_enable": (I, [V, I]),
            "fhd_timing_read": (I, [V, P(D), P(I)]),
            "fhd_timing_units": (I, [V, P(ctypes.c_longlong)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ctx(device: int):
    lib = load()
    c = _ctxs.get(device)
    if c is None:
        h = ctypes.c_void_p()
        _check(lib.fhd_create(ctypes.byref(h), device, None), None)
        c = h
        _ctxs[device] = c
    stream = torch.cuda.current_stream(device).cuda_stream
    _check(lib.fhd_set_stream(c, ctypes.c_void_p(stream)), c)
    return c


def _check(status, ctx):
    if status != FHD_OK:
        msg = load().fhd_last_error(ctx).decode() if ctx is not None else ""
        raise FHDError(status, msg)


def _dev(t, name, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise FHDError(FHD_EINVAL, f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise FHDError(FHD_EINVAL, f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise FHDError(FHD_EINVAL, f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def make_params(sigma_s=3.0, sigma_r=0.1, K=16, spatial="gaussian", radius=None,
                contract="fp32", coef="lsq", kmeans_max_iter=20, pinv_rtol=0.0, strict=False):
    p = Params()
    load().fhd_default_params(ctypes.byref(p))
    p.sigma_s = float(sigma_s if sigma_s is not None else 1.0)
    p.radius = -1 if radius is None else int(radius)
    p.sigma_r = float(sigma_r)
    p.K = int(K)
    p.spatial = SPATIAL[spatial]
    p.contract = CONTRACT[contract]
    p.coef = COEF[coef]
    p.kmeans_max_iter = int(kmeans_max_iter)
    p.pinv_rtol = float(pinv_rtol)
    p.strict = 1 if strict else 0
    return p


def _shape(f, guide):
    if not isinstance(f, torch.Tensor) or not f.is_cuda:
        raise FHDError(FHD_EINVAL, "images must be CUDA (HIP) tensors; there is no CPU path")
    if f.dim() != 3:
        raise FHDError(FHD_EINVAL, "images are (C, H, W)")
    g = f if guide is None else guide
    if g.dim() != 3 or g.shape[1:] != f.shape[1:]:
        raise FHDError(FHD_EINVAL, "guide must be (rho, H, W) with the image's H, W")
    return f.shape[0], g.shape[0], f.shape[1], f.shape[2], g


def _scalar(x):
    if isinstance(x, torch.Tensor):
        return x.dim() == 0
    try:
        len(x)
    except TypeError:
        return True
    return False


def _range(g, sigma_r):
    """A scalar sigma_r passes through; one value per guide dimension (the
    anisotropic kernel) becomes the guide scaled by fhd_scale_guide and
    sigma_r = 1."""
    if _scalar(sigma_r):
        return g, sigma_r
    return scale_guide(g, sigma_r), 1.0


def _saved_arg(saved):
    """(pointer, bytes) of a saved buffer: a uint8 device tensor, 256-byte aligned."""
    if saved is None:
        return None, 0
    if not isinstance(saved, torch.Tensor) or not saved.is_cuda or saved.dtype != torch.uint8:
        raise FHDError(FHD_EINVAL, "saved must be a uint8 CUDA (HIP) tensor (see saved_buffer)")
    if saved.data_ptr() % 256 != 0 or not saved.is_contiguous():
        raise FHDError(FHD_EINVAL, "saved must be contiguous and 256-byte aligned")
    return ctypes.c_void_p(saved.data_ptr()), saved.numel()


def saved_buffer(n, rho, H, W, K, device=0, sigma_s=3.0, sigma_r=0.1, spatial="gaussian", radius=None):
    """A device buffer (uint8 tensor) for a forward call to keep its
    intermediates for the adjoint (``fhd_saved_size``); ``H``, ``W`` lists for
    a batch (``fhd_saved_size_batch``)."""
    p = make_params(sigma_s, sigma_r, K, spatial, radius)
    b = ctypes.c_size_t()
    if isinstance(H, (list, tuple)):
        B = len(H)
        Ha, Wa = (ctypes.c_int * B)(*H), (ctypes.c_int * B)(*W)
        _check(load().fhd_saved_size_batch(ctypes.byref(p), B, Ha, Wa, n, rho, ctypes.byref(b)), None)
    else:
        _check(load().fhd_saved_size(ctypes.byref(p), n, rho, H, W, ctypes.byref(b)), None)
    return torch.empty(b.value, dtype=torch.uint8, device=torch.device("cuda", device))


def filter(f, guide=None, sigma_s=3.0, sigma_r=0.1, K=16, spatial="gaussian", radius=None,
           contract="fp32", coef="lsq", kmeans_max_iter=20, return_den=False,
           return_centers=False, info=False, strict=False, saved=None):
    """Algorithm 1 end to end: returns g_hat (n, H, W) [, den (H, W)]
    [, centers (K_eff, rho) on the host] [, info dict].  ``sigma_r`` is a
    number, or one value per guide dimension (anisotropic kernel; centers are
    then in the units of the scaled guide, see :func:`scale_guide`).  ``saved``
    (from :func:`saved_buffer`) keeps the intermediates for
    :func:`filter_backward`."""
    n, rho, H, W, g = _shape(f, guide)
    g, sigma_r = _range(g, sigma_r)
    ctx = _ctx(f.device.index)
    p = make_params(sigma_s, sigma_r, K, spatial, radius, contract, coef, kmeans_max_iter,
                    strict=strict)
    sp, sb = _saved_arg(saved)
    out = torch.empty_like(f)
    den = torch.empty((H, W), device=f.device, dtype=torch.float32) if return_den else None
    cen = torch.zeros((K, rho), dtype=torch.float32)
    inf = Info()
    lib = load()
    _check(lib.fhd_filter(ctx, _dev(f, "f"), n, _dev(g, "guide"), rho, H, W, ctypes.byref(p),
                          _dev(out, "out"), ctypes.c_void_p(cen.data_ptr()),
                          _dev(den, "den") if den is not None else None,
                          ctypes.byref(inf) if info else None, sp, sb), ctx)
    res = [out]
    if return_den:
        res.append(den)
    if return_centers:
        res.append(cen[:lib.fhd_last_k_eff(ctx)].clone())
    if info:
        res.append(inf.as_dict())
    return res[0] if len(res) == 1 else tuple(res)


def filter_volume(f, guide=None, sigma_s=3.0, sigma_r=0.1, K=16, spatial="gaussian", radius=None,
                  kmeans_max_iter=20, coef="lsq", return_den=False, return_centers=False, info=False,
                  strict=False):
    """Algorithm 1 on a volume: f (n, D, H, W), guide (rho, D, H, W) or None
    (the volume itself), window [-S,S]^3.  Returns g_hat [, den (D, H, W)]
    [, centers (K_eff, rho) on the host] [, info dict]."""
    if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dim() != 4:
        raise FHDError(FHD_EINVAL, "f must be an (n, D, H, W) CUDA (HIP) tensor; there is no CPU path")
    g = f if guide is None else guide
    if not isinstance(g, torch.Tensor) or g.dim() != 4 or g.shape[1:] != f.shape[1:]:
        raise FHDError(FHD_EINVAL, "guide must be (rho, D, H, W) with the volume's D, H, W")
    n, D, H, W = f.shape
    rho = g.shape[0]
    ctx = _ctx(f.device.index)
    p = make_params(sigma_s, sigma_r, K, spatial, radius, "fp32", coef, kmeans_max_iter, strict=strict)
    out = torch.empty_like(f)
    den = torch.empty((D, H, W), device=f.device, dtype=torch.float32) if return_den else None
    cen = torch.zeros((K, rho), dtype=torch.float32)
    inf = Info()
    _check(load().fhd_filter_volume(ctx, _dev(f, "f"), n, _dev(g, "guide"), rho, D, H, W, ctypes.byref(p),
                                    _dev(out, "out"), ctypes.c_void_p(cen.data_ptr()),
                                    _dev(den, "den") if den is not None else None,
                                    ctypes.byref(inf) if (info or return_centers) else None), ctx)
    res = [out]
    if return_den:
        res.append(den)
    if return_centers:
        res.append(cen[:inf.K_eff].clone())
    if info:
        res.append(inf.as_dict())
    return res[0] if len(res) == 1 else tuple(res)


def bruteforce_volume(f, guide=None, sigma_s=3.0, sigma_r=0.1, spatial="gaussian", radius=None,
                      return_den=False):
    """Eqs. (1)-(2) over [-S,S]^3 directly on the GPU (FP32); f (n, D, H, W)."""
    if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dim() != 4:
        raise FHDError(FHD_EINVAL, "f must be an (n, D, H, W) CUDA (HIP) tensor; there is no CPU path")
    g = f if guide is None else guide
    if not isinstance(g, torch.Tensor) or g.dim() != 4 or g.shape[1:] != f.shape[1:]:
        raise FHDError(FHD_EINVAL, "guide must be (rho, D, H, W) with the volume's D, H, W")
    n, D, H, W = f.shape
    ctx = _ctx(f.device.index)
    p = make_params(sigma_s, sigma_r, 1, spatial, radius)
    out = torch.empty_like(f)
    den = torch.empty((D, H, W), device=f.device, dtype=torch.float32) if return_den else None
    _check(load().fhd_bruteforce_volume(ctx, _dev(f, "f"), n, _dev(g, "guide"), g.shape[0], D, H, W,
                                        ctypes.byref(p), _dev(out, "out"),
                                        _dev(den, "den") if den is not None else None), ctx)
    return (out, den) if return_den else out


def filter_centers(f, guide, centers, sigma_s=3.0, sigma_r=0.1, spatial="gaussian", radius=None,
                   contract="fp32", coef="lsq", labels=None, return_den=False, info=False,
                   strict=False, saved=None):
    """Steps 2-5 with given centers (host or device (K, rho) float32); a
    per-dimension ``sigma_r`` as in :func:`filter` (centers in scaled units)."""
    n, rho, H, W, g = _shape(f, guide)
    g, sigma_r = _range(g, sigma_r)
    ctx = _ctx(f.device.index)
    c = torch.as_tensor(centers, dtype=torch.float32).detach().cpu().contiguous()
    K = c.shape[0]
    if c.dim() != 2 or c.shape[1] != rho:
        raise FHDError(FHD_EINVAL, "centers must be (K, rho)")
    p = make_params(sigma_s, sigma_r, K, spatial, radius, contract, coef, strict=strict)
    out = torch.empty_like(f)
    den = torch.empty((H, W), device=f.device, dtype=torch.float32) if return_den else None
    inf = Info()
    lab = _dev(labels, "labels", torch.int32) if labels is not None else None
    sp, sb = _saved_arg(saved)
    _check(load().fhd_filter_centers(ctx, _dev(f, "f"), n, _dev(g, "guide"), rho, H, W,
                                     ctypes.c_void_p(c.data_ptr()), K, lab, ctypes.byref(p),
                                     _dev(out, "out"),
                                     _dev(den, "den") if den is not None else None,
                                     ctypes.byref(inf) if info else None, sp, sb), ctx)
    res = [out]
    if return_den:
        res.append(den)
    if info:
        res.append(inf.as_dict())
    return res[0] if len(res) == 1 else tuple(res)


def filter_centers_noalloc(f, guide, centers, sigma_s=3.0, sigma_r=0.1, spatial="gaussian", radius=None,
                           contract="fp32", coef="lsq", labels=None, out=None, den=None, strict=False):
    """:func:`filter_centers` through ``fhd_filter_centers_noalloc``: the
    library allocates nothing (its scratch is a static device array of
    FHD_NOALLOC_SCRATCH_BYTES).  ``out`` (n, H, W) and ``den`` (H, W) may be
    given (then nothing is allocated here either); returns (out, den or None)."""
    n, rho, H, W, g = _shape(f, guide)
    if not _scalar(sigma_r):
        raise FHDError(FHD_EINVAL, "the allocation-free call takes a scalar sigma_r")
    ctx = _ctx(f.device.index)
    c = torch.as_tensor(centers, dtype=torch.float32).detach().cpu().contiguous()
    K = c.shape[0]
    if c.dim() != 2 or c.shape[1] != rho:
        raise FHDError(FHD_EINVAL, "centers must be (K, rho)")
    p = make_params(sigma_s, sigma_r, K, spatial, radius, contract, coef, strict=strict)
    out = torch.empty_like(f) if out is None else out
    lab = _dev(labels, "labels", torch.int32) if labels is not None else None
    _check(load().fhd_filter_centers_noalloc(ctx, _dev(f, "f"), n, _dev(g, "guide"), rho, H, W,
                                             ctypes.c_void_p(c.data_ptr()), K, lab, ctypes.byref(p),
                                             _dev(out, "out"), _dev(den, "den") if den is not None else None),
           ctx)
    return out, den


def filter_backward(f, guide, centers, out, den, grad_out, sigma_s=3.0, sigma_r=0.1,
                    spatial="gaussian", radius=None, need_f=True, need_guide=True, need_sigma_r=True,
                    need_sigma_s=False, need_centers=False, saved=None):
    """Adjoint of :func:`filter_centers` (least-squares coefficients): given
    G = dL/dg_hat and the forward call's (g_hat, r_hat), returns
    (dL/df or None, dL/dguide or None, dL/dsigma_r as float or None),
    followed by dL/dsigma_s (float) when ``need_sigma_s`` (Gaussian window)
    and dL/dcenters ((K, rho) float64 host tensor, clustering held fixed)
    when ``need_centers``."""
    n, rho, H, W, g = _shape(f, guide)
    ctx = _ctx(f.device.index)
    c = torch.as_tensor(centers, dtype=torch.float32).detach().cpu().contiguous()
    K = c.shape[0]
    if c.dim() != 2 or c.shape[1] != rho:
        raise FHDError(FHD_EINVAL, "centers must be (K, rho)")
    p = make_params(sigma_s, sigma_r, K, spatial, radius)
    gf = torch.empty_like(f) if need_f else None
    gg = torch.empty_like(g) if need_guide else None
    gs = ctypes.c_double(0.0)
    gss = ctypes.c_double(0.0)
    gmu = torch.zeros((K, rho), dtype=torch.float64) if need_centers else None
    _check(load().fhd_filter_backward(
        ctx, _dev(f, "f"), n, _dev(g, "guide"), rho, H, W, ctypes.c_void_p(c.data_ptr()), K,
        ctypes.byref(p), _dev(out, "out"), _dev(den, "den"), _dev(grad_out, "grad_out"),
        _dev(gf, "grad_f") if gf is not None else None,
        _dev(gg, "grad_guide") if gg is not None else None,
        ctypes.byref(gs) if need_sigma_r else None,
        ctypes.byref(gss) if need_sigma_s else None,
        ctypes.c_void_p(gmu.data_ptr()) if need_centers else None, *_saved_arg(saved)), ctx)
    res = (gf, gg, (gs.value if need_sigma_r else None))
    if need_sigma_s:
        res += (gss.value,)
    if need_centers:
        res += (gmu,)
    return res


class FilterFunction(torch.autograd.Function):
    """g_hat = filter_centers(f, guide, centers) with gradients with respect to
    f, guide, sigma_r and sigma_s (0-d tensors; sigma_s with the Gaussian
    window) and the centers (a (K, rho) tensor) from the library's adjoint.  Pass the same tensor as f and guide for joint
    filtering of an image by itself: autograd adds the two contributions."""

    @staticmethod
    def forward(ctx, f, guide, sigma_r, centers, sigma_s, spatial, radius, contract, keep=True):
        sr, ss = float(sigma_r), float(sigma_s)
        saved = None
        if keep and contract == "fp32":
            # the forward's intermediates for the adjoint, where the adjoint can use them
            try:
                saved = saved_buffer(f.shape[0], guide.shape[0], f.shape[1], f.shape[2], len(centers),
                                     f.device.index, sigma_s=ss, sigma_r=sr, spatial=spatial, radius=radius)
            except FHDError as e:
                if e.status != FHD_EUNSUPPORTED:
                    raise
        out, den = filter_centers(f.detach(), guide.detach(), centers, sigma_s=ss, sigma_r=sr,
                                  spatial=spatial, radius=radius, contract=contract, return_den=True,
                                  saved=saved)
        ctx.saved_buf = saved
        ctx.save_for_backward(f, guide, out, den)
        ctx.conf = (centers, ss, sr, spatial, radius)
        ctx.sr_tensor = isinstance(sigma_r, torch.Tensor)
        ctx.ss_tensor = isinstance(sigma_s, torch.Tensor)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        f, guide, out, den = ctx.saved_tensors
        centers, sigma_s, sr, spatial, radius = ctx.conf
        need_f, need_g, need_s = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        need_ss = ctx.needs_input_grad[4] and ctx.ss_tensor
        need_mu = ctx.needs_input_grad[3]
        cen = centers.detach() if isinstance(centers, torch.Tensor) else centers
        res = filter_backward(f.detach(), guide.detach(), cen, out, den,
                              grad_out.contiguous(), sigma_s=sigma_s, sigma_r=sr,
                              spatial=spatial, radius=radius, need_f=need_f, need_guide=need_g,
                              need_sigma_r=need_s and ctx.sr_tensor, need_sigma_s=need_ss,
                              need_centers=need_mu, saved=ctx.saved_buf)
        gf, gg, gs = res[:3]
        gsr = torch.tensor(gs, dtype=torch.float32) if need_s and ctx.sr_tensor else None
        gss = torch.tensor(res[3], dtype=torch.float32) if need_ss else None
        gmu = None
        if need_mu:
            gmu = res[-1].to(dtype=centers.dtype, device=centers.device)
        return gf, gg, gsr, gmu, gss, None, None, None, None


def filter_autograd(f, guide=None, sigma_s=3.0, sigma_r=0.1, K=16, spatial="gaussian",
                    radius=None, contract="fp32", centers=None, kmeans_max_iter=20, keep=True):
    """Differentiable Algorithm 1: the centers come from the bisecting K-means
    of the (detached) guide unless given, then :class:`FilterFunction`.
    ``sigma_r`` and ``sigma_s`` may be 0-d tensors that require grad; a
    ``sigma_r`` of one value per guide dimension (constants) filters the guide
    scaled by :class:`ScaleGuide` with sigma_r = 1, gradients flowing back to
    the unscaled guide.  ``keep`` lets the forward call keep its intermediates
    for the adjoint (:func:`saved_buffer`), where the adjoint can use them."""
    g = f if guide is None else guide
    if not _scalar(sigma_r):
        g, sigma_r = ScaleGuide.apply(g, sigma_r), 1.0
    if centers is None:
        centers, _ = cluster(g.detach(), K, max_iter=kmeans_max_iter)
    return FilterFunction.apply(f, g, sigma_r, centers, sigma_s, spatial, radius, contract, keep)


def pack_batch(images):
    """Concatenate (C, H_b, W_b) device tensors into the flat ragged layout of
    fhd_filter_batch; returns (flat tensor, [(H_b, W_b)])."""
    if not images:
        raise FHDError(FHD_EINVAL, "empty batch")
    C = images[0].shape[0]
    for t in images:
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dim() != 3 or t.shape[0] != C:
            raise FHDError(FHD_EINVAL, "batch images must be (C, H, W) CUDA tensors with one C")
    flat = torch.cat([t.reshape(-1) for t in images])
    return flat, [(int(t.shape[1]), int(t.shape[2])) for t in images]


def _batch_arrays(sizes):
    B = len(sizes)
    Ha = (ctypes.c_int * B)(*[h for h, _ in sizes])
    Wa = (ctypes.c_int * B)(*[w for _, w in sizes])
    offs, o = [], 0
    for h, w in sizes:
        offs.append(o)
        o += h * w
    Oa = (ctypes.c_longlong * B)(*offs)
    return B, Ha, Wa, Oa, o


def filter_batch(flat_f, sizes, n, flat_guide=None, rho=None, sigma_s=3.0, sigma_r=0.1, K=16,
                 spatial="gaussian", radius=None, contract="fp32", coef="lsq", kmeans_max_iter=20,
                 return_den=False, info=False, strict=False, saved=None):
    """Algorithm 1 on a ragged batch in the flat layout of :func:`pack_batch`.
    Returns (out flat, [den flat], centers (B, K, rho) host, K_eff list [, info list])."""
    B, Ha, Wa, Oa, N = _batch_arrays(sizes)
    g = flat_f if flat_guide is None else flat_guide
    rho = n if rho is None else rho
    if flat_f.numel() != n * N or g.numel() != rho * N:
        raise FHDError(FHD_EINVAL, "flat buffers do not match the sizes")
    ctx = _ctx(flat_f.device.index)
    p = make_params(sigma_s, sigma_r, K, spatial, radius, contract, coef, kmeans_max_iter, strict=strict)
    out = torch.empty_like(flat_f)
    den = torch.empty(N, device=flat_f.device, dtype=torch.float32) if return_den else None
    cen = torch.zeros((B, K, rho), dtype=torch.float32)
    keff = (ctypes.c_int * B)()
    infos = (Info * B)()
    _check(load().fhd_filter_batch(ctx, B, Ha, Wa, Oa, _dev(flat_f, "f"), n, _dev(g, "guide"), rho,
                                   ctypes.byref(p), _dev(out, "out"), ctypes.c_void_p(cen.data_ptr()),
                                   keff, _dev(den, "den") if den is not None else None,
                                   infos if info else None, *_saved_arg(saved)), ctx)
    res = [out]
    if return_den:
        res.append(den)
    res += [cen, list(keff)]
    if info:
        res.append([i.as_dict() for i in infos])
    return tuple(res)


def filter_batch_backward(flat_f, sizes, n, centers, K_eff, out, den, grad_out, flat_guide=None,
                          rho=None, sigma_s=3.0, sigma_r=0.1, spatial="gaussian", radius=None,
                          need_f=True, need_guide=True, need_sigma_r=True, need_sigma_s=False, saved=None):
    """Adjoint of :func:`filter_batch`: (dL/df flat or None, dL/dguide flat or
    None, dL/dsigma_r summed over the images or None), and dL/dsigma_s summed
    over the images as a fourth entry when ``need_sigma_s``."""
    B, Ha, Wa, Oa, N = _batch_arrays(sizes)
    g = flat_f if flat_guide is None else flat_guide
    rho = n if rho is None else rho
    ctx = _ctx(flat_f.device.index)
    c = torch.as_tensor(centers, dtype=torch.float32).detach().cpu().contiguous()
    K = c.shape[1]
    p = make_params(sigma_s, sigma_r, K, spatial, radius)
    keff = (ctypes.c_int * B)(*K_eff)
    gf = torch.empty_like(flat_f) if need_f else None
    gg = torch.empty_like(g) if need_guide else None
    gs = ctypes.c_double(0.0)
    gss = ctypes.c_double(0.0)
    _check(load().fhd_filter_batch_backward(
        ctx, B, Ha, Wa, Oa, _dev(flat_f, "f"), n, _dev(g, "guide"), rho, ctypes.c_void_p(c.data_ptr()),
        keff, ctypes.byref(p), _dev(out, "out"), _dev(den, "den"), _dev(grad_out, "grad_out"),
        _dev(gf, "grad_f") if gf is not None else None,
        _dev(gg, "grad_guide") if gg is not None else None,
        ctypes.byref(gs) if need_sigma_r else None,
        ctypes.byref(gss) if need_sigma_s else None, *_saved_arg(saved)), ctx)
    res = (gf, gg, (gs.value if need_sigma_r else None))
    return res + (gss.value,) if need_sigma_s else res


def cluster(guide, K, max_iter=20, labels=False):
    """Bisecting K-means of the guide vectors: (centers (K_eff, rho) host float32
    [, labels (H, W) int32 device], info)."""
    rho, H, W = guide.shape
    ctx = _ctx(guide.device.index)
    cen = torch.zeros((K, rho), dtype=torch.float32)
    lab = torch.empty((H, W), device=guide.device, dtype=torch.int32) if labels else None
    keff = ctypes.c_int()
    inf = Info()
    _check(load().fhd_cluster(ctx, _dev(guide, "guide"), rho, H, W, int(K), int(max_iter),
                              ctypes.c_void_p(cen.data_ptr()),
                              _dev(lab, "labels", torch.int32) if lab is not None else None,
                              ctypes.byref(keff), ctypes.byref(inf)), ctx)
    cen = cen[:keff.value].clone()
    if labels:
        return cen, lab, inf.as_dict()
    return cen, inf.as_dict()


def pinv(centers, sigma_r, rtol=0.0):
    """The K x K solve on the host (FP64): (A, A^+, rank, cond) as float64 tensors."""
    c = torch.as_tensor(centers, dtype=torch.float32).contiguous()
    K, rho = c.shape
    A = torch.empty((K, K), dtype=torch.float64)
    P = torch.empty((K, K), dtype=torch.float64)
    rank = ctypes.c_int()
    cond = ctypes.c_double()
    st = load().fhd_pinv(ctypes.c_void_p(c.data_ptr()), K, rho, float(sigma_r), float(rtol),
                         ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(P.data_ptr()),
                         ctypes.byref(rank), ctypes.byref(cond))
    _check(st, None)
    return A, P, rank.value, cond.value


def bruteforce(f, guide=None, sigma_s=3.0, sigma_r=0.1, spatial="gaussian", radius=None,
               return_den=False):
    """Eqs. (1)-(2) directly on the GPU (FP32); a per-dimension ``sigma_r`` as
    in :func:`filter`."""
    n, rho, H, W, g = _shape(f, guide)
    g, sigma_r = _range(g, sigma_r)
    ctx = _ctx(f.device.index)
    p = make_params(sigma_s, sigma_r, 1, spatial, radius)
    out = torch.empty_like(f)
    den = torch.empty((H, W), device=f.device, dtype=torch.float32) if return_den else None
    _check(load().fhd_bruteforce(ctx, _dev(f, "f"), n, _dev(g, "guide"), rho, H, W,
                                 ctypes.byref(p), _dev(out, "out"),
                                 _dev(den, "den") if den is not None else None), ctx)
    return (out, den) if return_den else out


def nlm_guide(f, patch=5, dims=16, eigvals=False):
    """Patch-PCA guide of nonlocal means: (dims, H, W) float32 on the device
    [, covariance eigenvalues (float64, descending)]."""
    if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dim() != 3:
        raise FHDError(FHD_EINVAL, "f must be a (C, H, W) CUDA (HIP) tensor")
    n, H, W = f.shape
    ctx = _ctx(f.device.index)
    g = torch.empty((dims, H, W), device=f.device, dtype=torch.float32)
    D = patch * patch * n
    ev = torch.zeros(D, dtype=torch.float64)
    _check(load().fhd_nlm_guide(ctx, _dev(f, "f"), n, H, W, int(patch), int(dims), _dev(g, "guide"),
                                ctypes.c_void_p(ev.data_ptr()) if eigvals else None), ctx)
    return (g, ev) if eigvals else g


def scale_guide(guide, sigma_d, out=None):
    """guide[d] / sigma_d per dimension on the device (``fhd_scale_guide``):
    filtering the result with sigma_r = 1 filters ``guide`` with the
    anisotropic range kernel exp(-sum_d x_d^2 / 2 sigma_d^2).  ``guide`` is
    (rho, ...) float32 on the device; ``sigma_d`` holds rho positive values;
    ``out`` may be ``guide`` itself."""
    if not isinstance(guide, torch.Tensor) or not guide.is_cuda or guide.dim() < 1:
        raise FHDError(FHD_EINVAL, "guide must be a (rho, ...) CUDA (HIP) tensor")
    rho = guide.shape[0]
    s = torch.as_tensor(sigma_d, dtype=torch.float32).detach().cpu().contiguous().reshape(-1)
    if s.numel() != rho:
        raise FHDError(FHD_EINVAL, f"sigma_d needs {rho} values (one per guide dimension)")
    ctx = _ctx(guide.device.index)
    res = torch.empty_like(guide) if out is None else out
    if res.shape != guide.shape:
        raise FHDError(FHD_EINVAL, "out must have the guide's shape")
    N = guide.numel() // rho if rho else 0
    _check(load().fhd_scale_guide(ctx, _dev(guide, "guide"), rho, N, ctypes.c_void_p(s.data_ptr()),
                                  _dev(res, "out")), ctx)
    return res


def approx_error(guide, centers, sigma_r=0.1, sigma_s=3.0, radius=None, spatial="gaussian",
                 pinv_rtol=0.0, per_pixel=True):
    """Error of the kernel approximation (``fhd_approx_error``): eq. (10) at
    c(i) = A^+ b(i) per pixel and its pixel mean E_ls (the averaged
    least-squares error of Sec. II-A, not the clustering error E_K of
    eq. (20)).  ``guide`` (rho, H, W) on the device, ``centers`` (K, rho),
    K <= 64.  Returns (err (H, W) or None, E_ls)."""
    if not isinstance(guide, torch.Tensor) or not guide.is_cuda or guide.dim() != 3:
        raise FHDError(FHD_EINVAL, "guide must be a (rho, H, W) CUDA (HIP) tensor")
    rho, H, W = guide.shape
    c = torch.as_tensor(centers, dtype=torch.float32).detach().cpu().contiguous()
    if c.dim() != 2 or c.shape[1] != rho:
        raise FHDError(FHD_EINVAL, "centers must be (K, rho)")
    ctx = _ctx(guide.device.index)
    p = make_params(sigma_s, sigma_r, c.shape[0], spatial, radius, pinv_rtol=pinv_rtol)
    err = torch.empty((H, W), device=guide.device, dtype=torch.float32) if per_pixel else None
    m = ctypes.c_double()
    _check(load().fhd_approx_error(ctx, _dev(guide, "guide"), rho, H, W, ctypes.c_void_p(c.data_ptr()),
                                   c.shape[0], ctypes.byref(p), _dev(err, "err") if err is not None else None,
                                   ctypes.byref(m)), ctx)
    return err, m.value


def exact_ls(guide, centers, sigma_r=0.1, sigma_s=3.0, radius=None, spatial="gaussian", pinv_rtol=0.0,
             coef=True, obj=True, obj11=True):
    """Eq. (10) solved at every pixel (``fhd_exact_ls``): the minimum-norm
    least-squares coefficients over the window's own guide samples (Sec.
    II-A), the fit that eq. (11)'s c = A^+ b(i) stands in for.  ``guide``
    (rho, H, W) on the device, ``centers`` (K, rho), K <= 32.  Returns
    (coef (K, H, W), obj (H, W): the minimum of eq. (10), obj11 (H, W):
    eq. (10) at A^+ b(i)); outputs not asked for are None."""
    if not isinstance(guide, torch.Tensor) or not guide.is_cuda or guide.dim() != 3:
        raise FHDError(FHD_EINVAL, "guide must be a (rho, H, W) CUDA (HIP) tensor")
    rho, H, W = guide.shape
    c = torch.as_tensor(centers, dtype=torch.float32).detach().cpu().contiguous()
    if c.dim() != 2 or c.shape[1] != rho:
        raise FHDError(FHD_EINVAL, "centers must be (K, rho)")
    K = c.shape[0]
    ctx = _ctx(guide.device.index)
    p = make_params(sigma_s, sigma_r, K, spatial, radius, pinv_rtol=pinv_rtol)
    dev = dict(device=guide.device, dtype=torch.float32)
    cf = torch.empty((K, H, W), **dev) if coef else None
    o10 = torch.empty((H, W), **dev) if obj else None
    o11 = torch.empty((H, W), **dev) if obj11 else None
    _check(load().fhd_exact_ls(ctx, _dev(guide, "guide"), rho, H, W, ctypes.c_void_p(c.data_ptr()), K,
                               ctypes.byref(p), _dev(cf, "coef") if cf is not None else None,
                               _dev(o10, "obj") if o10 is not None else None,
                               _dev(o11, "obj11") if o11 is not None else None), ctx)
    return cf, o10, o11


class ScaleGuide(torch.autograd.Function):
    """:func:`scale_guide` with its adjoint (the same diagonal map) for
    gradients with respect to the unscaled guide; ``sigma_d`` is a constant."""

    @staticmethod
    def forward(ctx, guide, sigma_d):
        ctx.sigma_d = torch.as_tensor(sigma_d, dtype=torch.float32).detach().cpu()
        return scale_guide(guide.detach().contiguous(), ctx.sigma_d)

    @staticmethod
    def backward(ctx, grad):
        return scale_guide(grad.contiguous(), ctx.sigma_d), None


def timing_enable(device=0, enable=True):
    """Record HIP events around each stage of later calls on `device`."""
    ctx = _ctx(device)
    _check(load().fhd_timing_enable(ctx, 1 if enable else 0), ctx)


def timing_read(device=0):
    """{stage: (total ms, launches)} since the last read (synchronises)."""
    ctx = _ctx(device)
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_int * len(STAGES))()
    _check(load().fhd_timing_read(ctx, ms, n), ctx)
    return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}


def timing_units(device=0):
    """{stage: algorithmic units} recorded since the last call (the points
    streamed by the clustering's assignment steps for "lloyd")."""
    ctx = _ctx(device)
    u = (ctypes.c_longlong * len(STAGES))()
    _check(load().fhd_timing_units(ctx, u), ctx)
    return {s: int(u[i]) for i, s in enumerate(STAGES)}
