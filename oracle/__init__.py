"""FP64 CPU oracle for fast high-dimensional bilateral / nonlocal-means filtering.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library ``paper_1811_02363_amd`` and never imports it.

Two independent references, both in FP64:

* **O-1** ``bruteforce``: the filter as defined by eqs. (1)-(2) (Sec. I-A).
* **O-2** ``fast_filter`` / ``fhd_filter``: the clustered approximation of
  Algorithm 1 (Sec. II-B) step by step: bisecting K-means of the range space
  eq. (8) (Sec. II-C), the kernel matrix and its pseudo-inverse eq. (12), the
  per-pixel weights b(i) and coefficients c(i) = A^+ b(i), the (n+1)K
  convolutions eqs. (13)-(14) and the recombination eqs. (15)-(16).

Also: the hard-assignment variant eqs. (17)-(18), the patch-PCA guide for
nonlocal means (Sec. III-C), the anisotropic range kernel (Sec. III, III-E) as a
direct brute force and as the scaled guide the method filters, the error of
the kernel approximation (eq. (10) at c = A^+ b, Sec. II-A), the per-pixel
minimisers of eq. (10) themselves (Sec. II-A's exact least squares), the brute force
and the fast filter on a 3-D domain (Sec. III-F), the PSNR of eq. (21).

The heavy loops (window sums) live in ``fhd_oracle.c`` (plain C + OpenMP),
compiled with gcc into ``liboracle.so`` beside this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fhd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

GAUSSIAN, BOX = 0, 1


def build(force: bool = True) -> str:
    """Compile ``fhd_oracle.c`` with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        lib.oracle_bruteforce.argtypes = [dp, c_int, dp, c_int, c_int, c_int,
                                          c_int, c_int, c_double, c_double, dp, dp]
        lib.oracle_bruteforce_at.argtypes = [dp, c_int, dp, c_int, c_int, c_int,
                                             c_int, c_int, c_double, c_double,
                                             ip, ip, c_int, dp, dp]
        lib.oracle_conv2d.argtypes = [dp, c_int, c_int, c_int, c_int, c_int,
                                      c_double, dp]
        lib.oracle_conv_separable.argtypes = [dp, c_int, c_int, c_int, c_int,
                                              c_int, c_double, dp]
        lib.oracle_cluster_images_at.argtypes = [dp, c_int, dp, c_int, c_int, c_int,
                                                 dp, c_int, c_int, c_int, c_double,
                                                 c_double, ip, ip, c_int, dp]
        for fn in ("oracle_bruteforce", "oracle_bruteforce_at", "oracle_conv2d",
                   "oracle_conv_separable", "oracle_cluster_images_at"):
            getattr(lib, fn).restype = None
        lib.oracle_set_threads.argtypes = [c_int]
        lib.oracle_set_threads.restype = None
        lib.oracle_get_threads.argtypes = []
        lib.oracle_get_threads.restype = c_int
        _lib = lib
    return _lib


def set_threads(t):
    """Threads of the C window sums (OpenMP); returns the previous count."""
    prev = _load().oracle_get_threads()
    _load().oracle_set_threads(int(t))
    return prev


def threads():
    return _load().oracle_get_threads()


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _spatial_code(spatial):
    if spatial in (0, "gaussian"):
        return GAUSSIAN
    if spatial in (1, "box"):
        return BOX
    raise ValueError(spatial)


def default_radius(sigma_s: float) -> int:
    """Window half-width S = 3 sigma_s (Sec. III), rounded up to an integer."""
    return int(np.ceil(3.0 * sigma_s - 1e-12))


# --------------------------------------------------------------------------
# Kernels (Sec. III)
# --------------------------------------------------------------------------

def phi(d2, sigma_r):
    """Gaussian range kernel exp(-|x|^2 / 2 sigma_r^2) of a squared distance;
    sigma_r = inf gives 1."""
    d2 = np.asarray(d2, dtype=np.float64)
    if np.isinf(sigma_r):
        return np.ones_like(d2)
    return np.exp(-d2 / (2.0 * sigma_r * sigma_r))


def spatial_kernel_2d(S, sigma_s, spatial="gaussian"):
    """omega(j) on [-S,S]^2: Gaussian exp(-|j|^2/2 sigma_s^2) or box (all 1)."""
    j = np.arange(-S, S + 1, dtype=np.float64)
    if _spatial_code(spatial) == BOX:
        return np.ones((2 * S + 1, 2 * S + 1))
    return np.exp(-(j[:, None] ** 2 + j[None, :] ** 2) / (2.0 * sigma_s ** 2))


# --------------------------------------------------------------------------
# O-1: brute force, eqs. (1)-(2)
# --------------------------------------------------------------------------

def bruteforce(f, guide, sigma_s, sigma_r, S=None, spatial="gaussian"):
    """Eqs. (1)-(2) over the whole image; returns (g, eta) as FP64 arrays."""
    f = _f64(f)
    guide = _f64(guide)
    n, H, W = f.shape
    rho = guide.shape[0]
    if S is None:
        S = default_radius(sigma_s)
    out = np.empty_like(f)
    den = np.empty((H, W))
    _load().oracle_bruteforce(_dp(f), n, _dp(guide), rho, H, W, int(S),
                              _spatial_code(spatial), float(sigma_s or 1.0),
                              float(sigma_r), _dp(out), _dp(den))
    return out, den


def bruteforce_at(f, guide, sigma_s, sigma_r, ys, xs, S=None, spatial="gaussian"):
    """Eqs. (1)-(2) at the listed pixels only; returns (g (M x n), eta (M))."""
    f = _f64(f)
    guide = _f64(guide)
    n, H, W = f.shape
    rho = guide.shape[0]
    if S is None:
        S = default_radius(sigma_s)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    M = len(ys)
    out = np.empty((M, n))
    den = np.empty(M)
    _load().oracle_bruteforce_at(_dp(f), n, _dp(guide), rho, H, W, int(S),
                                 _spatial_code(spatial), float(sigma_s or 1.0),
                                 float(sigma_r), _ip(ys), _ip(xs), M, _dp(out),
                                 _dp(den))
    return out, den


def anisotropic_scale(guide, sigma_d):
    """The guide as the method reads an anisotropic range kernel (Sec. III;
    the per-dimension sigma_r of Sec. III-E): phi(x) = exp(-sum_d x_d^2 /
    2 sigma_d^2) is the isotropic kernel with sigma_r = 1 of the guide divided
    by sigma_d per dimension, so the clustering and the whole of Algorithm 1
    run on that scaled guide.  Here the FP32 guide over the FP32 sigma_d,
    rounded once to FP32 (the FP64 quotient of two FP32 numbers rounds to the
    correctly rounded FP32 quotient)."""
    g = np.asarray(guide, dtype=np.float32).astype(np.float64)
    s = np.asarray(sigma_d, dtype=np.float32).astype(np.float64).reshape((-1,) + (1,) * (g.ndim - 1))
    assert s.shape[0] == g.shape[0] and np.all(s > 0) and np.all(np.isfinite(s))
    return (g / s).astype(np.float32)


def bruteforce_anisotropic(f, guide, sigma_s, sigma_d, S=None, spatial="gaussian"):
    """Eqs. (1)-(2) with the anisotropic range kernel exp(-sum_d x_d^2 /
    2 sigma_d^2) (Sec. III), written out in NumPy for small images: for every
    window offset j the neighbour image p(i - j), its per-dimension weighted
    squared distance to p(i), and both sums; out-of-image neighbours are left
    out of both.  Returns (g, eta) in FP64."""
    f = _f64(f)
    p = _f64(guide)
    n, H, W = f.shape
    s2 = np.asarray(sigma_d, dtype=np.float64).reshape(-1, 1, 1) ** 2
    if S is None:
        S = default_radius(sigma_s)
    om = spatial_kernel_2d(S, sigma_s, spatial)
    num = np.zeros((n, H, W))
    eta = np.zeros((H, W))
    for jy in range(-S, S + 1):
        for jx in range(-S, S + 1):
            # pixels i = (y, x) whose neighbour (y - jy, x - jx) is inside
            y0, y1 = max(0, jy), min(H, H + jy)
            x0, x1 = max(0, jx), min(W, W + jx)
            if y0 >= y1 or x0 >= x1:
                continue
            pi = p[:, y0:y1, x0:x1]
            pq = p[:, y0 - jy:y1 - jy, x0 - jx:x1 - jx]
            w = om[jy + S, jx + S] * np.exp(-(((pq - pi) ** 2) / (2.0 * s2)).sum(0))
            num[:, y0:y1, x0:x1] += w * f[:, y0 - jy:y1 - jy, x0 - jx:x1 - jx]
            eta[y0:y1, x0:x1] += w
    return num / eta, eta


def young_coefficients(sigma):
    """Coefficients of the recursive Gaussian of Young and van Vliet (1995),
    the O(1) convolution the paper uses for Gaussian windows (Sec. II-C):
    q from sigma (two published branches), then b0..b3 and the gain
    B = 1 - (b1 + b2 + b3) / b0.  Returns (B, b1/b0, b2/b0, b3/b0)."""
    s = float(sigma)
    if s >= 2.5:
        q = 0.98711 * s - 0.96330
    elif s >= 0.5:
        q = 3.97156 - 4.14554 * np.sqrt(1.0 - 0.26891 * s)
    else:
        raise ValueError("the recursive Gaussian needs sigma >= 0.5")
    b0 = 1.57825 + 2.44413 * q + 1.4281 * q ** 2 + 0.422205 * q ** 3
    b1 = 2.44413 * q + 2.85619 * q ** 2 + 1.26661 * q ** 3
    b2 = -(1.4281 * q ** 2 + 1.26661 * q ** 3)
    b3 = 0.422205 * q ** 3
    return 1.0 - (b1 + b2 + b3) / b0, b1 / b0, b2 / b0, b3 / b0


def young_1d(u, sigma, axis):
    """The recursive Gaussian along one axis of u (FP64): the causal pass
    w[t] = B u[t] + a1 w[t-1] + a2 w[t-2] + a3 w[t-3], then the anti-causal
    pass y[t] = B w[t] + a1 y[t+1] + a2 y[t+2] + a3 y[t+3], each from a zero
    state at its own end of the image (the paper does not say how the
    recursions start at the borders; zero states match its zero extension of
    the input, not of the causal output)."""
    B, a1, a2, a3 = young_coefficients(sigma)
    x = np.moveaxis(_f64(u), axis, 0)
    T = x.shape[0]
    w = np.zeros_like(x)
    p1 = p2 = p3 = np.zeros(x.shape[1:])
    for t in range(T):
        w[t] = B * x[t] + a1 * p1 + a2 * p2 + a3 * p3
        p1, p2, p3 = w[t], p1, p2
    y = np.zeros_like(x)
    p1 = p2 = p3 = np.zeros(x.shape[1:])
    for t in range(T - 1, -1, -1):
        y[t] = B * w[t] + a1 * p1 + a2 * p2 + a3 * p3
        p1, p2, p3 = y[t], p1, p2
    return np.moveaxis(y, 0, axis)


def young_conv(u, sigma):
    """The separable recursive Gaussian of a stack of planes (C,H,W): along
    the rows (x), then along the columns (y)."""
    return young_1d(young_1d(u, sigma, 2), sigma, 1)


def conv(u, S, sigma_s, spatial="gaussian", method="direct"):
    """omega * u for a stack of planes (C,H,W), zero-extended (eqs. (13)-(14))."""
    u = _f64(u)
    C, H, W = u.shape
    v = np.empty_like(u)
    fn = _load().oracle_conv2d if method == "direct" else _load().oracle_conv_separable
    fn(_dp(u), C, H, W, int(S), _spatial_code(spatial), float(sigma_s or 1.0), _dp(v))
    return v


# --------------------------------------------------------------------------
# Step 1: bisecting K-means of the range space (Alg. 1 step 1, Sec. II-C)
# --------------------------------------------------------------------------

@dataclass
class Node:
    heap: int              # root 1, children 2h (first seed) and 2h+1
    idx: np.ndarray        # pixel indices of the members, ascending
    mean: np.ndarray       # FP64 centroid
    sse: float             # sum of squared distances to the centroid
    splittable: bool       # two members differ (exact FP32 compare)
    children: tuple | None = None   # (Node, Node) once a 2-means split is computed
    lloyd_iters: int = 0


@dataclass
class Clustering:
    centers: np.ndarray            # K_eff x rho, FP64, leaves in heap-id order
    labels: np.ndarray             # N, index into centers
    leaf_heap: list                # heap ids of the leaves (ascending)
    leaf_sse: np.ndarray           # SSE of each leaf
    E_K: float                     # clustering error, eq. (20)
    split_order: list = field(default_factory=list)   # heap ids split, in order
    E_history: list = field(default_factory=list)     # E after each split


def _node(heap, idx, X, X32):
    Xc = X[idx]
    mean = Xc.mean(axis=0)
    sse = float(((Xc - mean) ** 2).sum())
    splittable = bool(np.any(X32[idx] != X32[idx[0]]))
    if not splittable:
        sse = 0.0
    return Node(heap, idx, mean, sse, splittable)


def _two_means(node, X, X32, max_iter):
    """2-means split of one cluster (Sec. II-C): start from a pair of far-apart
    members, then alternate assignment and centroid update.

    Seeds: a = the member farthest from the centroid, b = the member farthest
    from a (ties: lowest pixel index).  Assignment: x goes to the first child
    iff |x - c_a|^2 <= |x - c_b|^2 (FP64).  At most max_iter assignment steps;
    stop when no label changes.  An assignment that would empty a child (only
    possible through rounding) ends the loop and keeps the previous labels.
    """
    idx = node.idx
    Xc = X[idx]
    d = ((Xc - node.mean) ** 2).sum(axis=1)
    ia = int(np.argmax(d))
    a = Xc[ia].copy()
    db = ((Xc - a) ** 2).sum(axis=1)
    ib = int(np.argmax(db))
    ca, cb = a, Xc[ib].copy()
    lab = None
    iters = 0
    for _ in range(max_iter):
        da = ((Xc - ca) ** 2).sum(axis=1)
        dbb = ((Xc - cb) ** 2).sum(axis=1)
        new = da <= dbb
        if lab is not None and np.array_equal(new, lab):
            break
        if lab is not None and (new.all() or not new.any()):
            break
        lab = new
        iters += 1
        ca = Xc[lab].mean(axis=0)
        cb = Xc[~lab].mean(axis=0)
    A = _node(2 * node.heap, idx[lab], X, X32)
    B = _node(2 * node.heap + 1, idx[~lab], X, X32)
    node.children = (A, B)
    node.lloyd_iters = iters
    return A, B


def _split_key(nd):
    """Order of the split candidates (Sec. II-C, reading A6): the largest SSE
    first (not SSE per member), ties to the lower heap id."""
    return (-nd.sse, nd.heap)


def bisecting_kmeans(guide, K, max_iter=20, batched=False):
    """Bisecting K-means of the multiset {p(i)} (eq. (8)) into at most K
    clusters (Sec. II-C).

    Repeatedly the leaf with the largest SSE (sum of squared distances to its
    centroid; ties: lower heap id) is split by 2-means, until K leaves exist
    or no leaf has two distinct members.  ``batched=True`` computes the
    splits of all current leaves in rounds and then commits them in the same
    greedy order; it must return the same tree.
    """
    guide = np.asarray(guide)
    rho = guide.shape[0]
    X32 = np.ascontiguousarray(guide.reshape(rho, -1).T.astype(np.float32))
    X = X32.astype(np.float64)
    N = X.shape[0]
    if K < 1 or K > N:
        raise ValueError("K must be in [1, N]")
    root = _node(1, np.arange(N), X, X32)
    leaves = {1: root}
    order, hist = [], []

    def pick():
        cand = [nd for nd in leaves.values() if nd.splittable and nd.sse > 0.0]
        if not cand:
            return None
        return min(cand, key=_split_key)

    while len(leaves) < K:
        if batched:
            for nd in list(leaves.values()):
                if nd.splittable and nd.sse > 0.0 and nd.children is None:
                    _two_means(nd, X, X32, max_iter)
        nd = pick()
        if nd is None:
            break
        if nd.children is None:
            _two_means(nd, X, X32, max_iter)
        A, B = nd.children
        del leaves[nd.heap]
        leaves[A.heap] = A
        leaves[B.heap] = B
        order.append(nd.heap)
        hist.append(sum(x.sse for x in leaves.values()))

    heaps = sorted(leaves)
    centers = np.stack([leaves[h].mean for h in heaps])
    labels = np.empty(N, dtype=np.int32)
    for k, h in enumerate(heaps):
        labels[leaves[h].idx] = k
    sse = np.array([leaves[h].sse for h in heaps])
    return Clustering(centers, labels, heaps, sse, float(sse.sum()), order, hist)


def clustering_error(guide, centers, labels):
    """E_K of eq. (20): sum over pixels of |p(i) - mu_{cluster(i)}|^2."""
    rho = guide.shape[0]
    X = np.asarray(guide, dtype=np.float64).reshape(rho, -1).T
    return float(((X - np.asarray(centers, dtype=np.float64)[labels]) ** 2).sum())


# --------------------------------------------------------------------------
# Step 2: kernel matrix and pseudo-inverse, eq. (12)
# --------------------------------------------------------------------------

def kernel_matrix(centers, sigma_r):
    """A_kl = phi(mu_k - mu_l), eq. (12)."""
    mu = np.asarray(centers, dtype=np.float64)
    d2 = ((mu[:, None, :] - mu[None, :, :]) ** 2).sum(-1)
    return phi(d2, sigma_r)


def pinv(A, rtol=None):
    """Pseudo-inverse by the SVD, keeping singular values above
    max(size) * s_max * 2^-52 (the MATLAB pinv default the paper uses,
    Sec. II-C), or above rtol * s_max when rtol is given.
    Returns (A_pinv, rank, s)."""
    A = np.asarray(A, dtype=np.float64)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)  # the kept columns are those of the full SVD
    tol = (max(A.shape) * np.finfo(np.float64).eps if rtol is None else rtol) * s[0]
    keep = s > tol
    Ap = (Vt[keep].T / s[keep]) @ U[:, keep].T
    return Ap, int(keep.sum()), s


# --------------------------------------------------------------------------
# Steps 3-5: weights, coefficients, convolutions, recombination
# --------------------------------------------------------------------------

def range_weights(guide, centers, sigma_r):
    """b_k(i) = phi(mu_k - p(i)) of eq. (12), as an N x K array."""
    rho = guide.shape[0]
    X = np.asarray(guide, dtype=np.float64).reshape(rho, -1).T
    mu = np.asarray(centers, dtype=np.float64)
    N, K = X.shape[0], mu.shape[0]
    B = np.empty((N, K))
    step = max(1, (1 << 24) // max(1, K * rho))
    for s in range(0, N, step):
        d2 = ((X[s:s + step, None, :] - mu[None, :, :]) ** 2).sum(-1)
        B[s:s + step] = phi(d2, sigma_r)
    return B


def fast_filter(f, guide, centers, P, sigma_s, sigma_r, S=None,
                spatial="gaussian", conv_method="direct", coef="lsq",
                labels=None, return_terms=False):
    """Algorithm 1 from the centers on: b, c = P b, the convolutions
    v_k = omega * (b_k f), r_k = omega * b_k (eqs. (13)-(14)) and the
    recombination g = sum_k c_k v_k / sum_k c_k r_k (eqs. (15)-(16)).

    ``spatial='young'`` convolves with the recursive Gaussian of sigma_s
    (:func:`young_conv`, no radius).
    ``coef='hard'`` uses c_k(i) = 1 iff pixel i is in cluster k (eq. (17)),
    which gives eq. (18); ``labels`` must then be given.
    ``coef='exact'`` uses the per-pixel minimisers of eq. (10) over the
    filter's window (:func:`exact_ls`) in place of c = A^+ b of eq. (11).
    Returns (g (n,H,W), r_hat (H,W)) in FP64.  With ``return_terms`` it also
    returns the numerator v (n,H,W) of eq. (15) and the magnitudes of the
    sums that form v and r_hat, sum_k |c_k(i)| |v_k(i)| (n,H,W) and
    sum_k |c_k(i)| |r_k(i)| (H,W): the scale of the rounding error any
    finite-precision evaluation of the two sums carries.
    """
    f = _f64(f)
    n, H, W = f.shape
    if S is None and spatial != "young":
        S = default_radius(sigma_s)
    mu = np.asarray(centers, dtype=np.float64)
    K = mu.shape[0]
    B = range_weights(guide, mu, sigma_r)
    if coef == "lsq":
        C = B @ np.asarray(P, dtype=np.float64).T
    elif coef == "hard":
        C = np.zeros_like(B)
        C[np.arange(B.shape[0]), np.asarray(labels)] = 1.0
    elif coef == "exact":
        C = exact_ls(guide, mu, sigma_r, S, P=P)[0]
    else:
        raise ValueError(coef)
    F = f.reshape(n, -1)
    v = np.zeros((n, H * W))
    r = np.zeros(H * W)
    mv = np.zeros((n, H * W)) if return_terms else None
    mr = np.zeros(H * W) if return_terms else None
    for k in range(K):
        U = np.empty((n + 1, H * W))
        U[:n] = B[:, k] * F
        U[n] = B[:, k]
        if spatial == "young":
            V = young_conv(U.reshape(n + 1, H, W), sigma_s).reshape(n + 1, -1)
        else:
            V = conv(U.reshape(n + 1, H, W), S, sigma_s, spatial, conv_method).reshape(n + 1, -1)
        v += C[:, k] * V[:n]
        r += C[:, k] * V[n]
        if return_terms:
            mv += np.abs(C[:, k]) * np.abs(V[:n])
            mr += np.abs(C[:, k]) * np.abs(V[n])
    g, rh = (v / r).reshape(n, H, W), r.reshape(H, W)
    if return_terms:
        return g, rh, v.reshape(n, H, W), mv.reshape(n, H, W), mr.reshape(H, W)
    return g, rh


def _window_3d(S, sigma_s, spatial):
    """omega(j) on [-S,S]^3: Gaussian exp(-|j|^2/2 sigma_s^2) or box (all 1)."""
    j = np.arange(-S, S + 1, dtype=np.float64)
    if _spatial_code(spatial) == BOX:
        return np.ones((2 * S + 1,) * 3)
    r2 = j[:, None, None] ** 2 + j[None, :, None] ** 2 + j[None, None, :] ** 2
    return np.exp(-r2 / (2.0 * sigma_s ** 2))


def _offsets_3d(D, H, W, S):
    """Window offsets j = (jz, jy, jx) with the slices of the voxels i whose
    neighbour i - j lies in the volume, and of those neighbours (A1)."""
    for jz in range(-S, S + 1):
        for jy in range(-S, S + 1):
            for jx in range(-S, S + 1):
                lo = [max(0, jz), max(0, jy), max(0, jx)]
                hi = [min(D, D + jz), min(H, H + jy), min(W, W + jx)]
                if any(a >= b for a, b in zip(lo, hi)):
                    continue
                iv = tuple(slice(a, b) for a, b in zip(lo, hi))
                qv = tuple(slice(a - o, b - o) for a, b, o in zip(lo, hi, (jz, jy, jx)))
                yield (jz, jy, jx), iv, qv


def bruteforce_volume(f, guide, sigma_s, sigma_r, S, spatial="gaussian"):
    """Eqs. (1)-(2) on a 3-D domain (Sec. III-F filters a volume): the window
    [-S,S]^3, omega as in 2-D over |j|, neighbours outside the volume left
    out.  f (n, D, H, W), guide (rho, D, H, W).  Returns (g, eta) in FP64."""
    f = _f64(f)
    p = _f64(guide)
    n, D, H, W = f.shape
    om = _window_3d(S, sigma_s, spatial)
    num = np.zeros_like(f)
    eta = np.zeros((D, H, W))
    for (jz, jy, jx), iv, qv in _offsets_3d(D, H, W, S):
        w = om[jz + S, jy + S, jx + S] * phi(((p[(slice(None),) + qv] - p[(slice(None),) + iv]) ** 2).sum(0),
                                             sigma_r)
        num[(slice(None),) + iv] += w * f[(slice(None),) + qv]
        eta[iv] += w
    return num / eta, eta


def fast_filter_volume(f, guide, centers, P, sigma_s, sigma_r, S, spatial="gaussian", coef="lsq",
                       labels=None):
    """Algorithm 1 steps 3-5 on a 3-D domain in the paper's form: b_k(i) and
    c(i) = A^+ b(i) per voxel (eq. (12)), the (n+1)K window sums of
    omega(j) b_k(i - j) [f, 1](i - j) over [-S,S]^3 (eqs. (13)-(14), direct,
    neighbours outside the volume left out), and the ratio of eqs. (15)-(16).
    ``coef='hard'`` takes c_k(i) = 1 iff voxel i is in cluster k (eq. (17),
    ``labels`` per voxel in (z, y, x) order), which gives eq. (18).
    Returns (g, r_hat) in FP64."""
    f = _f64(f)
    p = _f64(guide)
    n, D, H, W = f.shape
    rho = p.shape[0]
    mu = np.asarray(centers, dtype=np.float64).reshape(-1, rho)
    K = mu.shape[0]
    X = p.reshape(rho, -1).T
    B = phi(((X[:, None, :] - mu[None, :, :]) ** 2).sum(-1), sigma_r).T.reshape(K, D, H, W)
    if coef == "lsq":
        C = (np.asarray(P, dtype=np.float64) @ B.reshape(K, -1)).reshape(K, D, H, W)
    elif coef == "hard":
        C = np.zeros((K, D * H * W))
        C[np.asarray(labels).reshape(-1), np.arange(D * H * W)] = 1.0
        C = C.reshape(K, D, H, W)
    else:
        raise ValueError(coef)
    U = np.concatenate([B[:, None] * f[None], B[:, None]], axis=1)  # K x (n+1) x D x H x W
    om = _window_3d(S, sigma_s, spatial)
    V = np.zeros_like(U)
    for (jz, jy, jx), iv, qv in _offsets_3d(D, H, W, S):
        V[(slice(None), slice(None)) + iv] += om[jz + S, jy + S, jx + S] * U[(slice(None), slice(None)) + qv]
    v = (C[:, None] * V).sum(0)
    return v[:n] / v[n], v[n]


def fhd_filter_volume(f, guide, sigma_s, sigma_r, K, S, spatial="gaussian", max_iter=20, coef="lsq"):
    """The whole of Algorithm 1 on a 3-D domain: the bisecting K-means of the
    voxels' guide vectors (the volume's voxels in (z, y, x) order, as one
    set), A and A^+, then :func:`fast_filter_volume` (least squares or the
    hard variant with the clustering's labels)."""
    rho, D, H, W = np.asarray(guide).shape
    cl = bisecting_kmeans(np.asarray(guide).reshape(rho, D * H, W), K, max_iter)
    A = kernel_matrix(cl.centers, sigma_r)
    P, rank, _ = pinv(A)
    out, den = fast_filter_volume(f, guide, cl.centers, P, sigma_s, sigma_r, S, spatial, coef,
                                  cl.labels.reshape(-1) if coef == "hard" else None)
    return FilterResult(out, den, cl, cl.centers, A, P, rank)


def approx_error(guide, centers, sigma_r, S, P=None):
    """The error of the kernel approximation eq. (9) at the pixels' own
    samples: for every pixel i, the objective of eq. (10) evaluated at the
    coefficients the method uses, c(i) = A^+ b(i) (eqs. (11)-(12)),
        err(i) = sum_{x in Theta_i} (phi(x - p(i)) - sum_k c_k(i) phi(x - mu_k))^2,
    Theta_i the guide values of the in-image pixels of the (2S+1)^2 window
    around i (A1; a multiset, A4).  Its mean over the pixels is the averaged
    least-squares error of Sec. II-A (E_ls here; the paper writes a script E
    indexed by K, distinct from the clustering error E_K of eq. (20)).
    Vectorised over the pixels, one window offset at a time.  Returns
    (err (H, W) FP64, E_ls)."""
    p = _f64(guide)
    rho, H, W = p.shape
    mu = np.asarray(centers, dtype=np.float64).reshape(-1, rho)
    K = mu.shape[0]
    if P is None:
        P, _, _ = pinv(kernel_matrix(mu, sigma_r))
    X = p.reshape(rho, -1).T
    B = phi(((X[:, None, :] - mu[None, :, :]) ** 2).sum(-1), sigma_r)  # b_k(i), N x K
    Bimg = B.T.reshape(K, H, W)
    Cimg = (B @ np.asarray(P, dtype=np.float64).T).T.reshape(K, H, W)  # c(i) = A^+ b(i)
    err = np.zeros((H, W))
    for jy in range(-S, S + 1):
        for jx in range(-S, S + 1):
            y0, y1 = max(0, jy), min(H, H + jy)
            x0, x1 = max(0, jx), min(W, W + jx)
            if y0 >= y1 or x0 >= x1:
                continue
            qy, qx = slice(y0 - jy, y1 - jy), slice(x0 - jx, x1 - jx)
            iy, ix = slice(y0, y1), slice(x0, x1)
            exact = phi(((p[:, qy, qx] - p[:, iy, ix]) ** 2).sum(0), sigma_r)
            fit = (Cimg[:, iy, ix] * Bimg[:, qy, qx]).sum(0)  # phi(x - mu_k) = b_k(q)
            err[iy, ix] += (exact - fit) ** 2
    return err, float(err.mean())


def exact_ls(guide, centers, sigma_r, S, pixels=None, P=None):
    """Eq. (10) solved at each pixel (Sec. II-A): c*(i) minimises
        sum_{x in Theta_i} (phi(x - p(i)) - sum_k c_k phi(x - mu_k))^2
    over the multiset Theta_i of the guide values of the in-image pixels of
    the (2S+1)^2 window around i (the readings of :func:`approx_error`).
    With the window's pixels q_1 .. q_m, row j of the design matrix M_i is
    [phi(p(q_j) - mu_k)]_k = b(q_j) (eq. (12)'s weights at q_j) and the target
    is y_j = phi(p(q_j) - p(i)); c*(i) = M_i^+ y_i, the minimum-norm minimiser,
    with the pseudo-inverse of :func:`pinv` (the MATLAB default tolerance, as
    for A^+).  ``pixels``: flat indices to solve (default: all).
    Returns (C (len, K): c*(i); obj (len,): the minimum of eq. (10);
    obj11 (len,): eq. (10) at the surrogate's coefficients c = A^+ b(i) of
    eq. (11)), all FP64."""
    p = _f64(guide)
    rho, H, W = p.shape
    mu = np.asarray(centers, dtype=np.float64).reshape(-1, rho)
    K = mu.shape[0]
    if P is None:
        P, _, _ = pinv(kernel_matrix(mu, sigma_r))
    P = np.asarray(P, dtype=np.float64)
    X = p.reshape(rho, -1).T
    B = range_weights(guide, mu, sigma_r)
    idx = np.arange(H * W) if pixels is None else np.asarray(pixels, dtype=np.int64).ravel()
    C = np.empty((len(idx), K))
    obj = np.empty(len(idx))
    obj11 = np.empty(len(idx))
    for t, i in enumerate(idx):
        iy, ix = divmod(int(i), W)
        ys = np.arange(max(0, iy - S), min(H, iy + S + 1))
        xs = np.arange(max(0, ix - S), min(W, ix + S + 1))
        q = (ys[:, None] * W + xs[None, :]).ravel()
        M = B[q]
        y = phi(((X[q] - X[i]) ** 2).sum(1), sigma_r)
        Mp, _, _ = pinv(M)
        c = Mp @ y
        C[t] = c
        obj[t] = ((y - M @ c) ** 2).sum()
        obj11[t] = ((y - M @ (P @ B[i])) ** 2).sum()
    return C, obj, obj11


def fast_filter_at(f, guide, centers, P, sigma_s, sigma_r, ys, xs, S=None,
                   spatial="gaussian"):
    """Eqs. (13)-(16) at the listed pixels only (direct window sums).
    Returns (g (M x n), r_hat (M))."""
    f = _f64(f)
    guide = _f64(guide)
    n, H, W = f.shape
    rho = guide.shape[0]
    if S is None:
        S = default_radius(sigma_s)
    mu = _f64(centers)
    K = mu.shape[0]
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    M = len(ys)
    V = np.empty((M, K, n + 1))
    _load().oracle_cluster_images_at(_dp(f), n, _dp(guide), rho, H, W, _dp(mu), K,
                                     int(S), _spatial_code(spatial),
                                     float(sigma_s or 1.0), float(sigma_r),
                                     _ip(ys), _ip(xs), M, _dp(V))
    p_at = guide.reshape(rho, -1)[:, ys.astype(np.int64) * W + xs].T
    d2 = ((p_at[:, None, :] - mu[None, :, :]) ** 2).sum(-1)
    Bm = phi(d2, sigma_r)
    Cm = Bm @ np.asarray(P, dtype=np.float64).T
    num = np.einsum("mk,mkc->mc", Cm, V[:, :, :n])
    den = np.einsum("mk,mk->m", Cm, V[:, :, n])
    return num / den[:, None], den


@dataclass
class FilterResult:
    out: np.ndarray
    den: np.ndarray
    clustering: Clustering
    centers: np.ndarray
    A: np.ndarray
    P: np.ndarray
    rank: int


def fhd_filter(f, guide, sigma_s, sigma_r, K, S=None, spatial="gaussian",
               max_iter=20, conv_method="direct", coef="lsq", centers=None):
    """The whole of Algorithm 1.  ``centers`` (optional) skips the clustering
    and uses the given centers (e.g. the GPU's, rounded to FP32)."""
    cl = bisecting_kmeans(guide, K, max_iter) if centers is None else None
    mu = cl.centers if centers is None else np.asarray(centers, dtype=np.float64)
    A = kernel_matrix(mu, sigma_r)
    P, rank, _ = pinv(A)
    labels = cl.labels if cl is not None else None
    out, den = fast_filter(f, guide, mu, P, sigma_s, sigma_r, S, spatial,
                           conv_method, coef, labels)
    return FilterResult(out, den, cl, mu, A, P, rank)


# --------------------------------------------------------------------------
# Nonlocal-means guide: PCA of color patches (Sec. I-A, Sec. III-C)
# --------------------------------------------------------------------------

def patches(f, m):
    """All m x m x n patches, one per pixel, flattened in (dy, dx, channel)
    order; the image is extended by half-sample symmetric reflection
    (index -1 maps to 0).  Returns N x (m*m*n) FP64."""
    f = np.asarray(f, dtype=np.float64)
    n, H, W = f.shape
    h = m // 2
    fp = np.pad(f, ((0, 0), (h, h), (h, h)), mode="symmetric")
    cols = []
    for dy in range(m):
        for dx in range(m):
            for c in range(n):
                cols.append(fp[c, dy:dy + H, dx:dx + W].reshape(-1))
    return np.stack(cols, axis=1)


def nlm_guide(f, m=5, dims=16):
    """Patch-PCA guide: project the mean-centred patches onto the `dims`
    leading eigenvectors of their covariance (FP64, no whitening).
    Returns (guide (dims,H,W), eigenvalues descending, basis (m*m*n x dims),
    patch mean)."""
    n, H, W = np.asarray(f).shape
    Pm = patches(f, m)
    mean = Pm.mean(axis=0)
    X = Pm - mean
    cov = (X.T @ X) / X.shape[0]
    lam, V = np.linalg.eigh(cov)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    basis = V[:, :dims]
    g = (X @ basis).T.reshape(dims, H, W)
    return g, lam, basis, mean


# --------------------------------------------------------------------------
# Quality, eq. (21)
# --------------------------------------------------------------------------

def mse(a, b):
    """|Omega|^-1 sum_i |a(i) - b(i)|^2 with the norm over channels, eq. (21)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    N = a.shape[-1] * a.shape[-2]
    return float(((a - b) ** 2).sum() / N)


def psnr(a, b):
    """PSNR = -10 log10(MSE) of eq. (21) (peak 1, channel-summed MSE)."""
    m = mse(a, b)
    return float("inf") if m == 0 else float(-10.0 * np.log10(m))
