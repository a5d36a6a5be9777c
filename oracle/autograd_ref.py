"""Differentiable FP64 transcriptions of the oracle for gradient checks.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``).

The paper does not differentiate its filter.  These plain PyTorch (CPU,
float64) transcriptions of eqs. (1)-(2) and of Algorithm 1 with fixed
centers let autograd provide reference gradients with respect to the image
f, the guide p, sigma_r and sigma_s.  Centers are constants (stop-gradient).
The window radius S is held fixed when sigma_s varies.
"""
from __future__ import annotations

import torch
import torch.nn.functional as F


def _omega2(S, sigma_s, spatial):
    j = torch.arange(-S, S + 1, dtype=torch.float64)
    if spatial == "box":
        return torch.ones(2 * S + 1, 2 * S + 1, dtype=torch.float64)
    return torch.exp(-(j[:, None] ** 2 + j[None, :] ** 2) / (2.0 * sigma_s ** 2))


def fast_filter_torch(f, p, centers, sigma_s, sigma_r, S, spatial="gaussian",
                      full_rank=True):
    """Algorithm 1 with given centers: b = phi(mu - p), c = A^+ b, the
    convolutions of eqs. (13)-(14), the ratio of eqs. (15)-(16).

    f: (n,H,W), p: (rho,H,W), centers: (K,rho), sigma_r / sigma_s: scalars or
    0-d tensors (may require grad).  A^+ = A^-1 when ``full_rank``.
    Returns (g, r_hat)."""
    n, H, W = f.shape
    rho = p.shape[0]
    mu = torch.as_tensor(centers, dtype=torch.float64)
    K = mu.shape[0]
    X = p.reshape(rho, -1).T
    d2 = ((X[:, None, :] - mu[None, :, :]) ** 2).sum(-1)
    B = torch.exp(-d2 / (2.0 * sigma_r ** 2))
    dm = ((mu[:, None, :] - mu[None, :, :]) ** 2).sum(-1)
    A = torch.exp(-dm / (2.0 * sigma_r ** 2))
    P = torch.linalg.inv(A) if full_rank else torch.linalg.pinv(A, hermitian=True)
    C = B @ P.T
    Fl = f.reshape(n, -1)
    U = torch.cat([B.T[:, None, :] * Fl[None, :, :], B.T[:, None, :]], dim=1)
    w = _omega2(S, sigma_s, spatial)
    V = F.conv2d(U.reshape(K * (n + 1), 1, H, W), w[None, None], padding=S)
    V = V.reshape(K, n + 1, H * W)
    v = (C.T[:, None, :] * V).sum(0)
    return (v[:n] / v[n]).reshape(n, H, W), v[n].reshape(H, W)


def bruteforce_torch(f, p, sigma_s, sigma_r, S, spatial="gaussian"):
    """Eqs. (1)-(2) with out-of-domain samples excluded.  Returns (g, eta)."""
    n, H, W = f.shape
    fp = F.pad(f[None], (S, S, S, S))[0]
    pp = F.pad(p[None], (S, S, S, S))[0]
    inside = F.pad(torch.ones(1, 1, H, W, dtype=torch.float64), (S, S, S, S))[0, 0]
    num = torch.zeros_like(f)
    eta = torch.zeros(H, W, dtype=torch.float64)
    for jy in range(-S, S + 1):
        for jx in range(-S, S + 1):
            # the sample q = i - j, read from the zero-padded copies
            ys, xs = slice(S - jy, S - jy + H), slice(S - jx, S - jx + W)
            if spatial == "box":
                w = 1.0
            else:
                w = torch.exp(torch.as_tensor(-(jy * jy + jx * jx), dtype=torch.float64)
                              / (2.0 * sigma_s ** 2))
            ph = torch.exp(-((pp[:, ys, xs] - p) ** 2).sum(0) / (2.0 * sigma_r ** 2))
            wt = w * ph * inside[ys, xs]
            num = num + wt * fp[:, ys, xs]
            eta = eta + wt
    return num / eta, eta


def sigma_r_shares(f, p, centers, sigma_s, sigma_r, S, G, spatial="gaussian", full_rank=True):
    """Per-pixel split of dL/dsigma_r for L = <G, g>, in FP64:
    share_b(i) = sum_k dL/db_k(i) * db_k(i)/dsigma_r (the weights' own
    dependence) and share_A(i) = dL/dc(i) . (dA^+/dsigma_r) b(i) (the pseudo-
    inverse's).  Their sum over pixels is the total gradient; the sum of their
    magnitudes sizes the rounding error of any evaluation of that total."""
    n, H, W = f.shape
    rho = p.shape[0]
    f = torch.as_tensor(f, dtype=torch.float64)
    p = torch.as_tensor(p, dtype=torch.float64)
    mu = torch.as_tensor(centers, dtype=torch.float64)
    X = p.reshape(rho, -1).T
    d2 = ((X[:, None, :] - mu[None, :, :]) ** 2).sum(-1)
    dm = ((mu[:, None, :] - mu[None, :, :]) ** 2).sum(-1)

    def pinv_of(s):
        A = torch.exp(-dm / (2.0 * s ** 2))
        return torch.linalg.inv(A) if full_rank else torch.linalg.pinv(A, hermitian=True)

    s0 = torch.tensor(float(sigma_r), dtype=torch.float64)
    B = torch.exp(-d2 / (2.0 * s0 ** 2)).requires_grad_(True)
    P = pinv_of(s0)
    C = B @ P.T
    C.retain_grad()
    Fl = f.reshape(n, -1)
    U = torch.cat([B.T[:, None, :] * Fl[None, :, :], B.T[:, None, :]], dim=1)
    w = _omega2(S, sigma_s, spatial)
    K = mu.shape[0]
    V = F.conv2d(U.reshape(K * (n + 1), 1, H, W), w[None, None], padding=S).reshape(K, n + 1, H * W)
    v = (C.T[:, None, :] * V).sum(0)
    g = v[:n] / v[n]
    (g * torch.as_tensor(G, dtype=torch.float64).reshape(n, -1)).sum().backward()
    dB = B.detach() * d2 / float(sigma_r) ** 3
    share_b = (B.grad * dB).sum(1)
    M = torch.autograd.functional.jacobian(pinv_of, s0)
    share_A = (C.grad * (B.detach() @ M.T)).sum(1)
    return share_b.numpy(), share_A.numpy()


def sigma_s_shares(f, p, centers, sigma_s, sigma_r, S, G, spatial="gaussian", full_rank=True):
    """Per-pixel split of dL/dsigma_s for L = <G, g>, in FP64: share(i) =
    G(i) . dg(i)/dsigma_s, the derivative image taken in forward mode through
    Algorithm 1 (the window's taps are the only dependence on sigma_s).  Their
    sum is the total gradient; the sum of their magnitudes sizes the rounding
    error of any evaluation of that total."""
    f = torch.as_tensor(f, dtype=torch.float64)
    p = torch.as_tensor(p, dtype=torch.float64)
    s0 = torch.tensor(float(sigma_s), dtype=torch.float64)

    def g_of(s):
        return fast_filter_torch(f, p, centers, s, sigma_r, S, spatial, full_rank)[0]

    _, dg = torch.autograd.functional.jvp(g_of, (s0,), (torch.ones((), dtype=torch.float64),))
    return (torch.as_tensor(G, dtype=torch.float64) * dg).sum(0).numpy()


def centers_abs_scale(f, p, centers, sigma_s, sigma_r, S, G, spatial="gaussian", full_rank=True):
    """Magnitude scale of the pixel terms behind dL/dmu, in FP64, per center
    coordinate (k, t): sum_i |w_k(i) (p_t(i) - mu_kt)| / sigma_r^2 (through
    the weights, w_k = dL/db_k b_k) plus sum_i |gamma(i)^T (dA^+/dmu_kt) b(i)|
    (through A^+, gamma = dL/dc).  The total is the sum of these terms with
    their signs; the sum of magnitudes sizes the rounding error of any
    evaluation of it."""
    n, H, W = f.shape
    rho = p.shape[0]
    f = torch.as_tensor(f, dtype=torch.float64)
    p = torch.as_tensor(p, dtype=torch.float64)
    mu = torch.as_tensor(centers, dtype=torch.float64)
    K = mu.shape[0]
    X = p.reshape(rho, -1).T
    d2 = ((X[:, None, :] - mu[None, :, :]) ** 2).sum(-1)
    B = torch.exp(-d2 / (2.0 * float(sigma_r) ** 2)).requires_grad_(True)

    def pinv_of(m):
        dm = ((m[:, None, :] - m[None, :, :]) ** 2).sum(-1)
        A = torch.exp(-dm / (2.0 * float(sigma_r) ** 2))
        return torch.linalg.inv(A) if full_rank else torch.linalg.pinv(A, hermitian=True)

    P = pinv_of(mu)
    C = B @ P.T
    C.retain_grad()
    Fl = f.reshape(n, -1)
    U = torch.cat([B.T[:, None, :] * Fl[None, :, :], B.T[:, None, :]], dim=1)
    w = _omega2(S, sigma_s, spatial)
    V = F.conv2d(U.reshape(K * (n + 1), 1, H, W), w[None, None], padding=S).reshape(K, n + 1, H * W)
    v = (C.T[:, None, :] * V).sum(0)
    g = v[:n] / v[n]
    (g * torch.as_tensor(G, dtype=torch.float64).reshape(n, -1)).sum().backward()
    wl = (B.grad * B.detach()).abs()                       # N x K
    diff = (X[:, None, :] - mu[None, :, :]).abs()           # N x K x rho
    sb = (wl[:, :, None] * diff).sum(0) / float(sigma_r) ** 2
    D = torch.autograd.functional.jacobian(pinv_of, mu)     # K x K x K x rho: d(A^+)_lm / dmu_kt
    gam, bb = C.grad, B.detach()
    sA = torch.zeros(K, rho, dtype=torch.float64)
    for k in range(K):
        for t in range(rho):
            # d(c_l)/dmu_kt = sum_m D[l, m, k, t] b_m  (c = A^+ b, A^+ symmetric up to rounding)
            sA[k, t] = (gam * (bb @ D[:, :, k, t].T)).sum(1).abs().sum()
    return sb.numpy(), sA.numpy()
