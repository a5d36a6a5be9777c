"""Pins of the FP64 gradient reference (``oracle/autograd_ref.py``) against
the oracle itself: central finite differences of ``oracle.fast_filter`` (the
NumPy transcription of Algorithm 1 with fixed centers) and the exact
linearity of the filter in the image.  The GPU adjoint is compared with this
reference, so a wrong reference gradient (a dropped term of the pseudo-inverse
derivative, a sign) must fail here first.

Finite differences: step h, truncation error O(h^2 |L'''|) and rounding error
O(eps |L| / h); with h = 1e-5 relative both are below 1e-8 of the gradient.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import autograd_ref as ar


def _setup(rho_guide=None, K=8, seed=3, H=18, W=21):
    # FP64 copies: a step of 1e-6 must not be rounded to the FP32 grid
    f = synth.voronoi_rgb(H, W, 6, 0.05, seed).astype(np.float64)
    g = f if rho_guide is None else synth.hyperspectral(H, W, rho_guide, 3, 0.5, 0.02, seed + 1).astype(np.float64)
    cen = oracle.bisecting_kmeans(g, K).centers.astype(np.float32).astype(np.float64)
    G = np.random.default_rng(seed + 7).standard_normal(f.shape)
    return f, g, cen, G


def _loss_oracle(f, g, cen, G, ss, sr, S, spatial="gaussian"):
    P, _, _ = oracle.pinv(oracle.kernel_matrix(cen, sr))
    out = oracle.fast_filter(f, g, cen, P, ss, sr, S, spatial)[0]
    return float((out * G).sum())


def _grads_ref(f, g, cen, G, ss, sr, S, spatial="gaussian", full_rank=True):
    ft = torch.tensor(f, dtype=torch.float64, requires_grad=True)
    gt = torch.tensor(g, dtype=torch.float64, requires_grad=True)
    st = torch.tensor(sr, dtype=torch.float64, requires_grad=True)
    out, _ = ar.fast_filter_torch(ft, gt, cen, ss, st, S, spatial, full_rank=full_rank)
    (out * torch.tensor(G)).sum().backward()
    return ft.grad.numpy(), gt.grad.numpy(), float(st.grad)


@pytest.mark.parametrize("spatial", ["gaussian", "box"])
def test_sigma_r_gradient_matches_finite_difference(spatial):
    f, g, cen, G = _setup(rho_guide=4, K=8)
    ss, sr, S = 2.0, 0.3, 4
    _, _, gs = _grads_ref(f, g, cen, G, ss, sr, S, spatial)
    h = 1e-5 * sr
    fd = (_loss_oracle(f, g, cen, G, ss, sr + h, S, spatial)
          - _loss_oracle(f, g, cen, G, ss, sr - h, S, spatial)) / (2 * h)
    assert abs(gs - fd) <= 1e-6 * max(1.0, abs(fd)), (gs, fd)


def test_guide_and_image_gradients_match_finite_difference():
    f, g, cen, G = _setup(rho_guide=3, K=6)
    ss, sr, S = 2.0, 0.25, 4
    gf, gg, _ = _grads_ref(f, g, cen, G, ss, sr, S)
    rng = np.random.default_rng(11)
    for _ in range(6):
        c, y, x = rng.integers(0, g.shape[0]), rng.integers(0, g.shape[1]), rng.integers(0, g.shape[2])
        h = 1e-6
        gp, gm = g.copy(), g.copy()
        gp[c, y, x] += h
        gm[c, y, x] -= h
        fd = (_loss_oracle(f, gp, cen, G, ss, sr, S) - _loss_oracle(f, gm, cen, G, ss, sr, S)) / (2 * h)
        assert abs(gg[c, y, x] - fd) <= 1e-6 * max(1.0, np.abs(gg).max()), (gg[c, y, x], fd)
    # the filter is linear in f: dL/df . delta = L(delta) exactly
    d = rng.standard_normal(f.shape)
    assert abs((gf * d).sum() - _loss_oracle(d, g, cen, G, ss, sr, S)) < 1e-9 * np.abs(gf).sum()


def test_rank_deficient_sigma_r_gradient():
    """Two identical centers: A has a zero eigenvalue for every sigma_r, the
    pseudo-inverse keeps rank K - 1, and the derivative of A^+ has the two
    extra terms of a rank-deficient matrix (the -A^+ dA A^+ term alone is
    wrong here)."""
    f, g, cen, G = _setup(rho_guide=3, K=6)
    cen = np.vstack([cen, cen[2:3]])
    ss, sr, S = 2.0, 0.3, 4
    assert oracle.pinv(oracle.kernel_matrix(cen, sr))[1] == cen.shape[0] - 1
    _, _, gs = _grads_ref(f, g, cen, G, ss, sr, S, full_rank=False)
    h = 1e-5 * sr
    fd = (_loss_oracle(f, g, cen, G, ss, sr + h, S) - _loss_oracle(f, g, cen, G, ss, sr - h, S)) / (2 * h)
    assert abs(gs - fd) <= 1e-6 * max(1.0, abs(fd)), (gs, fd)


def test_sigma_r_shares_sum_to_gradient():
    """The per-pixel split used to size the GPU tolerance adds up to the
    autograd total (full-rank and rank-deficient A)."""
    f, g, cen, G = _setup(rho_guide=3, K=6)
    for full, c in ((True, cen), (False, np.vstack([cen, cen[1:2]]))):
        _, _, gs = _grads_ref(f, g, c, G, 2.0, 0.3, 4, full_rank=full)
        sb, sa = ar.sigma_r_shares(f, g, c, 2.0, 0.3, 4, G, full_rank=full)
        assert abs(sb.sum() + sa.sum() - gs) <= 1e-10 * (np.abs(sb).sum() + np.abs(sa).sum())


def test_sigma_s_gradient_matches_finite_difference():
    """dL/dsigma_s through the window's taps (radius fixed) against central
    differences of the oracle in sigma_s, and its per-pixel split against the
    total."""
    f, g, cen, G = _setup(rho_guide=4, K=8)
    ss, sr, S = 2.0, 0.3, 5
    ft = torch.tensor(f)
    gt = torch.tensor(g)
    st = torch.tensor(ss, dtype=torch.float64, requires_grad=True)
    out, _ = ar.fast_filter_torch(ft, gt, cen, st, sr, S)
    (out * torch.tensor(G)).sum().backward()
    gss = float(st.grad)
    h = 1e-5 * ss
    fd = (_loss_oracle(f, g, cen, G, ss + h, sr, S) - _loss_oracle(f, g, cen, G, ss - h, sr, S)) / (2 * h)
    assert abs(gss - fd) <= 1e-6 * max(1.0, abs(fd)), (gss, fd)
    sh = ar.sigma_s_shares(f, g, cen, ss, sr, S, G)
    assert abs(sh.sum() - gss) <= 1e-10 * np.abs(sh).sum()


@pytest.mark.parametrize("full_rank", [True, False])
def test_centers_gradient_matches_finite_difference(full_rank):
    """dL/dmu (clustering held fixed: the centers enter through b and A)
    against central differences of the oracle in each center coordinate;
    full-rank A and a repeated center (rank K - 1, pseudo-inverse)."""
    f, g, cen, G = _setup(rho_guide=3, K=6)
    if not full_rank:
        cen = np.vstack([cen, cen[2:3]])
    ss, sr, S = 2.0, 0.3, 4
    ct = torch.tensor(cen, requires_grad=True)
    out, _ = ar.fast_filter_torch(torch.tensor(f), torch.tensor(g), ct, ss, sr, S, full_rank=full_rank)
    (out * torch.tensor(G)).sum().backward()
    gm = ct.grad.numpy()
    rows = [cen.shape[0] - 1, 0] if not full_rank else [0, 3]
    for k in rows:
        for t in range(cen.shape[1]):
            h = 1e-6
            cp, cm = cen.copy(), cen.copy()
            cp[k, t] += h
            cm[k, t] -= h
            if not full_rank:  # keep the pair identical: move both copies
                j = 2 if k == cen.shape[0] - 1 else (cen.shape[0] - 1 if k == 2 else None)
                if j is not None:
                    cp[j, t] += h
                    cm[j, t] -= h
            fd = (_loss_oracle(f, g, cp, G, ss, sr, S) - _loss_oracle(f, g, cm, G, ss, sr, S)) / (2 * h)
            ref = gm[k, t] + (gm[j, t] if (not full_rank and j is not None) else 0.0)
            assert abs(ref - fd) <= 1e-5 * max(1.0, np.abs(gm).max()), (k, t, ref, fd)
