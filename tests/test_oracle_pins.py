"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names the passage of the paper (or the mathematical fact) it
checks.  These run on the CPU only.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

import oracle
import synth
from oracle import autograd_ref as ar


def _rgb(H=24, W=28, seeds=6, noise=0.05, seed=7):
    return synth.voronoi_rgb(H, W, seeds, noise, seed)


# ---------------------------------------------------------------------------
# X11: brute force on a hand-worked example (eqs. (1)-(2))
# ---------------------------------------------------------------------------

def test_bruteforce_hand_worked(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "bruteforce_3px.json")))
    f = np.array(g["f"], dtype=np.float64).reshape(1, 1, 3)
    for case in g["cases"]:
        sr = math.inf if case["sigma_r"] == "inf" else case["sigma_r"]
        out, eta = oracle.bruteforce(f, f, case.get("sigma_s", 1.0), sr, S=case["S"],
                                     spatial=case["spatial"])
        np.testing.assert_allclose(out.ravel(), case["g"], rtol=0, atol=1e-15)
        np.testing.assert_allclose(eta.ravel(), case["eta"], rtol=0, atol=1e-15)


def test_bruteforce_torch_transcription_agrees():
    """The differentiable transcription of eqs. (1)-(2) and the C loop."""
    f = _rgb(12, 14)
    out, eta = oracle.bruteforce(f, f, 2.0, 0.15, S=6)
    t = torch.tensor(f, dtype=torch.float64)
    gt, et = ar.bruteforce_torch(t, t, 2.0, 0.15, 6)
    assert np.abs(gt.numpy() - out).max() < 1e-14
    assert np.abs(et.numpy() - eta).max() < 1e-12


# ---------------------------------------------------------------------------
# X1: a constant image is returned unchanged (eqs. (1)-(2), (15)-(16))
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K", [1, 4, 9])
def test_constant_image(K):
    guide = _rgb()
    f = np.empty((3,) + guide.shape[1:])
    f[:] = np.array([0.2, 0.5, 0.9])[:, None, None]
    out, _ = oracle.bruteforce(f, guide, 2.0, 0.1, S=6)
    assert np.abs(out - f).max() < 1e-13
    res = oracle.fhd_filter(f, guide, 2.0, 0.1, K, S=6)
    assert np.abs(res.out - f).max() < 1e-12
    # self-guided constant image: one distinct value -> one cluster, A = [1]
    res = oracle.fhd_filter(f, f, 2.0, 0.1, K, S=6)
    assert res.centers.shape[0] == 1 and res.A[0, 0] == 1.0
    assert np.abs(res.out - f).max() < 1e-13


# ---------------------------------------------------------------------------
# X2: sigma_r -> inf reduces both to the normalised spatial filter
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("spatial", ["gaussian", "box"])
def test_sigma_r_inf_is_normalised_convolution(spatial):
    f = _rgb(20, 23)
    S, ss = 5, 1.7
    w = oracle.spatial_kernel_2d(S, ss, spatial)
    one = np.ones(f.shape[1:])
    ref_den = ndi.convolve(one, w, mode="constant", cval=0.0)
    ref = np.stack([ndi.convolve(f[c].astype(np.float64), w, mode="constant", cval=0.0)
                    for c in range(3)]) / ref_den
    out, eta = oracle.bruteforce(f, f, ss, math.inf, S=S, spatial=spatial)
    assert np.abs(out - ref).max() < 1e-12
    assert np.abs(eta - ref_den).max() < 1e-11
    res = oracle.fhd_filter(f, f, ss, math.inf, 6, S=S, spatial=spatial)
    # A = J (all ones): rank 1, pinv J / K^2, c = 1/K
    K = res.centers.shape[0]
    assert res.rank == 1
    assert np.abs(res.P - np.full((K, K), 1.0 / K ** 2)).max() < 1e-14
    assert np.abs(res.out - ref).max() < 1e-12


# ---------------------------------------------------------------------------
# X3: K >= number of distinct guide values reproduces brute force exactly
# ---------------------------------------------------------------------------

def test_enough_clusters_is_exact():
    f = synth.voronoi_rgb(26, 30, 7, 0.0, 11)          # piecewise constant, no noise
    distinct = np.unique(f.reshape(3, -1).T, axis=0).shape[0]
    bf, _ = oracle.bruteforce(f, f, 2.5, 0.2, S=7)
    for K in (distinct, distinct + 3):
        res = oracle.fhd_filter(f, f, 2.5, 0.2, K, S=7)
        assert res.centers.shape[0] == distinct            # K_eff = #distinct
        assert res.rank == distinct
        assert np.abs(res.out - bf).max() < 1e-12


# ---------------------------------------------------------------------------
# X4: K = 1 is normalised convolution with certainty b
# ---------------------------------------------------------------------------

def test_single_cluster_is_normalised_convolution():
    f = _rgb(18, 21)
    S, ss, sr = 4, 1.5, 0.3
    res = oracle.fhd_filter(f, f, ss, sr, 1, S=S)
    X = f.reshape(3, -1).T.astype(np.float64)
    mu = X.mean(axis=0)
    assert np.abs(res.centers[0] - mu).max() < 1e-15
    b = np.exp(-((X - mu) ** 2).sum(1) / (2 * sr * sr)).reshape(f.shape[1:])
    w = oracle.spatial_kernel_2d(S, ss)
    den = ndi.convolve(b, w, mode="constant")
    ref = np.stack([ndi.convolve(b * f[c], w, mode="constant") for c in range(3)]) / den
    assert np.abs(res.out - ref).max() < 1e-12


# ---------------------------------------------------------------------------
# X5: the least-squares coefficients interpolate at the centers (eqs. (11)-(12))
# ---------------------------------------------------------------------------

def test_interpolation_identity_and_pinv():
    f = _rgb()
    cl = oracle.bisecting_kmeans(f, 12)
    A = oracle.kernel_matrix(cl.centers, 0.1)
    P, rank, s = oracle.pinv(A)
    assert rank == A.shape[0]
    B = oracle.range_weights(f, cl.centers, 0.1)
    C = B @ P.T
    resid = np.abs(C @ A.T - B).max()
    assert resid <= 1e-10 * np.abs(A).max() * np.abs(C).max()
    # against Gaussian elimination, a different library routine
    assert np.abs(P - np.linalg.solve(A, np.eye(A.shape[0]))).max() < 1e-8 * np.abs(P).max()


def test_pinv_rank_deficient_penrose_conditions():
    mu = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [0.5, 0.5, 0.5], [0.9, 0.1, 0.4]])
    A = oracle.kernel_matrix(mu, 0.2)
    P, rank, _ = oracle.pinv(A)
    assert rank == 3
    assert np.abs(A @ P @ A - A).max() < 1e-12
    assert np.abs(P @ A @ P - P).max() < 1e-12
    assert np.abs(A @ P - (A @ P).T).max() < 1e-12
    assert np.abs(P @ A - (P @ A).T).max() < 1e-12


# ---------------------------------------------------------------------------
# X6: Theorem 1 for the hard-assignment variant, eqs. (17)-(20)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("noise,K", [(1e-4, 10), (0.05, 6)])
def test_theorem1_per_pixel_bound(noise, K):
    f = synth.voronoi_rgb(22, 25, 6, noise, 5)
    S, ss, sr = 5, 2.0, 0.15
    cl = oracle.bisecting_kmeans(f, K)
    A = oracle.kernel_matrix(cl.centers, sr)
    P, _, _ = oracle.pinv(A)
    gh, _ = oracle.fast_filter(f, f, cl.centers, P, ss, sr, S, coef="hard", labels=cl.labels)
    g, eta = oracle.bruteforce(f, f, ss, sr, S=S)
    n, H, W = f.shape
    L = math.exp(-0.5) / sr                      # Lipschitz constant of phi
    one = np.ones((H, W))
    Omega_W = ndi.convolve(one, oracle.spatial_kernel_2d(S, ss), mode="constant")
    X = f.reshape(3, -1).T.astype(np.float64)
    dist = np.sqrt(((X - cl.centers[cl.labels]) ** 2).sum(1)).reshape(H, W)
    R = 1.0
    bound = 2.0 * math.sqrt(n) * R * L * Omega_W * dist / eta
    err = np.sqrt(((gh - g) ** 2).sum(0))
    assert np.all(err <= bound * (1 + 1e-9) + 1e-13)
    # the summed form of eq. (19) with C = 4 n R^2 (sum_W omega)^2 / eta_min^2
    total = (err ** 2).sum()
    assert total <= 4 * n * R * R * L * L * Omega_W.max() ** 2 * cl.E_K / eta.min() ** 2 + 1e-20
    if noise < 1e-3:
        assert err.max() < 1e-3                  # informative regime


# ---------------------------------------------------------------------------
# X7: bisecting K-means (Sec. II-C)
# ---------------------------------------------------------------------------

def test_bisecting_hand_worked(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "bisect_1d.json")))
    pts = np.array(g["points"], dtype=np.float32).reshape(1, 1, -1)
    cl = oracle.bisecting_kmeans(pts, g["K"])
    assert cl.leaf_heap == g["leaf_heap"]
    assert cl.split_order == g["split_order"]
    np.testing.assert_allclose(cl.centers.ravel(), g["centers"], atol=0)
    np.testing.assert_allclose(cl.leaf_sse, g["leaf_sse"], atol=1e-15)
    assert cl.E_K == g["E_K"]
    assert cl.labels.tolist() == g["labels"]


def _golden_select(golden_dir):
    return json.load(open(os.path.join(golden_dir, "bisect_select.json")))["cases"]


@pytest.mark.parametrize("batched", [False, True])
def test_bisecting_split_selection_golden(golden_dir, batched):
    """The split-selection rule, hand-worked (tests/golden/bisect_select.json):
    the largest SSE is split even when another leaf has the larger SSE per
    member, and equal SSEs go to the lower heap id."""
    for g in _golden_select(golden_dir):
        pts = np.array(g["points"], dtype=np.float32).reshape(1, 1, -1)
        cl = oracle.bisecting_kmeans(pts, g["K"], batched=batched)
        assert cl.leaf_heap == g["leaf_heap"], g["name"]
        assert cl.split_order == g["split_order"], g["name"]
        np.testing.assert_array_equal(cl.centers.ravel(), g["centers"])
        np.testing.assert_array_equal(cl.leaf_sse, g["leaf_sse"])
        assert cl.E_K == g["E_K"]
        assert cl.labels.tolist() == g["labels"]


@pytest.mark.parametrize("wrong", ["variance", "higher_heap"])
def test_bisecting_split_selection_golden_discriminates(golden_dir, monkeypatch, wrong):
    """A plausible misreading planted in the oracle (split the largest SSE per
    member, or break ties towards the higher heap id) fails the golden."""
    key = {"variance": lambda nd: (-nd.sse / len(nd.idx), nd.heap),
           "higher_heap": lambda nd: (-nd.sse, -nd.heap)}[wrong]
    monkeypatch.setattr(oracle, "_split_key", key)
    mismatched = 0
    for g in _golden_select(golden_dir):
        pts = np.array(g["points"], dtype=np.float32).reshape(1, 1, -1)
        cl = oracle.bisecting_kmeans(pts, g["K"])
        mismatched += cl.leaf_heap != g["leaf_heap"]
    assert mismatched >= 1


def test_bisecting_invariants():
    f = _rgb(40, 44, 9, 0.05, 3)
    K = 20
    cl = oracle.bisecting_kmeans(f, K)
    X = f.reshape(3, -1).T.astype(np.float64)
    assert cl.centers.shape[0] == K
    assert sorted(set(cl.labels.tolist())) == list(range(K))          # covers, no empty
    for k in range(K):
        assert np.abs(X[cl.labels == k].mean(0) - cl.centers[k]).max() < 1e-15
    assert abs(cl.E_K - oracle.clustering_error(f, cl.centers, cl.labels)) < 1e-12 * cl.E_K
    assert all(a >= b - 1e-12 for a, b in zip(cl.E_history, cl.E_history[1:]))
    # heap ids: each leaf has a unique ancestor chain back to the root
    assert all(h >= 2 for h in cl.leaf_heap)
    batched = oracle.bisecting_kmeans(f, K, batched=True)
    assert batched.leaf_heap == cl.leaf_heap
    assert np.array_equal(batched.labels, cl.labels)
    assert np.array_equal(batched.centers, cl.centers)


def test_bisecting_split_is_lloyd_fixed_point():
    """A converged 2-means split: each member is no farther from its own child
    center than from the sibling's (the assignment rule of Sec. II-C)."""
    f = _rgb(30, 30, 5, 0.05, 4)
    rho = 3
    X32 = f.reshape(rho, -1).T.astype(np.float32)
    X = X32.astype(np.float64)
    root = oracle._node(1, np.arange(X.shape[0]), X, X32)
    A, B = oracle._two_means(root, X, X32, 100)
    assert root.lloyd_iters < 100
    da = ((X[A.idx] - A.mean) ** 2).sum(1)
    db = ((X[A.idx] - B.mean) ** 2).sum(1)
    assert np.all(da <= db)
    da = ((X[B.idx] - A.mean) ** 2).sum(1)
    db = ((X[B.idx] - B.mean) ** 2).sum(1)
    assert np.all(db < da)
    # the SSE decomposition of a split
    nA, nB = len(A.idx), len(B.idx)
    merge = nA * nB / (nA + nB) * ((A.mean - B.mean) ** 2).sum()
    assert abs(root.sse - (A.sse + B.sse + merge)) < 1e-10 * root.sse


def test_bisecting_stops_without_distinct_values():
    f = np.zeros((3, 6, 6), dtype=np.float32)
    f[:, :3] = 0.25
    cl = oracle.bisecting_kmeans(f, 5)
    assert cl.centers.shape[0] == 2 and cl.E_K == 0.0


# ---------------------------------------------------------------------------
# X8: linearity in f;  X9: invariances of the guide
# ---------------------------------------------------------------------------

def test_linearity_in_f():
    guide = _rgb()
    f1 = _rgb(seed=21).astype(np.float64)
    f2 = _rgb(seed=22).astype(np.float64)
    cl = oracle.bisecting_kmeans(guide, 8)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(cl.centers, 0.1))
    g1, _ = oracle.fast_filter(f1, guide, cl.centers, P, 2.0, 0.1, 6)
    g2, _ = oracle.fast_filter(f2, guide, cl.centers, P, 2.0, 0.1, 6)
    g12, _ = oracle.fast_filter(0.3 * f1 - 1.7 * f2, guide, cl.centers,
                                P, 2.0, 0.1, 6)
    assert np.abs(g12 - (0.3 * g1 - 1.7 * g2)).max() < 1e-12


def test_guide_invariances():
    f = _rgb(20, 22)
    g0, _ = oracle.bruteforce(f, f, 2.0, 0.12, S=5)
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    pf = f.reshape(3, -1).astype(np.float64)
    variants = {
        "translate": (pf + np.array([[0.3], [-0.2], [5.0]]), 0.12),
        "rotate": (Q @ pf, 0.12),
        "permute": (pf[[2, 0, 1]], 0.12),
        "scale": (pf * 3.0, 0.36),
    }
    for name, (pg, sr) in variants.items():
        g, _ = oracle.bruteforce(f, pg.reshape(f.shape), 2.0, sr, S=5)
        assert np.abs(g - g0).max() < 1e-10, name
    # O-2 with centers mapped alongside the guide
    cl = oracle.bisecting_kmeans(f, 7)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(cl.centers, 0.12))
    base, _ = oracle.fast_filter(f, f, cl.centers, P, 2.0, 0.12, 5)
    t = np.array([0.3, -0.2, 5.0])
    out, _ = oracle.fast_filter(f, (pf + t[:, None]).reshape(f.shape), cl.centers + t, P,
                                2.0, 0.12, 5)
    assert np.abs(out - base).max() < 1e-10
    out, _ = oracle.fast_filter(f, (Q @ pf).reshape(f.shape), cl.centers @ Q.T, P, 2.0, 0.12, 5)
    assert np.abs(out - base).max() < 1e-10


def test_small_sigma_r_distinct_guide_is_identity():
    """X10: with all guide vectors distinct and sigma_r tiny, only the centre
    sample has weight 1, so g = f exactly."""
    H, W = 9, 11
    f = np.random.default_rng(1).uniform(size=(3, H, W))
    guide = np.arange(H * W, dtype=np.float64).reshape(1, H, W) * 1e-3
    out, eta = oracle.bruteforce(f, guide, 2.0, 1e-6, S=4)
    assert np.array_equal(out, f)
    assert np.all(eta == 1.0)


# ---------------------------------------------------------------------------
# Convolution forms and the sampled evaluator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("spatial", ["gaussian", "box"])
def test_conv_forms_agree_with_scipy(spatial):
    u = np.random.default_rng(3).normal(size=(2, 17, 23))
    w = oracle.spatial_kernel_2d(4, 1.3, spatial)
    ref = np.stack([ndi.convolve(u[c], w, mode="constant") for c in range(2)])
    assert np.abs(oracle.conv(u, 4, 1.3, spatial, "direct") - ref).max() < 1e-12
    assert np.abs(oracle.conv(u, 4, 1.3, spatial, "separable") - ref).max() < 1e-12


def test_sampled_evaluator_matches_full():
    f = _rgb(19, 27)
    res = oracle.fhd_filter(f, f, 2.0, 0.1, 9, S=6)
    ys = np.array([0, 3, 18, 10, 18])
    xs = np.array([0, 26, 0, 13, 26])
    g, den = oracle.fast_filter_at(f, f, res.centers, res.P, 2.0, 0.1, ys, xs, S=6)
    assert np.abs(g - res.out[:, ys, xs].T).max() < 1e-13
    assert np.abs(den - res.den[ys, xs]).max() < 1e-12
    gb, eb = oracle.bruteforce_at(f, f, 2.0, 0.1, ys, xs, S=6)
    full, eta = oracle.bruteforce(f, f, 2.0, 0.1, S=6)
    assert np.abs(gb - full[:, ys, xs].T).max() < 1e-15


def test_o2_torch_transcription_agrees():
    f = _rgb(14, 15)
    res = oracle.fhd_filter(f, f, 2.0, 0.1, 6, S=5)
    t = torch.tensor(f, dtype=torch.float64)
    g, r = ar.fast_filter_torch(t, t, res.centers, 2.0, 0.1, 5)
    assert np.abs(g.numpy() - res.out).max() < 1e-12


# ---------------------------------------------------------------------------
# X12: patch-PCA guide (Sec. III-C)
# ---------------------------------------------------------------------------

def test_patches_and_pca():
    f = _rgb(9, 10)
    P = oracle.patches(f, 5)
    # half-sample symmetric extension: pixel (0,0), offset (-2,-2) reads (1,1)
    assert P[0, 0] == f[0, 1, 1]
    # flatten order (dy, dx, c): entry for (dy=2, dx=2, c=1) is the pixel itself
    i = 4 * 10 + 7
    assert P[i, (2 * 5 + 2) * 3 + 1] == f[1, 4, 7]
    g, lam, basis, mean = oracle.nlm_guide(f, 5, 75)
    X = P - mean
    cov = X.T @ X / X.shape[0]
    assert np.abs(cov @ basis - basis * lam[None, :]).max() < 1e-10
    G = g.reshape(75, -1).T
    i, j = 3, 71
    assert abs(((G[i] - G[j]) ** 2).sum() - ((P[i] - P[j]) ** 2).sum()) < 1e-10
    assert np.all(np.diff(lam) <= 1e-15)


# ---------------------------------------------------------------------------
# eq. (21)
# ---------------------------------------------------------------------------

def test_psnr_definition():
    a = np.zeros((3, 4, 5))
    b = a + 0.1
    assert abs(oracle.mse(a, b) - 0.03) < 1e-15
    assert abs(oracle.psnr(a, b) - (-10 * math.log10(0.03))) < 1e-12


def test_generators_deterministic():
    a = synth.workload_input("bf_rgb_256")
    b = synth.workload_input("bf_rgb_256")
    assert a.shape == (3, 256, 256) and a.dtype == np.float32
    assert np.array_equal(a, b)
    assert a.min() >= 0 and a.max() <= 1
    h = synth.hyperspectral(16, 16, 32, 5, 0.5, 0.02, 1002)
    assert h.shape == (32, 16, 16)
    sizes = synth.batch_sizes()
    assert len(sizes) == 16 and sizes[0] == (384, 384) and sizes[-1] == (768, 1024)
