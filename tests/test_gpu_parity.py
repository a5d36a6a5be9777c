"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Steps 2-5 of Algorithm 1 are compared element by element with the oracle fed
the same FP32 centers (max-abs 1e-4 on the FP32 path).  The clustering
(step 1) is checked against the oracle's tree and against the invariants of
bisecting K-means.  The brute force is checked against the oracle's eqs.
(1)-(2).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def fhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_02363_amd as m
    m.load()
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _oracle_o2(f, guide, centers, ss, sr, S, spatial, coef="lsq", labels=None):
    A = oracle.kernel_matrix(np.asarray(centers, np.float64), sr)
    P, rank, _ = oracle.pinv(A)
    return oracle.fast_filter(f, guide, np.asarray(centers, np.float64), P, ss, sr, S, spatial,
                              conv_method="direct" if f.shape[1] * f.shape[2] <= 70000 else "separable",
                              coef=coef, labels=labels)


CASES = [
    # name, H, W, K, sigma_s, S, sigma_r, spatial
    ("c0_full_256", 256, 256, 16, 3.0, 9, 0.1, "gaussian"),
    ("ragged_77x93", 77, 93, 12, 2.0, 6, 0.12, "gaussian"),
    ("tall_301x40", 301, 40, 8, 5.0, 15, 0.1, "gaussian"),
    ("wide_33x517_S20", 33, 517, 10, 6.7, 21, 0.15, "gaussian"),
    ("box_120x130_S10", 120, 130, 16, None, 10, 0.2, "box"),
    ("large_radius_64x70_S40", 64, 70, 6, 13.3, 40, 0.2, "gaussian"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_filter_centers_rgb(fhd, case):
    name, H, W, K, ss, S, sr, spatial = case
    f = synth.voronoi_rgb(H, W, 24, 0.05, 1000 + H)
    cl = oracle.bisecting_kmeans(f, K)
    c32 = cl.centers.astype(np.float32)
    ref, rden = _oracle_o2(f, f, c32, ss, sr, S, spatial)
    fd = _dev(f)
    out, den = fhd.filter_centers(fd, fd, c32, sigma_s=ss, sigma_r=sr, spatial=spatial, radius=S,
                                  return_den=True)
    err = np.abs(out.cpu().numpy() - ref).max()
    derr = np.abs(den.cpu().numpy() - rden).max() / np.abs(rden).max()
    print(f"{name}: max-abs {err:.3e}, den rel {derr:.3e}")
    assert err < TOL
    assert derr < 1e-5


def test_filter_centers_joint_guide_materialized(fhd):
    """A 16-dimensional guide (weights pass + planes of b and c)."""
    H, W, K = 70, 90, 20
    f = synth.voronoi_rgb(H, W, 20, 0.05, 77)
    g = synth.hyperspectral(H, W, 16, 5, 0.5, 0.02, 78)
    cl = oracle.bisecting_kmeans(g, K)
    c32 = cl.centers.astype(np.float32)
    ref, _ = _oracle_o2(f, g, c32, 2.0, 0.25, 6, "gaussian")
    out = fhd.filter_centers(_dev(f), _dev(g), c32, sigma_s=2.0, sigma_r=0.25, radius=6)
    err = np.abs(out.cpu().numpy() - ref).max()
    print(f"joint 16-d guide: max-abs {err:.3e}")
    assert err < TOL


def test_filter_centers_hyperspectral(fhd):
    """n = rho = 32 (33 channels per cluster, several channel groups)."""
    H, W, K = 48, 52, 24
    f = synth.hyperspectral(H, W, 32, 5, 0.5, 0.02, 1002)
    cl = oracle.bisecting_kmeans(f, K)
    c32 = cl.centers.astype(np.float32)
    ref, _ = _oracle_o2(f, f, c32, 2.0, 0.2, 6, "gaussian")
    out = fhd.filter_centers(_dev(f), _dev(f), c32, sigma_s=2.0, sigma_r=0.2, radius=6)
    err = np.abs(out.cpu().numpy() - ref).max()
    print(f"hyperspectral 32 bands: max-abs {err:.3e}")
    assert err < TOL


@pytest.mark.parametrize("rho", [3, 16])
def test_filter_centers_hard_variant(fhd, rho):
    """Eqs. (17)-(18): coefficients are the cluster indicator."""
    H, W, K = 60, 75, 10
    f = synth.voronoi_rgb(H, W, 12, 0.05, 5)
    g = f if rho == 3 else synth.hyperspectral(H, W, 16, 5, 0.5, 0.02, 9)
    cl = oracle.bisecting_kmeans(g, K)
    c32 = cl.centers.astype(np.float32)
    ref, _ = _oracle_o2(f, g, c32, 2.0, 0.15, 6, "gaussian", coef="hard", labels=cl.labels)
    lab = torch.from_numpy(cl.labels.reshape(H, W).astype(np.int32)).cuda()
    out = fhd.filter_centers(_dev(f), _dev(g), c32, sigma_s=2.0, sigma_r=0.15, radius=6,
                             coef="hard", labels=lab)
    err = np.abs(out.cpu().numpy() - ref).max()
    print(f"hard rho={rho}: max-abs {err:.3e}")
    assert err < TOL


def _check_tree(fhd, g, K, name):
    gd = _dev(g)
    cen, lab, info = fhd.cluster(gd, K, labels=True)
    cl = oracle.bisecting_kmeans(g, K)
    lab = lab.cpu().numpy().reshape(-1)
    rho = g.shape[0]
    X = g.reshape(rho, -1).T.astype(np.float64)
    Ke = cen.shape[0]
    # partition covers the image; each center is the mean of its members
    assert sorted(set(lab.tolist())) == list(range(Ke))
    for k in range(Ke):
        m = X[lab == k].mean(0)
        assert np.abs(m - cen[k].numpy()).max() <= 1e-6 * max(1.0, np.abs(m).max())
    EK = oracle.clustering_error(g, cen.numpy().astype(np.float64), lab)
    print(f"{name}: K_eff {Ke} (oracle {len(cl.centers)}), E_K {info['E_K']:.6g} vs oracle "
          f"{cl.E_K:.6g}, rounds {info['kmeans_rounds']}, splits {info['kmeans_splits']}, "
          f"same labels {np.array_equal(lab, cl.labels)}")
    assert Ke == len(cl.centers)
    assert abs(info["E_K"] - EK) <= 1e-6 * EK + 1e-12
    assert 0.98 <= (info["E_K"] + 1e-30) / (cl.E_K + 1e-30) <= 1.02
    return cen, lab, cl


@pytest.mark.parametrize("shape,K", [((3, 64, 80), 16), ((3, 256, 256), 16), ((3, 97, 41), 40)])
def test_cluster_against_oracle(fhd, shape, K):
    g = synth.voronoi_rgb(shape[1], shape[2], 30, 0.05, 17 + K)
    _check_tree(fhd, g, K, f"rgb {shape} K={K}")


def test_cluster_high_dimensional(fhd):
    g = synth.hyperspectral(40, 44, 32, 5, 0.5, 0.02, 3)
    _check_tree(fhd, g, 24, "hyperspectral 32-d K=24")


def test_cluster_fewer_distinct_values(fhd):
    """K larger than the number of distinct guide vectors: K_eff = #distinct,
    E_K = 0 (X3 setting)."""
    g = synth.voronoi_rgb(50, 60, 7, 0.0, 11)
    distinct = np.unique(g.reshape(3, -1).T, axis=0).shape[0]
    cen, lab, cl = _check_tree(fhd, g, distinct + 5, "piecewise constant")
    assert cen.shape[0] == distinct


def test_enough_clusters_matches_bruteforce(fhd):
    """X3 on the GPU: a piecewise-constant guide with K >= #distinct values
    reproduces the brute force."""
    f = synth.voronoi_rgb(64, 72, 7, 0.0, 11)
    ref, _ = oracle.bruteforce(f, f, 2.5, 0.2, S=8)
    out = fhd.filter(_dev(f), sigma_s=2.5, sigma_r=0.2, K=12, radius=8)
    err = np.abs(out.cpu().numpy() - ref).max()
    print(f"K >= distinct vs brute force: max-abs {err:.3e}")
    assert err < 1e-5


def test_filter_end_to_end_c0(fhd):
    """The whole of Algorithm 1 on the 256x256 RGB workload vs the oracle's
    own clustering and filter, and its PSNR vs the brute force, eq. (21)."""
    f = synth.workload_input("bf_rgb_256")
    res = oracle.fhd_filter(f, f, 3.0, 0.1, 16, S=9)
    out, den, cen, info = fhd.filter(_dev(f), sigma_s=3.0, sigma_r=0.1, K=16, return_den=True,
                                     return_centers=True, info=True)
    cerr = np.abs(cen.numpy() - res.centers).max()
    err = np.abs(out.cpu().numpy() - res.out).max()
    bf, _ = oracle.bruteforce(f, f, 3.0, 0.1, S=9)
    p_gpu = oracle.psnr(out.cpu().numpy(), bf)
    p_ref = oracle.psnr(res.out, bf)
    print(f"c0 end to end: centers {cerr:.2e}, max-abs {err:.3e}, PSNR gpu {p_gpu:.3f} dB, "
          f"oracle {p_ref:.3f} dB, info {info}")
    assert cerr < 1e-6
    assert err < TOL
    assert abs(p_gpu - p_ref) < 0.01


def test_bruteforce_against_oracle(fhd):
    f = synth.voronoi_rgb(90, 110, 20, 0.05, 4)
    ref, eta = oracle.bruteforce(f, f, 3.0, 0.1, S=9)
    out, den = fhd.bruteforce(_dev(f), sigma_s=3.0, sigma_r=0.1, radius=9, return_den=True)
    err = np.abs(out.cpu().numpy() - ref).max()
    derr = np.abs(den.cpu().numpy() - eta).max() / eta.max()
    print(f"brute force: max-abs {err:.3e}, eta rel {derr:.3e}")
    assert err < TOL and derr < 1e-5
    g = synth.hyperspectral(40, 50, 32, 5, 0.5, 0.02, 8)
    ref, _ = oracle.bruteforce(g, g, 2.0, 0.2, S=6)
    out = fhd.bruteforce(_dev(g), sigma_s=2.0, sigma_r=0.2, radius=6)
    err = np.abs(out.cpu().numpy() - ref).max()
    print(f"brute force 32 bands: max-abs {err:.3e}")
    assert err < TOL


def test_edge_cases(fhd):
    # constant image: returned unchanged (X1)
    f = np.empty((3, 40, 50), np.float32)
    f[:] = np.array([0.2, 0.5, 0.9], np.float32)[:, None, None]
    g = synth.voronoi_rgb(40, 50, 10, 0.05, 1)
    out = fhd.filter(_dev(f), _dev(g), sigma_s=2.0, sigma_r=0.1, K=8)
    assert np.abs(out.cpu().numpy() - f).max() < 1e-6
    out = fhd.filter(_dev(f), sigma_s=2.0, sigma_r=0.1, K=8)      # self-guided: K_eff = 1
    assert np.abs(out.cpu().numpy() - f).max() < 1e-6
    # sigma_r = inf: the normalised spatial filter (X2)
    f = synth.voronoi_rgb(37, 45, 10, 0.05, 2)
    ref, _ = oracle.bruteforce(f, f, 2.0, math.inf, S=6)
    out = fhd.filter(_dev(f), sigma_s=2.0, sigma_r=math.inf, K=5, radius=6)
    assert np.abs(out.cpu().numpy() - ref).max() < TOL
    # K = 1 (X4)
    res = oracle.fhd_filter(f, f, 2.0, 0.2, 1, S=6)
    out = fhd.filter(_dev(f), sigma_s=2.0, sigma_r=0.2, K=1, radius=6)
    assert np.abs(out.cpu().numpy() - res.out).max() < TOL
    # tiny images: 1x1, one row, one column
    for (H, W) in [(1, 1), (1, 37), (29, 1), (5, 3)]:
        f = synth.voronoi_rgb(H, W, 3, 0.05, H * 100 + W)
        K = min(4, H * W)
        res = oracle.fhd_filter(f, f, 1.5, 0.2, K, S=4)
        out = fhd.filter_centers(_dev(f), _dev(f), res.centers.astype(np.float32), sigma_s=1.5,
                                 sigma_r=0.2, radius=4)
        err = np.abs(out.cpu().numpy() - _oracle_o2(f, f, res.centers.astype(np.float32), 1.5,
                                                   0.2, 4, "gaussian")[0]).max()
        print(f"tiny {H}x{W}: max-abs {err:.3e}")
        assert err < TOL
        out = fhd.filter(_dev(f), sigma_s=1.5, sigma_r=0.2, K=K, radius=4)
        assert np.isfinite(out.cpu().numpy()).all()


def test_invalid_arguments(fhd):
    f = _dev(synth.voronoi_rgb(16, 16, 4, 0.05, 1))
    for kw in [dict(K=0), dict(K=1000), dict(sigma_r=-1.0), dict(sigma_s=0.0)]:
        args = dict(sigma_s=2.0, sigma_r=0.1, K=4)
        args.update(kw)
        with pytest.raises(fhd.FHDError):
            fhd.filter(f, **args)
    with pytest.raises(fhd.FHDError):
        fhd.filter(f, K=300)                                   # K > pixels
    g = _dev(synth.voronoi_rgb(16, 16, 4, 0.05, 2))
    # output aliasing an input
    with pytest.raises(fhd.FHDError):
        p = fhd.make_params(sigma_s=2.0, sigma_r=0.1, K=4)
        ctx = fhd._ctx(0)
        fhd._check(fhd.load().fhd_filter(ctx, fhd._dev(f, "f"), 3, fhd._dev(g, "g"), 3, 16, 16,
                                         __import__("ctypes").byref(p), fhd._dev(f, "out"),
                                         None, None, None, None, 0), ctx)


def test_c1_full_size_sampled(fhd):
    """The 2048x2048 RGB workload in the benchmark's configuration: sampled
    outputs against the oracle's eqs. (13)-(16) evaluated pixel by pixel with
    the GPU's centers, plus brute-force samples for the PSNR estimate."""
    cfg = synth.WORKLOADS["bf_rgb_2048"]
    f = synth.workload_input("bf_rgb_2048")
    fd = _dev(f)
    out, cen, info = fhd.filter(fd, sigma_s=cfg["sigma_s"], sigma_r=cfg["sigma_r"], K=cfg["K"],
                                return_centers=True, info=True)
    out = out.cpu().numpy()
    rng = np.random.default_rng(5)
    ys = np.concatenate([rng.integers(0, 2048, 200), [0, 0, 2047, 2047, 1024]])
    xs = np.concatenate([rng.integers(0, 2048, 200), [0, 2047, 0, 2047, 7]])
    c = cen.numpy().astype(np.float64)
    A = oracle.kernel_matrix(c, cfg["sigma_r"])
    P, _, _ = oracle.pinv(A)
    ref, _ = oracle.fast_filter_at(f, f, c, P, cfg["sigma_s"], cfg["sigma_r"], ys, xs, S=cfg["S"])
    err = np.abs(out[:, ys, xs].T - ref).max()
    bf, _ = oracle.bruteforce_at(f, f, cfg["sigma_s"], cfg["sigma_r"], ys, xs, S=cfg["S"])
    mse = ((out[:, ys, xs].T - bf) ** 2).sum() / len(ys)
    print(f"c1 sampled: max-abs {err:.3e}, sampled PSNR vs brute {-10 * np.log10(mse):.2f} dB, "
          f"info {info}")
    assert err < TOL
