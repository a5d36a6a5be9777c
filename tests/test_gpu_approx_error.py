"""The error of the kernel approximation (fhd_approx_error: eq. (10) at
c(i) = A^+ b(i), its pixel mean E_ls of Sec. II-A) through the C ABI, against
the FP64 oracle fed the same FP32 centers.

Tolerance.  The GPU forms every residual r = phi(x - p(i)) - sum_k c_k phi(x -
mu_k) in FP32.  Its error is at most tau (1 + sum_l |c_l(i)| + sum_lk |A^+_lk|
b_k(i)) with tau = 1e-6 (a few FP32 roundings and the fast exponential's
relative error on the terms that make up c and the fit).  By the triangle
inequality on the vector of a pixel's residuals, |sqrt(err_gpu) -
sqrt(err_ref)| <= sqrt(|Theta_i|) times that bound; the test checks this per
pixel (the terms come from the oracle) and E_ls within the bound's mean.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TAU = 1e-6


@pytest.fixture(scope="module")
def fhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_02363_amd as m
    m.load()
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _bound(g, cen, sr, S):
    """Per-pixel bound on |sqrt(err_gpu) - sqrt(err_ref)|."""
    rho, H, W = g.shape
    mu = cen.astype(np.float64)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(mu, sr))
    X = g.reshape(rho, -1).T.astype(np.float64)
    B = oracle.phi(((X[:, None, :] - mu[None]) ** 2).sum(-1), sr)
    C = B @ P.T
    M = 1.0 + np.abs(C).sum(1) + B @ np.abs(P).sum(0)
    ys, xs = np.mgrid[0:H, 0:W]
    ny = np.minimum(ys + S, H - 1) - np.maximum(ys - S, 0) + 1
    nx = np.minimum(xs + S, W - 1) - np.maximum(xs - S, 0) + 1
    return np.sqrt(ny * nx) * TAU * M.reshape(H, W)


CASES = [
    # name, guide kind, H, W, rho, K, sigma_r, spatial, sigma_s, radius
    ("rgb_77x93_K12_gauss", "rgb", 77, 93, 3, 12, 0.12, "gaussian", 2.0, None),
    ("rgb_64x64_K64_box", "rgb", 64, 64, 3, 64, 0.2, "box", None, 4),
    ("rho7_45x50_K20", "hyper", 45, 50, 7, 20, 0.3, "gaussian", 1.5, None),
    ("rho32_40x37_K24_box", "hyper", 40, 37, 32, 24, 0.4, "box", None, 3),
    ("one_pixel_K1", "rgb", 1, 1, 3, 1, 0.1, "gaussian", 2.0, None),
    ("rho33_24x21_K64_box", "hyper", 24, 21, 33, 64, 0.5, "box", None, 2),  # largest LDS footprint
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_approx_error_parity(fhd, case):
    name, kind, H, W, rho, K, sr, spatial, ss, radius = case
    if kind == "rgb":
        g = synth.voronoi_rgb(H, W, 16, 0.05, 300 + H)
    else:
        g = synth.hyperspectral(H, W, rho, 4, 0.5, 0.02, 400 + rho)
    cen = oracle.bisecting_kmeans(g, K).centers.astype(np.float32)
    S = radius if radius is not None else oracle.default_radius(ss)
    ref, Els = oracle.approx_error(g, cen, sr, S)
    err, m = fhd.approx_error(_dev(g), cen, sigma_r=sr, sigma_s=ss if ss else 3.0, radius=radius,
                              spatial=spatial)
    torch.cuda.synchronize()
    e = err.cpu().numpy().astype(np.float64)
    bnd = _bound(g, cen, sr, S)
    dev = np.abs(np.sqrt(e) - np.sqrt(ref))
    ratio = float((dev / bnd).max())
    mbound = float(np.mean(bnd * (2.0 * np.sqrt(ref) + bnd)))
    print(f"{name}: E_ls gpu {m:.6e} oracle {Els:.6e}; max |sqrt err diff| / bound {ratio:.3f}")
    assert ratio <= 1.0
    assert abs(m - Els) <= mbound
    # the per-pixel values the GPU returned average to its own E_ls
    assert abs(e.mean() - m) <= 1e-6 * max(m, 1e-30) + 1e-12


def test_approx_error_exact_cases(fhd):
    rng = np.random.default_rng(8)
    vals = rng.uniform(0, 1, (5, 3)).astype(np.float32)
    lab = rng.integers(0, 5, (30, 41))
    g = np.ascontiguousarray(np.transpose(vals[lab], (2, 0, 1)))
    err, m = fhd.approx_error(_dev(g), vals, sigma_r=0.4, radius=3, spatial="box")
    assert m < 1e-9 and float(err.max()) < 1e-8
    f = synth.voronoi_rgb(20, 30, 6, 0.05, 9)
    cen = oracle.bisecting_kmeans(f, 4).centers.astype(np.float32)
    err, m = fhd.approx_error(_dev(f), cen, sigma_r=math.inf, radius=2, spatial="box")
    assert m < 1e-10


def test_approx_error_rejections(fhd):
    g = _dev(synth.voronoi_rgb(16, 16, 4, 0.05, 1))
    cen = np.zeros((65, 3), np.float32)
    with pytest.raises(fhd.FHDError) as e:
        fhd.approx_error(g, cen, sigma_r=0.1, radius=2, spatial="box")
    assert e.value.status == fhd.FHD_EUNSUPPORTED
    with pytest.raises(fhd.FHDError) as e:
        fhd.approx_error(g, cen[:4], sigma_r=0.1, spatial="young")
    assert e.value.status == fhd.FHD_EINVAL
    with pytest.raises(fhd.FHDError):
        fhd.approx_error(g, cen[:4, :2], sigma_r=0.1)
    _, m = fhd.approx_error(g, np.asarray(synth.voronoi_rgb(16, 16, 4, 0.05, 1)[:, 0, :4].T), sigma_r=0.1,
                            radius=1, spatial="box", per_pixel=False)
    assert np.isfinite(m)
