"""Algorithm 1 on a 3-D domain (fhd_filter_volume) through the C ABI, against
the FP64 oracle: the clustering tree (centers equal in FP32) and the output
of the oracle's own run of the whole algorithm, max-abs 1e-4 (the FP32
path's bar; cond(A) checked so that the bar is meaningful).  One slice equals
the 2-D path within the same bar.  The GPU brute force on volumes against
the oracle's, max-abs 1e-4 (and its normaliser 1e-5 relative).
"""
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


def _rgb_volume(D, H, W, seed):
    return np.stack([synth.voronoi_rgb(H, W, 8, 0.05, seed + z) for z in range(D)], axis=1)


CASES = [
    # name, D, H, W, K, sigma_s, radius, sigma_r, spatial, separate guide bands
    ("rgb_7x23x29_gauss", 7, 23, 29, 8, 1.5, None, 0.15, "gaussian", 0),
    ("rgb_5x16x40_box", 5, 16, 40, 12, None, 2, 0.2, "box", 0),
    ("guide5_4x19x21_gauss", 4, 19, 21, 10, 1.0, None, 0.3, "gaussian", 5),
    ("rgb_6x20x24_K24_cond500", 6, 20, 24, 24, 1.2, None, 0.3, "gaussian", 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_volume_end_to_end(fhd, case):
    name, D, H, W, K, ss, radius, sr, spatial, bands = case
    f = _rgb_volume(D, H, W, 700 if K == 24 else 500 + D)
    if bands:
        g = np.stack([synth.hyperspectral(H, W, bands, 3, 0.5, 0.02, 600 + z) for z in range(D)], axis=1)
    else:
        g = f
    S = radius if radius is not None else oracle.default_radius(ss)
    res = oracle.fhd_filter_volume(f, g, ss, sr, K, S, spatial)
    cond = float(np.linalg.cond(res.A))
    out, den, cen = fhd.filter_volume(_dev(f), None if not bands else _dev(g), sigma_s=ss if ss else 3.0,
                                      sigma_r=sr, K=K, spatial=spatial, radius=radius, return_den=True,
                                      return_centers=True)
    torch.cuda.synchronize()
    cerr = np.abs(cen.numpy() - res.centers).max()
    err = np.abs(out.cpu().numpy() - res.out).max()
    derr = np.abs(den.cpu().numpy() - res.den).max() / np.abs(res.den).max()
    bf, _ = oracle.bruteforce_volume(f, g, ss, sr, S, spatial)
    print(f"{name}: cond(A) {cond:.0f}, centers {cerr:.2e}, max-abs {err:.2e}, den rel {derr:.2e}, "
          f"PSNR vs 3-D brute force gpu {oracle.psnr(out.cpu().numpy(), bf):.2f} / oracle "
          f"{oracle.psnr(res.out, bf):.2f} dB")
    assert cond < 2e4
    assert cerr < 1e-6 and err < TOL and derr < 1e-5


@pytest.mark.parametrize("spatial,ss,radius", [("gaussian", 1.3, None), ("box", None, 2)])
def test_bruteforce_volume(fhd, spatial, ss, radius):
    f = _rgb_volume(5, 18, 22, 900)
    g = np.stack([synth.hyperspectral(18, 22, 4, 3, 0.5, 0.02, 950 + z) for z in range(5)], axis=1)
    S = radius if radius is not None else oracle.default_radius(ss)
    ref, eta = oracle.bruteforce_volume(f, g, ss, 0.25, S, spatial)
    out, den = fhd.bruteforce_volume(_dev(f), _dev(g), sigma_s=ss if ss else 3.0, sigma_r=0.25, spatial=spatial,
                                     radius=radius, return_den=True)
    torch.cuda.synchronize()
    err = np.abs(out.cpu().numpy() - ref).max()
    derr = np.abs(den.cpu().numpy() - eta).max() / eta.max()
    print(f"3-D brute force {spatial}: max-abs {err:.2e}, eta rel {derr:.2e}")
    assert err < TOL and derr < 1e-5


def test_volume_six_channels(fhd):
    """n = 6 (the brute force's two channel groups, six planes per cluster)."""
    f = np.stack([synth.hyperspectral(15, 18, 6, 3, 0.5, 0.02, 980 + z) for z in range(4)], axis=1)
    res = oracle.fhd_filter_volume(f, f, 1.0, 0.3, 10, 3)
    out, cen = fhd.filter_volume(_dev(f), sigma_s=1.0, sigma_r=0.3, K=10, return_centers=True)
    ref, _ = oracle.bruteforce_volume(f, f, 1.0, 0.3, 3)
    bf = fhd.bruteforce_volume(_dev(f), sigma_s=1.0, sigma_r=0.3)
    torch.cuda.synchronize()
    cerr = np.abs(cen.numpy() - res.centers).max()
    err = np.abs(out.cpu().numpy() - res.out).max()
    berr = np.abs(bf.cpu().numpy() - ref).max()
    print(f"six channels: cond(A) {np.linalg.cond(res.A):.0f}, centers {cerr:.2e}, max-abs {err:.2e}, "
          f"brute force max-abs {berr:.2e}")
    assert np.linalg.cond(res.A) < 2e4
    assert cerr < 1e-6 and err < TOL and berr < TOL


def test_volume_hard_variant(fhd):
    """Eqs. (17)-(18) on a volume: the indicator of each voxel's own cluster
    (labels from the library's clustering, equal to the oracle's)."""
    f = _rgb_volume(5, 21, 26, 820)
    res = oracle.fhd_filter_volume(f, f, 1.5, 0.15, 12, 4, coef="hard")
    out, cen = fhd.filter_volume(_dev(f), sigma_s=1.5, sigma_r=0.15, K=12, radius=4, coef="hard",
                                 return_centers=True)
    torch.cuda.synchronize()
    cerr = np.abs(cen.numpy() - res.centers).max()
    err = np.abs(out.cpu().numpy() - res.out).max()
    print(f"hard variant on a volume: centers {cerr:.2e}, max-abs {err:.2e}")
    assert cerr < 1e-6 and err < TOL


def test_one_slice_equals_the_2d_path(fhd):
    f = synth.voronoi_rgb(40, 52, 10, 0.05, 77)
    a = fhd.filter_volume(_dev(f[:, None]), sigma_s=2.0, sigma_r=0.15, K=12)
    b = fhd.filter(_dev(f), sigma_s=2.0, sigma_r=0.15, K=12)
    torch.cuda.synchronize()
    err = float((a[:, 0] - b).abs().max())
    print(f"one slice vs 2-D: max-abs {err:.2e}")
    assert err < TOL


def test_volume_rejections(fhd):
    v = _dev(_rgb_volume(2, 8, 8, 1))
    with pytest.raises(fhd.FHDError) as e:
        fhd.filter_volume(v, sigma_s=2.0, K=4, spatial="young")
    assert e.value.status == fhd.FHD_EUNSUPPORTED
    tall = _dev(np.zeros((1, 300, 300, 1)))
    with pytest.raises(fhd.FHDError) as e:
        fhd.filter_volume(tall, K=2)
    assert e.value.status == fhd.FHD_EUNSUPPORTED
    with pytest.raises(fhd.FHDError):
        fhd.filter_volume(v, _dev(np.zeros((3, 2, 8, 7))), K=4)
