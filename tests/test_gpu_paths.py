"""Parity of the window forms and call paths that the workloads do not reach,
through the C ABI, against the FP64 oracle fed the same FP32 centers.

* The box window (Sec. II-C) on every kernel that forms it: unit taps of the
  FIR kernels (rows below radius 26, columns below 8), the row pass's
  wave-scan running sum (radius 26 and above), the column running sum
  (radii 8..64, tiers up to 16, 32 and 64) and the generic column kernel
  beyond; rows split into several runs, ragged tiles, windows wider than the
  image.
* The generic Gaussian kernels (tap by tap) at radii beyond the unrolled
  1..32, with inline weights (3-d guide), materialised weight planes (12-d
  guide) and the hard variant of eq. (17), on ragged sizes, some smaller than
  the window.
* Radius 0 (the window is the pixel itself: g_hat = f wherever r_hat != 0),
  and radii above 96, where a row-pass block's halo run is longer than its
  threads.
* The normaliser diagnostics of fhd_info (den_min, den_nonpos, den_small,
  nonfinite) against the returned r_hat and output, and strict mode's
  FHD_ENUMERIC on a nonlocal-means crop whose r_hat goes through zero, with
  the signs of r_hat checked against the oracle's.
* A context moved between two streams (fhd_set_stream) orders the new
  stream after the work of the old one: outputs equal those of calls made
  one at a time.
* The split selection of the bisecting K-means on the hand-worked golden
  cases (largest SSE, not SSE per member; ties to the lower heap id).
"""
import json
import math
import os

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


def _dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _o2(f, guide, centers, ss, sr, S, spatial, coef="lsq", labels=None, terms=False):
    c = np.asarray(centers, np.float64)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(c, sr))
    return oracle.fast_filter(f, guide, c, P, ss, sr, S, spatial, conv_method="direct", coef=coef,
                              labels=labels, return_terms=terms)


GENERIC = [
    # name, H, W, guide dims, K, spatial, S, sigma_s, sigma_r, coef
    ("box_S1_inline_50x77", 50, 77, 3, 8, "box", 1, None, 0.15, "lsq"),
    ("box_S2_planes_45x61", 45, 61, 12, 9, "box", 2, None, 0.3, "lsq"),
    ("box_S10_inline_131x500", 131, 500, 3, 16, "box", 10, None, 0.15, "lsq"),
    ("box_S10_planes_97x301", 97, 301, 12, 10, "box", 10, None, 0.3, "lsq"),
    ("box_S10_hard_88x150", 88, 150, 3, 12, "box", 10, None, 0.15, "hard"),
    ("box_S16_hard_64x64", 64, 64, 3, 7, "box", 16, None, 0.15, "hard"),
    ("box_S17_inline_70x260", 70, 260, 3, 10, "box", 17, None, 0.15, "lsq"),
    ("box_S26_inline_90x530", 90, 530, 3, 12, "box", 26, None, 0.15, "lsq"),
    ("box_S28_hard_70x130", 70, 130, 3, 9, "box", 28, None, 0.15, "hard"),
    ("box_S32_inline_100x90", 100, 90, 3, 8, "box", 32, None, 0.2, "lsq"),
    ("box_S32_planes_40x300", 40, 300, 12, 8, "box", 32, None, 0.3, "lsq"),
    ("box_S40_inline_75x97", 75, 97, 3, 8, "box", 40, None, 0.15, "lsq"),
    ("box_S64_inline_150x140", 150, 140, 3, 8, "box", 64, None, 0.15, "lsq"),
    ("box_S70_planes_160x90", 160, 90, 12, 8, "box", 70, None, 0.3, "lsq"),
    ("box_S70_hard_150x150", 150, 150, 3, 8, "box", 70, None, 0.15, "hard"),
    ("box_S40_inline_150x131", 150, 131, 3, 12, "box", 40, None, 0.12, "lsq"),
    ("box_S33_planes_90x70", 90, 70, 12, 10, "box", 33, None, 0.3, "lsq"),
    ("box_S40_hard_80x101", 80, 101, 3, 9, "box", 40, None, 0.15, "hard"),
    ("gauss_S40_planes_70x83", 70, 83, 12, 10, "gaussian", 40, 13.3, 0.3, "lsq"),
    ("gauss_S45_inline_96x66", 96, 66, 3, 7, "gaussian", 45, 15.0, 0.2, "lsq"),
    ("box_S0_inline_41x57", 41, 57, 3, 6, "box", 0, None, 0.15, "lsq"),
    ("gauss_S0_inline_41x57", 41, 57, 3, 6, "gaussian", 0, 1.0, 0.15, "lsq"),
    ("box_S0_planes_33x45", 33, 45, 12, 8, "box", 0, None, 0.3, "lsq"),
    ("gauss_S0_hard_39x50", 39, 50, 3, 6, "gaussian", 0, 1.0, 0.15, "hard"),
    # radii above 96: the row pass's halo run (run + 2S) exceeds the block's
    # 256 threads, so its first phase takes the remaining halo pixels and
    # coefficient runs in loops
    ("gauss_S100_inline_48x300", 48, 300, 3, 8, "gaussian", 100, 33.3, 0.2, "lsq"),
    ("gauss_S128_hard_40x270", 40, 270, 3, 7, "gaussian", 128, 42.7, 0.15, "hard"),
    ("box_S110_planes_36x270", 36, 270, 12, 9, "box", 110, None, 0.3, "lsq"),
]


@pytest.mark.parametrize("case", GENERIC, ids=[c[0] for c in GENERIC])
def test_generic_windows(fhd, case):
    name, H, W, rho, K, spatial, S, ss, sr, coef = case
    f = synth.voronoi_rgb(H, W, 14, 0.05, 300 + H + W)
    g = f if rho == 3 else synth.hyperspectral(H, W, rho, 5, 0.5, 0.02, 400 + H)
    cl = oracle.bisecting_kmeans(g, K)
    c32 = cl.centers.astype(np.float32)
    lab = cl.labels if coef == "hard" else None
    ref, rden = _o2(f, g, c32, ss, sr, S, spatial, coef=coef, labels=lab)
    labd = _dev(cl.labels.reshape(H, W), np.int32) if coef == "hard" else None
    out, den = fhd.filter_centers(_dev(f), _dev(g), c32, sigma_s=ss if ss else 1.0, sigma_r=sr,
                                  spatial=spatial, radius=S, coef=coef, labels=labd, return_den=True)
    o = out.cpu().numpy()
    err = np.abs(o - ref).max()
    derr = np.abs(den.cpu().numpy() - rden).max() / np.abs(rden).max()
    print(f"{name}: max-abs {err:.3e}, den rel {derr:.3e}, den min {rden.min():.3e}")
    assert err < TOL
    assert derr < 1e-5
    if S == 0:
        # the window is the pixel itself: v = r_hat f, so g_hat = f
        assert np.abs(o - f).max() < 1e-5


def _stats(out, den):
    return dict(den_min=float(den.min()), den_nonpos=int((den <= 0).sum()),
                den_small=int((den < 1e-3).sum()), nonfinite=int((~torch.isfinite(out)).sum()))


def test_info_normaliser_diagnostics(fhd):
    """fhd_info's normaliser fields equal the statistics of the returned r_hat
    and g_hat, for fhd_filter, fhd_filter_centers and every image of a batch."""
    f = synth.voronoi_rgb(97, 113, 20, 0.05, 9)
    fd = _dev(f)
    out, den, cen, info = fhd.filter(fd, sigma_s=2.0, sigma_r=0.1, K=12, radius=6, return_den=True,
                                     return_centers=True, info=True)
    s = _stats(out, den)
    print("filter info", {k: info[k] for k in s}, "from outputs", s)
    for k in s:
        assert info[k] == s[k], k
    assert s["den_nonpos"] == 0 and s["den_min"] > 0
    out2, den2, info2 = fhd.filter_centers(fd, fd, cen, sigma_s=2.0, sigma_r=0.1, radius=6, return_den=True,
                                           info=True)
    s2 = _stats(out2, den2)
    for k in s2:
        assert info2[k] == s2[k], k
    # without a den output the library forms r_hat in its workspace
    _, info3 = fhd.filter_centers(fd, fd, cen, sigma_s=2.0, sigma_r=0.1, radius=6, info=True)
    for k in s2:
        assert info3[k] == s2[k], k
    imgs = [_dev(synth.voronoi_rgb(h, w, 10, 0.05, 70 + h)) for h, w in ((40, 50), (64, 33), (29, 71))]
    flat, sizes = fhd.pack_batch(imgs)
    bout, bden, _, _, binfo = fhd.filter_batch(flat, sizes, 3, sigma_s=2.0, sigma_r=0.1, K=8, radius=6,
                                               return_den=True, info=True)
    o = 0
    for b, (h, w) in enumerate(sizes):
        sb = _stats(bout[3 * o:3 * (o + h * w)], bden[o:o + h * w])
        o += h * w
        for k in sb:
            assert binfo[b][k] == sb[k], (b, k)


def _nlm_crop_with_negative_normaliser(fhd):
    """The 1024x1024 nonlocal-means workload: a 64x64 crop around a pixel
    whose r_hat is <= 0 (at least S = 10 pixels from the crop's border, so its
    window lies inside the crop), with the full image's centers."""
    cfg = synth.WORKLOADS["nlm_rgb_1024"]
    noisy, _ = synth.workload_input("nlm_rgb_1024")
    xd = _dev(noisy)
    g = fhd.nlm_guide(xd, patch=cfg["patch"], dims=cfg["dims"])
    kw = dict(sigma_r=cfg["sigma_r"], spatial="box", radius=cfg["S"])
    out, den, cen, info = fhd.filter(xd, g, K=cfg["K"], return_den=True, return_centers=True, info=True, **kw)
    s = _stats(out, den)
    for k in s:
        assert info[k] == s[k], k
    print(f"nlm 1024: den_min {info['den_min']:.4e}, den_nonpos {info['den_nonpos']}, "
          f"den_small {info['den_small']}, nonfinite {info['nonfinite']}")
    assert info["den_nonpos"] >= 1
    d = den.cpu().numpy()
    ys, xs = np.nonzero(d <= 0)
    inner = [(y, x) for y, x in zip(ys, xs) if 32 <= y < 1024 - 32 and 32 <= x < 1024 - 32]
    y, x = inner[0]
    y0, x0 = y - 32, x - 32
    fc = np.ascontiguousarray(noisy[:, y0:y0 + 64, x0:x0 + 64])
    gc = np.ascontiguousarray(g.cpu().numpy()[:, y0:y0 + 64, x0:x0 + 64])
    return fc, gc, cen.numpy(), kw, (32, 32), float(d[y, x])


def test_strict_mode_and_normaliser_signs_nlm_crop(fhd):
    fc, gc, cen, kw, (cy, cx), dfull = _nlm_crop_with_negative_normaliser(fhd)
    with pytest.raises(fhd.FHDError) as e:
        fhd.filter_centers(_dev(fc), _dev(gc), cen, strict=True, **kw)
    assert e.value.status == fhd.FHD_ENUMERIC
    out, den, info = fhd.filter_centers(_dev(fc), _dev(gc), cen, return_den=True, info=True, **kw)
    d = den.cpu().numpy()
    assert abs(d[cy, cx] - dfull) <= 1e-6 * max(1.0, abs(dfull))   # same window, same value
    ref, rden, _, _, mr = _o2(fc, gc, cen, None, kw["sigma_r"], kw["radius"], "box", terms=True)
    # sign of r_hat agrees wherever it is decided beyond the sums' rounding scale
    decided = np.abs(rden) > 1e-4 * mr
    agree = np.sign(d[decided]) == np.sign(rden[decided])
    print(f"crop: r_hat gpu {d[cy, cx]:.4e} oracle {rden[cy, cx]:.4e}; info {info}; "
          f"decided {decided.sum()} / {d.size}, sign agreement {agree.mean():.4f}")
    assert agree.all()
    assert info["den_nonpos"] == int((d <= 0).sum()) >= 1
    assert abs(d - rden).max() <= 1e-4 * mr.max()
    # the brute force's normaliser is >= 1, so strict mode accepts it
    fhd.bruteforce(_dev(fc), _dev(gc), sigma_r=kw["sigma_r"], spatial="box", radius=kw["radius"])


def test_stream_switch_orders_work(fhd):
    """Calls on two torch streams alternate on one context (one workspace);
    every output equals the output of the same call made on its own."""
    H, W = 1024, 1024
    fs = [synth.voronoi_rgb(H, W, 64, 0.05, 501 + i) for i in range(2)]
    ds = [_dev(f) for f in fs]
    kw = dict(sigma_s=5.0, sigma_r=0.12, radius=15)
    cens = [fhd.cluster(d, 32)[0] for d in ds]
    refs = []
    for d, c in zip(ds, cens):
        refs.append(fhd.filter_centers(d, d, c, **kw))
        torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.cuda.stream(s1):
            o1 = fhd.filter_centers(ds[0], ds[0], cens[0], **kw)
        with torch.cuda.stream(s2):
            o2 = fhd.filter_centers(ds[1], ds[1], cens[1], **kw)
        torch.cuda.synchronize()
        e1 = float((o1 - refs[0]).abs().max())
        e2 = float((o2 - refs[1]).abs().max())
        print(f"stream switch rep {rep}: {e1:.3e} {e2:.3e}")
        assert e1 == 0.0 and e2 == 0.0


def test_cluster_split_selection_golden(fhd, golden_dir):
    """The GPU's bisecting K-means on the hand-worked split-selection cases."""
    cases = json.load(open(os.path.join(golden_dir, "bisect_select.json")))["cases"]
    for g in cases:
        pts = np.array(g["points"], dtype=np.float32).reshape(1, 1, -1)
        cen, lab, info = fhd.cluster(_dev(pts), g["K"], labels=True)
        print(g["name"], cen.numpy().ravel(), lab.cpu().numpy().ravel(), info["E_K"])
        assert cen.numpy().ravel().tolist() == g["centers"]
        assert lab.cpu().numpy().ravel().tolist() == g["labels"]
        assert info["E_K"] == g["E_K"]
