"""Eq. (10) solved per pixel on the GPU (fhd_exact_ls, coef='exact') against
the FP64 oracle fed the same FP32 guide and centers, through the C ABI.

* Objectives (the minimum of eq. (10), and eq. (10) at the surrogate's
  c = A^+ b(i) of eq. (11)) at every pixel within 1e-9 of the window's
  sample count plus 1e-6 relative: both sides run in FP64, the outputs are
  FP32.
* Coefficients at every pixel whose design matrix has a clear rank (kept
  singular values >= 1e-8 s_max, dropped ones below a tenth of the
  tolerance): relative L2 <= 1e-5; elsewhere the minimiser is not
  well-determined in floating point and only the objective is compared.
* Shapes: RGB and 12-d guides, K 1, 8, 16, 32 (the three kernel tiers), box
  and Gaussian windows, windows with fewer samples than clusters (rank
  deficient: the minimum-norm solution), borders.
* The filter with coef='exact' against the oracle's fast_filter with the
  same per-pixel minimisers: max-abs 1e-4 where the recombination cancels
  little, else the numerator and r_hat within 1e-5 of the sums of their
  terms' magnitudes (the minimisers can be large and of mixed sign).
* The surrogate is never better than the exact fit, and the calls that do
  not take coef='exact' reject it.
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_02363_amd as m
    m.load()
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _design(p, mu, sr, S, i):
    rho, H, W = p.shape
    iy, ix = divmod(i, W)
    ys = np.arange(max(0, iy - S), min(H, iy + S + 1))
    xs = np.arange(max(0, ix - S), min(W, ix + S + 1))
    q = (ys[:, None] * W + xs[None, :]).ravel()
    X = p.reshape(rho, -1).T.astype(np.float64)
    M = np.exp(-((X[q][:, None, :] - mu[None, :, :]) ** 2).sum(-1) / (2 * sr * sr))
    return M


CASES = [
    # name, H, W, guide dims, K, spatial, S, sigma_s, sigma_r
    ("rgb_K8_box_S3_40x52", 40, 52, 3, 8, "box", 3, None, 0.2),
    ("rgb_K1_gauss_37x29", 37, 29, 3, 1, "gaussian", None, 1.0, 0.25),
    ("g12_K16_box_S4_24x30", 24, 30, 12, 16, "box", 4, None, 0.5),
    ("rgb_K32_box_S4_20x24", 20, 24, 3, 32, "box", 4, None, 0.25),
    ("rgb_K16_box_S1_18x21_rank_deficient", 18, 21, 3, 16, "box", 1, None, 0.2),
    ("g5_K12_gauss_S2_31x17", 31, 17, 5, 12, "gaussian", 2, 0.8, 0.3),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_exact_ls_against_oracle(fhd, case):
    name, H, W, rho, K, spatial, S, ss, sr = case
    g = synth.voronoi_rgb(H, W, 10, 0.05, 900 + H) if rho == 3 else synth.hyperspectral(H, W, rho, 4, 0.5, 0.02,
                                                                                       910 + H)
    cen = oracle.bisecting_kmeans(g, K).centers.astype(np.float32)
    K = cen.shape[0]
    Sr = S if S is not None else oracle.default_radius(ss)
    cf, o10, o11 = fhd.exact_ls(_dev(g), cen, sigma_r=sr, sigma_s=ss if ss else 1.0, radius=S, spatial=spatial)
    C, obj, obj11 = oracle.exact_ls(g, cen.astype(np.float64), sr, Sr)
    gc = cf.cpu().numpy().reshape(K, -1).T.astype(np.float64)
    go, go11 = o10.cpu().numpy().ravel().astype(np.float64), o11.cpu().numpy().ravel().astype(np.float64)
    mu = cen.astype(np.float64)
    worst_obj = worst_c = 0.0
    compared = 0
    for i in range(H * W):
        M = _design(g, mu, sr, Sr, i)
        m = M.shape[0]
        tol_o = 1e-9 * m
        worst_obj = max(worst_obj, abs(go[i] - obj[i]) / (tol_o + 1e-6 * obj[i]))
        worst_obj = max(worst_obj, abs(go11[i] - obj11[i]) / (tol_o + 1e-6 * obj11[i]))
        s = np.linalg.svd(M, compute_uv=False)
        tol = max(m, K) * np.finfo(np.float64).eps * s[0]
        kept, dropped = s[s > tol], s[s <= tol]
        if kept.min() >= 1e-8 * s[0] and (dropped.size == 0 or dropped.max() <= 0.1 * tol):
            compared += 1
            e = np.linalg.norm(gc[i] - C[i]) / max(np.linalg.norm(C[i]), 1e-30)
            worst_c = max(worst_c, e / 1e-5)
    print(f"{name}: objective err / tol {worst_obj:.3f}, coefficient err / tol {worst_c:.3f} "
          f"({compared} of {H * W} pixels compared), mean eq.(10) exact {obj.mean():.4e} vs at A^+b "
          f"{obj11.mean():.4e}")
    assert worst_obj <= 1.0
    assert worst_c <= 1.0
    assert compared >= H * W // 4
    # the exact fit is never worse than the surrogate's
    assert np.all(go <= go11 * (1 + 1e-5) + 1e-7)


def test_exact_coefficients_in_the_filter(fhd):
    H, W = 36, 47
    f = synth.voronoi_rgb(H, W, 9, 0.05, 931)
    cen = oracle.bisecting_kmeans(f, 8).centers.astype(np.float32)
    kw = dict(sigma_s=1.2, sigma_r=0.2, radius=3)
    out, den = fhd.filter_centers(_dev(f), _dev(f), cen, coef="exact", return_den=True, **kw)
    c = cen.astype(np.float64)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(c, 0.2))
    ref, rden, v, mv, mr = oracle.fast_filter(f, f, c, P, 1.2, 0.2, 3, coef="exact", return_terms=True)
    o, d = out.cpu().numpy().astype(np.float64), den.cpu().numpy().astype(np.float64)
    # The per-pixel minimisers can be large and cancel in the recombination,
    # so FP32 rounding scales with sum_k |c_k| |terms| (mv, mr), not |r_hat|:
    # g_hat within 1e-4 where that sum is within 10 |r_hat| (little
    # cancellation), else the numerator and r_hat within 1e-5 of it.
    mild = mr <= 10.0 * np.abs(rden)
    err = np.abs(o - ref)[:, mild].max()
    ev = (np.abs(o * d - v) / np.maximum(mv, 1e-30))[:, ~mild]
    er = (np.abs(d - rden) / np.maximum(mr, 1e-30))
    print(f"filter with eq. (10) coefficients: max-abs {err:.3e} on {mild.sum()} of {H * W} pixels "
          f"(mild cancellation; worst anywhere {np.abs(o - ref).max():.3e}), numerator err / magnitude "
          f"{ev.max() if ev.size else 0.0:.2e} elsewhere, r_hat err / magnitude {er.max():.2e}")
    assert mild.sum() >= H * W // 2
    assert err < 1e-4
    assert ev.size == 0 or ev.max() < 1e-5
    assert er.max() < 1e-5
    # fhd_filter takes it too (its own clustering)
    out2, cen2 = fhd.filter(_dev(f), coef="exact", K=8, return_centers=True, **kw)
    assert np.array_equal(cen2.numpy(), cen)
    assert torch.equal(out2, out)


def test_exact_rejected_where_not_built(fhd):
    f = _dev(synth.voronoi_rgb(30, 30, 5, 0.05, 940))
    kw = dict(sigma_s=1.0, sigma_r=0.2, radius=2)

    def expect(status, fn):
        with pytest.raises(fhd.FHDError) as e:
            fn()
        assert e.value.status == status

    expect(fhd.FHD_EUNSUPPORTED, lambda: fhd.filter(f, coef="exact", K=33, **kw))
    expect(fhd.FHD_EUNSUPPORTED, lambda: fhd.filter(f, coef="exact", K=8, contract="bf16", **kw))
    expect(fhd.FHD_EUNSUPPORTED, lambda: fhd.filter(f, coef="exact", K=8, sigma_s=2.0, sigma_r=0.2,
                                                    spatial="young"))
    flat, sizes = fhd.pack_batch([f, f])
    expect(fhd.FHD_EUNSUPPORTED, lambda: fhd.filter_batch(flat, sizes, 3, coef="exact", K=8, **kw))
    expect(fhd.FHD_EUNSUPPORTED, lambda: fhd.exact_ls(f, np.zeros((33, 3), np.float32), sigma_r=0.2, radius=2,
                                                      spatial="box"))


def test_centers_without_info(fhd):
    """fhd_filter's centers come back without fhd_info (fhd_last_k_eff): an
    image of three colours gives three centers at K 8."""
    img = np.zeros((3, 20, 30), np.float32)
    img[:, :, 10:20] = 0.5
    img[:, :, 20:] = 1.0
    out, cen = fhd.filter(_dev(img), K=8, sigma_s=1.0, sigma_r=0.2, radius=2, return_centers=True)
    out2, cen2, info = fhd.filter(_dev(img), K=8, sigma_s=1.0, sigma_r=0.2, radius=2, return_centers=True,
                                  info=True)
    assert cen.shape == (3, 3) and info["K_eff"] == 3
    assert np.array_equal(cen.numpy(), cen2.numpy())
    assert torch.equal(out, out2)
