"""The hand-written adjoint (fhd_filter_backward) through the C ABI, against
the FP64 gradient reference (``oracle/autograd_ref.py``, itself pinned to
finite differences of the oracle) fed the same FP32 centers.

Tolerance: relative L2 error <= 1e-4 for dL/df and dL/dguide.  The adjoint
runs in FP32: each gradient entry sums (2S+1)^2 K products whose terms carry
A^+ (cond(A) <= 2e4 in these cases, checked), so the FP32 rounding (6e-8 per
operation) grows to about 1e-5..1e-4 relative; 1e-4 holds with a margin in
these cases while still catching any dropped term (those change the gradient at the 1e-2..1
level).  dL/dsigma_r and dL/dsigma_s are sums over all pixels of per-pixel
shares that largely cancel, so their errors are bounded by the same 1e-4
times the sum of the shares' magnitudes (from the FP64 per-pixel split of
the reference), not times the total.  (1e-4 relative L2 is also the gradient bar of the method's
parity targets.)
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import autograd_ref as ar

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


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-30))


def _ref(f, g, cen, G, ss, sr, S, spatial, full_rank=True):
    ft = torch.tensor(f, dtype=torch.float64, requires_grad=True)
    gt = torch.tensor(g, dtype=torch.float64, requires_grad=True)
    st = torch.tensor(float(sr), dtype=torch.float64, requires_grad=True)
    out, _ = ar.fast_filter_torch(ft, gt, np.asarray(cen, np.float64), ss, st, S, spatial,
                                  full_rank=full_rank)
    (out * torch.tensor(G, dtype=torch.float64)).sum().backward()
    return ft.grad.numpy(), gt.grad.numpy(), float(st.grad)


def _sigma_scale(f, g, cen, G, ss, sr, S, spatial, full_rank=True):
    sb, sa = ar.sigma_r_shares(f, g, np.asarray(cen, np.float64), ss, sr, S, G, spatial, full_rank)
    return float(np.abs(sb).sum() + np.abs(sa).sum())


def _gpu(fhd, f, g, cen, G, ss, sr, S, spatial):
    fd, gd = _dev(f), _dev(g)
    out, den = fhd.filter_centers(fd, gd, cen, sigma_s=ss, sigma_r=sr, radius=S, spatial=spatial,
                                  return_den=True)
    gf, gg, gs = fhd.filter_backward(fd, gd, cen, out, den, _dev(G), sigma_s=ss, sigma_r=sr,
                                     spatial=spatial, radius=S)
    torch.cuda.synchronize()
    return gf.cpu().numpy(), gg.cpu().numpy(), gs


CASES = [
    # (H, W, rho of a separate guide, K, sigma_s, S, sigma_r, window)
    (37, 53, 3, 16, 2.0, 6, 0.3, "gaussian"),
    (29, 70, 5, 48, 1.5, 4, 0.15, "gaussian"),  # K > 32: two final-kernel launches
    (33, 41, 12, 24, None, 3, 0.3, "box"),
    (40, 47, 3, 12, None, 28, 0.3, "box"),   # the running-sum row pass
    (45, 38, 3, 8, 3.0, 9, 0.25, "gaussian"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-rho{c[2]}-K{c[3]}-{c[7]}S{c[5]}")
def test_adjoint_against_fp64_autograd(fhd, case):
    H, W, rho, K, ss, S, sr, spatial = case
    f = synth.voronoi_rgb(H, W, 9, 0.05, 10 + K)
    g = synth.hyperspectral(H, W, rho, 4, 0.5, 0.02, 20 + K)
    cen = oracle.bisecting_kmeans(g, K).centers.astype(np.float32)
    assert fhd.pinv(cen, sr)[3] < 2e4  # FP32 carries the gradient only for a well-conditioned A
    G = np.random.default_rng(K).standard_normal(f.shape).astype(np.float32)
    rf, rg, rs = _ref(f, g, cen, G, ss, sr, S, spatial)
    gf, gg, gs = _gpu(fhd, f, g, cen, G, ss, sr, S, spatial)
    scale = _sigma_scale(f, g, cen, G, ss, sr, S, spatial)
    ef, eg, es = _rel(gf, rf), _rel(gg, rg), abs(gs - rs) / scale
    print(f"{case}: rel L2 df {ef:.2e}, dguide {eg:.2e}; dsigma_r {gs:.6e} vs {rs:.6e} "
          f"(err / sum|shares| {es:.2e}, cancellation {scale / abs(rs):.1f}x)")
    assert ef < TOL and eg < TOL and es < TOL


def test_adjoint_is_transpose_in_f(fhd):
    """The filter is linear in f for a fixed guide: <G, F(delta)> = <F^T G, delta>
    with both sides from the GPU."""
    f = synth.voronoi_rgb(64, 90, 12, 0.05, 4)
    g = synth.hyperspectral(64, 90, 4, 4, 0.5, 0.02, 5)
    cen = oracle.bisecting_kmeans(g, 16).centers.astype(np.float32)
    rng = np.random.default_rng(6)
    G = rng.standard_normal(f.shape).astype(np.float32)
    d = rng.standard_normal(f.shape).astype(np.float32)
    gf, _, _ = _gpu(fhd, f, g, cen, G, 2.5, 0.3, 8, "gaussian")
    Fd = fhd.filter_centers(_dev(d), _dev(g), cen, sigma_s=2.5, sigma_r=0.3, radius=8).cpu().numpy()
    lhs = float((G.astype(np.float64) * Fd).sum())
    rhs = float((gf.astype(np.float64) * d).sum())
    print(f"<G, F d> {lhs:.8e}  <F^T G, d> {rhs:.8e}")
    assert abs(lhs - rhs) <= 1e-5 * np.abs(G * Fd).sum()


def test_sigma_r_gradient_rank_deficient(fhd):
    """A repeated center: A^+ keeps rank K - 1 and its derivative has the
    extra terms of a rank-deficient matrix."""
    f = synth.voronoi_rgb(31, 44, 8, 0.05, 7)
    g = synth.hyperspectral(31, 44, 3, 3, 0.5, 0.02, 8)
    cen = oracle.bisecting_kmeans(g, 10).centers.astype(np.float32)
    cen = np.vstack([cen, cen[3:4]])
    A, P, rank, cond = fhd.pinv(cen, 0.3)
    assert rank == cen.shape[0] - 1
    G = np.random.default_rng(9).standard_normal(f.shape).astype(np.float32)
    rf, rg, rs = _ref(f, g, cen, G, 2.0, 0.3, 5, "gaussian", full_rank=False)
    gf, gg, gs = _gpu(fhd, f, g, cen, G, 2.0, 0.3, 5, "gaussian")
    scale = _sigma_scale(f, g, cen, G, 2.0, 0.3, 5, "gaussian", full_rank=False)
    print(f"rank-deficient: df {_rel(gf, rf):.2e} dguide {_rel(gg, rg):.2e} dsigma {gs:.6e} vs {rs:.6e} "
          f"(err / sum|shares| {abs(gs - rs) / scale:.2e})")
    assert _rel(gf, rf) < TOL and _rel(gg, rg) < TOL and abs(gs - rs) < TOL * scale


def test_exact_case_image_gradient_equals_bruteforce(fhd):
    """X3 for the adjoint: with one center per distinct guide value the fast
    filter is the brute-force filter for every image, so dL/df equals the
    brute-force gradient (eqs. (1)-(2), autograd in FP64)."""
    H, W = 30, 36
    rng = np.random.default_rng(12)
    levels = np.array([[0.1, 0.2, 0.3], [0.7, 0.4, 0.2], [0.3, 0.8, 0.6], [0.9, 0.9, 0.1]], np.float32)
    lab = rng.integers(0, 4, (H, W))
    g = levels[lab].transpose(2, 0, 1).copy()
    f = rng.random((3, H, W)).astype(np.float32)
    G = rng.standard_normal(f.shape).astype(np.float32)
    ft = torch.tensor(f, dtype=torch.float64, requires_grad=True)
    out, _ = ar.bruteforce_torch(ft, torch.tensor(g, dtype=torch.float64), 2.0, 0.2, 5)
    (out * torch.tensor(G, dtype=torch.float64)).sum().backward()
    gf, _, _ = _gpu(fhd, f, g, levels, G, 2.0, 0.2, 5, "gaussian")
    e = _rel(gf, ft.grad.numpy())
    print(f"exact case: rel L2 df vs brute force {e:.2e}")
    assert e < TOL


def test_autograd_function_joint(fhd):
    """filter_autograd with the image as its own guide: autograd adds the
    image and guide contributions; sigma_r is a tensor with a gradient."""
    f = synth.voronoi_rgb(40, 48, 10, 0.05, 13)
    fd = _dev(f).requires_grad_(True)
    sr = torch.tensor(0.2, requires_grad=True)
    cen, _ = fhd.cluster(fd.detach(), 12)
    out = fhd.filter_autograd(fd, None, sigma_s=2.0, sigma_r=sr, centers=cen, radius=6)
    G = np.random.default_rng(14).standard_normal(f.shape).astype(np.float32)
    (out * _dev(G)).sum().backward()
    ft = torch.tensor(f, dtype=torch.float64, requires_grad=True)
    st = torch.tensor(0.2, dtype=torch.float64, requires_grad=True)
    ro, _ = ar.fast_filter_torch(ft, ft, cen.numpy().astype(np.float64), 2.0, st, 6)
    (ro * torch.tensor(G, dtype=torch.float64)).sum().backward()
    e = _rel(fd.grad.cpu().numpy(), ft.grad.numpy())
    scale = _sigma_scale(f, f, cen.numpy(), G, 2.0, 0.2, 6, "gaussian")
    es = abs(float(sr.grad) - float(st.grad)) / scale
    print(f"joint autograd: rel L2 df {e:.2e}; dsigma_r {float(sr.grad):.6e} vs {float(st.grad):.6e}")
    assert e < TOL and es < TOL


def test_adjoint_rejects_unsupported(fhd):
    f = _dev(synth.voronoi_rgb(16, 16, 4, 0.05, 1))
    cen = np.random.default_rng(0).random((8, 3)).astype(np.float32)
    out, den = fhd.filter_centers(f, f, cen, sigma_s=2.0, sigma_r=0.3, radius=4, return_den=True)
    with pytest.raises(fhd.FHDError, match="FHD_EUNSUPPORTED"):
        fhd.filter_backward(f, f, cen, out, den, out.clone(), sigma_s=2.0, sigma_r=0.3, radius=40)
    cen70 = np.random.default_rng(0).random((70, 3)).astype(np.float32)
    with pytest.raises(fhd.FHDError, match="FHD_EUNSUPPORTED"):
        fhd.filter_backward(f, f, cen70, out, den, out.clone(), sigma_s=2.0, sigma_r=0.3, radius=4)
    # dL/dsigma_s: the box window has no sigma_s
    ob, db = fhd.filter_centers(f, f, cen, sigma_r=0.3, radius=4, spatial="box", return_den=True)
    with pytest.raises(fhd.FHDError, match="FHD_EUNSUPPORTED"):
        fhd.filter_backward(f, f, cen, ob, db, ob.clone(), sigma_r=0.3, radius=4, spatial="box",
                            need_sigma_s=True)


SIGMA_S_CASES = [
    # (H, W, rho of a separate guide, K, sigma_s, S, sigma_r)
    (37, 53, 3, 16, 2.0, 6, 0.3),
    (29, 70, 5, 48, 1.5, 4, 0.15),  # K > 32: two final-kernel launches
    (45, 38, 3, 8, 3.0, 9, 0.25),
]


@pytest.mark.parametrize("case", SIGMA_S_CASES, ids=lambda c: f"{c[0]}x{c[1]}-rho{c[2]}-K{c[3]}-S{c[5]}")
def test_sigma_s_gradient_against_fp64_autograd(fhd, case):
    """dL/dsigma_s (window taps differentiated, radius fixed) against FP64
    autograd; the other gradients of the same call are unchanged by asking
    for it."""
    H, W, rho, K, ss, S, sr = case
    f = synth.voronoi_rgb(H, W, 9, 0.05, 10 + K)
    g = synth.hyperspectral(H, W, rho, 4, 0.5, 0.02, 20 + K)
    cen = oracle.bisecting_kmeans(g, K).centers.astype(np.float32)
    G = np.random.default_rng(K).standard_normal(f.shape).astype(np.float32)
    ft = torch.tensor(f, dtype=torch.float64)
    gt = torch.tensor(g, dtype=torch.float64)
    st = torch.tensor(float(ss), dtype=torch.float64, requires_grad=True)
    out64, _ = ar.fast_filter_torch(ft, gt, np.asarray(cen, np.float64), st, sr, S)
    (out64 * torch.tensor(G, dtype=torch.float64)).sum().backward()
    rss = float(st.grad)
    scale = float(np.abs(ar.sigma_s_shares(f, g, np.asarray(cen, np.float64), ss, sr, S, G)).sum())
    fd, gd = _dev(f), _dev(g)
    out, den = fhd.filter_centers(fd, gd, cen, sigma_s=ss, sigma_r=sr, radius=S, return_den=True)
    gf, gg, gs, gss = fhd.filter_backward(fd, gd, cen, out, den, _dev(G), sigma_s=ss, sigma_r=sr, radius=S,
                                          need_sigma_s=True)
    gf0, gg0, gs0 = fhd.filter_backward(fd, gd, cen, out, den, _dev(G), sigma_s=ss, sigma_r=sr, radius=S)
    es = abs(gss - rss) / scale
    print(f"{case}: dsigma_s {gss:.6e} vs {rss:.6e} (err / sum|shares| {es:.2e}, "
          f"cancellation {scale / abs(rss):.1f}x)")
    assert es < TOL
    assert torch.equal(gf, gf0) and torch.equal(gg, gg0) and gs == gs0


def test_sigma_s_autograd_function(fhd):
    """FilterFunction: a 0-d sigma_s tensor receives the adjoint's value."""
    f = synth.voronoi_rgb(40, 48, 8, 0.05, 3)
    cen = oracle.bisecting_kmeans(f, 12).centers.astype(np.float32)
    fd = _dev(f)
    ss = torch.tensor(2.5, requires_grad=True)
    out = fhd.FilterFunction.apply(fd, fd, 0.2, cen, ss, "gaussian", 7, "fp32")
    G = torch.randn_like(out)
    (out * G).sum().backward()
    o2, d2 = fhd.filter_centers(fd, fd, cen, sigma_s=2.5, sigma_r=0.2, radius=7, return_den=True)
    ref = fhd.filter_backward(fd, fd, cen, o2, d2, G, sigma_s=2.5, sigma_r=0.2, radius=7,
                              need_f=False, need_guide=False, need_sigma_r=False, need_sigma_s=True)[3]
    assert abs(float(ss.grad) - ref) <= 1e-6 * abs(ref)


@pytest.mark.parametrize("case", SIGMA_S_CASES, ids=lambda c: f"{c[0]}x{c[1]}-rho{c[2]}-K{c[3]}-S{c[5]}")
def test_centers_gradient_against_fp64_autograd(fhd, case):
    """dL/dmu (the clustering held fixed) against FP64 autograd through the
    oracle's transcription; error per entry within 1e-4 of the sum of the
    magnitudes of its per-pixel terms (through b and through A^+, FP64), since
    those terms cancel."""
    H, W, rho, K, ss, S, sr = case
    f = synth.voronoi_rgb(H, W, 9, 0.05, 10 + K)
    g = synth.hyperspectral(H, W, rho, 4, 0.5, 0.02, 20 + K)
    cen = oracle.bisecting_kmeans(g, K).centers.astype(np.float32)
    G = np.random.default_rng(K).standard_normal(f.shape).astype(np.float32)
    ct = torch.tensor(np.asarray(cen, np.float64), requires_grad=True)
    out64, _ = ar.fast_filter_torch(torch.tensor(f, dtype=torch.float64), torch.tensor(g, dtype=torch.float64),
                                    ct, ss, sr, S)
    (out64 * torch.tensor(G, dtype=torch.float64)).sum().backward()
    ref = ct.grad.numpy()
    sb, sA = ar.centers_abs_scale(f, g, np.asarray(cen, np.float64), ss, sr, S, G)
    fd, gd = _dev(f), _dev(g)
    out, den = fhd.filter_centers(fd, gd, cen, sigma_s=ss, sigma_r=sr, radius=S, return_den=True)
    res = fhd.filter_backward(fd, gd, cen, out, den, _dev(G), sigma_s=ss, sigma_r=sr, radius=S,
                              need_centers=True)
    gmu = res[3].numpy()
    scale = sb + sA
    err = np.abs(gmu - ref) / scale
    print(f"{case}: dmu rel L2 {_rel(gmu, ref):.2e}, max err / scale {err.max():.2e}, "
          f"|ref| max {np.abs(ref).max():.3e}")
    assert err.max() < TOL


def test_centers_gradient_autograd_function(fhd):
    """FilterFunction: a (K, rho) centers tensor receives the adjoint's value."""
    f = synth.voronoi_rgb(40, 48, 8, 0.05, 3)
    cen = oracle.bisecting_kmeans(f, 12).centers.astype(np.float32)
    fd = _dev(f)
    ct = torch.tensor(cen, requires_grad=True)
    out = fhd.FilterFunction.apply(fd, fd, 0.2, ct, 2.5, "gaussian", 7, "fp32")
    G = torch.randn_like(out)
    (out * G).sum().backward()
    o2, d2 = fhd.filter_centers(fd, fd, cen, sigma_s=2.5, sigma_r=0.2, radius=7, return_den=True)
    ref = fhd.filter_backward(fd, fd, cen, o2, d2, G, sigma_s=2.5, sigma_r=0.2, radius=7, need_f=False,
                              need_guide=False, need_sigma_r=False, need_centers=True)[3]
    assert torch.allclose(ct.grad.double(), ref, rtol=1e-6, atol=0.0)
