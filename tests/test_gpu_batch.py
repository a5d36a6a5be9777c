"""The ragged batch entry points (fhd_filter_batch, fhd_filter_batch_backward)
through the C ABI.

One tree per image with every clustering pass launched once for all images:
the partition of each image's points into blocks, and so every FP64 sum, is
the same as when the image is clustered alone, so centers and outputs must be
bit-identical to the single-image calls; each image is also checked against
the FP64 oracle (max-abs 1e-4).  The batch adjoint must equal the per-image
adjoint (bit-identical image and guide gradients; sigma_r summed over images,
1e-12 relative), on both of its paths.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

SIZES = [(40, 52), (33, 61), (64, 64), (17, 90), (48, 35)]


@pytest.fixture(scope="module")
def fhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_02363_amd as m
    m.load()
    return m


def _images(seed0=1400):
    return [synth.voronoi_rgb(h, w, 12, 0.05, seed0 + b) for b, (h, w) in enumerate(SIZES)]


def _split(flat, sizes, C):
    outs, o = [], 0
    for h, w in sizes:
        outs.append(flat[o * C:(o + h * w) * C].reshape(C, h, w))
        o += h * w
    return outs


@pytest.mark.parametrize("spatial,coef,S", [("gaussian", "lsq", 9), ("gaussian", "hard", 9), ("box", "lsq", 9),
                                            ("box", "hard", 9), ("box", "lsq", 28), ("box", "hard", 28)])
def test_batch_equals_single_image_calls(fhd, spatial, coef, S):
    imgs = _images()
    dev = [torch.from_numpy(x).cuda() for x in imgs]
    flat, sizes = fhd.pack_batch(dev)
    kw = dict(sigma_s=3.0, sigma_r=0.1, K=16, radius=S, spatial=spatial, coef=coef)
    out, den, cen, keff = fhd.filter_batch(flat, sizes, 3, return_den=True, **kw)
    outs = _split(out, sizes, 3)
    dens = _split(den, sizes, 1)
    if spatial == "box":  # the running-sum kernels against the oracle's direct window sums
        for b, x in enumerate(imgs):
            c = cen[b, :keff[b]].numpy().astype(np.float64)
            P, _, _ = oracle.pinv(oracle.kernel_matrix(c, 0.1))
            lab = oracle.bisecting_kmeans(x, 16).labels if coef == "hard" else None
            ref = oracle.fast_filter(x, x, c, P, None, 0.1, S, "box", coef=coef, labels=lab)[0]
            err = float(np.abs(outs[b].cpu().numpy() - ref).max())
            assert err < 1e-4, f"image {b}: max-abs {err:.3e} against the oracle"
    for b, x in enumerate(dev):
        o1, d1, c1 = fhd.filter(x, return_den=True, return_centers=True, **kw)
        assert keff[b] == c1.shape[0]
        assert torch.equal(cen[b, :keff[b]], c1), f"image {b}: centers differ"
        assert torch.equal(outs[b], o1), f"image {b}: output differs"
        assert torch.equal(dens[b][0], d1), f"image {b}: normaliser differs"


def test_batch_against_oracle(fhd):
    imgs = _images(1500)
    dev = [torch.from_numpy(x).cuda() for x in imgs]
    flat, sizes = fhd.pack_batch(dev)
    out, cen, keff = fhd.filter_batch(flat, sizes, 3, sigma_s=3.0, sigma_r=0.1, K=32, radius=9)
    outs = _split(out, sizes, 3)
    worst = 0.0
    for b, x in enumerate(imgs):
        c = cen[b, :keff[b]].numpy().astype(np.float64)
        P, _, _ = oracle.pinv(oracle.kernel_matrix(c, 0.1))
        ref = oracle.fast_filter(x, x, c, P, 3.0, 0.1, 9)[0]
        worst = max(worst, float(np.abs(outs[b].cpu().numpy() - ref).max()))
        # the tree of each image is the oracle's tree
        cl = oracle.bisecting_kmeans(x, 32)
        assert np.array_equal(cl.centers.astype(np.float32), cen[b, :keff[b]].numpy())
    print(f"batch of {len(imgs)}: max-abs vs oracle {worst:.3e}")
    assert worst < 1e-4


@pytest.mark.parametrize("K,spatial,S", [(32, "gaussian", 9), (48, "gaussian", 9), (32, "box", 9), (32, "box", 28)])
def test_batch_backward_equals_per_image(fhd, K, spatial, S):
    """K 32: one launch per pass for all images; K 48: the images spread over
    streams, one adjoint each."""
    imgs = _images(1600)
    dev = [torch.from_numpy(x).cuda() for x in imgs]
    flat, sizes = fhd.pack_batch(dev)
    kw = dict(sigma_s=3.0, sigma_r=0.1, radius=S, spatial=spatial)
    out, den, cen, keff = fhd.filter_batch(flat, sizes, 3, K=K, return_den=True, **kw)
    G = torch.from_numpy(np.random.default_rng(3).standard_normal(flat.numel()).astype(np.float32)).cuda()
    gf, gg, gs = fhd.filter_batch_backward(flat, sizes, 3, cen, keff, out, den, G, **kw)
    gfs, ggs, Gs = _split(gf, sizes, 3), _split(gg, sizes, 3), _split(G, sizes, 3)
    outs, dens = _split(out, sizes, 3), _split(den, sizes, 1)
    total = 0.0
    for b, x in enumerate(dev):
        c = cen[b, :keff[b]]
        f1, g1, s1 = fhd.filter_backward(x, x, c, outs[b].contiguous(), dens[b][0].contiguous(),
                                         Gs[b].contiguous(), **kw)
        assert torch.equal(gfs[b], f1) and torch.equal(ggs[b], g1), f"image {b}: gradients differ"
        total += s1
    print(f"batch dsigma_r {gs:.10e} vs per-image sum {total:.10e}")
    assert abs(gs - total) <= 1e-12 * max(1.0, abs(total))


def test_batch_backward_sigma_s(fhd):
    """dL/dsigma_s of the batch is the sum of the per-image values (the other
    gradients are unchanged by asking for it)."""
    imgs = _images(1700)
    dev = [torch.from_numpy(x).cuda() for x in imgs]
    flat, sizes = fhd.pack_batch(dev)
    out, den, cen, keff = fhd.filter_batch(flat, sizes, 3, sigma_s=3.0, sigma_r=0.1, K=16, radius=9,
                                           return_den=True)
    G = torch.from_numpy(np.random.default_rng(5).standard_normal(flat.numel()).astype(np.float32)).cuda()
    kw = dict(sigma_s=3.0, sigma_r=0.1, radius=9)
    gf, gg, gs, gss = fhd.filter_batch_backward(flat, sizes, 3, cen, keff, out, den, G, need_sigma_s=True, **kw)
    gf0, gg0, gs0 = fhd.filter_batch_backward(flat, sizes, 3, cen, keff, out, den, G, **kw)
    assert torch.equal(gf, gf0) and torch.equal(gg, gg0)
    assert abs(gs - gs0) <= 1e-12 * max(1.0, abs(gs0))
    outs, dens, Gs = _split(out, sizes, 3), _split(den, sizes, 1), _split(G, sizes, 3)
    total = 0.0
    for b, x in enumerate(dev):
        r = fhd.filter_backward(x, x, cen[b, :keff[b]], outs[b].contiguous(), dens[b][0].contiguous(),
                                Gs[b].contiguous(), need_f=False, need_guide=False, need_sigma_r=False,
                                need_sigma_s=True, **kw)
        total += r[3]
    print(f"batch dsigma_s {gss:.10e} vs per-image sum {total:.10e}")
    assert abs(gss - total) <= 1e-12 * max(1.0, abs(total))


def test_batch_rejects_gaps(fhd):
    import ctypes
    lib = fhd.load()
    x = torch.zeros(3 * 100, device="cuda")
    o = torch.empty_like(x)
    p = fhd.make_params(K=4, sigma_s=1.0, radius=2)
    Ha = (ctypes.c_int * 2)(5, 5)
    Wa = (ctypes.c_int * 2)(10, 10)
    Oa = (ctypes.c_longlong * 2)(0, 60)   # a gap of 10 pixels
    ctx = fhd._ctx(0)
    st = lib.fhd_filter_batch(ctx, 2, Ha, Wa, Oa, ctypes.c_void_p(x.data_ptr()), 3, ctypes.c_void_p(x.data_ptr()),
                              3, ctypes.byref(p), ctypes.c_void_p(o.data_ptr()), None, None, None, None, None, 0)
    assert st == fhd.FHD_EINVAL
    assert b"back to back" in lib.fhd_last_error(ctx)
