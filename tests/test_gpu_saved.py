"""The forward call's intermediates kept for the adjoint (fhd_saved_size and
the `saved` arguments), through the C ABI.

* With a saved buffer the adjoint reuses the forward call's row-filtered
  planes of c_l [f, 1] and its coefficient (and weight) planes instead of
  recomputing them; its gradients equal those of the adjoint without one:
  bit for bit where both sides form the same values (weights materialised,
  long guides), and within FP32 rounding of c = A^+ b where the forward row
  pass forms c on the matrix cores and the adjoint's weights pass on the
  vector units (relative L2 1e-6).  Single images (given centers and the
  whole of Algorithm 1), with the sigma_s gradient, and the ragged batch.
* Misuse is rejected: a buffer from a call with other arguments, one that a
  later call overwrote, one too small, and forms the adjoint does not cover.
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


def _rel(a, b):
    a, b = a.double(), b.double()
    return float((a - b).norm() / max(float(b.norm()), 1e-30))


CASES = [
    # name, H, W, guide dims, K, spatial, S, sigma_s
    ("rgb_inline_97x131", 97, 131, 3, 16, "gaussian", 6, 2.0),
    ("box_inline_64x90", 64, 90, 3, 12, "box", 5, None),
    ("box_rows_inline_60x150", 60, 150, 3, 12, "box", 28, None),
    ("planes_rho12_70x66", 70, 66, 12, 20, "gaussian", 4, 1.5),
    ("planes_K40_80x72", 80, 72, 3, 40, "gaussian", 5, 1.7),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_saved_adjoint_matches_recomputed(fhd, case):
    name, H, W, rho, K, spatial, S, ss = case
    f = synth.voronoi_rgb(H, W, 18, 0.05, 600 + H)
    g = f if rho == 3 else synth.hyperspectral(H, W, rho, 5, 0.5, 0.02, 700 + H)
    cen = oracle.bisecting_kmeans(g, K).centers.astype(np.float32)
    fd, gd = _dev(f), _dev(g)
    kw = dict(sigma_s=ss if ss else 1.0, sigma_r=0.2, spatial=spatial, radius=S)
    sv = fhd.saved_buffer(3, rho, H, W, len(cen), sigma_s=kw["sigma_s"], sigma_r=0.2, spatial=spatial, radius=S)
    out, den = fhd.filter_centers(fd, gd, cen, return_den=True, **kw)
    out2, den2 = fhd.filter_centers(fd, gd, cen, return_den=True, saved=sv, **kw)
    assert torch.equal(out, out2) and torch.equal(den, den2)
    G = _dev(np.random.default_rng(3).standard_normal(f.shape))
    need_s = spatial == "gaussian"
    ref = fhd.filter_backward(fd, gd, cen, out, den, G, need_sigma_s=need_s, **kw)
    got = fhd.filter_backward(fd, gd, cen, out, den, G, need_sigma_s=need_s, saved=sv, **kw)
    ef, eg = _rel(got[0], ref[0]), _rel(got[1], ref[1])
    es = abs(got[2] - ref[2]) / max(abs(ref[2]), 1e-30)
    ess = abs(got[3] - ref[3]) / max(abs(ref[3]), 1e-30) if need_s else 0.0
    print(f"{name}: rel dL/df {ef:.2e}, dL/dguide {eg:.2e}, dL/dsigma_r {es:.2e}, dL/dsigma_s {ess:.2e}")
    tol = 0.0 if (rho > 8 or K > 32) else 1e-6
    assert ef <= tol and eg <= tol and es <= max(tol, 1e-9) and ess <= max(tol, 1e-9)


def test_saved_whole_algorithm(fhd):
    """fhd_filter (clustering included) keeps its intermediates for the
    adjoint of the centers it returns."""
    cfg = synth.WORKLOADS["bf_rgb_256"]
    f = synth.workload_input("bf_rgb_256")
    fd = _dev(f)
    kw = dict(sigma_s=cfg["sigma_s"], sigma_r=cfg["sigma_r"], radius=cfg["S"])
    sv = fhd.saved_buffer(3, 3, 256, 256, cfg["K"], **kw)
    out, den, cen = fhd.filter(fd, K=cfg["K"], return_den=True, return_centers=True, saved=sv, **kw)
    G = _dev(np.random.default_rng(5).standard_normal(f.shape))
    ref = fhd.filter_backward(fd, fd, cen, out, den, G, **kw)
    got = fhd.filter_backward(fd, fd, cen, out, den, G, saved=sv, **kw)
    print(f"whole algorithm: rel dL/df {_rel(got[0], ref[0]):.2e}, dL/dguide {_rel(got[1], ref[1]):.2e}")
    assert _rel(got[0], ref[0]) <= 1e-6 and _rel(got[1], ref[1]) <= 1e-6
    assert abs(got[2] - ref[2]) <= 1e-6 * abs(ref[2])


def test_saved_batch(fhd):
    cfg = synth.WORKLOADS["bf_rgb_batch16"]
    imgs = [_dev(synth.voronoi_rgb(h, w, 20, 0.05, 800 + h + w)) for h, w in ((96, 130), (150, 77), (64, 64))]
    flat, sizes = fhd.pack_batch(imgs)
    kw = dict(sigma_s=cfg["sigma_s"], sigma_r=cfg["sigma_r"], radius=cfg["S"])
    K = 24
    sv = fhd.saved_buffer(3, 3, [h for h, _ in sizes], [w for _, w in sizes], K, **kw)
    out, den, cen, keff = fhd.filter_batch(flat, sizes, 3, K=K, return_den=True, saved=sv, **kw)
    G = torch.from_numpy(np.random.default_rng(9).standard_normal(flat.numel()).astype(np.float32)).cuda()
    ref = fhd.filter_batch_backward(flat, sizes, 3, cen, keff, out, den, G, **kw)
    got = fhd.filter_batch_backward(flat, sizes, 3, cen, keff, out, den, G, saved=sv, **kw)
    print(f"batch: rel dL/df {_rel(got[0], ref[0]):.2e}, dL/dguide {_rel(got[1], ref[1]):.2e}, "
          f"dL/dsigma_r {got[2]:.6e} vs {ref[2]:.6e}")
    assert _rel(got[0], ref[0]) <= 1e-6 and _rel(got[1], ref[1]) <= 1e-6
    assert abs(got[2] - ref[2]) <= 1e-6 * abs(ref[2])


def test_saved_misuse_rejected(fhd):
    f1 = _dev(synth.voronoi_rgb(60, 70, 10, 0.05, 1))
    f2 = _dev(synth.voronoi_rgb(60, 70, 10, 0.05, 2))
    kw = dict(sigma_s=2.0, sigma_r=0.15, radius=6)
    c1, _ = fhd.cluster(f1, 8)
    c2, _ = fhd.cluster(f2, 8)
    sv = fhd.saved_buffer(3, 3, 60, 70, 8, **kw)
    o1, d1 = fhd.filter_centers(f1, f1, c1, return_den=True, saved=sv, **kw)
    G = torch.ones_like(f1)

    def expect_einval(fn):
        with pytest.raises(fhd.FHDError) as e:
            fn()
        assert e.value.status == fhd.FHD_EINVAL

    # other centers, other image, other window, other sigma_r
    expect_einval(lambda: fhd.filter_backward(f1, f1, c2, o1, d1, G, saved=sv, **kw))
    expect_einval(lambda: fhd.filter_backward(f2, f2, c1, o1, d1, G, saved=sv, **kw))
    expect_einval(lambda: fhd.filter_backward(f1, f1, c1, o1, d1, G, saved=sv, sigma_s=2.0, sigma_r=0.15,
                                              radius=5))
    expect_einval(lambda: fhd.filter_backward(f1, f1, c1, o1, d1, G, saved=sv, sigma_s=2.0, sigma_r=0.2,
                                              radius=6))
    # the same buffer overwritten by a later forward call
    fhd.filter_centers(f2, f2, c2, saved=sv, **kw)
    expect_einval(lambda: fhd.filter_backward(f1, f1, c1, o1, d1, G, saved=sv, **kw))
    # a buffer never written
    blank = torch.empty_like(sv)
    expect_einval(lambda: fhd.filter_backward(f1, f1, c1, o1, d1, G, saved=blank, **kw))
    # too small
    expect_einval(lambda: fhd.filter_centers(f1, f1, c1, saved=sv[:1024], **kw))
    # forms the adjoint does not cover
    with pytest.raises(fhd.FHDError) as e:
        fhd.filter_centers(f1, f1, c1, contract="bf16", saved=sv, **kw)
    assert e.value.status == fhd.FHD_EUNSUPPORTED
    with pytest.raises(fhd.FHDError) as e:
        fhd.saved_buffer(3, 3, 60, 70, 8, sigma_s=2.0, sigma_r=0.15, spatial="young")
    assert e.value.status == fhd.FHD_EUNSUPPORTED


def test_saved_autograd(fhd):
    """The autograd function keeps the intermediates by default; its gradients
    equal those of the function without them."""
    f = synth.voronoi_rgb(50, 64, 10, 0.05, 12)
    grads = []
    for keep in (True, False):
        x = _dev(f).requires_grad_(True)
        sr = torch.tensor(0.15, requires_grad=True)
        y = fhd.filter_autograd(x, sigma_s=2.0, sigma_r=sr, K=10, radius=6, keep=keep)
        (y * torch.linspace(-1, 1, y.numel(), device=y.device).reshape(y.shape)).sum().backward()
        grads.append((x.grad.clone(), float(sr.grad)))
    print(f"autograd: rel dL/df {_rel(grads[0][0], grads[1][0]):.2e}, sigma_r {grads[0][1]:.6e} vs {grads[1][1]:.6e}")
    assert _rel(grads[0][0], grads[1][0]) <= 1e-6
    assert abs(grads[0][1] - grads[1][1]) <= 1e-6 * abs(grads[1][1])
