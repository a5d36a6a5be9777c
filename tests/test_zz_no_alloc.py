"""The allocation-free entry point fhd_filter_centers_noalloc (static device
scratch, constants through the context's fixed pinned buffer) against
fhd_filter_centers, through the C ABI: two calls in a row, the second on a
smaller input, each within the FP32 parity bar of the library's own entry
point (1e-4; the kernels are the same, so the outputs are expected to be
equal), an image too large for the scratch rejected with FHD_ENOMEM, and
strict mode."""
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


def _case(H, W, rho, K, seed):
    f = synth.voronoi_rgb(H, W, 20, 0.05, seed)
    g = f if rho == 3 else synth.hyperspectral(H, W, rho, 5, 0.5, 0.02, seed + 1)
    cen = oracle.bisecting_kmeans(g, K).centers.astype(np.float32)
    return _dev(f), _dev(g), cen


def test_noalloc_matches_filter_centers(fhd):
    cases = [
        # 256x256 RGB, K 16, radius 9 (inline weights), then a smaller
        # 12-band guide with weight planes
        (256, 256, 3, 16, dict(sigma_s=3.0, sigma_r=0.1, radius=9), 31),
        (97, 131, 12, 12, dict(sigma_s=2.0, sigma_r=0.3, radius=6), 32),
    ]
    for H, W, rho, K, kw, seed in cases:
        f, g, cen = _case(H, W, rho, K, seed)
        ref, rden = fhd.filter_centers(f, g, cen, return_den=True, **kw)
        out = torch.full_like(f, float("nan"))
        den = torch.full((H, W), float("nan"), device=f.device)
        fhd.filter_centers_noalloc(f, g, cen, out=out, den=den, **kw)
        torch.cuda.synchronize()
        e = float((out - ref).abs().max())
        ed = float((den - rden).abs().max())
        print(f"noalloc {H}x{W} rho {rho} K {K}: max-abs vs filter_centers {e:.3e}, den {ed:.3e}")
        assert e <= TOL and ed <= TOL
        # without a den output
        out2, _ = fhd.filter_centers_noalloc(f, g, cen, **kw)
        torch.cuda.synchronize()
        assert float((out2 - ref).abs().max()) <= TOL
        # strict mode on a well-conditioned image passes
        fhd.filter_centers_noalloc(f, g, cen, strict=True, **kw)


def test_noalloc_rejects_images_beyond_the_scratch(fhd):
    f, g, cen = _case(1024, 1024, 3, 32, 33)
    with pytest.raises(fhd.FHDError) as e:
        fhd.filter_centers_noalloc(f, g, cen, sigma_s=5.0, sigma_r=0.12, radius=15)
    assert e.value.status == fhd.FHD_ENOMEM
    assert "static scratch" in str(e.value)
    # the context still works afterwards
    f, g, cen = _case(64, 80, 3, 8, 34)
    ref = fhd.filter_centers(f, g, cen, sigma_s=2.0, sigma_r=0.1, radius=6)
    out, _ = fhd.filter_centers_noalloc(f, g, cen, sigma_s=2.0, sigma_r=0.1, radius=6)
    torch.cuda.synchronize()
    assert float((out - ref).abs().max()) <= TOL
