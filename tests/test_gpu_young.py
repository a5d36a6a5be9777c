"""The recursive Gaussian window (Young and van Vliet; the paper's O(1)
Gaussian convolution) through the C ABI, against the oracle's FP64
transcription of the same recursions (``oracle.young_conv``) fed the same
FP32 centers: max-abs <= 1e-4 (FP32 path), least-squares and hard
coefficients, including rows and columns long enough for the FP32 recursion
to accumulate rounding over hundreds of steps."""
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


CASES = [
    # (H, W, rho of a separate guide or None, K, sigma_s, sigma_r)
    (40, 57, None, 8, 2.0, 0.2),
    (31, 300, None, 16, 5.0, 0.15),   # long rows
    (260, 23, 4, 12, 3.5, 0.3),       # long columns, separate guide
    (48, 64, None, 40, 1.2, 0.1),     # K > 32, sigma in the lower q branch
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-K{c[3]}-s{c[4]}")
def test_young_against_oracle(fhd, case):
    H, W, rho, K, ss, sr = case
    f = synth.voronoi_rgb(H, W, 10, 0.05, H + W)
    g = f if rho is None else synth.hyperspectral(H, W, rho, 3, 0.5, 0.02, H)
    cl = oracle.bisecting_kmeans(g, K)
    cen = cl.centers.astype(np.float32)
    c64 = cen.astype(np.float64)
    A = oracle.kernel_matrix(c64, sr)
    assert np.linalg.cond(A) < 2e4  # FP32 coefficients carry 1e-4 only for a well-conditioned A
    P, _, _ = oracle.pinv(A)
    ref, rref = oracle.fast_filter(f, g, c64, P, ss, sr, spatial="young")
    out, den = fhd.filter_centers(_dev(f), _dev(g), cen, sigma_s=ss, sigma_r=sr, spatial="young",
                                  return_den=True)
    err = float(np.abs(out.cpu().numpy() - ref).max())
    # r_hat = sum_l c_l (omega * b_l): its terms cancel through A^+, so its
    # error is sized by the sum of their magnitudes (FP64)
    Bw = oracle.range_weights(g, c64, sr)
    Cw = Bw @ P.T
    Vn = oracle.young_conv(Bw.T.reshape(K, H, W), ss).reshape(K, -1)
    scale = (np.abs(Cw.T) * np.abs(Vn)).sum(0).reshape(H, W)
    eden = float((np.abs(den.cpu().numpy() - rref) / scale).max())
    print(f"{case}: max-abs {err:.2e}, normaliser error / sum of |terms| {eden:.2e}, "
          f"cond(A) {np.linalg.cond(A):.1e}")
    assert err < TOL and eden < TOL


def test_young_hard_and_full_call(fhd):
    """The hard variant (eq. (18)) with the recursive window, and the whole
    fhd_filter call (clustering on the GPU) against the oracle with the
    GPU's centers."""
    f = synth.voronoi_rgb(50, 70, 10, 0.05, 9)
    out, cen = fhd.filter(_dev(f), sigma_s=2.5, sigma_r=0.2, K=12, spatial="young", return_centers=True)
    c64 = cen.numpy().astype(np.float64)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(c64, 0.2))
    ref, _ = oracle.fast_filter(f, f, c64, P, 2.5, 0.2, spatial="young")
    e1 = float(np.abs(out.cpu().numpy() - ref).max())
    cl = oracle.bisecting_kmeans(f, 12)
    assert np.array_equal(cl.centers.astype(np.float32), cen.numpy())
    oh = fhd.filter(_dev(f), sigma_s=2.5, sigma_r=0.2, K=12, spatial="young", coef="hard")
    refh, _ = oracle.fast_filter(f, f, cl.centers, None, 2.5, 0.2, spatial="young", coef="hard",
                                 labels=cl.labels)
    e2 = float(np.abs(oh.cpu().numpy() - refh).max())
    print(f"full call max-abs {e1:.2e}, hard {e2:.2e}")
    assert e1 < TOL and e2 < TOL


def test_young_rejections(fhd):
    f = _dev(synth.voronoi_rgb(16, 16, 4, 0.05, 1))
    cen = np.random.default_rng(0).random((6, 3)).astype(np.float32)
    out, den = fhd.filter_centers(f, f, cen, sigma_s=2.0, sigma_r=0.3, spatial="young", return_den=True)
    with pytest.raises(fhd.FHDError, match="FHD_EUNSUPPORTED"):
        fhd.filter_backward(f, f, cen, out, den, out.clone(), sigma_s=2.0, sigma_r=0.3, spatial="young")
    with pytest.raises(fhd.FHDError, match="FHD_EUNSUPPORTED"):
        fhd.bruteforce(f, sigma_s=2.0, sigma_r=0.3, spatial="young")
    with pytest.raises(fhd.FHDError, match="FHD_EINVAL"):
        fhd.filter_centers(f, f, cen, sigma_s=0.3, sigma_r=0.3, spatial="young")
