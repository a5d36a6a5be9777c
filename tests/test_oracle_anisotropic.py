"""Pins of the oracle's anisotropic range kernel (Sec. III; the per-dimension
sigma_r of Sec. III-E).

* The direct NumPy brute force with exp(-sum_d x_d^2 / 2 sigma_d^2) equals
  the C brute force (isotropic, sigma_r = 1) of the guide divided by sigma_d:
  two separate implementations meeting through an identity of the kernel.
  Distinct sigma_d per dimension make a sigma applied to the wrong dimension,
  a dropped square or a missing factor 2 fail it.
* Equal sigma_d reduce it to the isotropic brute force with that sigma_r.
* The scaled guide is the correctly rounded FP32 quotient (NumPy's own FP32
  division agrees bit for bit).
"""
import numpy as np

import oracle
import synth


def _case(H, W, rho, seed):
    f = synth.voronoi_rgb(H, W, 7, 0.05, seed)
    g = synth.hyperspectral(H, W, rho, 3, 0.5, 0.02, seed + 1)
    return f, g


def test_anisotropic_bruteforce_is_scaled_isotropic():
    f, g = _case(23, 19, 4, 5)
    sd = np.array([0.15, 0.4, 0.07, 1.3])
    for spatial, ss, S in (("gaussian", 1.5, 4), ("box", None, 3)):
        out, eta = oracle.bruteforce_anisotropic(f, g, ss, sd, S=S, spatial=spatial)
        ref, reta = oracle.bruteforce(f, g.astype(np.float64) / sd[:, None, None], ss, 1.0, S=S,
                                      spatial=spatial)
        assert np.max(np.abs(eta - reta) / reta) < 1e-12
        assert np.max(np.abs(out - ref)) < 1e-12
    # a sigma applied to the wrong dimension is visible
    wrong, _ = oracle.bruteforce_anisotropic(f, g, 1.5, sd[::-1], S=4)
    ref, _ = oracle.bruteforce(f, g.astype(np.float64) / sd[:, None, None], 1.5, 1.0, S=4)
    assert np.max(np.abs(wrong - ref)) > 1e-3


def test_equal_sigmas_are_the_isotropic_kernel():
    f, g = _case(17, 21, 3, 9)
    out, eta = oracle.bruteforce_anisotropic(f, g, 2.0, [0.2, 0.2, 0.2], S=5)
    ref, reta = oracle.bruteforce(f, g, 2.0, 0.2, S=5)
    assert np.max(np.abs(out - ref)) < 1e-12
    assert np.max(np.abs(eta - reta) / reta) < 1e-12


def test_scaled_guide_is_correctly_rounded_fp32():
    rng = np.random.default_rng(3)
    g = (rng.standard_normal((5, 31, 17)) * rng.uniform(0.01, 100, (5, 1, 1))).astype(np.float32)
    sd = np.array([0.3, 7.0, 1e-3, 50.0, 0.1], dtype=np.float32)
    a = oracle.anisotropic_scale(g, sd)
    b = g / sd[:, None, None]  # NumPy FP32 division (IEEE, correctly rounded)
    assert a.dtype == np.float32 and b.dtype == np.float32
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
