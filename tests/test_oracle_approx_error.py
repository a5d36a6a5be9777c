"""Pins of the oracle's kernel-approximation error (eq. (10) evaluated at the
method's coefficients c(i) = A^+ b(i); its pixel mean is the averaged
least-squares error E_ls of Sec. II-A, not the clustering error E_K).

* A plain triple loop over pixels, window offsets and centers on tiny images
  (math.exp, scalar sums) gives the same per-pixel errors as the vectorised
  oracle, for an invertible A and for a rank-deficient one.
* Exact cases: with K equal to the number of distinct guide values every
  sample of every Theta_i is a center, the fit interpolates there (A c = b),
  and the error vanishes; sigma_r = inf (phi = 1) fits exactly with any K.
* Translating the guide and the centers together leaves it unchanged (only
  differences enter); a wrong sign or index in a difference breaks that.
"""
import math

import numpy as np

import oracle
import synth


def _loops(guide, centers, sigma_r, S):
    rho, H, W = guide.shape
    K = len(centers)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(np.asarray(centers, np.float64), sigma_r))

    def ph(a, b):
        return math.exp(-sum((float(a[d]) - float(b[d])) ** 2 for d in range(rho)) / (2 * sigma_r ** 2))

    err = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            pi = guide[:, y, x]
            b = [ph(centers[k], pi) for k in range(K)]
            c = [sum(P[l][k] * b[k] for k in range(K)) for l in range(K)]
            e = 0.0
            for dy in range(-S, S + 1):
                for dx in range(-S, S + 1):
                    yy, xx = y - dy, x - dx
                    if 0 <= yy < H and 0 <= xx < W:
                        xq = guide[:, yy, xx]
                        fit = sum(c[k] * ph(xq, centers[k]) for k in range(K))
                        e += (ph(xq, pi) - fit) ** 2
            err[y, x] = e
    return err


def test_matches_loops_on_tiny_images():
    g = synth.voronoi_rgb(6, 7, 5, 0.05, 77).astype(np.float64)
    cen = oracle.bisecting_kmeans(g, 4).centers
    for sr in (0.3, 0.08):
        err, Els = oracle.approx_error(g, cen, sr, 2)
        ref = _loops(g, cen, sr, 2)
        assert np.max(np.abs(err - ref)) < 1e-12 * max(1.0, ref.max())
        assert abs(Els - ref.mean()) < 1e-12 * max(1.0, ref.mean())
        assert ref.max() > 1e-6  # not a trivially exact case
    # rank-deficient A: two coincident centers
    cen2 = np.vstack([cen[:3], cen[2:3]])
    err, _ = oracle.approx_error(g, cen2, 0.3, 1)
    assert np.max(np.abs(err - _loops(g, cen2, 0.3, 1))) < 1e-12


def test_exact_cases():
    rng = np.random.default_rng(5)
    vals = rng.uniform(0, 1, (5, 3))
    lab = rng.integers(0, 5, (9, 11))
    g = np.transpose(vals[lab], (2, 0, 1))
    err, Els = oracle.approx_error(g, vals, 0.4, 3)
    assert Els < 1e-18 and err.max() < 1e-16
    g2 = synth.voronoi_rgb(10, 9, 6, 0.05, 3)
    cen = oracle.bisecting_kmeans(g2, 3).centers
    err, Els = oracle.approx_error(g2, cen, np.inf, 2)
    assert err.max() < 1e-20


def test_translation_invariance():
    g = synth.hyperspectral(12, 10, 4, 3, 0.5, 0.02, 9).astype(np.float64)
    cen = oracle.bisecting_kmeans(g, 6).centers
    t = np.array([0.3, -1.2, 5.0, 0.01])
    e1, _ = oracle.approx_error(g, cen, 0.2, 3)
    e2, _ = oracle.approx_error(g + t[:, None, None], cen + t[None, :], 0.2, 3)
    assert np.max(np.abs(e1 - e2)) < 1e-9 * max(1.0, e1.max())
    assert e1.max() > 1e-6
