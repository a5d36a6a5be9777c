"""Pins of the oracle's per-pixel least squares, eq. (10) (Sec. II-A), against
facts that do not come from its own code:

* K = 1: the scalar least-squares fit, c = sum_j b_j y_j / sum_j b_j^2 and
  minimum sum_j y_j^2 - (sum_j b_j y_j)^2 / sum_j b_j^2, written out with
  explicit loops over the window's in-image pixels (catches a window that
  reaches outside the image, a wrong offset, a wrong target).
* A window whose samples are the K centers, each once: then the fit of
  eq. (10) is the fit of eq. (11), so c*(i) = A^+ b(i) and both objectives
  agree (catches a transposed design matrix and a target taken at the wrong
  point).
* p(i) equal to a center mu_m: phi(x - p(i)) is the m-th basis function, so
  c*(i) = e_m and the minimum is 0 (catches a sign or index error between
  the target and the basis).
* Two equal centers: the minimum-norm minimiser splits the weight of the
  shared basis function evenly, and the two halves add up to that center's
  coefficient in the fit without the copy (the pseudo-inverse reading).
* Optimality: the minimum is no larger than eq. (10) at the surrogate's
  c = A^+ b(i) nor at random perturbations of c*(i) (objective evaluated by
  an explicit loop).
"""
import math

import numpy as np

import oracle


def _phi(d2, sr):
    return math.exp(-d2 / (2.0 * sr * sr))


def _window(H, W, iy, ix, S):
    for qy in range(iy - S, iy + S + 1):
        for qx in range(ix - S, ix + S + 1):
            if 0 <= qy < H and 0 <= qx < W:
                yield qy, qx


def _objective_loop(p, mu, sr, S, iy, ix, c):
    rho, H, W = p.shape
    tot = 0.0
    for qy, qx in _window(H, W, iy, ix, S):
        x = p[:, qy, qx]
        target = _phi(float(((x - p[:, iy, ix]) ** 2).sum()), sr)
        fit = sum(c[k] * _phi(float(((x - mu[k]) ** 2).sum()), sr) for k in range(len(mu)))
        tot += (target - fit) ** 2
    return tot


def test_single_center_closed_form():
    rng = np.random.default_rng(1)
    p = rng.uniform(0, 1, (3, 7, 9))
    mu = np.array([[0.4, 0.5, 0.6]])
    sr, S = 0.35, 2
    C, obj, _ = oracle.exact_ls(p, mu, sr, S)
    for iy, ix in [(0, 0), (3, 4), (6, 8), (0, 5), (4, 0)]:
        sbb = sby = syy = 0.0
        for qy, qx in _window(7, 9, iy, ix, S):
            b = _phi(float(((p[:, qy, qx] - mu[0]) ** 2).sum()), sr)
            y = _phi(float(((p[:, qy, qx] - p[:, iy, ix]) ** 2).sum()), sr)
            sbb += b * b
            sby += b * y
            syy += y * y
        t = iy * 9 + ix
        assert abs(C[t, 0] - sby / sbb) <= 1e-12 * abs(sby / sbb)
        assert abs(obj[t] - (syy - sby * sby / sbb)) <= 1e-12 * syy


def test_window_of_centers_reduces_to_surrogate():
    """One row of K pixels whose guide values are the K centers; a window
    reaching across the row makes Theta_i = Lambda for every pixel."""
    rng = np.random.default_rng(2)
    K, sr = 6, 0.3
    mu = rng.uniform(0, 1, (K, 2))
    order = rng.permutation(K)
    p = mu[order].T.reshape(2, 1, K)
    C, obj, obj11 = oracle.exact_ls(p, mu, sr, S=K)
    A = oracle.kernel_matrix(mu, sr)
    assert np.linalg.cond(A) < 1e6
    P, rank, _ = oracle.pinv(A)
    assert rank == K
    B = oracle.range_weights(p, mu, sr)
    np.testing.assert_allclose(C, B @ P.T, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(obj, obj11, rtol=1e-7, atol=1e-12)
    # the surrogate fits its own samples exactly: the minimum is 0
    assert obj.max() < 1e-12


def test_pixel_at_a_center_is_exact():
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 1, (3, 8, 8))
    iy, ix = 4, 3
    mu = np.vstack([rng.uniform(0, 1, (4, 3)), p[:, iy, ix][None, :], rng.uniform(0, 1, (2, 3))])
    m = 4
    C, obj, _ = oracle.exact_ls(p, mu, 0.4, 2, pixels=[iy * 8 + ix])
    e = np.zeros(len(mu))
    e[m] = 1.0
    np.testing.assert_allclose(C[0], e, atol=1e-8)
    assert obj[0] < 1e-20


def test_duplicate_centers_share_the_weight():
    rng = np.random.default_rng(4)
    p = rng.uniform(0, 1, (3, 9, 10))
    base = rng.uniform(0, 1, (5, 3))
    dup = np.vstack([base[:1], base])  # center 0 twice
    pix = [0, 17, 44, 89]
    Cd, od, _ = oracle.exact_ls(p, dup, 0.3, 2, pixels=pix)
    Cb, ob, _ = oracle.exact_ls(p, base, 0.3, 2, pixels=pix)
    np.testing.assert_allclose(Cd[:, 0], Cd[:, 1], rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(Cd[:, 0] + Cd[:, 1], Cb[:, 0], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(Cd[:, 2:], Cb[:, 1:], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(od, ob, rtol=1e-8, atol=1e-14)


def test_minimum_is_optimal():
    rng = np.random.default_rng(5)
    p = rng.uniform(0, 1, (3, 6, 7))
    mu = rng.uniform(0, 1, (5, 3))
    sr, S = 0.3, 2
    C, obj, obj11 = oracle.exact_ls(p, mu, sr, S)
    assert np.all(obj <= obj11 * (1 + 1e-9) + 1e-15)
    for iy, ix in [(0, 0), (2, 3), (5, 6)]:
        t = iy * 7 + ix
        c = C[t]
        base = _objective_loop(p, mu, sr, S, iy, ix, c)
        assert abs(base - obj[t]) <= 1e-9 * max(base, 1e-12)
        for _ in range(5):
            d = rng.standard_normal(len(mu)) * 1e-3
            assert _objective_loop(p, mu, sr, S, iy, ix, c + d) >= base - 1e-15


def test_exact_coefficients_in_the_filter():
    """fast_filter with coef='exact' equals the recombination of eqs. (13)-(16)
    with the per-pixel minimisers, written out at one pixel."""
    rng = np.random.default_rng(6)
    f = rng.uniform(0, 1, (3, 9, 11))
    mu = rng.uniform(0, 1, (4, 3))
    sr, ss, S = 0.3, 1.5, 2
    P, _, _ = oracle.pinv(oracle.kernel_matrix(mu, sr))
    g, rh = oracle.fast_filter(f, f, mu, P, ss, sr, S, coef="exact")
    C, _, _ = oracle.exact_ls(f, mu, sr, S)
    iy, ix = 4, 5
    c = C[iy * 11 + ix]
    v = np.zeros(3)
    r = 0.0
    for qy, qx in _window(9, 11, iy, ix, S):
        w = math.exp(-((qy - iy) ** 2 + (qx - ix) ** 2) / (2 * ss * ss))
        for k in range(4):
            b = _phi(float(((f[:, qy, qx] - mu[k]) ** 2).sum()), sr)
            v += c[k] * w * b * f[:, qy, qx]
            r += c[k] * w * b
    np.testing.assert_allclose(rh[iy, ix], r, rtol=1e-10)
    np.testing.assert_allclose(g[:, iy, ix], v / r, rtol=1e-9)
