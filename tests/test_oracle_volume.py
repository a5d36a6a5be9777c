"""Pins of the oracle on a 3-D domain (Sec. III-F filters a volume).

* One slice (D = 1) reduces the 3-D brute force to the C brute force of
  eqs. (1)-(2) and the 3-D fast filter to the 2-D fast filter (both pinned
  on their own).
* Exchanging two axes of the volume commutes with both filters (the window
  and omega are isotropic): an index or a stride tied to the wrong axis
  breaks it.
* With K equal to the number of distinct guide vectors the fast filter is
  the brute force exactly (A c = b interpolates at every guide value).
* A constant volume is returned unchanged.
"""
import numpy as np

import oracle
import synth


def _vol(D, H, W, seed, n=3):
    sl = [synth.voronoi_rgb(H, W, 6, 0.05, seed + z) for z in range(D)]
    return np.stack(sl, axis=1)[:n]  # (n, D, H, W)


def test_one_slice_is_the_2d_filter():
    f = synth.voronoi_rgb(13, 17, 6, 0.05, 3)
    cen = oracle.bisecting_kmeans(f, 5).centers
    P, _, _ = oracle.pinv(oracle.kernel_matrix(cen, 0.2))
    for spatial, ss, S in (("gaussian", 1.5, 4), ("box", None, 2)):
        b3, e3 = oracle.bruteforce_volume(f[:, None], f[:, None], ss, 0.2, S, spatial)
        b2, e2 = oracle.bruteforce(f, f, ss, 0.2, S=S, spatial=spatial)
        assert np.max(np.abs(b3[:, 0] - b2)) < 1e-12 and np.max(np.abs(e3[0] - e2)) < 1e-12
        g3, r3 = oracle.fast_filter_volume(f[:, None], f[:, None], cen, P, ss, 0.2, S, spatial)
        g2, r2 = oracle.fast_filter(f, f, cen, P, ss, 0.2, S, spatial, conv_method="direct")
        assert np.max(np.abs(g3[:, 0] - g2)) < 1e-10 and np.max(np.abs(r3[0] - r2)) < 1e-10


def test_axis_exchange_commutes():
    f = _vol(4, 6, 7, 20)
    cen = oracle.bisecting_kmeans(f.reshape(3, 24, 7), 6).centers
    P, _, _ = oracle.pinv(oracle.kernel_matrix(cen, 0.25))
    g, _ = oracle.fast_filter_volume(f, f, cen, P, 1.2, 0.25, 2)
    b, _ = oracle.bruteforce_volume(f, f, 1.2, 0.25, 2)
    for perm in ((0, 2, 1, 3), (0, 1, 3, 2), (0, 3, 2, 1)):
        ft = np.ascontiguousarray(np.transpose(f, perm))
        gt, _ = oracle.fast_filter_volume(ft, ft, cen, P, 1.2, 0.25, 2)
        bt, _ = oracle.bruteforce_volume(ft, ft, 1.2, 0.25, 2)
        assert np.max(np.abs(gt - np.transpose(g, perm))) < 1e-12
        assert np.max(np.abs(bt - np.transpose(b, perm))) < 1e-12


def test_enough_clusters_is_the_bruteforce():
    rng = np.random.default_rng(4)
    vals = rng.uniform(0, 1, (5, 3))
    lab = rng.integers(0, 5, (3, 8, 9))
    g = np.transpose(vals[lab], (3, 0, 1, 2))
    f = rng.uniform(0, 1, (2, 3, 8, 9))
    P, rank, _ = oracle.pinv(oracle.kernel_matrix(vals, 0.3))
    assert rank == 5
    out, _ = oracle.fast_filter_volume(f, g, vals, P, 1.0, 0.3, 2)
    ref, _ = oracle.bruteforce_volume(f, g, 1.0, 0.3, 2)
    assert np.max(np.abs(out - ref)) < 1e-10
    # and the whole of Algorithm 1 finds those values as its clusters
    res = oracle.fhd_filter_volume(f, g, 1.0, 0.3, 5, 2)
    assert np.max(np.abs(res.out - ref)) < 1e-9


def test_hard_variant():
    """Eqs. (17)-(18) on a volume: one slice is the 2-D hard variant, and with
    every voxel equal to its cluster's center (E_K = 0) it is the brute force
    (Theorem 1's bound vanishes)."""
    f = synth.voronoi_rgb(12, 14, 5, 0.05, 8)
    cl = oracle.bisecting_kmeans(f, 4)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(cl.centers, 0.2))
    g3, _ = oracle.fast_filter_volume(f[:, None], f[:, None], cl.centers, P, 1.5, 0.2, 3, coef="hard",
                                      labels=cl.labels)
    g2, _ = oracle.fast_filter(f, f, cl.centers, P, 1.5, 0.2, 3, conv_method="direct", coef="hard",
                               labels=cl.labels)
    assert np.max(np.abs(g3[:, 0] - g2)) < 1e-10
    rng = np.random.default_rng(6)
    vals = rng.uniform(0, 1, (4, 2))
    lab = rng.integers(0, 4, (3, 7, 8))
    g = np.transpose(vals[lab], (3, 0, 1, 2))
    fv = rng.uniform(0, 1, (2, 3, 7, 8))
    res = oracle.fhd_filter_volume(fv, g, 1.0, 0.25, 4, 2, coef="hard")
    ref, _ = oracle.bruteforce_volume(fv, g, 1.0, 0.25, 2)
    assert np.max(np.abs(res.out - ref)) < 1e-7


def test_constant_volume():
    f = np.full((2, 3, 5, 4), 0.37)
    out, _ = oracle.fast_filter_volume(f, f, np.array([[0.37, 0.37]]), np.array([[1.0]]), 1.0, 0.1, 2)
    assert np.max(np.abs(out - 0.37)) < 1e-15
