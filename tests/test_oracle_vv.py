"""Pins of the oracle's velocity cross-correlation (Results section: the
velocity correlation of two chains against their separation |R_cc'|).

* a simple cubic lattice (spacing a, also under a Lees-Edwards offset that
  is a whole number of spacings) has, per particle, r_3(m) neighbours at
  distance a sqrt(m) (6, 12, 8, 6, 24, ... counted here by enumerating
  integer vectors): the pair counts per bin are n/2 times those numbers;
  a uniform velocity c gives sum = count |c|^2 exactly;
* random boxes with an arbitrary offset: the pair set and bins against a
  brute-force search over the explicit image lattice
  R_j + a Lx x + b (Ly y + delta x) + c Lz z (nearest image by distance,
  bins from r itself), a different route to the same definition;
* zero offset: the pair set from scipy's periodic k-d tree;
* the flow flag removes kappa (y - Ly/2) from the x velocity: an affine
  Couette field plus a constant gives sum = count |c|^2 to rounding;
* cell-list and brute-force pair searches give identical results.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1808_06381_amd import inputs


def lattice_shell_counts(a, r_max, nbins, reach=6):
    """neighbours per particle of an infinite simple cubic lattice, per bin"""
    g = np.arange(-reach, reach + 1)
    v = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    r = a * np.sqrt((v * v).sum(1))
    r = r[(r > 0) & (r < r_max)]
    k = np.floor(r / (r_max / nbins)).astype(int)
    return np.bincount(k, minlength=nbins)


@pytest.mark.parametrize("shift_cells", [0, 2, 5])
def test_lattice_shells(shift_cells):
    n1, a = 8, 1.25
    L = n1 * a
    cfg = inputs.base_params(n=n1 ** 3, box=(L, L, L), shear_rate=0.0)
    pos = inputs.lattice_positions((n1, n1, n1), a, origin=(0.3, 0.41, 0.17))
    # bins of 0.35 a: no shell radius a sqrt(m) lies within 1e-3 a of an edge
    r_max, nbins = 3.5 * a, 10
    c = np.array([1.0, 2.0, -0.5])
    vel = np.tile(c, (len(pos), 1))
    s, cnt, u2 = oracle.velocity_correlation(cfg, shift_cells * a, pos, vel, r_max, nbins,
                                             flow=False, cells=False)
    want = lattice_shell_counts(a, r_max, nbins) * len(pos) // 2
    np.testing.assert_array_equal(cnt, want)
    np.testing.assert_array_equal(s, cnt * 5.25)
    assert u2 == len(pos) * 5.25


def image_search(box, delta, pos, r_max, nbins, u):
    """pairs, bins and u.u by explicit images of every j, nearest by distance"""
    Lx, Ly, Lz = box
    imgs = np.array([[a * Lx + b * delta, b * Ly, c * Lz]
                     for a, b, c in itertools.product(range(-2, 3), range(-1, 2), range(-1, 2))])
    n = len(pos)
    sums = np.zeros(nbins)
    cnt = np.zeros(nbins, dtype=np.int64)
    for i in range(n - 1):
        d = pos[i][None, None, :] - (pos[i + 1:][:, None, :] + imgs[None, :, :])
        r = np.sqrt((d * d).sum(-1)).min(axis=1)
        j = np.nonzero(r < r_max)[0]
        k = np.minimum(np.floor(r[j] * nbins / r_max).astype(int), nbins - 1)
        np.add.at(cnt, k, 1)
        np.add.at(sums, k, (u[i][None, :] * u[i + 1 + j]).sum(1))
    return sums, cnt


@pytest.mark.parametrize("delta_frac", [0.0, 0.23, 0.5, 0.91])
def test_random_box_against_explicit_images(delta_frac):
    box = (9.0, 7.0, 8.0)
    cfg = inputs.base_params(n=400, box=box, shear_rate=0.3)
    rng = np.random.default_rng(11)
    pos = rng.uniform(0, 1, size=(400, 3)) * box
    vel = rng.normal(size=(400, 3))
    delta = delta_frac * box[0]
    r_max, nbins = 3.4, 17
    s, cnt, u2 = oracle.velocity_correlation(cfg, delta, pos, vel, r_max, nbins, flow=True,
                                             cells=False)
    u = vel.copy()
    u[:, 0] -= 0.3 * (pos[:, 1] - 0.5 * box[1])
    s_ref, cnt_ref = image_search(box, delta, pos, r_max, nbins, u)
    np.testing.assert_array_equal(cnt, cnt_ref)
    np.testing.assert_allclose(s, s_ref, rtol=1e-12, atol=1e-12 * np.abs(u).max() ** 2 * cnt.max())
    assert u2 == pytest.approx((u * u).sum(), rel=1e-13)


def test_zero_offset_against_periodic_kdtree():
    spatial = pytest.importorskip("scipy.spatial")
    cfg = inputs.cube_params(6000, 0.0, seed=3)
    L = cfg["box"][0]
    pos = inputs.uniform_positions(6000, cfg["box"], 3)
    vel = np.random.default_rng(4).normal(size=(6000, 3))
    r_max, nbins = 2.5, 25
    s, cnt, _ = oracle.velocity_correlation(cfg, 0.0, pos, vel, r_max, nbins, flow=False)
    tree = spatial.cKDTree(pos, boxsize=L * (1 + 1e-15))
    pr = np.array(sorted(tree.query_pairs(r_max)))
    d = pos[pr[:, 0]] - pos[pr[:, 1]]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(1))
    keep = r < r_max
    k = np.minimum(np.floor(r[keep] * nbins / r_max).astype(int), nbins - 1)
    np.testing.assert_array_equal(cnt, np.bincount(k, minlength=nbins))
    uu = (vel[pr[keep, 0]] * vel[pr[keep, 1]]).sum(1)
    np.testing.assert_allclose(s, np.bincount(k, weights=uu, minlength=nbins), rtol=1e-10,
                               atol=1e-9)


def test_flow_flag_removes_the_couette_field():
    cfg = inputs.cube_params(3000, 0.7, seed=5)
    Ly = cfg["box"][1]
    pos = inputs.uniform_positions(3000, cfg["box"], 5)
    c = np.array([0.5, -1.0, 2.0])
    vel = np.tile(c, (3000, 1))
    vel[:, 0] += 0.7 * (pos[:, 1] - 0.5 * Ly)
    s, cnt, u2 = oracle.velocity_correlation(cfg, 4.1, pos, vel, 2.0, 8, flow=True)
    np.testing.assert_allclose(s, cnt * 5.25, rtol=1e-12)
    assert u2 == pytest.approx(3000 * 5.25, rel=1e-12)
    s0, cnt0, _ = oracle.velocity_correlation(cfg, 4.1, pos, vel, 2.0, 8, flow=False)
    np.testing.assert_array_equal(cnt0, cnt)
    assert not np.allclose(s0, s)


def test_cells_equal_brute_force():
    cfg = inputs.cube_params(2500, 0.4, seed=8)
    pos = inputs.uniform_positions(2500, cfg["box"], 8)
    vel = np.random.default_rng(9).normal(size=(2500, 3))
    for delta in (0.0, 3.3, cfg["box"][0] - 1e-9):
        a = oracle.velocity_correlation(cfg, delta, pos, vel, 3.1, 31, cells=False)
        b = oracle.velocity_correlation(cfg, delta, pos, vel, 3.1, 31, cells=True)
        np.testing.assert_array_equal(a[1], b[1])
        np.testing.assert_array_equal(a[0], b[0])


def test_bad_arguments():
    cfg = inputs.cube_params(10, 0.1)
    pos = inputs.uniform_positions(10, cfg["box"], 1)
    with pytest.raises(ValueError):
        oracle.velocity_correlation(cfg, 0.0, pos, pos, 1.0, 0)
    with pytest.raises(ValueError):
        oracle.velocity_correlation(cfg, 0.0, pos, pos, -1.0, 4)
