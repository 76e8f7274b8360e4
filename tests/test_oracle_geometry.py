"""Pins of the oracle's Lees-Edwards geometry and truncated pair set.

The reference for the minimum image is the definition of Lees-Edwards
boundaries written as an explicit image sum: the periodic copy of particle j
in the box ny rows above sits at R_j + (nx*Lx + ny*delta, ny*Ly, nz*Lz)
(Method section: "standard Lees-Edwards boundary conditions"; image index of
Eq. 8).  The pair set is the set of pairs with r < rc (Method section: weights
below the threshold are dropped)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1808_06381_amd import inputs


def image_min(ri, rj, box, delta):
    """Nearest periodic/Lees-Edwards image of j seen from i: (d, ny, r2)."""
    Lx, Ly, Lz = box
    best = None
    for ny, nz, nx in itertools.product((-1, 0, 1), (-1, 0, 1), range(-3, 4)):
        img = np.array([rj[0] + nx * Lx + ny * delta, rj[1] + ny * Ly, rj[2] + nz * Lz])
        d = np.asarray(ri) - img
        r2 = float(d @ d)
        if best is None or r2 < best[2]:
            best = (d, ny, r2)
    return best


def brute_images(pos, box, delta, rc):
    """Independent O(N^2 * images) pair search in numpy (vectorised)."""
    Lx, Ly, Lz = box
    n = len(pos)
    r2min = np.full((n, n), np.inf)
    for ny, nz, nx in itertools.product((-1, 0, 1), (-1, 0, 1), range(-3, 4)):
        shift = np.array([nx * Lx + ny * delta, ny * Ly, nz * Lz])
        d = pos[:, None, :] - (pos[None, :, :] + shift)
        r2min = np.minimum(r2min, np.einsum("ijk,ijk->ij", d, d))
    iu = np.triu_indices(n, 1)
    return r2min[iu], np.stack(iu, 1)


def cfg_for(n, box, rc=1.0):
    return inputs.base_params(n=n, box=box, rc=rc)


@pytest.mark.parametrize("box", [(10.0, 10.0, 10.0), (7.3, 5.1, 4.4), (12.0, 3.1, 6.0)])
@pytest.mark.parametrize("delta_frac", [0.0, 0.37, 1.0 - 1e-13])
def test_separation_is_nearest_image(box, delta_frac):
    rng = np.random.default_rng(5)
    cfg = cfg_for(2, box)
    delta = delta_frac * box[0]
    for _ in range(400):
        ri = rng.uniform(0, 1, 3) * box
        # mostly close pairs, many straddling faces
        rj = ri + rng.normal(0, 0.6, 3)
        rj = np.mod(rj, box)
        d, s = oracle.separation(cfg, delta, ri, rj)
        dref, ny, r2 = image_min(ri, rj, box, delta)
        if r2 < (0.49 * min(box)) ** 2:
            assert s == ny
            np.testing.assert_allclose(d, dref, rtol=0, atol=1e-12)
        assert float(d @ d) >= r2 - 1e-12
        # sign symmetry, bit for bit
        d2, s2 = oracle.separation(cfg, delta, rj, ri)
        assert s2 == -s and np.array_equal(d2, -d)
        assert np.all(np.abs(d) <= 0.5 * np.asarray(box))


@pytest.mark.parametrize("n,box,delta_frac", [
    (300, (6.0, 6.0, 6.0), 0.0),
    (300, (6.0, 6.0, 6.0), 0.37),
    (250, (7.0, 4.5, 5.0), 0.81),
    (64, (2.6, 2.3, 2.9), 0.5),
])
def test_pairs_brute_matches_image_sum(n, box, delta_frac):
    pos = inputs.uniform_positions(n, box, seed=11)
    delta = delta_frac * box[0]
    cfg = cfg_for(n, box)
    got = oracle.pairs(cfg, pos, delta, "brute")
    r2, ij = brute_images(pos, box, delta, 1.0)
    # no pair sits on the cut-off to rounding precision, so the sets are unique
    assert np.all(np.abs(r2 - 1.0) > 1e-9)
    ref = ij[r2 < 1.0]
    assert got.shape == ref.shape and np.array_equal(got, ref)


@pytest.mark.parametrize("n,box,delta_frac,seed", [
    (2000, (13.0, 12.0, 13.0), 0.0, 1),
    (2000, (13.0, 12.0, 13.0), 0.37, 2),
    (2000, (13.0, 12.0, 13.0), 1.0 - 1e-12, 3),
    (1500, (20.0, 5.0, 15.0), 0.6, 4),
    (300, (2.5, 9.0, 2.2), 0.2, 5),    # x and z have fewer than three cells
    (300, (9.0, 2.1, 9.0), 0.9, 6),    # y has fewer than three cells
    (2, (4.0, 4.0, 4.0), 0.3, 7),
    (3, (4.0, 4.0, 4.0), 0.0, 8),
])
def test_pairs_cells_equal_brute(n, box, delta_frac, seed):
    pos = inputs.uniform_positions(n, box, seed)
    cfg = cfg_for(n, box)
    delta = delta_frac * box[0]
    a = oracle.pairs(cfg, pos, delta, "brute")
    b = oracle.pairs(cfg, pos, delta, "cells")
    assert np.array_equal(a, b)


def test_pairs_clusters_on_every_face():
    """Particles packed around all six faces, edges and the corner."""
    box = (9.0, 8.0, 7.0)
    rng = np.random.default_rng(3)
    pts = []
    for centre in [(0, 4, 3.5), (9, 4, 3.5), (4.5, 0, 3.5), (4.5, 8, 3.5), (4.5, 4, 0),
                   (4.5, 4, 7), (0, 0, 0), (9, 8, 7), (0, 8, 0)]:
        pts.append(np.asarray(centre, float) + rng.normal(0, 0.5, (40, 3)))
    pos = np.mod(np.concatenate(pts), box)
    cfg = cfg_for(len(pos), box)
    for delta in (0.0, 2.2, 8.999999999):
        a = oracle.pairs(cfg, pos, delta, "brute")
        b = oracle.pairs(cfg, pos, delta, "cells")
        assert np.array_equal(a, b) and len(a) > 100
        r2, ij = brute_images(pos, box, delta, 1.0)
        keep = np.abs(r2 - 1.0) > 1e-9
        ref = ij[(r2 < 1.0) & keep]
        got = set(map(tuple, a))
        assert set(map(tuple, ref)) <= got
        assert len(got - set(map(tuple, ref))) == int(np.sum(~keep & (r2 < 1.0)))


def test_cutoff_is_strict_and_boundary_positions():
    box = (5.0, 5.0, 5.0)
    # separation exactly rc = 1.0 along x (all values exact in binary)
    pos = np.array([[1.0, 2.0, 2.0], [2.0, 2.0, 2.0], [3.0 - 2**-40, 2.0, 2.0],
                    [5.0, 5.0, 5.0], [0.25, 0.0, 0.0]])
    cfg = cfg_for(len(pos), box)
    got = set(map(tuple, oracle.pairs(cfg, pos, 0.0, "brute")))
    assert (0, 1) not in got          # r == rc exactly: not a pair
    assert (1, 2) in got              # r just below rc
    assert (3, 4) in got              # x = L is the same point as x = 0 (r = 0.25)
    assert got == set(map(tuple, oracle.pairs(cfg, pos, 0.0, "cells")))


def test_le_offset_closed_form():
    cfg = inputs.base_params(box=(10.0, 10.0, 10.0), shear_rate=0.5, dt=0.1)
    assert oracle.le_offset(cfg, 0) == 0.0
    assert oracle.le_offset(cfg, 3) == pytest.approx(1.5, abs=1e-15)
    assert oracle.le_offset(cfg, 25) == pytest.approx(2.5, abs=1e-12)   # 12.5 mod 10
    cfg0 = dict(cfg, shear_rate=0.0)
    assert oracle.le_offset(cfg0, 1000) == 0.0


def test_wrap_crossings():
    cfg = inputs.base_params(n=4, box=(10.0, 10.0, 10.0), shear_rate=0.5, dt=0.1)
    # after step 3 the offset is 1.5
    pos = np.array([[5.0, 10.25, 5.0],    # leaves through the top: x -= delta
                    [0.5, -0.25, 5.0],    # leaves through the bottom: x += delta
                    [0.5, 10.5, -0.5],    # top crossing that also wraps x and z
                    [10.25, 3.0, 10.0]])  # plain periodic x; z == Lz stays (is Lz)
    out = oracle.wrap(cfg, pos, 3)
    np.testing.assert_allclose(out[0], [3.5, 0.25, 5.0], atol=1e-14)
    np.testing.assert_allclose(out[1], [2.0, 9.75, 5.0], atol=1e-14)
    np.testing.assert_allclose(out[2], [9.0, 0.5, 9.5], atol=1e-14)
    np.testing.assert_allclose(out[3], [0.25, 3.0, 0.0], atol=1e-14)
