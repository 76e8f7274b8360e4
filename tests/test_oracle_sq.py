"""Pins of the oracle's structure factor S(q) (Results section, Eq. Sfactor)
on the Lees-Edwards-compatible wavevector grid.

* the wavevectors meet the image conditions q.(Lx,0,0) = 2 pi mx,
  q.(delta,Ly,0) = 2 pi my, q.(0,0,Lz) = 2 pi mz (stated as dot products
  with the image lattice, not as the grid formula);
* q = 0 gives S = C; one particle gives 1 for every q; two particles give
  the closed form 2 + 2 cos(q.(R1 - R2));
* a simple cubic lattice sheared with the box (lattice vectors (a,0,0),
  (delta/n, a, 0), (0,0,a), n cells a side) has S = C on its reciprocal
  lattice (mx, my, mz all multiples of n) and 0 elsewhere (Laue): a wrong
  sign or size of the shear term in qy breaks it;
* replacing particles by Lees-Edwards images leaves S unchanged;
* uniform random positions have mean S = 1 over q != 0.
"""
import math

import numpy as np
import pytest

from oracle import sq

BOX = (12.0, 9.0, 7.5)


def test_wavevectors_meet_the_image_conditions():
    rng = np.random.default_rng(1)
    m = rng.integers(-20, 21, size=(200, 3))
    for delta in (0.0, 3.7, 11.999):
        q = sq.le_wavevectors(BOX, delta, m)
        Lx, Ly, Lz = BOX
        np.testing.assert_allclose(q @ np.array([Lx, 0, 0]), 2 * math.pi * m[:, 0], atol=1e-11)
        np.testing.assert_allclose(q @ np.array([delta, Ly, 0]), 2 * math.pi * m[:, 1], atol=1e-11)
        np.testing.assert_allclose(q @ np.array([0, 0, Lz]), 2 * math.pi * m[:, 2], atol=1e-11)


def test_zero_vector_one_and_two_particles():
    rng = np.random.default_rng(2)
    pos = rng.uniform(0, 1, size=(50, 3)) * BOX
    assert sq.structure_factor(BOX, 2.5, pos, [[0, 0, 0]])[0] == pytest.approx(50, rel=1e-14)
    m = rng.integers(-8, 9, size=(100, 3))
    s1 = sq.structure_factor(BOX, 2.5, pos[:1], m)
    np.testing.assert_allclose(s1, 1.0, rtol=1e-13)
    q = sq.le_wavevectors(BOX, 2.5, m)
    s2 = sq.structure_factor(BOX, 2.5, pos[:2], m)
    # |e^{-i q.R1} + e^{-i q.R2}|^2 / 2 = (2 + 2 cos(q.(R1 - R2))) / 2
    np.testing.assert_allclose(s2, 1.0 + np.cos(q @ (pos[0] - pos[1])), atol=1e-13)


@pytest.mark.parametrize("delta_frac", [0.0, 0.31, 0.77])
def test_sheared_lattice_gives_laue_peaks(delta_frac):
    n, a = 6, 1.5
    L = n * a
    box = (L, L, L)
    delta = delta_frac * L
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    pos = np.stack([a * i + (delta / n) * j, a * j, a * k], axis=1) + 0.1
    pos[:, 0] %= L   # any image of each particle: S must not care
    m = np.stack(np.meshgrid(np.arange(-7, 8), np.arange(-7, 8), np.arange(-1, 2),
                             indexing="ij"), -1).reshape(-1, 3)
    s = sq.structure_factor(box, delta, pos, m)
    peak = np.all(m % n == 0, axis=1)
    np.testing.assert_allclose(s[peak], n ** 3, rtol=1e-10)
    assert np.max(s[~peak]) < 1e-9


def test_images_leave_s_unchanged():
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 1, size=(300, 3)) * BOX
    delta = 4.2
    m = rng.integers(-10, 11, size=(150, 3))
    s0 = sq.structure_factor(BOX, delta, pos, m)
    moved = pos.copy()
    sel = rng.random(300) < 0.5
    moved[sel] += np.array([delta, BOX[1], 0.0])          # through the sheared y face
    sel2 = rng.random(300) < 0.3
    moved[sel2] += np.array([-BOX[0], 0.0, BOX[2]])       # x and z faces
    s1 = sq.structure_factor(BOX, delta, moved, m)
    np.testing.assert_allclose(s1, s0, rtol=1e-9, atol=1e-9)
    # a plain (unsheared) image in y is not an image of this box: S changes
    wrong = pos.copy()
    wrong[sel] += np.array([0.0, BOX[1], 0.0])
    assert np.max(np.abs(sq.structure_factor(BOX, delta, wrong, m) - s0)) > 1e-3


def test_uniform_random_mean_is_one():
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, 1, size=(4000, 3)) * BOX
    m = sq.grid_triples(12, 12, 1)
    s = sq.structure_factor(BOX, 1.3, pos, m)
    # S(q) of independent uniform positions is exponential with mean 1
    assert abs(s.mean() - 1.0) < 5.0 / math.sqrt(len(s))


def test_chunking_and_grid_layout():
    rng = np.random.default_rng(5)
    pos = rng.uniform(0, 1, size=(1000, 3)) * BOX
    m = sq.grid_triples(5, 3, 2)
    assert m.shape == (5 * 7, 3)
    assert m[0].tolist() == [0, -3, 2] and m[6].tolist() == [0, 3, 2] and m[7].tolist() == [1, -3, 2]
    np.testing.assert_allclose(sq.structure_factor(BOX, 0.7, pos, m, chunk=7),
                               sq.structure_factor(BOX, 0.7, pos, m), rtol=1e-12)
