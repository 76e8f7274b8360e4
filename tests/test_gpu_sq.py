"""Structure factor S(q) (Results section, Eq. Sfactor) of the library
against the oracle, on the Lees-Edwards-compatible grid.

Tolerance from the arithmetic: each side forms the phase 2 pi (mx sx + my sy
+ mz sz) (library) or q . R (oracle) in FP64, an error of at most about
2 pi |m| * 4 eps per term (|m| = |mx| + |my| + |mz|, eps = 2^-53), and the
library's tables take up to 7 complex multiplications by a unit step after
each sincospi (<= 16 eps more): dtheta = 2 pi |m| 4 eps + 16 eps per term,
so rho = sum_c exp(-i q.R_c) may differ by N dtheta at most and
S = |rho|^2 / N by 2 dtheta sqrt(N S) (+ dtheta^2 N); the sum order adds
N eps per term at most, far less.  The tests allow twice that bound.

* a ragged grid (nx = 40 < 64, 2 my_max + 1 = 41 > 32 spans two tiles) on
  evolved boxes, every output;
* a batch of uneven replicas (row chunks of 4096 split within replicas);
* N = 10^6 (L = 100) with sampled outputs;
* a lattice sheared with the box (Laue peaks), q = 0 (S = N), determinism
  and argument checks.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import sq as osq
from paper_1808_06381_amd import inputs
from paper_1808_06381_amd import sim as S

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


def bound(m, n, s_ref):
    mag = np.abs(m).sum(axis=1)
    dth = 2 * math.pi * np.maximum(mag, 1) * 4 * EPS + 16 * EPS
    return 2 * (2 * dth * np.sqrt(n * np.maximum(s_ref, 0)) + dth * dth * n) + 1e-14


def check(cfg, pos, step, got, nx, my_max, mz, sample=None):
    m = osq.grid_triples(nx, my_max, mz)
    flat = got.reshape(-1)
    if sample is not None:
        m, flat = m[sample], flat[sample]
    ref = osq.structure_factor(cfg["box"], oracle.le_offset(cfg, step), pos, m)
    err = np.abs(flat - ref)
    tol = bound(m, len(pos), ref)
    assert np.all(err <= tol), (np.max(err / tol), m[np.argmax(err / tol)])
    return ref


@pytest.mark.parametrize("shear,steps", [(0.0, 0), (0.5, 3)])
def test_ragged_grid_matches_oracle(shear, steps):
    cfg = inputs.cube_params(3000, shear, seed=5)
    pos0 = inputs.uniform_positions(cfg["n"], cfg["box"], 5)
    with S.Sim(cfg, pos0) as sim:
        if steps:
            sim.step(steps)
        pos, _, meta = sim.state()
        got = sim.structure_factor(40, 20, mz=1)
    assert got.shape == (1, 40, 41)
    if steps:
        assert meta["le_offset"] != 0.0
    check(cfg, pos, steps, got[0], 40, 20, 1)


def test_batch_of_uneven_replicas():
    cfgs, pos = [], []
    for r, (n, shear) in enumerate([(5000, 0.3), (700, 1.0), (9000, 0.05)]):
        c = inputs.cube_params(n, shear, seed=40 + r)
        c["stream"] = r
        cfgs.append(c)
        pos.append(inputs.uniform_positions(n, c["box"], 40 + r))
    with S.Sim(cfgs, np.concatenate(pos)) as sim:
        sim.step(2)
        p, _, _ = sim.state()
        got = sim.structure_factor(70, 18, mz=0)
    off = np.cumsum([0] + [c["n"] for c in cfgs])
    for r, c in enumerate(cfgs):
        check(c, p[off[r]:off[r + 1]], 2, got[r], 70, 18, 0)


def test_full_size_sampled():
    cfg = inputs.single_box(shear_rate=0.5, seed=3, n=1_000_000, L=100.0)["params"]
    pos0 = inputs.uniform_positions(cfg["n"], cfg["box"], 3)
    nx, my_max = 64, 64
    with S.Sim(cfg, pos0, tol=1e-8) as sim:
        sim.step(2)
        pos, _, _ = sim.state()
        got, ms = sim.structure_factor(nx, my_max, timed=True)
    assert ms > 0
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([[0, nx * (2 * my_max + 1) - 1, my_max],
                                       rng.integers(0, nx * (2 * my_max + 1), 30)]))
    ref = check(cfg, pos, 2, got[0], nx, my_max, 0, sample=sample)
    assert got[0, 0, my_max] == pytest.approx(1_000_000, rel=1e-15)   # q = 0


def test_sheared_lattice_laue_peaks_and_determinism():
    counts, a = (8, 8, 8), 1.25
    L = counts[0] * a
    cfg = inputs.base_params(n=512, box=(L, L, L), shear_rate=0.0, kT=0.0, seed=2)
    pos0 = inputs.lattice_positions(counts, a, origin=(0.3, 0.3, 0.3))
    with S.Sim(cfg, pos0) as sim:
        got = sim.structure_factor(20, 20, mz=8)
        again = sim.structure_factor(20, 20, mz=8)
    assert np.array_equal(got, again)
    m = osq.grid_triples(20, 20, 8)
    peak = np.all(m % 8 == 0, axis=1)
    s = got[0].reshape(-1)
    np.testing.assert_allclose(s[peak], 512.0, rtol=1e-12)
    assert np.max(s[~peak]) < 1e-10


def test_invalid_arguments():
    cfg = inputs.cube_params(100, 0.1, seed=1)
    pos0 = inputs.uniform_positions(100, cfg["box"], 1)
    with S.Sim(cfg, pos0) as sim:
        for args in [(0, 4, 0), (257, 4, 0), (8, -1, 0), (8, 129, 0), (8, 4, 300)]:
            with pytest.raises(S.SimError):
                sim.structure_factor(*args)


def test_largest_grid():
    # nx = 256, my_max = 128, |mz| = 256: the limits of the call, sampled outputs
    cfg = inputs.cube_params(1500, 0.7, seed=9)
    pos0 = inputs.uniform_positions(1500, cfg["box"], 9)
    with S.Sim(cfg, pos0) as sim:
        sim.step(2)
        pos, _, _ = sim.state()
        got = sim.structure_factor(256, 128, mz=-256)
    assert got.shape == (1, 256, 257)
    rng = np.random.default_rng(3)
    sample = np.unique(np.concatenate([[0, 256 * 257 - 1, 128, 255 * 257 + 128],
                                       rng.integers(0, 256 * 257, 200)]))
    check(cfg, pos, 2, got[0], 256, 128, -256, sample=sample)
