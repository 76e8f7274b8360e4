"""Pins of the oracle's counter-based generator (Philox4x64-10) and of the
Box-Muller Gaussians built on it.  These are not the paper's: the paper only
says the thermal force is a Wiener process (Method, Eq. 6a)."""
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox4x64_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 6, 7, 8), (123, 456)),
    ((2**63, 2**64 - 1, 3, 2**40), (2**64 - 1, 17)),
    ((99, 1, 2**33, 5), (20240101, 3)),
])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox bit generator increments the counter, then emits the block
    c0 = np.array(ctr, dtype=np.uint64)
    c0[0] -= np.uint64(1)
    bg = np.random.Philox(counter=c0, key=np.array(key, dtype=np.uint64))
    ref = bg.random_raw(4)
    out = oracle.philox4x64_10(ctr, key)
    assert [int(x) for x in out] == [int(x) for x in ref]


def _draws(m):
    cfg = dict(n=1, box=(1, 1, 1), kT=1, gamma0=1, alpha=0, shear_rate=0, dt=1, rc=0.1,
               seed=42, stream=3)
    return np.array([oracle.gauss4(cfg, s, 0, i, 0) for s in range(m // 64) for i in range(64)])


def test_gaussian_moments_and_ks():
    g = _draws(80_000)
    for c in range(4):
        x = g[:, c]
        assert abs(x.mean()) < 5 / np.sqrt(len(x))
        assert abs(x.var() - 1) < 5 * np.sqrt(2 / len(x))
        assert abs(np.mean(x ** 4) - 3) < 5 * np.sqrt(96 / len(x))
        assert stats.kstest(x, "norm").pvalue > 1e-4
    cc = np.corrcoef(g.T)
    assert np.all(np.abs(cc - np.eye(4)) < 5 / np.sqrt(len(g)))


def test_gaussian_counter_dependence():
    cfg = dict(n=1, box=(1, 1, 1), kT=1, gamma0=1, alpha=0, shear_rate=0, dt=1, rc=0.1, seed=1)
    a = oracle.gauss4(cfg, 3, 1, 10, 20)
    assert np.array_equal(a, oracle.gauss4(cfg, 3, 1, 10, 20))
    for other in [(4, 1, 10, 20), (3, 0, 10, 20), (3, 1, 11, 20), (3, 1, 10, 21)]:
        assert not np.array_equal(a, oracle.gauss4(cfg, *other))
    cfg2 = dict(cfg, stream=1)
    assert not np.array_equal(a, oracle.gauss4(cfg2, 3, 1, 10, 20))
