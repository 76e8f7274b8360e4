"""Pins of the oracle's conjugate-gradient solve of Eq. 9 against dense
linear algebra (numpy/LAPACK), exact-factorisation special cases and the
limits of the method (Method and Results sections)."""
import numpy as np
import pytest

import oracle
from paper_1808_06381_amd import inputs


def case(n=600, L=8.5, seed=3, **over):
    cfg = inputs.base_params(n=n, box=(L, L, L), shear_rate=0.2, seed=seed, **over)
    pos = inputs.uniform_positions(n, cfg["box"], seed)
    return cfg, pos, oracle.build_system(cfg, pos, 2)


@pytest.mark.parametrize("precond", ["jacobi", "none", "ic0"])
def test_pcg_matches_dense_cholesky(precond):
    cfg, pos, s = case(alpha=3.0)
    A = oracle.dense(s)
    ref = np.linalg.solve(A, s["rhs"])
    c = np.linalg.cholesky(A)
    ref2 = np.linalg.solve(c.T, np.linalg.solve(c, s["rhs"]))
    np.testing.assert_allclose(ref, ref2, rtol=1e-12, atol=1e-12)
    x, its, rel = oracle.pcg(s, tol=1e-13, precond=precond)
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(x - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.all(err <= kappa * 1e-13 * 2)
    assert np.all(rel <= 1e-13)
    true_res = np.linalg.norm(s["rhs"] - A @ x, axis=0) / np.linalg.norm(s["rhs"], axis=0)
    assert np.all(true_res <= 1e-13)


def test_preconditioners_reduce_iterations():
    cfg, pos, s = case(alpha=3.0, n=900, L=8.0)
    its = {p: oracle.pcg(s, tol=1e-10, precond=p)[1] for p in ("none", "jacobi", "ic0")}
    assert max(its["ic0"]) < min(its["jacobi"]) <= max(its["jacobi"]) < min(its["none"]) + 5


def test_ic0_is_exact_on_a_tree():
    """A chain of particles (graph = path) has no fill-in: IC(0) is the
    exact Cholesky factor and PCG converges in one iteration."""
    n = 40
    box = (n * 0.8, 5.0, 5.0)
    pos = np.stack([np.arange(n) * 0.8 + 0.1, np.full(n, 2.5), np.full(n, 2.5)], 1)
    cfg = inputs.base_params(n=n, box=box, alpha=2.0, rc=1.0, shear_rate=0.3)
    s = oracle.build_system(cfg, pos, 0)
    assert s["npairs"] == n   # closed ring through the periodic x boundary
    # open the ring: remove the periodic pair by a longer box
    box2 = (n * 0.8 + 1.0, 5.0, 5.0)
    cfg2 = dict(cfg, box=box2)
    s2 = oracle.build_system(cfg2, pos, 0)
    assert s2["npairs"] == n - 1
    x, its, _ = oracle.pcg(s2, tol=1e-12, precond="ic0")
    assert its == [1, 1, 1]
    np.testing.assert_allclose(x, np.linalg.solve(oracle.dense(s2), s2["rhs"]), rtol=1e-11)


def test_given_exact_inverse_converges_in_one_iteration():
    cfg, pos, s = case(n=120, L=4.5)
    Ainv = np.linalg.inv(oracle.dense(s))
    n = len(Ainv)
    rows, cols = np.nonzero(~np.eye(n, dtype=bool))
    m = dict(rowptr=np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int64), col=cols.astype(np.int64),
             val=Ainv[rows, cols].copy(), diag=np.diag(Ainv).copy())
    x, its, _ = oracle.pcg(s, tol=1e-10, precond="given", m=m)
    assert its == [1, 1, 1]


def test_zero_rhs_and_alpha_zero():
    cfg, pos, s = case(n=200, L=6.0)
    x, its, rel = oracle.pcg(s, rhs=np.zeros((200, 3)))
    assert its == [0, 0, 0] and not np.any(x)
    # alpha = 0: A = gamma0 I, v = b / gamma0, one Jacobi iteration
    cfg0, pos0, s0 = case(n=200, L=6.0, alpha=0.0)
    x0, its0, _ = oracle.pcg(s0, tol=1e-12)
    np.testing.assert_allclose(x0, s0["rhs"] / cfg0["gamma0"], rtol=1e-15)
    assert its0 == [1, 1, 1]


def test_solid_body_limit():
    """alpha -> infinity couples a connected cluster into one solid body
    (Results section): all its velocities tend to sum(b) / (m gamma0), and
    the deviation from that rigid motion falls like 1/alpha."""
    m = 30
    rng = np.random.default_rng(1)
    pos = 5.0 + np.cumsum(rng.normal(0, 0.25, (m, 3)), 0)   # a connected random walk
    devs = []
    for alpha in (1e4, 1e6):
        cfg = inputs.base_params(n=m, box=(40.0, 40.0, 40.0), alpha=alpha, gamma0=0.5, rc=1.0,
                                 shear_rate=0.4, potential="soft", noise="off")
        s = oracle.build_system(cfg, pos, 0)
        A = oracle.dense(s)
        ev = np.linalg.eigvalsh(A - cfg["gamma0"] * np.eye(m))
        assert np.sum(ev < 1e-9 * alpha) == 1        # connected: one zero mode of L
        x, _, _ = oracle.pcg(s, tol=1e-8, maxit=100000)
        mean = s["rhs"].sum(0) / (m * cfg["gamma0"])
        devs.append(np.max(np.abs(x - mean)) / np.max(np.abs(mean)))
    assert devs[1] < 1e-2
    assert devs[1] == pytest.approx(devs[0] / 100, rel=0.05)


def test_ic0_factor_reproduces_a_on_its_pattern():
    """IC(0): (L L^T)_ij = A_ij wherever A_ij != 0 (the definition), L lower
    triangular with a positive diagonal, and fill outside the pattern."""
    cfg = inputs.base_params(n=300, box=(6.0, 6.0, 6.0), seed=2)
    pos = inputs.uniform_positions(300, cfg["box"], 2)
    s = oracle.build_system(cfg, pos, 0)
    lrow, lcol, lval = oracle.ic0(s)
    A = oracle.dense(s)
    L = np.zeros_like(A)
    for i in range(cfg["n"]):
        for q in range(lrow[i], lrow[i + 1]):
            L[i, lcol[q]] = lval[q]
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) > 0)
    E = L @ L.T - A
    assert np.abs(E[A != 0]).max() <= 1e-14 * np.abs(A).max()
    assert np.abs(E[A == 0]).max() > 1e-3      # IC(0) is incomplete here
