"""Pins of the oracle's learned-preconditioner network (FP64): analytic
gradient against central finite differences, a symmetric M^-1 with a
positive diagonal for arbitrary weights, the two-term Neumann series of A^-1
at the initial head weights (closed form and positive definiteness), and
bfloat16 rounding against torch's conversion."""
import numpy as np
import pytest
import torch

import oracle
from paper_1808_06381_amd import inputs, precond


def small_system(n=60, seed=3, alpha=1.5):
    cfg = inputs.base_params(n=n, box=(3.6, 3.7, 3.5), alpha=alpha, shear_rate=0.2, seed=seed)
    pos = inputs.uniform_positions(n, cfg["box"], seed)
    s = oracle.build_system(cfg, pos, 1)
    er = oracle.edge_r(cfg, pos, s, 1)
    return cfg, pos, s, er


def random_theta(seed):
    th = precond.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for name in ("v", "v0", "z", "ze", "z0"):
        off, shape = precond.LAYOUT[name]
        th[off:off + int(np.prod(shape))] = rng.normal(0, 0.3, int(np.prod(shape)))
    return th


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-3, 200), [0.0, -0.0, 1.0,
                         1.00390625, 1.01171875, 3.0e38, -2.5e-40]]).astype(np.float32)
    ref = torch.tensor(xs).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.bf16(x) for x in xs])
    assert np.array_equal(got, ref)


def test_minv_symmetric_with_positive_diagonal():
    cfg, pos, s, er = small_system()
    for seed in range(3):
        th = random_theta(seed)
        mdiag, moff = oracle.mpnn_forward(s, er, cfg["alpha"], th)
        M = oracle.dense(dict(s, val=moff, diag=mdiag))
        assert np.array_equal(M, M.T)
        assert np.all(np.diag(M) > 0)
        # the sparsity of A
        A = oracle.dense(s)
        assert np.all((M != 0) <= (A != 0))


def test_minv_is_the_neumann_series_at_initial_heads():
    """v = z = 0, ze = (0, 0, 1), z0 = 0: S_ij = What_ij and lam = softplus(v0)
    + 0.3 (= 1 up to the bf16 rounding of v0), i.e. M^-1 = D^-1/2 (lam I +
    What) D^-1/2; with lam = 1 this is D^-1 + D^-1 (D - A) D^-1, the first two
    terms of A^-1 = sum_k (D^-1 (D - A))^k D^-1.  Positive definite: the
    spectral radius of What is below 1 because A is strictly diagonally
    dominant (gamma0 > 0)."""
    cfg, pos, s, er = small_system()
    th = precond.init_params(4)
    mdiag, moff = oracle.mpnn_forward(s, er, cfg["alpha"], th)
    rows = np.repeat(np.arange(cfg["n"]), np.diff(s["rowptr"]))
    ref = -s["val"] / (s["diag"][rows] * s["diag"][s["col"]])
    np.testing.assert_allclose(moff, ref, rtol=1e-14)
    v0 = oracle.bf16(th[precond.LAYOUT["v0"][0]])
    lam = np.log1p(np.exp(v0)) + 0.3
    np.testing.assert_allclose(mdiag * s["diag"], lam, rtol=1e-14)
    assert abs(lam - 1.0) < 4e-3
    A = oracle.dense(s)
    D = np.diag(s["diag"])
    Dinv = np.diag(1.0 / s["diag"])
    neumann = Dinv + Dinv @ (D - A) @ Dinv + (lam - 1.0) * Dinv
    M = oracle.dense(dict(s, val=moff, diag=mdiag))
    np.testing.assert_allclose(M, neumann, rtol=1e-13, atol=1e-15 * np.abs(M).max())
    assert np.linalg.eigvalsh(M)[0] > 0
    # I - M A = (I - D^-1 A)^2 at lam = 1: the series' remainder
    E = np.eye(cfg["n"]) - (Dinv + Dinv @ (D - A) @ Dinv) @ A
    R = np.eye(cfg["n"]) - Dinv @ A
    np.testing.assert_allclose(E, R @ R, atol=1e-12)


@pytest.mark.parametrize("norm", ["A", "2"])
def test_loss_definition(norm):
    cfg, pos, s, er = small_system()
    th = random_theta(1)
    rng = np.random.default_rng(2)
    xstar = rng.normal(size=(cfg["n"], 3))
    A = oracle.dense(s)
    b = A @ xstar
    loss = oracle.mpnn_loss_grad(s, er, cfg["alpha"], th, b, xstar, grad=False, norm=norm)
    mdiag, moff = oracle.mpnn_forward(s, er, cfg["alpha"], th)
    M = oracle.dense(dict(s, val=moff, diag=mdiag))
    e = M @ b - xstar
    W = A if norm == "A" else np.eye(cfg["n"])
    ref = np.einsum("ic,ij,jc->", e, W, e) / np.einsum("ic,ij,jc->", xstar, W, xstar)
    assert loss == pytest.approx(ref, rel=1e-12)
    # with b = A x* the loss is the probe form ||(M A - I) x*||^2 / ||x*||^2
    E = (M @ A - np.eye(cfg["n"])) @ xstar
    assert loss == pytest.approx(np.einsum("ic,ij,jc->", E, W, E) /
                                 np.einsum("ic,ij,jc->", xstar, W, xstar), rel=1e-10)


@pytest.mark.parametrize("norm", ["A", "2"])
def test_gradient_matches_finite_differences(norm):
    cfg, pos, s, er = small_system()
    th = random_theta(7)
    rng = np.random.default_rng(5)
    xstar = rng.normal(size=(cfg["n"], 3))
    b = oracle.dense(s) @ xstar + rng.normal(0, 0.1, size=(cfg["n"], 3))
    oracle.mpnn_set_bf16(False)
    try:
        loss, g = oracle.mpnn_loss_grad(s, er, cfg["alpha"], th, b, xstar, norm=norm)
        picks = []
        for name, (off, shape) in precond.LAYOUT.items():
            size = int(np.prod(shape))
            picks += list(off + rng.choice(size, size=min(3, size), replace=False))
        checked = 0
        for k in picks:
            h = 1e-5 * max(1.0, abs(float(th[k])))
            tp = th.copy(); tp[k] += np.float32(h)
            tm = th.copy(); tm[k] -= np.float32(h)
            hp = float(tp[k]) - float(th[k]); hm = float(th[k]) - float(tm[k])
            lp = oracle.mpnn_loss_grad(s, er, cfg["alpha"], tp, b, xstar, grad=False, norm=norm)
            lm = oracle.mpnn_loss_grad(s, er, cfg["alpha"], tm, b, xstar, grad=False, norm=norm)
            fd = (lp - lm) / (hp + hm)
            assert g[k] == pytest.approx(fd, rel=2e-3, abs=1e-7 * max(1.0, abs(loss))), k
            checked += 1
        assert checked >= 60
        assert np.count_nonzero(g) > 0.5 * g.size
    finally:
        oracle.mpnn_set_bf16(True)
