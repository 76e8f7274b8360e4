"""Pins of the oracle's learned-preconditioner network (FP64): analytic
gradient against central finite differences, symmetric positive definite
M^-1 for arbitrary weights, the closed form of M^-1 at g = 1, and bfloat16
rounding against torch's conversion."""
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


def test_minv_symmetric_positive_definite():
    cfg, pos, s, er = small_system()
    for seed in range(3):
        th = random_theta(seed)
        mdiag, moff = oracle.mpnn_forward(s, er, cfg["alpha"], th)
        M = oracle.dense(dict(s, val=moff, diag=mdiag))
        assert np.array_equal(M, M.T)
        assert np.linalg.eigvalsh(M)[0] > 0
        # diagonal dominance of D^1/2 M D^1/2 (the construction)
        dh = np.sqrt(s["diag"])
        Mh = M * dh[:, None] * dh[None, :]
        off = np.abs(Mh - np.diag(np.diag(Mh))).sum(1)
        assert np.all(np.diag(Mh) > off)


def test_minv_offdiagonal_closed_form_at_unit_gain():
    """z = ze = z0 = 0 gives g = 1: M^-1_ij = alpha w_ij / (D_i D_j), the second
    term of the Neumann series of A^-1."""
    cfg, pos, s, er = small_system()
    th = precond.init_params(4)
    mdiag, moff = oracle.mpnn_forward(s, er, cfg["alpha"], th)
    rows = np.repeat(np.arange(cfg["n"]), np.diff(s["rowptr"]))
    ref = -s["val"] / (s["diag"][rows] * s["diag"][s["col"]])
    np.testing.assert_allclose(moff, ref, rtol=1e-14)
    what = -s["val"] / np.sqrt(s["diag"][rows] * s["diag"][s["col"]])
    a = np.bincount(rows, weights=what, minlength=cfg["n"])
    lam = mdiag * s["diag"]
    assert np.all(lam > a)          # lam_i = sum_j S_ij + softplus(.) + eps


def test_loss_definition():
    cfg, pos, s, er = small_system()
    th = random_theta(1)
    rng = np.random.default_rng(2)
    xstar = rng.normal(size=(cfg["n"], 3))
    A = oracle.dense(s)
    b = A @ xstar
    loss = oracle.mpnn_loss_grad(s, er, cfg["alpha"], th, b, xstar, grad=False)
    mdiag, moff = oracle.mpnn_forward(s, er, cfg["alpha"], th)
    M = oracle.dense(dict(s, val=moff, diag=mdiag))
    e = M @ b - xstar
    ref = np.einsum("ic,ij,jc->", e, A, e) / np.einsum("ic,ij,jc->", xstar, A, xstar)
    assert loss == pytest.approx(ref, rel=1e-12)


def test_gradient_matches_finite_differences():
    cfg, pos, s, er = small_system()
    th = random_theta(7)
    rng = np.random.default_rng(5)
    xstar = rng.normal(size=(cfg["n"], 3))
    b = oracle.dense(s) @ xstar + rng.normal(0, 0.1, size=(cfg["n"], 3))
    oracle.mpnn_set_bf16(False)
    try:
        loss, g = oracle.mpnn_loss_grad(s, er, cfg["alpha"], th, b, xstar)
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
            lp = oracle.mpnn_loss_grad(s, er, cfg["alpha"], tp, b, xstar, grad=False)
            lm = oracle.mpnn_loss_grad(s, er, cfg["alpha"], tm, b, xstar, grad=False)
            fd = (lp - lm) / (hp + hm)
            assert g[k] == pytest.approx(fd, rel=2e-3, abs=1e-7 * max(1.0, abs(loss))), k
            checked += 1
        assert checked >= 60
        assert np.count_nonzero(g) > 0.5 * g.size
    finally:
        oracle.mpnn_set_bf16(True)
