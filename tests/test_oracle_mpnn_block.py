"""Pins of the oracle's learned preconditioner on the anisotropic block system
(3 x 3 heads, M^-1 = R Xh R with R = blockdiag(A_ii^-1/2)): with isotropic
friction it is the scalar network times I_3 for any anisotropy weights; at
the initial heads it is the two-term Neumann series of the block-Jacobi
splitting (closed form, positive definite; a wrong root R fails it); it is
symmetric and turns with the system under a rotation (a root that is not
the symmetric one fails it); the loss is its definition and the analytic
gradient matches central finite differences."""
import numpy as np
import pytest

import oracle
from paper_1808_06381_amd import inputs, precond


def block_case(n=60, seed=3, alpha=1.5, a_par=2.0, a_perp=0.5):
    cfg = inputs.base_params(n=n, box=(3.6, 3.7, 3.5), alpha=alpha, shear_rate=0.2, seed=seed)
    pos = inputs.uniform_positions(n, cfg["box"], seed)
    bs = oracle.build_block_system(cfg, pos, a_par, a_perp, 1)
    er = oracle.edge_r(cfg, pos, bs, 1)
    return cfg, pos, bs, er


def random_block_theta(seed):
    th = precond.block_params(precond.init_params(seed))
    rng = np.random.default_rng(seed + 100)
    for name in ("v", "v0", "z", "ze", "z0", "u", "u0", "s", "se", "s0"):
        off, shape = precond.BLOCK_LAYOUT[name]
        th[off:off + int(np.prod(shape))] = rng.normal(0, 0.3, int(np.prod(shape)))
    return th


def dense_blocks(bs, mdiag, moff):
    return oracle.block_dense(dict(bs, bdiag=mdiag, bval=moff))


def test_layout_sizes_agree():
    assert oracle.mpnn_block_nparams() == precond.NPARAMS_BLOCK
    assert precond.BLOCK_LAYOUT["s0"][0] == precond.NPARAMS_BLOCK - 1
    th = precond.block_params()
    assert th[precond.BLOCK_LAYOUT["s0"][0]] == 1.0
    assert np.array_equal(th[:precond.NPARAMS], precond.init_params(0))


def test_isotropic_friction_reduces_to_the_scalar_network():
    """a_par = a_perp = 1: every block of A is a multiple of I_3, the trunk sees
    exactly the scalar system, both anisotropy terms vanish, so M^-1 is the
    scalar network's times I_3 whatever the anisotropy weights; the loss is
    the scalar loss and its gradient the scalar gradient (zero for u, s)."""
    cfg, pos, bs, er = block_case(a_par=1.0, a_perp=1.0)
    s = oracle.build_system(cfg, pos, 1)
    assert np.array_equal(s["col"], bs["col"]) and np.array_equal(s["rowptr"], bs["rowptr"])
    th = random_block_theta(5)
    mdiag, moff = oracle.mpnn_block_forward(bs, er, cfg["alpha"], th)
    sd, so = oracle.mpnn_forward(s, er, cfg["alpha"], th[:precond.NPARAMS])
    I3 = np.eye(3)
    np.testing.assert_allclose(mdiag, sd[:, None, None] * I3, rtol=1e-12,
                               atol=1e-13 * np.abs(sd).max())
    np.testing.assert_allclose(moff, so[:, None, None] * I3, rtol=1e-12,
                               atol=1e-13 * np.abs(so).max())
    rng = np.random.default_rng(1)
    xstar = rng.normal(size=(cfg["n"], 3))
    b = oracle.dense(s) @ xstar
    for norm in ("2", "A"):
        lb, gb = oracle.mpnn_block_loss_grad(bs, er, cfg["alpha"], th, b, xstar, norm=norm)
        ls, gs = oracle.mpnn_loss_grad(s, er, cfg["alpha"], th[:precond.NPARAMS], b, xstar,
                                       norm=norm)
        assert lb == pytest.approx(ls, rel=1e-11)
        scale = np.abs(gs).max()
        np.testing.assert_allclose(gb[:precond.NPARAMS], gs, rtol=1e-8, atol=1e-10 * scale)
        assert np.abs(gb[precond.NPARAMS:]).max() <= 1e-10 * scale


def test_initial_heads_are_the_block_neumann_series():
    """v = z = z0 = 0, ze = (0, 0, 1), mu = 0, sig = 1: Xh_ii = lam I and
    Xh_ij = What_ij I + (Nh_ij - What_ij I) = R_i W_ij R_j, so with
    R^2 = B = D^-1, D = blockdiag(A_ii): M^-1 = lam B + B (D - A) B; at lam = 1
    the first two terms of A^-1 = sum_k (D^-1 (D - A))^k D^-1.  Positive
    definite: 2D - A = gamma0 I + sum over pairs of [[W, W], [W, W]]."""
    cfg, pos, bs, er = block_case()
    oracle.mpnn_set_bf16(False)
    try:
        th = precond.block_params(precond.init_params(4))
        lam = float(np.log1p(np.exp(np.float64(th[precond.LAYOUT["v0"][0]])))) + 0.3
        assert abs(lam - 1.0) < 1e-6
        mdiag, moff = oracle.mpnn_block_forward(bs, er, cfg["alpha"], th)
    finally:
        oracle.mpnn_set_bf16(True)
    A = oracle.block_dense(bs)
    n = cfg["n"]
    D = np.zeros_like(A)
    for i in range(n):
        D[3 * i:3 * i + 3, 3 * i:3 * i + 3] = bs["bdiag"][i]
    Binv = np.linalg.inv(D)
    ref = lam * Binv + Binv @ (D - A) @ Binv
    M = dense_blocks(bs, mdiag, moff)
    np.testing.assert_allclose(M, ref, rtol=1e-10, atol=1e-13 * np.abs(ref).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0
    assert np.linalg.eigvalsh(2 * D - A)[0] > 0
    # the remainder of the series at lam = 1: I - M A = (I - B A)^2
    M1 = Binv + Binv @ (D - A) @ Binv
    R = np.eye(3 * n) - Binv @ A
    np.testing.assert_allclose(np.eye(3 * n) - M1 @ A, R @ R, atol=1e-12)


def test_minv_symmetric_in_the_block_pattern():
    cfg, pos, bs, er = block_case()
    A = oracle.block_dense(bs)
    for seed in range(3):
        th = random_block_theta(seed)
        mdiag, moff = oracle.mpnn_block_forward(bs, er, cfg["alpha"], th)
        M = dense_blocks(bs, mdiag, moff)
        np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-13 * np.abs(M).max())
        assert np.all((M != 0) <= (A != 0))
        # genuine 3 x 3 blocks: not multiples of I_3
        off = moff - np.trace(moff, axis1=1, axis2=2)[:, None, None] / 3 * np.eye(3)
        assert np.abs(off).max() > 1e-3 * np.abs(moff).max()


def test_rotation_equivariance():
    """Rotating every block of A (A_ij -> R A_ij R^T, the system of the rotated
    configuration) rotates every block of M^-1 the same way: the heads use
    only I and A's blocks, the trunk only traces."""
    cfg, pos, bs, er = block_case()
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    rot = dict(bs, bval=np.einsum("ab,ebc,dc->ead", Q, bs["bval"], Q),
               bdiag=np.einsum("ab,ebc,dc->ead", Q, bs["bdiag"], Q))
    th = random_block_theta(2)
    md, mo = oracle.mpnn_block_forward(bs, er, cfg["alpha"], th)
    rd, ro = oracle.mpnn_block_forward(rot, er, cfg["alpha"], th)
    np.testing.assert_allclose(rd, np.einsum("ab,ebc,dc->ead", Q, md, Q), rtol=1e-9,
                               atol=1e-12 * np.abs(md).max())
    np.testing.assert_allclose(ro, np.einsum("ab,ebc,dc->ead", Q, mo, Q), rtol=1e-9,
                               atol=1e-12 * np.abs(mo).max())


@pytest.mark.parametrize("norm", ["A", "2"])
def test_block_loss_definition(norm):
    cfg, pos, bs, er = block_case()
    th = random_block_theta(1)
    rng = np.random.default_rng(2)
    xstar = rng.normal(size=(cfg["n"], 3))
    A = oracle.block_dense(bs)
    b = (A @ xstar.reshape(-1)).reshape(-1, 3)
    loss = oracle.mpnn_block_loss_grad(bs, er, cfg["alpha"], th, b, xstar, grad=False,
                                       norm=norm)
    mdiag, moff = oracle.mpnn_block_forward(bs, er, cfg["alpha"], th)
    M = dense_blocks(bs, mdiag, moff)
    e = M @ b.reshape(-1) - xstar.reshape(-1)
    W = A if norm == "A" else np.eye(A.shape[0])
    x = xstar.reshape(-1)
    assert loss == pytest.approx(e @ W @ e / (x @ W @ x), rel=1e-11)


@pytest.mark.parametrize("norm", ["A", "2"])
def test_block_gradient_matches_finite_differences(norm):
    cfg, pos, bs, er = block_case(n=50)
    th = random_block_theta(7)
    rng = np.random.default_rng(5)
    xstar = rng.normal(size=(cfg["n"], 3))
    A = oracle.block_dense(bs)
    b = (A @ xstar.reshape(-1)).reshape(-1, 3) + rng.normal(0, 0.1, size=(cfg["n"], 3))
    oracle.mpnn_set_bf16(False)
    try:
        loss, g = oracle.mpnn_block_loss_grad(bs, er, cfg["alpha"], th, b, xstar, norm=norm)
        picks = []
        for name, (off, shape) in precond.BLOCK_LAYOUT.items():
            size = int(np.prod(shape))
            picks += list(off + rng.choice(size, size=min(3, size), replace=False))
        for k in picks:
            h = 1e-5 * max(1.0, abs(float(th[k])))
            tp = th.copy(); tp[k] += np.float32(h)
            tm = th.copy(); tm[k] -= np.float32(h)
            hp = float(tp[k]) - float(th[k]); hm = float(th[k]) - float(tm[k])
            lp = oracle.mpnn_block_loss_grad(bs, er, cfg["alpha"], tp, b, xstar, grad=False,
                                             norm=norm)
            lm = oracle.mpnn_block_loss_grad(bs, er, cfg["alpha"], tm, b, xstar, grad=False,
                                             norm=norm)
            fd = (lp - lm) / (hp + hm)
            assert g[k] == pytest.approx(fd, rel=2e-3, abs=1e-7 * max(1.0, abs(loss))), k
        assert len(picks) >= 60
        for name in ("u", "u0", "s", "se", "s0"):
            off, shape = precond.BLOCK_LAYOUT[name]
            assert np.any(g[off:off + int(np.prod(shape))] != 0), name
    finally:
        oracle.mpnn_set_bf16(True)


def test_scalar_trained_weights_stay_definite_on_anisotropic_blocks():
    """The frame of R = A_ii^-1/2 is where the scalar network's S_ij was
    trained (D^-1/2 A D^-1/2 with unit diagonal): with the shipped weights and
    the default anisotropy heads (mu = 0, sig = 1) M^-1 stays positive
    definite on strongly anisotropic boxes.  (Scaling the isotropic part of
    each pair block by A_ii^-1 instead of A_ii^-1/2 makes it indefinite there:
    the weak directions of A_ii get d_i / a times too much coupling.)"""
    import os
    path = os.path.join(os.path.dirname(precond.__file__), "weights", "precond_n1e5.bin")
    th = precond.block_params(precond.load(path))
    for a_par, a_perp in ((3.0, 0.5), (0.5, 2.0)):
        # the training boxes' physics: density 1, the friction-matrix workload
        cfg = inputs.cube_params(800, 0.3, seed=41)
        pos = inputs.uniform_positions(800, cfg["box"], 41)
        bs = oracle.build_block_system(cfg, pos, a_par, a_perp, 0)
        er = oracle.edge_r(cfg, pos, bs, 0)
        mdiag, moff = oracle.mpnn_block_forward(bs, er, cfg["alpha"], th)
        M = dense_blocks(bs, mdiag, moff)
        assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0, (a_par, a_perp)
