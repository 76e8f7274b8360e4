"""GPU parity of the learned preconditioner (through the C ABI) against the
oracle's FP64 network: M^-1 entry by entry, the training loss and its
gradient; solves with the learned preconditioner against dense LAPACK; the
forced Jacobi fallback; an indefinite M^-1 (random head weights), which the
true-residual test and the fallback turn into the same answer; and what
training gains over Jacobi.

Tolerances: with activations kept in FP32 (round_act off) the GPU network is
an FP32 evaluation of the oracle's FP64 one on the same bfloat16 weights:
1e-4 relative on M^-1 and the loss, 1e-3 on the gradient norm and on the
gradient of every parameter tensor against that tensor's own norm.  With the
default bfloat16 activations the products see inputs rounded to 2^-9
relative, fan-in <= 64: 3e-2 relative on M^-1."""
import numpy as np
import pytest

import oracle
from paper_1808_06381_amd import inputs, precond
from paper_1808_06381_amd import sim as S

pytestmark = pytest.mark.gpu


def case(n=2000, seed=3, alpha=1.0):
    cfg = inputs.cube_params(n, 0.3, seed=seed, alpha=alpha)
    pos = inputs.uniform_positions(n, cfg["box"], seed)
    return cfg, pos


def random_theta(seed, scale=0.3):
    th = precond.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for name in ("v", "v0", "z", "ze", "z0"):
        off, shape = precond.LAYOUT[name]
        th[off:off + int(np.prod(shape))] = rng.normal(0, scale, int(np.prod(shape)))
    return th


def oracle_minv(cfg, pos, theta, step=0):
    s = oracle.build_system(cfg, pos, step)
    er = oracle.edge_r(cfg, pos, s, step)
    mdiag, moff = oracle.mpnn_forward(s, er, cfg["alpha"], theta)
    rows = np.repeat(np.arange(cfg["n"]), np.diff(s["rowptr"]))
    return s, er, mdiag, rows, s["col"], moff


def sorted_triples(rows, cols, vals):
    o = np.lexsort((cols, rows))
    return rows[o], cols[o], vals[o]


@pytest.mark.parametrize("round_act,rtol", [(False, 1e-4), (True, 3e-2)])
def test_minv_matches_oracle(round_act, rtol):
    cfg, pos = case()
    th = random_theta(1)
    with S.Sim(cfg, pos, precond="learned") as sim:
        sim.set_weights(th)
        sim.precond_config(round_act=round_act)
        gr, gc, gv, gd = sim.precond_matrix()
    s, er, md, orow, ocol, ov = oracle_minv(cfg, pos, th)
    gr, gc, gv = sorted_triples(gr, gc, gv)
    orow, ocol, ov = sorted_triples(orow, ocol, ov)
    assert np.array_equal(gr, orow) and np.array_equal(gc, ocol)
    np.testing.assert_allclose(gd, md, rtol=rtol)
    np.testing.assert_allclose(gv, ov, rtol=rtol, atol=rtol * np.abs(ov).max())


def test_minv_symmetric_with_positive_diagonal():
    cfg, pos = case(n=600, seed=5)
    for th, spd in ((random_theta(2, scale=1.0), False), (precond.init_params(2), True)):
        with S.Sim(cfg, pos, precond="learned") as sim:
            sim.set_weights(th)
            r, c, v, d = sim.precond_matrix()
        M = np.diag(d)
        M[r, c] = v
        assert np.array_equal(M, M.T) and np.all(d > 0)
        if spd:  # the initial heads: the two-term Neumann series
            assert np.linalg.eigvalsh(M)[0] > 0


def test_indefinite_preconditioner_still_gives_the_answer():
    cfg, pos = case(n=3000, seed=9)
    th = random_theta(5, scale=1.0)
    s, er, md, orow, ocol, ov = oracle_minv(cfg, pos, th)
    M = oracle.dense(dict(s, val=ov, diag=md))
    assert np.linalg.eigvalsh(M)[0] < 0     # the case this test is about
    b = np.random.default_rng(4).normal(size=(cfg["n"], 3))
    with S.Sim(cfg, pos, tol=1e-10, maxit=3000, precond="learned") as sim:
        sim.set_weights(th)
        v, st = sim.solve(b)
    A = oracle.dense(s)
    res = np.linalg.norm(b - A @ v, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(res <= 1e-10 * 1.001), (res, st)


def test_loss_and_gradient_match_oracle():
    cfg, pos = case(n=2000, seed=7)
    th = random_theta(3)
    b = np.random.default_rng(0).normal(size=(cfg["n"], 3))
    with S.Sim(cfg, pos, tol=1e-12, precond="jacobi") as sim:
        sim.set_weights(th)
        sim.precond_config(round_act=False)
        v, _ = sim.solve(b)
        loss = sim.train_step(0.0)
        g = sim.precond_grad().astype(np.float64)
    s = oracle.build_system(cfg, pos, 0)
    er = oracle.edge_r(cfg, pos, s, 0)
    lo, go = oracle.mpnn_loss_grad(s, er, cfg["alpha"], th, b, v)
    assert loss == pytest.approx(lo, rel=1e-4)
    assert np.linalg.norm(g - go) <= 1e-3 * np.linalg.norm(go)
    assert_grad_per_tensor(g, go)


def assert_grad_per_tensor(g, go):
    """Every parameter tensor's gradient against its own norm, so that an
    error in a small tensor (v0, z0, ze, a layer's Q or c) cannot hide under
    the 32 x 32 matrices: 1e-3 relative (an FP32 evaluation of the FP64
    oracle on the same weights), plus 1e-7 of the whole gradient's norm
    (FP32 rounding of the sums that feed a tensor whose own gradient is
    small)."""
    floor = 1e-7 * np.linalg.norm(go)
    for name, (off, shape) in precond.LAYOUT.items():
        sl = slice(off, off + int(np.prod(shape)))
        err = np.linalg.norm(g[sl] - go[sl])
        ref = np.linalg.norm(go[sl])
        assert ref > 0.0 or name in ("z0",), name
        assert err <= 1e-3 * ref + floor, (name, err, ref)


def oracle_probe(cfg, seed, index):
    """z of the white-noise probe from the oracle's own Philox: counter
    (index, 3, id, 0), key (seed, stream)."""
    c = dict(cfg, seed=seed)
    return np.array([oracle.gauss4(c, index, 3, i, 0)[:3] for i in range(cfg["n"])])


@pytest.mark.parametrize("batch,norm", [(False, "A"), (True, "A"), (False, "2"), (True, "2")])
def test_probe_loss_and_gradient_match_oracle(batch, norm):
    cfg, pos = case(n=1500, seed=13)
    th = random_theta(6)
    cfgs, poss = [cfg], [pos]
    if batch:
        c2, p2 = case(n=900, seed=14)
        c2["stream"] = 1
        cfgs.append(c2)
        poss.append(p2)
    b0 = np.random.default_rng(1).normal(size=(sum(c["n"] for c in cfgs), 3))
    with S.Sim(cfgs if batch else cfg, np.concatenate(poss), tol=1e-10) as sim:
        sim.set_weights(th)
        sim.precond_config(round_act=False)
        v0, _ = sim.solve(b0)
        loss = sim.train_probe(0.0, seed=77, index=5, norm=norm)
        g = sim.precond_grad().astype(np.float64)
        v1, _ = sim.solve(b0)
    assert np.array_equal(v0, v1)            # the solve's own vectors are untouched
    num = den = 0.0
    go = np.zeros_like(g)
    for c, p in zip(cfgs, poss):
        s = oracle.build_system(c, p, 0)
        er = oracle.edge_r(c, p, s, 0)
        z = oracle_probe(c, 77, 5)
        A = oracle.dense(s)
        b = A @ z
        lo, gr = oracle.mpnn_loss_grad(s, er, c["alpha"], th, b, z, norm=norm)
        dz = np.einsum("ic,ij,jc->", z, A, z) if norm == "A" else np.sum(z * z)
        num += lo * dz
        den += dz
        go += gr * dz
    assert loss == pytest.approx(num / den, rel=1e-4)
    go /= den
    assert np.linalg.norm(g - go) <= 1e-3 * np.linalg.norm(go)
    assert_grad_per_tensor(g, go)


def test_optimizer_state_moves_between_handles():
    cfg, pos = case(n=1200, seed=15)
    with S.Sim(cfg, pos, tol=1e-8) as a:
        a.set_weights(precond.init_params(1))
        a.step(1)
        for k in range(3):
            a.train_probe(1e-3, seed=1, index=k)
        th, st = a.get_weights(), a.get_optimizer()
        a.train_probe(1e-3, seed=1, index=3)
        ref = a.get_weights()
    assert st[2] == 3 and np.any(st[0] != 0) and np.all(st[1] >= 0)
    with S.Sim(cfg, pos, tol=1e-8) as b:
        b.set_weights(th)
        b.set_optimizer(st)
        b.step(1)
        b.train_probe(1e-3, seed=1, index=3)
        assert np.array_equal(b.get_weights(), ref)


def test_learned_solve_matches_dense_and_converges():
    cfg, pos = case(n=3000, seed=9)
    b = np.random.default_rng(2).normal(size=(cfg["n"], 3))
    with S.Sim(cfg, pos, tol=1e-10, precond="learned") as sim:
        sim.set_weights(precond.init_params(4))
        v, st = sim.solve(b)
    A = oracle.dense(oracle.build_system(cfg, pos, 0))
    x = np.linalg.solve(A, b)
    assert st["fallback"] == 0
    assert np.all(np.linalg.norm(b - A @ v, axis=0) / np.linalg.norm(b, axis=0) <= 1e-10 * 1.001)
    assert np.all(np.linalg.norm(v - x, axis=0) / np.linalg.norm(x, axis=0)
                  <= np.linalg.cond(A) * 1e-10)


def test_forced_fallback_gives_the_same_answer():
    cfg, pos = case(n=2000, seed=11)
    b = np.random.default_rng(3).normal(size=(cfg["n"], 3))
    with S.Sim(cfg, pos, tol=1e-10, precond="learned") as sim:
        sim.precond_config(round_act=True, learned_maxit=1)
        v, st = sim.solve(b)
    with S.Sim(cfg, pos, tol=1e-10, precond="jacobi") as ref:
        vj, _ = ref.solve(b)
    assert st["fallback"] == 1
    np.testing.assert_allclose(v, vj, rtol=0, atol=1e-8 * np.abs(vj).max())


def test_learned_trajectory_matches_oracle():
    """The preconditioner changes iteration counts, not the converged answer."""
    cfg = inputs.small_case(seed=1)["params"]
    pos0 = inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"])
    with S.Sim(cfg, pos0, tol=1e-10, precond="learned") as sim:
        sim.set_weights(precond.init_params(0))
        sim.step(5)
        pg, vg, _ = sim.state()
    po, vo, _ = oracle.run(cfg, pos0, 5, tol=1e-10)
    rel = np.linalg.norm(vg - vo, axis=0) / np.linalg.norm(vo, axis=0)
    assert np.all(rel < 1e-8)


def iterations(cfg, pos, precond_name, theta, steps=3):
    its = []
    with S.Sim(cfg, pos, tol=1e-8, precond=precond_name) as sim:
        if theta is not None:
            sim.set_weights(theta)
        for _ in range(steps):
            st = sim.step(1)
            its.append(max(st["iters"]))
            assert st["fallback"] == 0
    return np.mean(its)


def test_training_gain_over_jacobi():
    """A short training run on the simulation's own systems lowers the loss,
    and the trained preconditioner needs fewer CG iterations than Jacobi on
    held-out boxes (other seeds and shear rates)."""
    theta, losses = precond.train(160, n=8000, lr=3e-3, seed=0, episode=40)
    assert np.mean(losses[-20:]) < 0.8 * np.mean(losses[:20])
    for seed, kappa in ((9001, 0.02), (9002, 0.5)):
        cfg = inputs.cube_params(8000, kappa, seed=seed)
        pos = inputs.uniform_positions(8000, cfg["box"], seed)
        jac = iterations(cfg, pos, "jacobi", None)
        lrn = iterations(cfg, pos, "learned", theta)
        assert lrn < 0.75 * jac, (seed, jac, lrn)
