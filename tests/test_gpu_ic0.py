"""IC(0)-preconditioned CG on the GPU (multicolour order) against the
oracle's sequential IC(0) of the same ordering.

The ordering is computed here from the positions alone: cell coordinates
floor(x n_c / L) per axis (n_c = floor(L / r_c) cells, one cell where that
is below three, one fewer where it is odd and at least five, so that the
axis keeps two colours), colour per axis = coordinate parity, 2 for the
last cell of an odd axis (three cells), rows sorted by (colour, linear cell
index z-major x fastest, particle id).  The oracle factors and solves the
permuted system.

Checks: the factor L entry by entry (same operations in the same order:
1e-13 relative), iteration counts within 2 of the oracle's PCG, converged
velocities within kappa(A) * tol of dense LAPACK and within 1e-8 of the
Jacobi trajectory, batches and step graphs with IC(0), and the
unpreconditioned variant (u = r)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1808_06381_amd import inputs
from paper_1808_06381_amd import sim as S

pytestmark = pytest.mark.gpu


def ic_order(cfg, pos):
    """rank -> original id of the IC(0) ordering"""
    n = cfg["n"]
    nc, cell = [], []
    for k in range(3):
        m = int(np.floor(cfg["box"][k] / (cfg["rc"] * (1.0 + 1e-9))))
        m = 1 if m < 3 else m
        m = m - 1 if (m >= 5 and m % 2 == 1) else m
        c = np.floor(pos[:, k] * (m / cfg["box"][k])).astype(np.int64)
        nc.append(m)
        cell.append(np.clip(c, 0, m - 1))

    def axc(c, m):
        return np.where((m > 1) & (m % 2 == 1) & (c == m - 1), 2, c % 2)

    color = axc(cell[0], nc[0]) + 3 * (axc(cell[1], nc[1]) + 3 * axc(cell[2], nc[2]))
    lin = (cell[2] * nc[1] + cell[1]) * nc[0] + cell[0]
    return np.lexsort((np.arange(n), lin, color))


def permuted(s, perm):
    n = len(perm)
    A = sp.csr_matrix((s["val"], s["col"], s["rowptr"]), shape=(n, n))
    Ap = A[perm][:, perm].tocsr()
    Ap.sort_indices()
    return dict(rowptr=Ap.indptr.astype(np.int64), col=Ap.indices.astype(np.int64),
                val=Ap.data.copy(), diag=s["diag"][perm].copy(), rhs=s["rhs"][perm].copy())


CASES = {
    "even_cells": inputs.base_params(n=3000, box=(14.4, 14.4, 14.4), shear_rate=0.3, seed=11),
    "odd_cells": inputs.base_params(n=2300, box=(13.5, 13.2, 12.9), shear_rate=0.7, seed=12),
    "thin_axes": inputs.base_params(n=200, box=(2.6, 9.0, 2.2), shear_rate=0.8, seed=5),
    "three_cells": inputs.base_params(n=250, box=(3.4, 9.3, 7.6), shear_rate=0.5, seed=6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_ic0_factor_matches_oracle(name):
    cfg = CASES[name]
    pos0 = inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"])
    with S.Sim(cfg, pos0, precond="ic0") as sim:
        sim.step(3)                       # a non-zero Lees-Edwards offset
        pos = sim.state()[0]
        gr, gc, gv, gd = sim.precond_matrix()
    s = oracle.build_system(cfg, pos, 3)
    perm = ic_order(cfg, pos)
    lrow, lcol, lval = oracle.ic0(permuted(s, perm))
    rows, cols, vals, diag = [], [], [], np.zeros(cfg["n"])
    for k in range(cfg["n"]):
        q0, q1 = lrow[k], lrow[k + 1] - 1
        diag[perm[k]] = lval[q1]
        rows += [perm[k]] * (q1 - q0)
        cols += list(perm[lcol[q0:q1]])
        vals += list(lval[q0:q1])
    o_ = np.lexsort((cols, rows))
    rows, cols, vals = np.array(rows)[o_], np.array(cols)[o_], np.array(vals)[o_]
    g_ = np.lexsort((gc, gr))
    assert np.array_equal(gr[g_], rows) and np.array_equal(gc[g_], cols)
    np.testing.assert_allclose(gv[g_], vals, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(gd, diag, rtol=1e-13)


@pytest.mark.parametrize("name", ["even_cells", "odd_cells"])
def test_ic0_solve_matches_dense_and_oracle_iterations(name):
    cfg = CASES[name]
    n = cfg["n"]
    pos = inputs.uniform_positions(n, cfg["box"], cfg["seed"])
    b = np.random.default_rng(3).normal(size=(n, 3))
    with S.Sim(cfg, pos, tol=1e-10, precond="ic0") as sim:
        v, st = sim.solve(b)
    with S.Sim(cfg, pos, tol=1e-10) as sim:
        _, stj = sim.solve(b)
    s = oracle.build_system(cfg, pos, 0)
    A = oracle.dense(s)
    x = np.linalg.solve(A, b)
    err = np.linalg.norm(v - x, axis=0) / np.linalg.norm(x, axis=0)
    assert np.all(err <= np.linalg.cond(A) * 1e-10), err
    assert max(st["relres"]) <= 1e-10
    perm = ic_order(cfg, pos)
    _, its, _ = oracle.pcg(permuted(s, perm), rhs=b[perm], tol=1e-10, precond="ic0")
    assert max(abs(a - c) for a, c in zip(its, st["iters"])) <= 2, (its, st["iters"])
    assert max(st["iters"]) < min(stj["iters"])


def test_ic0_batch_trajectory_and_graphs():
    cfgs, pos = [], []
    for r, name in enumerate(["even_cells", "odd_cells"]):
        c = dict(CASES[name], stream=r)
        cfgs.append(c)
        pos.append(inputs.uniform_positions(c["n"], c["box"], c["seed"]))
    pos0 = np.concatenate(pos)
    out = []
    for graph in (False, True):
        with S.Sim(cfgs, pos0, tol=1e-10, precond="ic0") as sim:
            if graph:
                sim.graph_mode(True)
            for _ in range(5):
                st = sim.step(1)
                assert max(st["relres"]) <= 1e-10
            out.append(sim.state()[:2])
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    off = 0
    for c, p in zip(cfgs, pos):
        po = p.copy()
        for k in range(5):
            po, vo, _ = oracle.step(c, po, k, tol=1e-10)
        vg = out[0][1][off:off + c["n"]]
        rel = np.linalg.norm(vg - vo, axis=0) / np.linalg.norm(vo, axis=0)
        assert np.all(rel < 1e-8), rel
        off += c["n"]


def test_unpreconditioned_cg_matches_oracle():
    cfg = CASES["even_cells"]
    pos = inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"])
    b = np.random.default_rng(4).normal(size=(cfg["n"], 3))
    with S.Sim(cfg, pos, tol=1e-10, precond="none") as sim:
        v, st = sim.solve(b)
    s = oracle.build_system(cfg, pos, 0)
    xo, its, _ = oracle.pcg(s, rhs=b, tol=1e-10, precond="none")
    A = oracle.dense(s)
    assert np.all(np.linalg.norm(b - A @ v, axis=0) / np.linalg.norm(b, axis=0) <= 1e-10 * 1.001)
    assert max(abs(a - c) for a, c in zip(its, st["iters"])) <= 2, (its, st["iters"])
