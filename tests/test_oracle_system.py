"""Pins of the oracle's friction system (Method section, Eq. 6-9).

A = gamma0*I + alpha*L(w): symmetric, non-positive off-diagonal, zero row sums
of L, smallest eigenvalue gamma0 on the uniform vector.  The right-hand side
pairs are antisymmetric (momentum), the conservative force is minus the
gradient of the paper's potential, and the thermal force satisfies the
fluctuation-dissipation identity Cov(f) = (2kT/dt) A."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1808_06381_amd import inputs


def small_cfg(**over):
    p = inputs.base_params(n=300, box=(6.0, 6.0, 6.0), shear_rate=0.3, seed=4)
    p.update(over)
    return p


def system(cfg, pos, step=0, **kw):
    return oracle.build_system(cfg, pos, step, **kw)


@pytest.mark.parametrize("law", ["poly2", "gauss"])
def test_matrix_structure(law):
    cfg = small_cfg(weight_law=law, lam=0.45, rc=1.0, alpha=2.5, gamma0=0.3)
    pos = inputs.uniform_positions(cfg["n"], cfg["box"], 9)
    s = system(cfg, pos, step=7)
    A = oracle.dense(s)
    assert np.array_equal(A, A.T)                     # bitwise symmetric
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0) and np.count_nonzero(off) == 2 * s["npairs"]
    rows = A.sum(1) - cfg["gamma0"]                   # zero row sums of L
    assert np.max(np.abs(rows)) <= 1e-13 * np.max(np.diag(A))
    ev = np.linalg.eigvalsh(A)
    assert ev[0] == pytest.approx(cfg["gamma0"], rel=1e-11)
    assert ev[-1] <= np.max(2 * np.diag(A) - cfg["gamma0"]) * (1 + 1e-12)   # Gershgorin


def test_weight_values():
    # w = (1 - r/rc)^2 at r = 0.5, rc = 1 is 1/4; the Gaussian at the 5 % cut-off is 0.05
    box = (10.0, 10.0, 10.0)
    pos = np.array([[2.0, 2.0, 2.0], [2.5, 2.0, 2.0]])
    cfg = inputs.base_params(n=2, box=box, alpha=1.0, rc=1.0, weight_law="poly2")
    s = system(cfg, pos)
    assert s["val"].tolist() == [-0.25, -0.25]
    rc = inputs.gauss_cutoff(1.0, 0.05)
    pos2 = np.array([[2.0, 2.0, 2.0], [2.0 + rc * (1 - 1e-12), 2.0, 2.0]])
    cfg2 = inputs.base_params(n=2, box=box, alpha=1.0, rc=rc, lam=1.0, weight_law="gauss")
    s2 = system(cfg2, pos2)
    assert -s2["val"][0] == pytest.approx(0.05, rel=1e-10)
    # pair strength alpha multiplies the envelope; the diagonal is gamma0 + alpha*w
    cfg3 = dict(cfg, alpha=4.0, gamma0=0.7)
    s3 = system(cfg3, pos)
    assert s3["val"][0] == -1.0 and s3["diag"].tolist() == [1.7, 1.7]


def potential_energy(cfg, pos, delta):
    """Sum of the pair potential over pairs, written from the paper's forms."""
    ij = oracle.pairs(cfg, pos, delta)
    e = 0.0
    for i, j in ij:
        d, _ = oracle.separation(cfg, delta, pos[i], pos[j])
        r2 = float(d @ d)
        if cfg["potential"] == "gauss_core":
            # U = kT * (v / lambda^3) * exp(-r^2 / (2 lambda^2)) gives Eq. 6b's force
            e += cfg["kT"] * cfg["u_amp"] * np.exp(-r2 / (2 * cfg["lam"] ** 2))
        else:
            e += cfg["u_amp"] * (1 - np.sqrt(r2) / cfg["rc"]) ** 2
    return e


@pytest.mark.parametrize("pot,lam,kT", [("gauss_core", 1.3, 1.7), ("soft", 1.0, 1.0)])
def test_conservative_force_is_minus_gradient(pot, lam, kT):
    cfg = small_cfg(n=60, box=(4.0, 4.0, 4.0), potential=pot, lam=lam, kT=kT, u_amp=0.8,
                    rc=1.9, noise="off", shear_rate=0.0)
    pos = inputs.uniform_positions(60, cfg["box"], 2)
    s = system(cfg, pos, step=0)
    h = 1e-6
    for i in (0, 7, 33):
        for c in range(3):
            pp = pos.copy(); pp[i, c] += h
            pm = pos.copy(); pm[i, c] -= h
            # keep the pair set fixed: skip coordinates whose shift changes it
            if (len(oracle.pairs(cfg, pp)) != len(oracle.pairs(cfg, pos))
                    or len(oracle.pairs(cfg, pm)) != len(oracle.pairs(cfg, pos))):
                continue
            g = (potential_energy(cfg, pp, 0.0) - potential_energy(cfg, pm, 0.0)) / (2 * h)
            assert s["fcons"][i, c] == pytest.approx(-g, rel=1e-6, abs=1e-8)


def test_pair_terms_are_antisymmetric():
    cfg = small_cfg(kT=1.0, dt=0.01, potential="soft", noise="fdt", shear_rate=0.7)
    n = cfg["n"]
    pos = inputs.uniform_positions(n, cfg["box"], 21)
    rng = np.random.default_rng(0)
    xi = rng.normal(size=(n, 3))
    m = oracle.build_system(cfg, pos, 5)["npairs"]
    eta = rng.normal(size=(m, 3))
    s = system(cfg, pos, step=5, xi=xi, eta=eta)
    assert np.max(np.abs(s["fcons"].sum(0))) < 1e-12
    # every pair term cancels in the total; what is left are the node terms
    Ly = cfg["box"][1]
    node = np.zeros(3)
    node[0] = cfg["gamma0"] * cfg["shear_rate"] * np.sum(pos[:, 1] - 0.5 * Ly)
    node += np.sqrt(2 * cfg["kT"] / cfg["dt"]) * np.sqrt(cfg["gamma0"]) * xi.sum(0)
    np.testing.assert_allclose(s["rhs"].sum(0), node, rtol=0, atol=1e-9)


def noise_map(cfg, pos, step=3):
    """Linear map G from (xi, eta) to the thermal force (rows: 3n outputs)."""
    n = cfg["n"]
    det = dict(cfg, noise="off")
    base = system(det, pos, step)["rhs"].reshape(-1)
    m = system(cfg, pos, step)["npairs"]
    cols = []
    for k in range(3 * n + 3 * m):
        xi = np.zeros(3 * n)
        eta = np.zeros(3 * max(m, 1))
        if k < 3 * n:
            xi[k] = 1.0
        else:
            eta[k - 3 * n] = 1.0
        f = system(cfg, pos, step, xi=xi.reshape(n, 3), eta=eta[:3 * m].reshape(m, 3))["rhs"]
        cols.append(f.reshape(-1) - base)
    return np.array(cols).T


@pytest.mark.parametrize("law", ["poly2", "gauss"])
def test_fdt_identity_deterministic(law):
    """G G^T = (2kT/dt) (A (x) I3): the incidence-matrix noise is FDT-consistent."""
    n = 14
    cfg = inputs.base_params(n=n, box=(2.6, 2.4, 2.5), kT=0.35, dt=0.02, alpha=1.7, gamma0=0.4,
                             rc=1.2, lam=0.6, weight_law=law, potential="soft", shear_rate=0.2)
    pos = inputs.uniform_positions(n, cfg["box"], 8)
    s = system(cfg, pos, 3)
    assert s["npairs"] > 20
    G = noise_map(cfg, pos)
    A3 = np.kron(oracle.dense(s), np.eye(3))
    np.testing.assert_allclose(G @ G.T, (2 * cfg["kT"] / cfg["dt"]) * A3, rtol=0, atol=1e-12)
    # the paper's node-only noise gives (2 gamma0 kT/dt) I instead: not FDT for alpha > 0
    Gp = noise_map(dict(cfg, noise="paper"), pos)
    np.testing.assert_allclose(Gp @ Gp.T, (2 * cfg["gamma0"] * cfg["kT"] / cfg["dt"]) *
                               np.eye(3 * n), atol=1e-12)
    assert np.max(np.abs(Gp @ Gp.T - (2 * cfg["kT"] / cfg["dt"]) * A3)) > 1e-3


def test_fdt_covariance_statistical():
    """Sampled Cov(f) dt/(2kT) == A entry-wise within 5 sigma (generator path)."""
    n = 8
    cfg = inputs.base_params(n=n, box=(2.2, 2.2, 2.2), kT=0.5, dt=0.01, alpha=1.3, gamma0=0.2,
                             rc=1.05, shear_rate=0.0, potential="none", seed=77)
    pos = inputs.uniform_positions(n, cfg["box"], 4)
    s = system(dict(cfg, noise="off"), pos, 0)
    A = oracle.dense(s)
    M = 40_000
    f = np.array([system(cfg, pos, step)["rhs"] for step in range(M)])  # positions fixed
    f -= s["rhs"][None]
    scale = cfg["dt"] / (2 * cfg["kT"])
    for c in range(3):
        cov = (f[:, :, c].T @ f[:, :, c]) / M * scale
        sig = np.sqrt((np.outer(np.diag(A), np.diag(A)) + A * A) / M)
        assert np.all(np.abs(cov - A) < 5 * sig + 1e-12)
    # components are independent
    cross = (f[:, :, 0].T @ f[:, :, 1]) / M * scale
    sig = np.sqrt(np.outer(np.diag(A), np.diag(A)) / M)
    assert np.all(np.abs(cross) < 5 * sig)
