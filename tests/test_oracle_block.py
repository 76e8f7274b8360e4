"""Pins of the oracle's anisotropic friction system (block.c): pair friction
W_ij = alpha w (a_perp I + (a_par - a_perp) d d^T / r^2), so that A of Eq. 9
has 3 x 3 blocks.

* a_par = a_perp = 1: the blocks are the isotropic system's values times I3
  (bitwise off the diagonal sums), the right-hand side that of the isotropic
  assembly;
* any a: A symmetric, every block row of the pair part sums to zero, A maps
  a uniform translation to gamma0 times itself (lambda_min = gamma0), all
  eigenvalues >= gamma0;
* two particles (no potential, no noise, no shear): the relative velocity
  under opposite forces f along / across the line of centres is
  2 f / (gamma0 + 2 alpha w a_par) / 2 f / (gamma0 + 2 alpha w a_perp);
* rotating the positions rotates every block (Q W Q^T);
* FDT: over many noise draws the covariance of b (two particles, zero shear,
  no potential) is (2 kT / dt) A within five standard errors;
* an affine Couette field on a lattice whose spacing divides the box solves
  the system exactly (boundary pairs included): a wrong sign or image of the
  tensor drag W V breaks it;
* the block CG against a dense solve.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1808_06381_amd import inputs


def test_isotropic_reduction():
    cfg = inputs.cube_params(400, 0.4, seed=3)
    pos = inputs.uniform_positions(400, cfg["box"], 3)
    blk = oracle.build_block_system(cfg, pos, 1.0, 1.0, step=5)
    iso = oracle.build_system(cfg, pos, step=5)
    np.testing.assert_array_equal(blk["rowptr"], iso["rowptr"])
    np.testing.assert_array_equal(blk["col"], iso["col"])
    eye = np.eye(3)
    np.testing.assert_array_equal(blk["bval"], iso["val"][:, None, None] * eye)
    np.testing.assert_allclose(blk["bdiag"], iso["diag"][:, None, None] * eye, rtol=1e-14)
    scale = np.abs(iso["rhs"]).max()
    np.testing.assert_allclose(blk["rhs"], iso["rhs"], rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("a_par,a_perp", [(3.0, 0.5), (0.2, 2.0)])
def test_structure_and_spectrum(a_par, a_perp):
    cfg = inputs.cube_params(120, 0.3, seed=4)
    pos = inputs.uniform_positions(120, cfg["box"], 4)
    sys_ = oracle.build_block_system(cfg, pos, a_par, a_perp, step=2)
    A = oracle.block_dense(sys_)
    assert np.array_equal(A, A.T)
    n = 120
    for i in range(n):
        rowsum = sys_["bdiag"][i] - cfg["gamma0"] * np.eye(3)
        for e in range(sys_["rowptr"][i], sys_["rowptr"][i + 1]):
            rowsum = rowsum + sys_["bval"][e]
        assert np.abs(rowsum).max() <= 1e-14 * max(1.0, np.abs(sys_["bdiag"][i]).max())
    for c in range(3):
        t = np.zeros((n, 3))
        t[:, c] = 1.0
        np.testing.assert_allclose(A @ t.ravel(), cfg["gamma0"] * t.ravel(), atol=1e-13)
    assert np.linalg.eigvalsh(A).min() >= cfg["gamma0"] * (1 - 1e-12)
    x, _ = oracle.block_pcg(sys_, tol=1e-13)
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(A, sys_["rhs"].ravel()), rtol=1e-10,
                               atol=1e-10 * np.abs(x).max())


def two_particles(d, a_par, a_perp, alpha=2.0):
    cfg = inputs.base_params(n=2, box=(10.0, 10.0, 10.0), shear_rate=0.0, kT=0.0, alpha=alpha,
                             potential="none", noise="off")
    p0 = np.array([5.0, 5.0, 5.0])
    return cfg, np.stack([p0, p0 - d])


@pytest.mark.parametrize("a_par,a_perp", [(1.0, 1.0), (4.0, 0.5), (0.3, 2.5)])
def test_two_particles_closed_form(a_par, a_perp):
    rng = np.random.default_rng(7)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    d = 0.6 * u
    cfg, pos = two_particles(d, a_par, a_perp)
    sys_ = oracle.build_block_system(cfg, pos, a_par, a_perp)
    w = (1.0 - 0.6 / cfg["rc"]) ** 2
    g0, aw = cfg["gamma0"], cfg["alpha"] * w
    perp = np.cross(u, [0.0, 0.0, 1.0])
    perp /= np.linalg.norm(perp)
    for direction, a in ((u, a_par), (perp, a_perp)):
        f = 0.7 * direction
        b = np.stack([f, -f])
        x, _ = oracle.block_pcg(sys_, rhs=b, tol=1e-14)
        np.testing.assert_allclose(x[0] - x[1], 2 * f / (g0 + 2 * aw * a), rtol=1e-12, atol=1e-13)


def test_rotation_covariance():
    rng = np.random.default_rng(9)
    cfg = inputs.base_params(n=40, box=(40.0, 40.0, 40.0), shear_rate=0.0, noise="off")
    pos = 20.0 + rng.uniform(-1.5, 1.5, size=(40, 3))   # a cluster far from the faces
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    pos_r = 20.0 + (pos - 20.0) @ q.T
    a = oracle.build_block_system(cfg, pos, 2.5, 0.4)
    b = oracle.build_block_system(cfg, pos_r, 2.5, 0.4)
    np.testing.assert_array_equal(a["col"], b["col"])
    rot = np.einsum("kl,elm,nm->ekn", q, a["bval"], q)
    np.testing.assert_allclose(b["bval"], rot, atol=1e-12)


def test_noise_covariance_is_fdt():
    d = np.array([0.3, -0.25, 0.4])
    cfg, pos = two_particles(d, 3.0, 0.4)
    cfg = dict(cfg, kT=1.0, noise="fdt", dt=0.5)
    M = 8000
    bs = np.stack([oracle.build_block_system(cfg, pos, 3.0, 0.4, step=k)["rhs"].ravel()
                   for k in range(M)])
    cov = np.cov(bs.T, bias=True)
    A = oracle.block_dense(oracle.build_block_system(cfg, pos, 3.0, 0.4))
    want = (2 * cfg["kT"] / cfg["dt"]) * A
    diag = np.diag(want)
    se = np.sqrt((np.outer(diag, diag) + want ** 2) / M)
    assert np.all(np.abs(cov - want) <= 5 * se + 1e-12)
    # the isotropic-noise covariance is not: the anisotropy is in the noise
    iso = (2 * cfg["kT"] / cfg["dt"]) * oracle.block_dense(
        oracle.build_block_system(cfg, pos, 1.0, 1.0))
    assert np.any(np.abs(cov - iso) > 8 * se)


@pytest.mark.parametrize("delta_cells", [0, 3])
def test_affine_couette_lattice(delta_cells):
    n1, a = 6, 1.0
    L = n1 * a
    kappa = 0.3
    cfg = inputs.base_params(n=n1 ** 3, box=(L, L, L), shear_rate=kappa, kT=0.0, rc=1.5,
                             potential="none", noise="off", dt=1.0)
    # steps such that the offset is a whole number of spacings: kappa*L*t = delta_cells*a
    step = int(round(delta_cells * a / (kappa * L * cfg["dt"])))
    cfg = dict(cfg, dt=(delta_cells * a / (kappa * L * step)) if step else 1.0)
    pos = inputs.lattice_positions((n1, n1, n1), a, origin=(0.5, 0.5, 0.5))
    sys_ = oracle.build_block_system(cfg, pos, 2.0, 0.5, step=step)
    x, _ = oracle.block_pcg(sys_, tol=1e-14)
    want = np.zeros_like(pos)
    want[:, 0] = kappa * (pos[:, 1] - 0.5 * L)
    np.testing.assert_allclose(x, want, atol=1e-11)
