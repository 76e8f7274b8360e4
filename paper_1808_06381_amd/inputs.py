"""Seeded synthetic inputs and workload parameter sets.

This module is the one place both the GPU path's callers and the CPU oracle's
tests take inputs from.  It holds no step arithmetic: only positions drawn
from numpy's seeded generator, lattices, and the parameter dicts of the
workloads (plain numbers).

Parameter dict keys (shared vocabulary of both bindings):
    n            particles
    box          (Lx, Ly, Lz); flow along x, velocity gradient along y
    kT           temperature
    gamma0       background friction (zeta of the paper's Eq. 6 and 7)
    alpha        pair-friction strength (alpha of Eq. 7)
    shear_rate   kappa (Eq. 6c, Eq. 8)
    dt           time step
    rc           pair cut-off (pairs with r < rc)
    lam          Gaussian width lambda (Gaussian weight and Gaussian core)
    u_amp        potential amplitude: v/lambda^3 (Gaussian core, Eq. 6b) or
                 epsilon (soft (1 - r/rc)^2 potential)
    weight_law   'gauss' (paper) or 'poly2' ((1 - r/rc)^2)
    potential    'gauss_core' (paper), 'soft' or 'none'
    noise        'fdt' (weighted incidence + node), 'paper' (node only), 'off'
    seed, stream Philox key words
"""
import math

import numpy as np


def gauss_cutoff(lam, threshold):
    """Distance at which exp(-r^2 / (2 lam^2)) falls to `threshold`."""
    return lam * math.sqrt(2.0 * math.log(1.0 / threshold))


def uniform_positions(n, box, seed):
    """n x 3 positions, uniform in [0, L) per axis, numpy PCG64 seeded."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(int(n), 3)) * np.asarray(box, dtype=np.float64)[None, :]


def lattice_positions(counts, spacing, origin=(0.0, 0.0, 0.0)):
    """Simple-cubic lattice, counts = (nx, ny, nz), ids in x-fastest order."""
    nx, ny, nz = counts
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    g = g.transpose(2, 1, 0, 3).reshape(-1, 3).astype(np.float64)
    return g * float(spacing) + np.asarray(origin, dtype=np.float64)[None, :]


def base_params(**over):
    """Friction-matrix workload physics: density 1, r_c = 1, (1 - r/rc)^2
    weight, soft (1 - r/rc)^2 potential of amplitude 1 kT, background
    friction 0.1, kT = 1, dt = 0.01, fluctuation-dissipation noise."""
    p = dict(n=1000, box=(10.0, 10.0, 10.0), kT=1.0, gamma0=0.1, alpha=1.0, shear_rate=0.05,
             dt=0.01, rc=1.0, lam=1.0, u_amp=1.0, weight_law="poly2", potential="soft",
             noise="fdt", seed=1, stream=0)
    p.update(over)
    return p


def cube_params(n, shear_rate, seed=1, density=1.0, **over):
    """Cubic box of side (n/density)^(1/3) with the base physics."""
    L = (n / density) ** (1.0 / 3.0)
    return base_params(n=int(n), box=(L, L, L), shear_rate=shear_rate, seed=seed, **over)


# Workloads ------------------------------------------------------------------

def small_case(seed=1):
    """N = 1000 in L = 10, kappa = 0.05, 100 steps, Jacobi-PCG to 1e-10."""
    return dict(params=base_params(n=1000, box=(10.0, 10.0, 10.0), shear_rate=0.05, seed=seed),
                steps=100, tol=1e-10)


def single_box(shear_rate=0.1, seed=1, n=1_000_000, L=100.0):
    """N = 10^6 in L = 100 (density 1), kappa in {0.01, 0.1, 0.5}, tol 1e-8."""
    return dict(params=base_params(n=int(n), box=(L, L, L), shear_rate=shear_rate, seed=seed),
                steps=1000, tol=1e-8)


def batch_replicas(count=64, seed=7, nmin=1e4, nmax=2e5, kmin=0.005, kmax=1.0):
    """`count` independent boxes, N log-uniform in [nmin, nmax] (density 1,
    cubic), shear rate log-uniform in [kmin, kmax]; one params dict each."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count))).astype(np.int64)
    ks = np.exp(rng.uniform(math.log(kmin), math.log(kmax), size=count))
    return [cube_params(int(n), float(k), seed=1000 + r, stream=r) for r, (n, k) in
            enumerate(zip(ns, ks))]


def paper_box(shear_rate=0.05, seed=1):
    """The paper's own box: 87.6 x 43.6 x 22 lambda^3 at overlap density 1,
    C = 3V/(4 pi lambda^3) chains, Gaussian weight cut at 5 %, Gaussian core
    v/lambda^3 = 0.1, zeta = 1, alpha = 4 (Method and Results sections)."""
    box = (87.6, 43.6, 22.0)
    n = int(round(3.0 * box[0] * box[1] * box[2] / (4.0 * math.pi)))
    return base_params(n=n, box=box, gamma0=1.0, alpha=4.0, shear_rate=shear_rate,
                       rc=gauss_cutoff(1.0, 0.05), lam=1.0, u_amp=0.1, weight_law="gauss",
                       potential="gauss_core", seed=seed)
