"""Learned preconditioner: parameter layout, initial weights, weight files and
the training driver.  The network and its gradients run in the library's HIP
kernels (sim_train_step / sim_precond_eval); this module only sequences calls.

Network (hidden 32, three message-passing layers on the pair graph of A):
    h0_i = relu(W0 x_i + b0)                     x_i = (t_i, a_i, deg_i/8)
    layer: y_j = P h_j,  m_i = 1/8 sum_j relu(y_j + Q e_ij + c),
           h_i <- h_i + relu(U h_i + V m_i + d)  e_ij = (r_ij/rc, w_ij, What_ij)
    heads: lam'_i = softplus(v.h_i + v0),  g_ij = 2 sigmoid(z.(h_i*h_j) + ze.e_ij + z0)
    M^-1 = D^-1/2 (diag(lam) + S) D^-1/2,  S_ij = g_ij What_ij,
    lam_i = sum_j S_ij + lam'_i + 1e-3   (SPD by diagonal dominance)
With z = ze = z0 = 0 and lam'_i = 1 - sum_j What_ij it is the two-term Neumann
series D^-1 + D^-1 W D^-1 of A^-1.
"""
import math
import struct

import numpy as np

H, FN, FE, NL = 32, 3, 3, 3
L_SIZE = H * H + H * FE + H + H * H + H * H + H


def layout():
    """name -> (offset, shape) of the flat FP32 parameter vector."""
    out = {}
    off = 0

    def add(name, shape):
        nonlocal off
        out[name] = (off, shape)
        off += int(np.prod(shape))

    add("W0", (H, FN))
    add("b0", (H,))
    for l in range(NL):
        add(f"P{l}", (H, H))
        add(f"Q{l}", (H, FE))
        add(f"c{l}", (H,))
        add(f"U{l}", (H, H))
        add(f"V{l}", (H, H))
        add(f"d{l}", (H,))
    add("v", (H,))
    add("v0", (1,))
    add("z", (H,))
    add("ze", (FE,))
    add("z0", (1,))
    return out, off


LAYOUT, NPARAMS = layout()


def init_params(seed=0, scale=0.5):
    """Small random weights; heads start at g = 1 and lam' ~ 0.6 (close to the
    two-term Neumann series)."""
    rng = np.random.default_rng(seed)
    theta = np.zeros(NPARAMS, dtype=np.float32)
    for name, (off, shape) in LAYOUT.items():
        if len(shape) == 2:
            fan_in = shape[1]
            w = rng.normal(0.0, scale / math.sqrt(fan_in), size=shape)
            theta[off:off + w.size] = w.reshape(-1)
    off, _ = LAYOUT["b0"]
    theta[off:off + H] = 0.1
    off, _ = LAYOUT["v0"]
    theta[off] = math.log(math.expm1(0.6))
    for name in ("v", "z", "ze", "z0"):
        off, shape = LAYOUT[name]
        theta[off:off + int(np.prod(shape))] = 0.0
    return theta


MAGIC = b"SIMPC001"


def save(path, theta):
    theta = np.ascontiguousarray(theta, dtype=np.float32)
    with open(path, "wb") as f:
        f.write(MAGIC + struct.pack("<q", theta.size) + theta.tobytes())


def load(path):
    with open(path, "rb") as f:
        head = f.read(16)
        if head[:8] != MAGIC:
            raise ValueError("not a preconditioner weight file")
        (n,) = struct.unpack("<q", head[8:])
        theta = np.frombuffer(f.read(4 * n), dtype=np.float32).copy()
    if theta.size != NPARAMS:
        raise ValueError("weight count mismatch")
    return theta


def train(steps, n=100_000, lr=3e-3, seed=0, episode=100, shear_range=(0.01, 1.0),
          theta=None, tol=1e-10, log_every=0):
    """Train the network on (A, b, x*) triples that the simulation generates:
    boxes of n particles (density 1, the friction-matrix workload physics), a
    new box with a log-uniform shear rate every `episode` steps; each step's
    Jacobi-PCG solve (tolerance `tol`) supplies one triple and one Adam step.
    Returns (theta, losses)."""
    from . import inputs
    from . import sim as S

    rng = np.random.default_rng(seed)
    theta = init_params(seed) if theta is None else np.asarray(theta, dtype=np.float32)
    lo, hi = math.log(shear_range[0]), math.log(shear_range[1])
    losses = []
    done = 0
    while done < steps:
        kappa = math.exp(rng.uniform(lo, hi))
        box_seed = int(rng.integers(1, 2**31))
        cfg = inputs.cube_params(n, kappa, seed=box_seed)
        pos = inputs.uniform_positions(n, cfg["box"], box_seed)
        with S.Sim(cfg, pos, tol=tol, precond="jacobi") as sm:
            sm.set_weights(theta)
            for _ in range(min(episode, steps - done)):
                sm.step(1)
                losses.append(sm.train_step(lr))
                done += 1
                if log_every and done % log_every == 0:
                    print(f"train step {done}: loss {np.mean(losses[-log_every:]):.4f}",
                          flush=True)
            theta = sm.get_weights()
    return theta, np.array(losses)
