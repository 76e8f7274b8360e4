"""Learned preconditioner: parameter layout, initial weights, weight files and
the training driver.  The network and its gradients run in the library's HIP
kernels (sim_train_step / sim_precond_eval); this module only sequences calls.

Network (hidden 32, three message-passing layers on the pair graph of A):
    h0_i = relu(W0 x_i + b0)                     x_i = (t_i, a_i, deg_i/8)
    layer: y_j = P h_j,  m_i = 1/8 sum_j relu(y_j + Q e_ij + c),
           h_i <- h_i + relu(U h_i + V m_i + d)  e_ij = (r_ij/rc, w_ij, What_ij)
    heads: lam_i = softplus(v.h_i + v0) + 0.3,  S_ij = z.(h_i*h_j) + ze.e_ij + z0
    M^-1 = D^-1/2 (diag(lam) + S) D^-1/2   (symmetric, positive diagonal)
With v = z = z0 = 0, ze = (0, 0, 1) and lam = 1 it is the two-term Neumann
series D^-1 + D^-1 (D - A) D^-1 of A^-1 (positive definite), the initial
point of training.  The head is deliberately not constrained to diagonal
dominance: the best preconditioners with A's sparsity are not diagonally
dominant, and the solver's true-residual test and Jacobi fallback make an
indefinite M^-1 cost time, never correctness.  The floor 0.3 of lam adds
0.3 D^-1 to M^-1: a margin for the rare strongly coupled clusters where the
trained S outweighs lam, which grow more likely with the box (on pre-sheared
boxes at shear 0.5 it steadies N = 8e6 at 28.6 mean CG iterations against
32.2 with the floor 0.1, at a cost of 0.7 iterations at N = 1e6).
"""
import math
import struct

import numpy as np

H, FN, FE, NL = 32, 3, 3, 3
LAM_FLOOR = 0.3  # lam_i = softplus(.) + LAM_FLOOR
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


def block_layout():
    """The parameters of the 3 x 3 heads on the anisotropic block system,
    appended after the scalar network's (the trunk and the scalar heads
    lam_i and S_ij are shared):
        mu_i   = u . h_i + u0                      node anisotropy
        sig_ij = s . (h_i * h_j) + se . e_ij + s0  edge anisotropy
    In the frame R = blockdiag(A_ii^-1/2) (symmetric roots):
    Xh_ii = lam_i I + mu_i (d_i A_ii^-1 - I),
    Xh_ij = S_ij I + sig_ij (R_i W_ij R_j - What_ij I),  M^-1 = R Xh R,
    d_i = tr A_ii / 3, omega_ij = tr W_ij / 3 (A_ij = -W_ij),
    What_ij = omega_ij / sqrt(d_i d_j); the trunk sees the traces."""
    out = dict(LAYOUT)
    off = NPARAMS
    for name, shape in (("u", (H,)), ("u0", (1,)), ("s", (H,)), ("se", (FE,)), ("s0", (1,))):
        out[name] = (off, shape)
        off += int(np.prod(shape))
    return out, off


BLOCK_LAYOUT, NPARAMS_BLOCK = block_layout()


def block_params(theta=None, seed=0):
    """Weights of the block form: the scalar network's (theta, or the initial
    ones) and anisotropy heads mu = 0, sig = 1, which keep the anisotropic
    part of every normalised pair block R_i W_ij R_j: with the initial scalar
    heads M^-1 = D^-1 + D^-1 (D - A) D^-1, D = blockdiag(A_ii), the block
    two-term Neumann series (positive definite)."""
    base = init_params(seed) if theta is None else np.asarray(theta, dtype=np.float32)
    if base.size == NPARAMS_BLOCK:
        return base.copy()
    if base.size != NPARAMS:
        raise ValueError("weight count mismatch")
    out = np.zeros(NPARAMS_BLOCK, dtype=np.float32)
    out[:NPARAMS] = base
    out[BLOCK_LAYOUT["s0"][0]] = 1.0
    return out


def init_params(seed=0, scale=0.5):
    """Small random weights; the heads start at lam = softplus(v0) + eps = 1
    and S_ij = What_ij, i.e. the two-term Neumann series
    M^-1 = D^-1 + D^-1 (D - A) D^-1 (positive definite)."""
    rng = np.random.default_rng(seed)
    theta = np.zeros(NPARAMS, dtype=np.float32)
    for name, (off, shape) in LAYOUT.items():
        if len(shape) == 2:
            fan_in = shape[1]
            w = rng.normal(0.0, scale / math.sqrt(fan_in), size=shape)
            theta[off:off + w.size] = w.reshape(-1)
    off, _ = LAYOUT["b0"]
    theta[off:off + H] = 0.1
    for name in ("v", "z", "ze", "z0"):
        off, shape = LAYOUT[name]
        theta[off:off + int(np.prod(shape))] = 0.0
    off, _ = LAYOUT["v0"]
    theta[off] = math.log(math.expm1(1.0 - LAM_FLOOR))
    off, _ = LAYOUT["ze"]
    theta[off + 2] = 1.0  # edge feature 2 is What_ij
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
    if theta.size not in (NPARAMS, NPARAMS_BLOCK):
        raise ValueError("weight count mismatch")
    return theta


def train(steps, n=100_000, lr=3e-3, seed=0, episode=100, shear_range=(0.01, 1.0),
          theta=None, tol=1e-8, log_every=0, loss="probe", replicas=1, probe_seed=None,
          norm="2", lr_final=0.1):
    """Train the network on friction matrices that the simulation generates:
    boxes of n particles in total (density 1, the friction-matrix workload
    physics; `replicas` boxes of n / replicas each in one handle), new boxes
    with log-uniform shear rates every `episode` steps.  Every training step
    advances the simulation one step (Jacobi-PCG to `tol`) and takes one Adam
    step on
      loss = "probe":    ||(M^-1 A - I) z||^2 / ||z||^2, z white noise, in the
                         Euclidean (norm "2") or the A-norm (sim_train_probe), or
      loss = "solution": ||M^-1 b - x*||_A^2 / ||x*||_A^2 on the step's own
                         b and solution (sim_train_step; one replica).
    The learning rate follows a cosine from lr down to lr_final * lr; the Adam
    state carries over between boxes.  Returns (theta, losses)."""
    from . import inputs
    from . import sim as S

    if loss not in ("probe", "solution"):
        raise ValueError("loss must be 'probe' or 'solution'")
    if loss == "solution" and replicas != 1:
        raise ValueError("the solution loss trains on one replica")
    rng = np.random.default_rng(seed)
    probe_seed = seed + 0x5EED if probe_seed is None else probe_seed
    theta = init_params(seed) if theta is None else np.asarray(theta, dtype=np.float32)
    lo, hi = math.log(shear_range[0]), math.log(shear_range[1])
    losses = []
    opt = None
    done = 0
    while done < steps:
        cfgs, poss = [], []
        for r in range(replicas):
            kappa = math.exp(rng.uniform(lo, hi))
            box_seed = int(rng.integers(1, 2**31))
            c = inputs.cube_params(n // replicas, kappa, seed=box_seed)
            c["stream"] = r
            cfgs.append(c)
            poss.append(inputs.uniform_positions(c["n"], c["box"], box_seed))
        with S.Sim(cfgs if replicas > 1 else cfgs[0], np.concatenate(poss), tol=tol,
                   precond="jacobi") as sm:
            sm.set_weights(theta)
            if opt is not None:
                sm.set_optimizer(opt)
            for _ in range(min(episode, steps - done)):
                sm.step(1)
                lr_t = lr * (lr_final + (1.0 - lr_final) * 0.5 * (1.0 + math.cos(math.pi * done / steps)))
                if loss == "probe":
                    losses.append(sm.train_probe(lr_t, probe_seed, done, norm=norm))
                else:
                    losses.append(sm.train_step(lr_t))
                done += 1
                if log_every and done % log_every == 0:
                    print(f"train step {done}: loss {np.mean(losses[-log_every:]):.4f}",
                          flush=True)
            theta = sm.get_weights()
            opt = sm.get_optimizer()
    return theta, np.array(losses)
