"""Long runs in the paper's own geometry (Results section): the box of
87.6 x 43.6 x 22 lambda^3 at overlap density 1 (C = 20,060 chains), Gaussian
weight cut at 5 %, Gaussian core v/lambda^3 = 0.1, zeta = 1, alpha = 4,
dt = 0.01 tau, at the four shear rates kappa tau = 0, 0.005, 0.05, 0.5, all
four advanced together as one batch of replicas on the GPU.

After `discard` steps (the start-up trajectory the paper drops) the run
samples, every `every` steps, per replica:
* the structure factor S(q) (Eq. 5) on the Lees-Edwards grid in the
  flow-gradient plane q_z = 0 (q_x = 2 pi m_x / L_x, m_x = 0..nx-1;
  q_y from m_y = -my..my), averaged over the samples;
* the velocity cross-correlation against separation (pair sums of u.u and
  counts up to r_max = 10.9 < L_z / 2, u relative to the Couette flow).

The summary checks what the paper reports qualitatively:
* zero shear: the radially averaged S(q) has a minimum near q lambda = 2.3
  (the first shell of neighbours);
* shear: more neighbours in quadrants 2 and 4 of the flow-gradient plane
  than in 1 and 3 (the pair correlation skewed backwards);
* shear: the intensity at small q along the flow (q_x lambda of about 0.1;
  the box allows 0.072 and 0.143) grows with the shear rate, by about 20x
  between zero and the highest shear in the paper;
* the velocity correlation at alpha = 4 persists over many lambda.

Noise: the paper's thermal force acts on the background friction only
(`noise="paper"`, the default here); `--noise fdt` uses the
fluctuation-dissipation form instead.

    python -m paper_1808_06381_amd.paper_runs --steps 20000 --out run.json
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs
from . import sim as S

SHEARS = (0.0, 0.005, 0.05, 0.5)


def make_batch(noise="paper", seed=11, shears=SHEARS):
    cfgs, pos = [], []
    for r, k in enumerate(shears):
        c = inputs.paper_box(shear_rate=k, seed=seed + r)
        c["noise"] = noise
        c["stream"] = r
        cfgs.append(c)
        pos.append(inputs.uniform_positions(c["n"], c["box"], seed + 100 + r))
    return cfgs, np.concatenate(pos)


def radial(box, s_plane, my_max, dq=0.1, qmax=4.0):
    """ring average of one replica's S(m_x, m_y) plane at q_z = 0 (the
    offset-free grid of the unsheared box: q_y = 2 pi m_y / L_y)"""
    nx = s_plane.shape[0]
    mx, my = np.meshgrid(np.arange(nx), np.arange(-my_max, my_max + 1), indexing="ij")
    q = np.hypot(2 * math.pi * mx / box[0], 2 * math.pi * my / box[1])
    edges = np.arange(0.0, qmax + dq, dq)
    k = np.digitize(q.ravel(), edges) - 1
    ok = (k >= 0) & (k < len(edges) - 1) & (q.ravel() > 0)
    tot = np.bincount(k[ok], weights=s_plane.ravel()[ok], minlength=len(edges) - 1)
    cnt = np.bincount(k[ok], minlength=len(edges) - 1)
    mid = 0.5 * (edges[1:] + edges[:-1])
    good = cnt > 0
    return mid[good], tot[good] / cnt[good]


def quadrant_counts(sim, cfgs):
    """per replica, the interacting pairs whose separation lies in quadrants
    2 and 4 of the flow-gradient plane (d_x d_y < 0) and in 1 and 3 (> 0),
    from the library's pair list and positions (Lees-Edwards nearest image;
    the pair export rebuilds the system, so it runs after the other samples)"""
    pos, _, meta = sim.state()
    pr = sim.pairs()
    off = np.cumsum([0] + [c["n"] for c in cfgs])
    out = np.zeros((len(cfgs), 2))
    for r, c in enumerate(cfgs):
        sel = pr[pr[:, 0] == r]
        a = pos[off[r] + sel[:, 1]]
        b = pos[off[r] + sel[:, 2]]
        Lx, Ly, Lz = c["box"]
        delta = math.fmod(c["shear_rate"] * Ly * (meta["step"] * c["dt"]), Lx)
        dy = a[:, 1] - b[:, 1]
        sy = (dy > 0.5 * Ly).astype(float) - (dy < -0.5 * Ly).astype(float)
        dy = dy - sy * Ly
        dx = a[:, 0] - b[:, 0] - sy * delta
        dx = dx - Lx * np.round(dx / Lx)
        out[r] = [(dx * dy < 0).sum(), (dx * dy > 0).sum()]
    return out


def run(steps=20000, discard=10000, every=100, noise="paper", nx=48, my_max=24, r_max=10.9,
        nbins=109, tol=1e-8, seed=11, shears=SHEARS, log=sys.stderr):
    cfgs, pos0 = make_batch(noise, seed, shears)
    R = len(cfgs)
    box = cfgs[0]["box"]
    s_acc = np.zeros((R, nx, 2 * my_max + 1))
    vv_s = np.zeros((R, nbins))
    vv_c = np.zeros((R, nbins), dtype=np.int64)
    vv_u2 = np.zeros(R)
    quad = np.zeros((R, 2))   # neighbour pairs with d_x d_y < 0 (quadrants 2, 4) and > 0
    samples = 0
    t0 = time.perf_counter()
    with S.Sim(cfgs, pos0, tol=tol) as sim:
        sim.graph_mode(True)
        done = 0
        while done < steps:
            k = min(every, steps - done)
            sim.step(k)
            done += k
            if done > discard:
                s_acc += sim.structure_factor(nx, my_max, mz=0)
                s, c, u2 = sim.velocity_correlation(r_max, nbins, flow=True)
                vv_s += s
                vv_c += c
                vv_u2 += u2
                quad += quadrant_counts(sim, cfgs)
                samples += 1
            if done % (10 * every) == 0 or done == steps:
                print(f"# {done} steps, {time.perf_counter() - t0:.1f} s", file=log, flush=True)
        wall = time.perf_counter() - t0
    s_mean = s_acc / max(samples, 1)
    out = dict(workload="paper box 87.6 x 43.6 x 22, C = %d per replica, alpha 4, gamma0 1, "
                        "Gaussian weight cut at 5 %%, Gaussian core 0.1 kT, dt 0.01, noise %s"
                        % (cfgs[0]["n"], noise),
               shears=list(shears), steps=steps, discard=discard, every=every, samples=samples,
               wall_s=round(wall, 2),
               particle_steps_per_s=round(sum(c["n"] for c in cfgs) * steps / wall, 1))
    # zero shear: radial S(q) and its minimum in 1 < q lambda < 4
    q, sr = radial(box, s_mean[0], my_max)
    sel = (q > 1.0) & (q < 4.0)
    out["zero_shear_radial"] = dict(q=[round(float(x), 3) for x in q],
                                    s=[round(float(x), 4) for x in sr])
    out["zero_shear_min_q"] = round(float(q[sel][np.argmin(sr[sel])]), 3)
    # small q along the flow: m_x = 1, 2 at m_y = 0 (q_x = 0.072, 0.143)
    low = s_mean[:, 1:3, my_max]
    out["s_flow_qx"] = [round(2 * math.pi * m / box[0], 4) for m in (1, 2)]
    out["s_flow"] = [[round(float(x), 4) for x in row] for row in low]
    out["s_flow_growth_vs_zero_shear"] = [round(float(low[r].max() / low[0].max()), 3)
                                          for r in range(R)]
    # the brightest small-q wavevector of each replica's plane (|q| < 0.5, q != 0)
    mx, my = np.meshgrid(np.arange(nx), np.arange(-my_max, my_max + 1), indexing="ij")
    qx = 2 * math.pi * mx / box[0]
    qy = 2 * math.pi * my / box[1]
    win = (np.hypot(qx, qy) < 0.5) & ~((mx == 0) & (my == 0))
    peaks = []
    for r in range(R):
        i = np.argmax(np.where(win, s_mean[r], -np.inf))
        peaks.append(dict(s=round(float(s_mean[r].ravel()[i]), 4), mx=int(mx.ravel()[i]),
                          my=int(my.ravel()[i])))
    out["small_q_peak"] = peaks
    # mean over the small-q window of the plane (|q| < 0.3, q != 0): a
    # steadier measure of the intensity than single wavevectors
    win3 = (np.hypot(qx, qy) < 0.3) & ~((mx == 0) & (my == 0))
    wmean = [float(s_mean[r][win3].mean()) for r in range(R)]
    out["small_q_window_mean"] = [round(x, 4) for x in wmean]
    out["small_q_window_growth"] = [round(x / wmean[0], 3) for x in wmean]
    # neighbours skewed backwards under shear: (N_24 - N_13) / (N_24 + N_13)
    out["quadrant_asymmetry"] = [round(float((q[0] - q[1]) / max(q.sum(), 1)), 5) for q in quad]
    # velocity correlation, normalised by the mean square relative velocity
    n = cfgs[0]["n"]
    corr = (vv_s / np.maximum(vv_c, 1)) / (vv_u2[:, None] / (n * max(samples, 1)))
    rr = (np.arange(nbins) + 0.5) * r_max / nbins
    out["vv_r"] = [round(float(x), 3) for x in rr[::5]]
    out["vv_corr"] = [[round(float(x), 4) for x in row[::5]] for row in corr]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--discard", type=int, default=None, help="default: half of --steps")
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--noise", default="paper", choices=["paper", "fdt"])
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--out", default=None, help="write the summary JSON here")
    a = ap.parse_args(argv)
    res = run(steps=a.steps, discard=a.steps // 2 if a.discard is None else a.discard,
              every=a.every, noise=a.noise, seed=a.seed)
    txt = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(txt)


if __name__ == "__main__":
    main()
