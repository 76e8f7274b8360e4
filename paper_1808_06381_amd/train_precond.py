"""Train and evaluate the learned preconditioner on the GPU.

Training data are the friction matrices of the simulation itself: boxes of
N particles at density 1 with the friction-matrix workload physics, new
boxes with log-uniform shear rates every `episode` steps; each simulation
step supplies one matrix A and one Adam step on a white-noise probe loss
||(M^-1 A - I) z||^2 / ||z||^2 (Euclidean by default, --norm A for the
A-norm; or on the step's own b and solution with
--loss solution; all arithmetic in the library's kernels, see
``precond.train``).

Evaluation runs held-out boxes (seeds 9001..) at several shear rates with the
trained network and with Jacobi from identical initial states, and reports
CG iterations per step and the final true relative residual of each form
(--eval-only: the weights of --out as they are, at the library's floor).

    python -m paper_1808_06381_amd.train_precond --steps 20000 --n 100000 \
        --replicas 4 --out paper_1808_06381_amd/weights/precond_n1e5.bin \
        --eval-json paper_1808_06381_amd/weights/precond_n1e5.eval.json
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1808_06381_amd import inputs, precond  # noqa: E402
from paper_1808_06381_amd import sim as S  # noqa: E402


def evaluate(theta, n, seeds, shears, steps=5, tol=1e-8):
    rows = []
    for seed in seeds:
        for kappa in shears:
            cfg = inputs.cube_params(n, kappa, seed=seed)
            pos = inputs.uniform_positions(n, cfg["box"], seed)
            rec = dict(seed=seed, shear=kappa)
            for name in ("jacobi", "learned"):
                its, res, fb = [], [], 0
                with S.Sim(cfg, pos, tol=tol, precond=name) as sim:
                    if name == "learned":
                        sim.set_weights(theta)
                    for _ in range(steps):
                        st = sim.step(1)
                        its.append(max(st["iters"]))
                        res.append(max(st["relres"]))
                        fb += st["fallback"]
                rec[name] = dict(iters=float(np.mean(its)), max_relres=float(np.max(res)),
                                 fallbacks=fb)
            rows.append(rec)
            print(f"eval seed {seed} shear {kappa}: jacobi {rec['jacobi']['iters']:.1f} it, "
                  f"learned {rec['learned']['iters']:.1f} it", flush=True)
    jac = np.mean([r["jacobi"]["iters"] for r in rows])
    lrn = np.mean([r["learned"]["iters"] for r in rows])
    return dict(n=n, tol=tol, steps_per_box=steps, cases=rows, mean_iters_jacobi=float(jac),
                mean_iters_learned=float(lrn), iteration_ratio=float(lrn / jac))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lr-final", type=float, default=0.1, help="final / initial learning rate")
    ap.add_argument("--episode", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--loss", choices=("probe", "solution"), default="probe")
    ap.add_argument("--replicas", type=int, default=4)
    ap.add_argument("--norm", choices=("2", "A"), default="2")
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_1808_06381_amd", "weights",
                                                  "precond_n1e5.bin"))
    ap.add_argument("--init", default=None, help="start from these weights")
    ap.add_argument("--eval-json", default=None)
    ap.add_argument("--eval-seeds", type=int, default=10)
    ap.add_argument("--eval-only", action="store_true",
                    help="evaluate the weights of --out (no training) with the library's "
                         "current head floor; training fields of an existing --eval-json "
                         "are kept")
    args = ap.parse_args()
    if args.eval_only:
        theta = precond.load(args.out)
        ev = evaluate(theta, args.n, seeds=list(range(9001, 9001 + args.eval_seeds)),
                      shears=(0.01, 0.1, 1.0))
        old = {}
        if args.eval_json and os.path.exists(args.eval_json):
            with open(args.eval_json) as f:
                old = json.load(f)
        keep = {k: v for k, v in old.items() if k not in ev}
        ev.update(keep)
        ev["eval_lam_floor"] = precond.LAM_FLOOR
        if args.eval_json:
            with open(args.eval_json, "w") as f:
                json.dump(ev, f, indent=1)
        print(f"held-out mean CG iterations at head floor {precond.LAM_FLOOR}: jacobi "
              f"{ev['mean_iters_jacobi']:.2f}, learned {ev['mean_iters_learned']:.2f} "
              f"(ratio {ev['iteration_ratio']:.3f})", flush=True)
        return
    theta = precond.load(args.init) if args.init else None
    t0 = time.time()
    theta, losses = precond.train(args.steps, n=args.n, lr=args.lr, seed=args.seed,
                                  episode=args.episode, theta=theta, loss=args.loss,
                                  replicas=args.replicas, norm=args.norm, lr_final=args.lr_final,
                                  log_every=max(1, args.steps // 20))
    t1 = time.time()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    precond.save(args.out, theta)
    print(f"trained {args.steps} steps in {t1 - t0:.1f} s; loss first 5% "
          f"{losses[:max(1, len(losses) // 20)].mean():.4f} last 5% "
          f"{losses[-max(1, len(losses) // 20):].mean():.4f}; weights -> {args.out}", flush=True)
    if args.eval_json:
        ev = evaluate(theta, args.n, seeds=list(range(9001, 9001 + args.eval_seeds)),
                      shears=(0.01, 0.1, 1.0))
        ev.update(train_steps=args.steps, train_n=args.n, lr=args.lr, lr_final=args.lr_final,
                  episode=args.episode,
                  loss=args.loss, replicas=args.replicas, norm=args.norm,
                  train_seconds=t1 - t0, loss_first=float(losses[:len(losses) // 20].mean()),
                  loss_last=float(losses[-len(losses) // 20:].mean()))
        with open(args.eval_json, "w") as f:
            json.dump(ev, f, indent=1)
        print(f"held-out mean CG iterations: jacobi {ev['mean_iters_jacobi']:.2f}, learned "
              f"{ev['mean_iters_learned']:.2f} (ratio {ev['iteration_ratio']:.3f})", flush=True)


if __name__ == "__main__":
    main()
