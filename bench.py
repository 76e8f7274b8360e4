"""Benchmark of the sheared mesoscale blob step on one MI355X.

Workload (default): three single boxes of N = 10^6 particles, L = 100
(density 1, r_c = 1, (1 - r/r_c)^2 friction weight, soft potential,
background friction 0.1, kT = 1, dt = 0.01, fluctuation-dissipation noise),
one per shear rate 0.01, 0.1 and 0.5, Jacobi-PCG to a true relative residual
of 1e-8 per component, FP64.  One bench step advances each of the three
boxes by one time step (3 x 10^6 particle-steps); inputs are resident in HBM.

Each form (plain Jacobi-PCG, learned-PCG) is timed with whole steps
replayed as HIP graphs; every --probe-every-th step runs eagerly with its CG
kernels bracketed by HIP events, which gives the per-kernel durations.  A
second workload, 64 replicas of uneven size in one handle (N log-uniform in
[1e4, 2e5], shear log-uniform in [0.005, 1]), is timed the same way and
reported under "batch".

Prints one JSON line: particle-steps/s over the timed steps, the roofline of
the dominant CG kernel (algorithmic bytes per launch over its event-timed
mean duration, sampled inside the timed region), and the oracle's own
throughput on the host cores for a bounded sample of the same workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec at CG rel. residual 1e-8; learned-PCG vs plain-PCG, same GPU"
PEAK_HBM_GBS = 8000.0
# FP64 vector FMA peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
PEAK_FP64_TFLOPS = 78.6
# FP64 vector instructions: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (an add or
# multiply is one op; the 78.6 TFLOP/s figure counts a fused multiply-add as two)
PEAK_FP64_TOPS = 39.3
SHEARS = (0.01, 0.1, 0.5)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--probe-every", type=int, default=8,
                    help="every k-th step runs eagerly with every k-th CG iteration timed")
    ap.add_argument("--no-graph", action="store_true", help="eager steps only")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default lane widths of the CSR products")
    ap.add_argument("--batch", type=int, default=64, help="replicas of the batch workload (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--c5", action="store_true",
                    help="the scale workloads instead: one N = 8e6 box (L = 200) and 16 replicas "
                         "of N = 5e5, shear 0.5, from a pre-sheared state")
    ap.add_argument("--c5-preshear", type=int, default=2000,
                    help="plain steps at shear 0.5 before timing (from uniform positions)")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-spmv", action="store_true")
    ap.add_argument("--no-aniso", action="store_true",
                    help="skip the anisotropic-friction (3x3 block) measurement")
    ap.add_argument("--forms", default="plain,learned,ic0",
                    help="comma list of CG forms to time: plain (Jacobi-PCG), learned, ic0")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1808_06381_amd", "weights",
                                                      "precond_n1e5.bin"))
    ap.set_defaults(event_over_us=0.0)  # set from the event probe before any timing
    return ap.parse_args()


def kernel_source_sha():
    """Hash of the sources of the CG kernels the traffic record covers."""
    h = hashlib.sha256()
    for f in ("cg.hip", "sim_dev.h"):
        with open(os.path.join(ROOT, "paper_1808_06381_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload_key, form):
    """HBM traffic per launch of `kernel` from the committed counter summary,
    if it was taken on the current kernel sources, workload and CG form
    (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("#") or "=" not in line:
            continue
        k, v = line.split("=", 1)
        rec[k.strip()] = v.strip()
    if (rec.get("workload") != workload_key or rec.get("form") != form or
            rec.get("source_sha") != kernel_source_sha()):
        return None
    try:
        return float(rec[f"{kernel}.traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, pos0, steps, tol):
    import oracle

    t0 = time.perf_counter()
    oracle.run(cfg, pos0, steps, tol=tol)
    dt = time.perf_counter() - t0
    return dict(value=cfg["n"] * steps / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{steps} steps of the N={cfg['n']} box at shear {cfg['shear_rate']} "
                       f"from the same initial positions, single-threaded FP64 oracle, "
                       f"{dt:.1f} s")


def measure_sq(sim, n, np, nx=64, my_max=64, reps=3):
    """Structure factor of the final state (Eq. Sfactor, 64 x 129 wavevectors,
    mz = 0): the contraction kernel's event-timed duration less the event
    overhead, and its FP64 rate at 8 flops (one complex multiply-add) per
    particle and wavevector."""
    sim.structure_factor(nx, my_max)  # untimed first call (scratch, code load)
    ms = []
    for _ in range(reps):
        s, t = sim.structure_factor(nx, my_max, timed=True)
        ms.append(t)
    ny = 2 * my_max + 1
    kernel_ms = float(np.mean(ms))
    flops = 8.0 * n * nx * ny
    return dict(grid=f"mx 0..{nx - 1} x my -{my_max}..{my_max}, mz 0", particles=n,
                kernel_ms_events=round(kernel_ms, 4), flops_per_call=flops,
                s_q0=float(s[0, 0, my_max]))


# FP64 operations of one accepted pair in the velocity correlation:
# separation 3, r^2 5, cut-off compare 1, bin scale 1, u_i . u_j 5,
# fixed-point scale and rounding 2
VV_OPS_PER_PAIR = 17


def measure_vv(sim, n, np, r_max=10.0, nbins=100, reps=3):
    """Velocity cross-correlation of the last step (Results section), pairs
    with r < r_max = 10 in bins of 0.1: the pair kernel's event-timed
    duration and its rate in accepted pairs (each unordered pair is tested
    once)."""
    sim.velocity_correlation(r_max, nbins)  # untimed first call (scratch)
    ms = []
    for _ in range(reps):
        s, c, u2, t = sim.velocity_correlation(r_max, nbins, timed=True)
        ms.append(t)
    pairs = int(c.sum())
    norm = (s[0] / np.maximum(c[0], 1)) / (u2[0] / n)
    return dict(r_max=r_max, nbins=nbins, particles=n, pairs=pairs,
                kernel_ms_events=round(float(np.mean(ms)), 4),
                corr_bins_0_to_2=[round(float(x), 5) for x in norm[:20]])


def measure_aniso(args, S, inputs, np, a_par=2.0, a_perp=0.5, warm=3, steps=10):
    """Anisotropic pair friction (3 x 3 blocks, block-Jacobi CG over the 3n
    coupled unknowns) on the shear-0.1 box: eager steps, whole-step rate."""
    cfg = inputs.single_box(shear_rate=0.1, seed=1, n=args.n, L=round(args.n ** (1 / 3), 6))["params"]
    cfg = dict(cfg, friction_par=a_par, friction_perp=a_perp)
    pos0 = inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"])
    with S.Sim(cfg, pos0, tol=args.tol) as sim:
        sim.step(warm)
        its = []
        t0 = time.perf_counter()
        for _ in range(steps):
            st = sim.step(1)
            its.append(st["iters"][0])
        dt = time.perf_counter() - t0
        nnz = st["nnz"]
        rows = (cfg["n"] + 1023) // 1024 * 1024   # rows padded to whole 1024-row tiles
    return dict(workload=f"the N={cfg['n']} box at shear 0.1 with pair friction a_par={a_par} "
                         f"along and a_perp={a_perp} across the line of centres",
                value=round(cfg["n"] * steps / dt, 1), unit="particle-steps/s",
                ms_per_step=round(dt / steps * 1e3, 3), steps=steps,
                mean_cg_iters=round(float(np.mean(its)), 2),
                # block product per launch: row pointers 8, own vector 24,
                # diagonal block 48, result 24 B per row; block 48 + column 4 B
                # per entry (each gathered vector counted once)
                k_bcg_spmv_bytes_per_launch=104 * rows + 52 * nnz)


def time_form(args, S, cfgs, pos0s, form, theta, stream, torch, np, steps=None, label="",
              after=None):
    """Warm up, then time `steps` bench steps of the systems (one handle per
    entry of cfgs; an entry may be a list of replicas) with one CG form."""
    steps = args.steps if steps is None else steps
    sims = []
    for cfg, pos0 in zip(cfgs, pos0s):
        sim = S.Sim(cfg, pos0, tol=args.tol, maxit=5000,
                    spmv_fp32=1 if args.fp32_spmv else 0, stream=stream,
                    precond={"plain": "jacobi"}.get(form, form))
        if form == "learned":
            sim.set_weights(theta)
        if not args.no_graph:
            sim.graph_mode(True)
        sims.append(sim)
    print(f"# {label}form {form}: warmup {args.warmup}, timed {steps}", file=sys.stderr, flush=True)
    for k in range(args.warmup):
        for sim in sims:
            sim.step(1)
    tuning = []
    if not args.no_autotune:
        for sim in sims:
            tuning.append(sim.autotune(reps=10))
            sim.step(1)  # re-records the step graph with the chosen variants
    for sim in sims:
        sim.profile_read(reset=True)
        sim.profile_enable(args.probe_every)
    iters, fallbacks = [], 0
    rowstat = [None] * len(sims)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        for q, sim in enumerate(sims):
            st = sim.step(1)
            iters.append(max(st["iters"]))
            fallbacks += st["fallback"]
            rowstat[q] = (st["nnz"], st["max_row"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    extra = after(sims) if after else None
    prof = {}
    graphs = dict(captures=0, replays=0)
    for sim in sims:
        for k, v in sim.graph_info().items():
            graphs[k] += v
        for name, rec in sim.profile_read(reset=True).items():
            acc = prof.setdefault(name, dict(launches=0, ms=0.0, bytes=0.0))
            for f in ("launches", "ms", "bytes"):
                acc[f] += rec[f]
        sim.close()
    print(f"# {label}form {form}: {steps} steps x {len(sims)} handles in {elapsed:.3f} s; "
          f"mean CG iterations {np.mean(iters):.1f}; graphs {graphs}", file=sys.stderr, flush=True)
    kernels = {}
    for name, rec in prof.items():
        if rec["launches"] == 0:
            continue
        ms_ev = rec["ms"] / rec["launches"]
        # the launch-bound event pair adds args.event_over_us to each timed
        # launch (measured live by the event probe): the kernel's own time
        ms = ms_ev - args.event_over_us * 1e-3
        bpl = rec["bytes"] / rec["launches"]
        kernels[name] = dict(launches=rec["launches"], mean_us=ms * 1e3,
                             mean_us_events=ms_ev * 1e3, bytes_per_launch=bpl,
                             gbs=bpl / (ms * 1e-3) / 1e9, total_ms=rec["ms"])
    particles = sum(sum(r["n"] for r in (c if isinstance(c, list) else [c])) for c in cfgs)
    value = steps * particles / elapsed
    tuned = [dict(spmv=S.CSR_VARIANTS[t["spmv_variant"]], apply=S.CSR_VARIANTS[t["apply_variant"]],
                  spmv_us=[round(u, 1) for u in t["spmv_us"]],
                  apply_us=[round(u, 1) for u in t["apply_us"]]) for t in tuning]
    ns = [sum(r["n"] for r in (c if isinstance(c, list) else [c])) for c in cfgs]
    rows = dict(mean_offdiag_per_row=round(sum(r[0] for r in rowstat) / sum(ns), 3),
                max_row=max(r[1] for r in rowstat))
    return dict(value=value, elapsed=elapsed, iters=iters, kernels=kernels, fallbacks=fallbacks,
                graphs=graphs, particles=particles, steps=steps, tuning=tuned, rows=rows,
                extra=extra)


def run_c5(args, S, inputs, theta, forms, stream, torch, np, copy_gbs):
    """Scale workloads: one N = 8e6 box (L = 200) and 16 replicas of N = 5e5
    (L = 79.37), shear 0.5, each from a state pre-sheared with plain steps;
    every form starts from the same pre-sheared positions."""
    import math
    out_w = {}
    single = inputs.single_box(shear_rate=0.5, seed=51, n=8_000_000, L=200.0)["params"]
    batch = [dict(inputs.cube_params(500_000, 0.5, seed=60 + r), stream=r) for r in range(16)]
    for name, cfg in (("single_n8e6", single), ("batch_16x5e5", batch)):
        cl = cfg if isinstance(cfg, list) else [cfg]
        pos = np.concatenate([inputs.uniform_positions(c["n"], c["box"], c["seed"]) for c in cl])
        print(f"# c5 {name}: pre-shearing {args.c5_preshear} steps", file=sys.stderr, flush=True)
        with S.Sim(cfg, pos, tol=args.tol, maxit=5000, stream=stream) as sim:
            sim.graph_mode(True)
            for k in range(args.c5_preshear):
                sim.step(1)
                if (k + 1) % 50 == 0:
                    print(f"# c5 {name}: pre-shear step {k + 1}", file=sys.stderr, flush=True)
            pos = sim.state()[0]
        runs = {f: time_form(args, S, [cfg], [pos], f, theta, stream, torch, np, label=f"c5 {name} ")
                for f in forms}
        out_w[name] = {f: dict(value=round(r["value"], 1),
                               ms_per_step=round(r["elapsed"] / r["steps"] * 1e3, 3),
                               mean_cg_iters=round(float(np.mean(r["iters"])), 2),
                               fallbacks=r["fallbacks"], rows=r["rows"],
                               kernels={k: dict(mean_us=round(v["mean_us"], 2),
                                                gbs=round(v["gbs"], 1),
                                                frac=round(v["gbs"] / PEAK_HBM_GBS, 4))
                                        for k, v in r["kernels"].items()})
                       for f, r in runs.items()}
        if "learned" in runs and "plain" in runs:
            out_w[name]["learned_vs_plain"] = round(runs["learned"]["value"] /
                                                    runs["plain"]["value"], 4)
    head = "learned" if "learned" in forms else forms[0]
    v = out_w["single_n8e6"][head]
    dom = max(v["kernels"], key=lambda k: v["kernels"][k]["mean_us"]) if v["kernels"] else None
    out = {
        "metric": METRIC, "value": v["value"], "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": v["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-spmv/f64" if args.fp32_spmv else "f64", "data": "synthetic",
        "config": {"workload": f"scale workloads: one box N=8000000, L=200, and 16 replicas N=500000 "
                               f"(L=79.37), shear 0.5, density 1, r_c 1, gamma0 0.1, alpha 1, kT 1, dt 0.01, each pre-sheared "
                               f"{args.c5_preshear} plain steps from uniform positions; value = the "
                               f"N=8e6 box, {head} form",
                   "precond": head, "cg_tol": args.tol, "parallelism": "single GPU"},
        "roofline": None if dom is None else {
            "bound": "hbm", "achieved": v["kernels"][dom]["gbs"], "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": v["kernels"][dom]["frac"], "traffic": None, "kernel": dom,
            "mean_us": v["kernels"][dom]["mean_us"], "event_overhead_us": round(args.event_over_us, 2),
            "copy_probe_gbs": round(copy_gbs, 1)},
        "cpu_baseline": None,
        "c5": out_w,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(each GPU would own whole boxes; see the sharding notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1808_06381_amd import inputs
    from paper_1808_06381_amd import sim as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    L = (args.n) ** (1.0 / 3.0) if args.n != 1_000_000 else 100.0
    # achievable HBM bandwidth: a plain 1 GiB device copy (read + write)
    nbytes = 1 << 30
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    copy_ms = S.copy_probe(src, dst, reps=10, stream=stream)
    copy_gbs = 2 * nbytes / (copy_ms * 1e-3) / 1e9
    # what the probe's launch-bound events add per timed launch: the same
    # copy (64 MB, a CG kernel's duration) timed in a chain and one by one
    ev_chain, ev_each = S.event_probe(src[:8 << 20], dst[:8 << 20], reps=64, stream=stream)
    args.event_over_us = max(0.0, (ev_each - ev_chain) * 1e3)
    print(f"# event probe: copy {ev_chain * 1e3:.2f} us in a chain, {ev_each * 1e3:.2f} us timed "
          f"one by one: {args.event_over_us:.2f} us per timed launch", file=sys.stderr, flush=True)
    del src, dst
    cfgs, pos0s = [], []
    for k, shear in enumerate(SHEARS):
        cfg = inputs.single_box(shear_rate=shear, seed=1 + k, n=args.n, L=L)["params"]
        cfgs.append(cfg)
        pos0s.append(inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"]))
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    theta = None
    if "learned" in forms:
        if not os.path.exists(args.weights):
            print(f"# no weights at {args.weights}: skipping the learned form", file=sys.stderr)
            forms = [f for f in forms if f != "learned"]
        else:
            from paper_1808_06381_amd import precond
            theta = precond.load(args.weights)
    if args.c5:
        run_c5(args, S, inputs, theta, [f for f in forms if f != "ic0"], stream, torch, np,
               copy_gbs)
        return
    runs = {}
    head = "learned" if "learned" in forms else forms[0]
    for form in forms:
        after = (lambda sims: dict(sq=measure_sq(sims[0], cfgs[0]["n"], np),
                                   vv=measure_vv(sims[0], cfgs[0]["n"], np))) if form == head else None
        runs[form] = time_form(args, S, cfgs, pos0s, form, theta, stream, torch, np, after=after)
    hr = runs[head]
    value = hr["value"]
    elapsed = hr["elapsed"]
    iters = hr["iters"]
    kernels = hr["kernels"]
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
        kr = kernels[dom]
        wl_key = f"single_n{args.n}"
        traffic = read_traffic(dom, wl_key, head)
        roofline = dict(bound="hbm", achieved=round(kr["gbs"], 1), peak=PEAK_HBM_GBS, unit="GB/s",
                        frac=round(kr["gbs"] / PEAK_HBM_GBS, 4),
                        copy_probe_gbs=round(copy_gbs, 1),
                        traffic=traffic, kernel=dom,
                        bytes_per_launch=kr["bytes_per_launch"], mean_us=round(kr["mean_us"], 2),
                        mean_us_events=round(kr["mean_us_events"], 2),
                        event_overhead_us=round(args.event_over_us, 2))

    cpu = None
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfgs[1], pos0s[1], args.cpu_steps, args.tol)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-spmv/f64" if args.fp32_spmv else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"three single boxes N={args.n}, L={L:.4g}, density 1, shear rates "
                        f"{list(SHEARS)}, r_c=1, (1-r/r_c)^2 weight, soft potential eps=1kT, "
                        f"gamma0=0.1, kT=1, dt=0.01, FDT noise; one bench step = one time step "
                        f"of each box",
            "precond": head,
            "cg_tol": args.tol,
            "particles_per_step": sum(c["n"] for c in cfgs),
            "mean_cg_iters": round(float(np.mean(iters)), 2),
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "kernels": {k: {f: (round(v, 3) if isinstance(v, float) else v) for f, v in r.items()}
                    for k, r in kernels.items()},
        "cpu_baseline": cpu,
        "forms": {f: dict(value=round(r["value"], 1), ms_per_step=round(r["elapsed"] / args.steps * 1e3, 4),
                          mean_cg_iters=round(float(np.mean(r["iters"])), 2), fallbacks=r["fallbacks"],
                          graphs=r["graphs"], tuning=r["tuning"])
                  for f, r in runs.items()},
        "graph_steps": not args.no_graph,
    }
    extra = hr.get("extra") or {}
    sqm = extra.get("sq")
    if sqm:
        # structure factor of the first box's final state: the contraction
        # runs on the FP64 matrix cores (the 24 bytes of a particle feed
        # nx * ny complex multiply-adds)
        ms = sqm["kernel_ms_events"] - args.event_over_us * 1e-3
        tf = sqm["flops_per_call"] / (ms * 1e-3) / 1e12
        out["structure_factor"] = dict(
            sqm, kernel="k_sq_partial", kernel_ms=round(ms, 4),
            roofline=dict(bound="mfma", achieved=round(tf, 2), peak=PEAK_FP64_TFLOPS,
                          unit="TFLOP/s", frac=round(tf / PEAK_FP64_TFLOPS, 4)))
    vvm = extra.get("vv")
    if vvm:
        # velocity correlation of the first box's last step: pair tests and
        # accepted-pair arithmetic on the FP64 vector units
        ms = vvm["kernel_ms_events"] - args.event_over_us * 1e-3
        tops = VV_OPS_PER_PAIR * vvm["pairs"] / (ms * 1e-3) / 1e12
        out["velocity_correlation"] = dict(
            vvm, kernel="k_vv_pairs", kernel_ms=round(ms, 4),
            pairs_per_s=round(vvm["pairs"] / (ms * 1e-3), 1),
            roofline=dict(bound="alu", achieved=round(tops, 3), peak=PEAK_FP64_TOPS,
                          unit="Top/s", frac=round(tops / PEAK_FP64_TOPS, 4),
                          ops_per_pair=VV_OPS_PER_PAIR))
    if "learned" in runs and "plain" in runs:
        out["learned_vs_plain"] = round(runs["learned"]["value"] / runs["plain"]["value"], 4)
    if not args.no_aniso:
        out["anisotropic"] = measure_aniso(args, S, inputs, np)
    if args.batch > 0:
        bcfgs = inputs.batch_replicas(count=args.batch, seed=7)
        bpos = np.concatenate([inputs.uniform_positions(c["n"], c["box"], c["seed"]) for c in bcfgs])
        bruns = {form: time_form(args, S, [bcfgs], [bpos], form, theta, stream, torch, np,
                                 steps=args.batch_steps, label="batch ")
                 for form in forms}
        out["batch"] = {
            "workload": f"{args.batch} replicas in one handle, N log-uniform in [1e4, 2e5] "
                        f"(sum {bruns[forms[0]]['particles']}), density 1, shear log-uniform in "
                        f"[0.005, 1], same physics; one bench step = one time step of every "
                        f"replica",
            "steps": args.batch_steps,
            "forms": {f: dict(value=round(r["value"], 1),
                              ms_per_step=round(r["elapsed"] / r["steps"] * 1e3, 4),
                              mean_cg_iters=round(float(np.mean(r["iters"])), 2),
                              fallbacks=r["fallbacks"], graphs=r["graphs"], tuning=r["tuning"])
                      for f, r in bruns.items()},
        }
        if "learned" in bruns and "plain" in bruns:
            out["batch"]["learned_vs_plain"] = round(bruns["learned"]["value"] /
                                                     bruns["plain"]["value"], 4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
