"""Benchmark of the sheared mesoscale blob step on one MI355X.

Headline workload: one box of N = 8e6 particles, L = 200 (density 1,
r_c = 1, (1 - r/r_c)^2 friction weight, soft potential, background friction
0.1, kT = 1, dt = 0.01, fluctuation-dissipation noise) at shear rate 0.5,
pre-sheared with 2000 plain steps from uniform positions, then timed with
the learned preconditioner (headline value) and with Jacobi-PCG (plain),
both to a true relative residual of 1e-8 per component, FP64.  One bench
step = one time step of the box.  Beside it, a batch of 16 replicas of
N = 5e5 (L = 79.37) prepared the same way.  Inputs are resident in HBM for
the whole timed region.

Each form is timed over whole steps replayed as HIP graphs; every
--probe-every-th step runs eagerly with HIP events: alternately the CG
kernels launch by launch, and a run of whole CG iterations (all kernels,
the finisher and the gaps) between one event pair.  The roofline of the
line is the CG iteration: its algorithmic bytes (matrix 12(k+1)+4 and
vectors 200 per particle, plus one matrix pass for the learned M^-1
product) over its measured time, against 8 TB/s.

Further keys: the three N = 1e6 boxes at shear 0.01 / 0.1 / 0.5 (plain,
learned, IC(0)) with the structure factor and the velocity correlation of
the final state, the 64-replica uneven batch, the N = 1000 small case, the
paper's own box (4 x 20060 at its four shear rates), anisotropic friction,
and the oracle's own throughput on the host cores (1 and all) for a bounded
sample of the pre-sheared scale workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--only c5|c5-single|c2|small|aniso]
                  [--no-cpu-baseline] [--c5-preshear 2000]
"""
import argparse
import hashlib
import json
import os
import platform
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
CG_KERNELS = ("k_cg_vec", "k_cg_spmv", "k_cg_apply")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--probe-every", type=int, default=4,
                    help="every k-th step runs eagerly with HIP events on the CG")
    ap.add_argument("--no-graph", action="store_true", help="eager steps only")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default lane widths of the CSR products")
    ap.add_argument("--tuning", default="",
                    help="spmv,apply,vec variant indices to use instead of the autotuner "
                         "(e.g. 7,6,1; for counter runs that must match a timed run)")
    ap.add_argument("--preshear-cache", default="",
                    help="directory for pre-sheared states (profiling runs share one)")
    ap.add_argument("--c5-preshear", type=int, default=2000,
                    help="plain steps at shear 0.5 before timing (from uniform positions)")
    ap.add_argument("--only", default="",
                    help="c5: the scale workloads only; c5-single: the N = 8e6 box only; "
                         "small: the N = 1000 case and the paper's box only; c2: the N = 1e6 "
                         "boxes with S(q) and the velocity correlation only; aniso: the "
                         "anisotropic-friction box only (no headline line for small, c2 and "
                         "aniso)")
    ap.add_argument("--c2-steps", type=int, default=20)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-spmv", action="store_true")
    ap.add_argument("--forms", default="plain,learned",
                    help="CG forms of the scale workloads: plain (Jacobi-PCG), learned")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1808_06381_amd", "weights",
                                                      "precond_n1e5.bin"))
    ap.set_defaults(event_over_us=0.0)  # set from the event probe before any timing
    return ap.parse_args()


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the sources of the CG kernels the traffic record covers."""
    h = hashlib.sha256()
    for f in ("cg.hip", "sim_dev.h"):
        with open(os.path.join(ROOT, "paper_1808_06381_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload_key, form):
    """HBM bytes per CG iteration and per kernel launch from the committed
    counter summary, if it was taken on the current kernel sources, this
    workload and CG form (else None)."""
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
        out = dict(bytes_per_iteration=float(rec["cg_iteration.traffic_bytes"]),
                   algorithmic_bytes_per_iteration=float(rec["cg_iteration.algorithmic_bytes"]))
        for k in CG_KERNELS + ("k_cg_finish",):
            if f"{k}.traffic_bytes_per_launch" in rec:
                out[k] = float(rec[f"{k}.traffic_bytes_per_launch"])
        return out
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def time_oracle_step(cfg, pos, step_index, tol, threads):
    import oracle
    used = oracle.set_threads(threads)
    t0 = time.perf_counter()
    oracle.step(cfg, pos, step_index, tol=tol)
    return time.perf_counter() - t0, used


def cpu_baseline(cfg, pos, step_index, tol):
    """The oracle on the host cores: one step of one replica (N = 5e5) of the
    pre-sheared 16-replica scale batch, sequential and on every core (the
    OpenMP build spreads the solve's row loops; the pair search and the
    assembly stay sequential; the result bits are the same)."""
    ncores = os.cpu_count() or 1
    dt1, _ = time_oracle_step(cfg, pos, step_index, tol, 1)
    dtn, used = time_oracle_step(cfg, pos, step_index, tol, ncores)
    n = cfg["n"]
    return dict(value=round(n / dtn, 1), unit="particle-steps/s", cores=used, kind="oracle",
                sample=f"1 step (step {step_index}) of one N={n} replica of the 16 x 5e5 scale "
                       f"batch after {step_index} pre-shear steps at shear 0.5, FP64 oracle, "
                       f"tol {tol}: {dtn:.1f} s on {used} threads, {dt1:.1f} s on 1",
                single_core=dict(value=round(n / dt1, 1), cores=1, seconds=round(dt1, 2)),
                seconds=round(dtn, 2), cpu_model=cpu_model(), host_cpus=ncores)


def measure_sq(sim, n, np, nx=64, my_max=64, reps=3):
    """Structure factor of the final state (Eq. Sfactor, 64 x 129 wavevectors,
    mz = 0): the contraction kernel's event-timed duration, 8 flops (one
    complex multiply-add) per particle and wavevector."""
    sim.structure_factor(nx, my_max)  # untimed first call (scratch, code load)
    ms = []
    for _ in range(reps):
        s, t = sim.structure_factor(nx, my_max, timed=True)
        ms.append(t)
    ny = 2 * my_max + 1
    return dict(grid=f"mx 0..{nx - 1} x my -{my_max}..{my_max}, mz 0", particles=n,
                kernel_ms_events=round(float(np.mean(ms)), 4), flops_per_call=8.0 * n * nx * ny,
                s_q0=float(s[0, 0, my_max]))


# FP64 operations of one accepted pair in the velocity correlation:
# separation 3, r^2 5, cut-off compare 1, bin scale 1, u_i . u_j 5,
# fixed-point scale and rounding 2
VV_OPS_PER_PAIR = 17


def measure_vv(sim, n, np, r_max=10.0, nbins=100, reps=3):
    """Velocity cross-correlation of the last step (Results section), pairs
    with r < r_max = 10 in bins of 0.1: the pair kernel's event-timed
    duration and its rate in accepted pairs (each unordered pair once)."""
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
    coupled unknowns) on the N = 1e6 shear-0.1 box: eager steps, with FP64
    blocks and with FP32-valued iteration products (spmv_fp32)."""
    cfg0 = inputs.single_box(shear_rate=0.1, seed=1)["params"]
    pos0 = inputs.uniform_positions(cfg0["n"], cfg0["box"], cfg0["seed"])
    res = {}
    for fp32 in (0, 1):
        cfg = dict(cfg0, friction_par=a_par, friction_perp=a_perp, spmv_fp32=fp32)
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
        res[fp32] = dict(value=round(cfg["n"] * steps / dt, 1),
                         ms_per_step=round(dt / steps * 1e3, 3),
                         mean_cg_iters=round(float(np.mean(its)), 2),
                         # block product per launch: row pointers 8, own vector
                         # 24, diagonal block 48, result 24 B per row; block 48
                         # (FP32: 24) + column 4 B per entry (each gathered
                         # vector counted once)
                         k_bcg_spmv_bytes_per_launch=104 * rows + (28 if fp32 else 52) * nnz)
    out = dict(workload=f"the N={cfg0['n']} box at shear 0.1 with pair friction a_par={a_par} "
                        f"along and a_perp={a_perp} across the line of centres",
               unit="particle-steps/s", steps=steps, **res[0])
    out["fp32_product"] = res[1]
    return out


def time_form(args, S, cfgs, pos0s, form, theta, stream, torch, np, steps=None, label="",
              after=None, warmup=None, probe_every=None, tol=None):
    """Warm up, then time `steps` bench steps of the systems (one handle per
    entry of cfgs; an entry may be a list of replicas) with one CG form."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    probe_every = args.probe_every if probe_every is None else probe_every
    tol = args.tol if tol is None else tol
    sims = []
    for cfg, pos0 in zip(cfgs, pos0s):
        sim = S.Sim(cfg, pos0, tol=tol, maxit=5000,
                    spmv_fp32=1 if args.fp32_spmv else 0, stream=stream,
                    precond={"plain": "jacobi"}.get(form, form))
        if form == "learned":
            sim.set_weights(theta)
        if not args.no_graph:
            sim.graph_mode(True)
        sims.append(sim)
    log(f"{label}form {form}: warmup {warmup}, timed {steps}")
    for k in range(warmup):
        for sim in sims:
            sim.step(1)
    tuning = []
    if args.tuning:
        sv, av, vv = (int(x) for x in args.tuning.split(","))
        for sim in sims:
            sim.set_tuning(spmv_variant=sv, apply_variant=av, vec_variant=vv)
            sim.step(1)
    elif not args.no_autotune:
        for sim in sims:
            tuning.append(sim.autotune(reps=10))
            sim.step(1)  # re-records the step graph with the chosen variants
    for sim in sims:
        sim.profile_read(reset=True)
        sim.profile_enable(probe_every)
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
    log(f"{label}form {form}: {steps} steps x {len(sims)} handles in {elapsed:.3f} s; "
        f"mean CG iterations {np.mean(iters):.1f}; graphs {graphs}")
    kernels = {}
    for name, rec in prof.items():
        if rec["launches"] == 0:
            continue
        ms_ev = rec["ms"] / rec["launches"]
        # a launch-bound event pair adds args.event_over_us to each timed
        # launch (measured live by the event probe); the iteration record is
        # one pair around many launches, left as measured
        ms = ms_ev if name == "cg_iteration" else ms_ev - args.event_over_us * 1e-3
        bpl = rec["bytes"] / rec["launches"]
        kernels[name] = dict(launches=rec["launches"], mean_us=ms * 1e3,
                             mean_us_events=ms_ev * 1e3, bytes_per_launch=bpl,
                             gbs=bpl / (ms * 1e-3) / 1e9, total_ms=rec["ms"])
    particles = sum(sum(r["n"] for r in (c if isinstance(c, list) else [c])) for c in cfgs)
    tuned = [dict(spmv=S.CSR_VARIANTS[t["spmv_variant"]], apply=S.CSR_VARIANTS[t["apply_variant"]],
                  spmv_us=[round(u, 1) for u in t["spmv_us"]],
                  apply_us=[round(u, 1) for u in t["apply_us"]],
                  vec="nontemporal" if t["vec_variant"] else "ordinary",
                  vec_us=[round(u, 1) for u in t["vec_us"]]) for t in tuning]
    ns = [sum(r["n"] for r in (c if isinstance(c, list) else [c])) for c in cfgs]
    rows = dict(mean_offdiag_per_row=round(sum(r[0] for r in rowstat) / sum(ns), 3),
                max_row=max(r[1] for r in rowstat))
    return dict(value=steps * particles / elapsed, elapsed=elapsed, iters=iters, kernels=kernels,
                fallbacks=fallbacks, graphs=graphs, particles=particles, steps=steps, tuning=tuned,
                rows=rows, extra=extra)


def form_summary(r, np):
    return dict(value=round(r["value"], 1), ms_per_step=round(r["elapsed"] / r["steps"] * 1e3, 3),
                mean_cg_iters=round(float(np.mean(r["iters"])), 2), fallbacks=r["fallbacks"],
                rows=r["rows"], graphs=r["graphs"], tuning=r["tuning"],
                kernels={k: dict(launches=v["launches"], mean_us=round(v["mean_us"], 2),
                                 bytes_per_launch=round(v["bytes_per_launch"], 1),
                                 gbs=round(v["gbs"], 1),
                                 frac=round(v["gbs"] / PEAK_HBM_GBS, 4))
                         for k, v in r["kernels"].items()})


def preshear(args, S, cfg, pos, stream, name):
    """Plain graph steps at the workload's shear from uniform positions.  With
    --preshear-cache DIR the state is read from / written to DIR (the steps
    are deterministic, so a cached state is the state a fresh run reaches)."""
    import numpy as np

    cache = None
    if args.preshear_cache:
        os.makedirs(args.preshear_cache, exist_ok=True)
        cache = os.path.join(args.preshear_cache,
                             f"{name}_n{cfg['n']}_seed{cfg['seed']}_steps{args.c5_preshear}.npy")
        if os.path.exists(cache):
            log(f"{name}: pre-sheared state from {cache}")
            return np.load(cache)
    log(f"{name}: pre-shearing {args.c5_preshear} steps")
    t0 = time.perf_counter()
    with S.Sim(cfg, pos, tol=args.tol, maxit=5000, stream=stream) as sim:
        sim.graph_mode(True)
        for k in range(args.c5_preshear):
            sim.step(1)
            if (k + 1) % 50 == 0:
                log(f"{name}: pre-shear step {k + 1} ({time.perf_counter() - t0:.0f} s)")
        out = sim.state()[0]
    if cache:
        np.save(cache, out)
    return out


def iteration_roofline(r, copy_gbs, traffic):
    """The CG iteration measured as a whole against the HBM peak, with the
    dominant single kernel beside it."""
    it = r["kernels"].get("cg_iteration")
    if not it:
        return None
    dom = max((k for k in CG_KERNELS if k in r["kernels"]),
              key=lambda k: r["kernels"][k]["mean_us"], default=None)
    out = dict(bound="hbm", achieved=round(it["gbs"], 1), peak=PEAK_HBM_GBS, unit="GB/s",
               frac=round(it["gbs"] / PEAK_HBM_GBS, 4),
               traffic=None if traffic is None else traffic["bytes_per_iteration"],
               kernel="cg_iteration: k_cg_vec + k_cg_apply + k_cg_spmv + k_cg_finish and the "
                      "gaps between them",
               basis="algorithmic bytes per CG iteration: 12(k+1)+4 (matrix) + 200 (vectors) per "
                     "particle, + 12(k+1)+4 for the learned M^-1 product",
               k_offdiag_per_row=r["rows"]["mean_offdiag_per_row"],
               bytes_per_iteration=round(it["bytes_per_launch"], 1),
               us_per_iteration=round(it["mean_us"], 2), iterations_timed=it["launches"],
               copy_probe_gbs=round(copy_gbs, 1),
               frac_of_copy_probe=round(it["gbs"] / copy_gbs, 4))
    if dom:
        d = r["kernels"][dom]
        out["dominant_kernel"] = dict(kernel=dom, achieved=round(d["gbs"], 1),
                                      frac=round(d["gbs"] / PEAK_HBM_GBS, 4),
                                      bytes_per_launch=round(d["bytes_per_launch"], 1),
                                      mean_us=round(d["mean_us"], 2),
                                      traffic=None if traffic is None else traffic.get(dom))
    if traffic is not None:
        out["traffic_over_algorithmic"] = round(
            traffic["bytes_per_iteration"] / traffic["algorithmic_bytes_per_iteration"], 4)
    return out


def run_c2(args, S, inputs, theta, forms, head, stream, torch, np, copy_gbs):
    """The three N = 1e6 boxes (plain, learned, IC(0)), S(q) and the velocity
    correlation of the first box's final state."""
    out = {}
    cfgs, pos0s = [], []
    for k, shear in enumerate(SHEARS):
        cfg = inputs.single_box(shear_rate=shear, seed=1 + k)["params"]
        cfgs.append(cfg)
        pos0s.append(inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"]))
    c2 = {}
    for form in forms + ["ic0"]:
        after = (lambda sims: dict(sq=measure_sq(sims[0], cfgs[0]["n"], np),
                                   vv=measure_vv(sims[0], cfgs[0]["n"], np))) \
            if form == head else None
        c2[form] = time_form(args, S, cfgs, pos0s, form, theta, stream, torch, np,
                             steps=args.c2_steps, after=after, label="c2 ")
    out["single_n1e6_x3"] = dict(
        workload=f"three boxes N=1000000, L=100, shear rates {list(SHEARS)}, same physics, "
                 f"from uniform positions; one bench step = one time step of each box",
        forms={f: form_summary(r, np) for f, r in c2.items()},
        roofline=iteration_roofline(c2[head], copy_gbs, None))
    if "learned" in c2 and "plain" in c2:
        out["single_n1e6_x3"]["learned_vs_plain"] = round(c2["learned"]["value"] /
                                                          c2["plain"]["value"], 4)
    extra = c2[head].get("extra") or {}
    sqm = extra.get("sq")
    if sqm:
        ms = sqm["kernel_ms_events"] - args.event_over_us * 1e-3
        tf = sqm["flops_per_call"] / (ms * 1e-3) / 1e12
        out["structure_factor"] = dict(
            sqm, kernel="k_sq_partial", kernel_ms=round(ms, 4),
            roofline=dict(bound="mfma", achieved=round(tf, 2), peak=PEAK_FP64_TFLOPS,
                          unit="TFLOP/s", frac=round(tf / PEAK_FP64_TFLOPS, 4)))
    vvm = extra.get("vv")
    if vvm:
        ms = vvm["kernel_ms_events"] - args.event_over_us * 1e-3
        tops = VV_OPS_PER_PAIR * vvm["pairs"] / (ms * 1e-3) / 1e12
        out["velocity_correlation"] = dict(
            vvm, kernel="k_vv_pairs", kernel_ms=round(ms, 4),
            pairs_per_s=round(vvm["pairs"] / (ms * 1e-3), 1),
            roofline=dict(bound="alu", achieved=round(tops, 3), peak=PEAK_FP64_TOPS,
                          unit="Top/s", frac=round(tops / PEAK_FP64_TOPS, 4),
                          ops_per_pair=VV_OPS_PER_PAIR))
    return out


def run_c5(args, S, inputs, theta, forms, stream, torch, np, copy_gbs):
    """Scale workloads: one N = 8e6 box (L = 200) and 16 replicas of N = 5e5
    (L = 79.37), shear 0.5, each pre-sheared from uniform positions; every
    form starts from the same pre-sheared positions."""
    single = inputs.single_box(shear_rate=0.5, seed=51, n=8_000_000, L=200.0)["params"]
    batch = [dict(inputs.cube_params(500_000, 0.5, seed=60 + r), stream=r) for r in range(16)]
    workloads = [("single_n8e6", single)]
    if args.only != "c5-single":
        workloads.append(("batch_16x5e5", batch))
    out, batch_state = {}, None
    for name, cfg in workloads:
        cl = cfg if isinstance(cfg, list) else [cfg]
        pos = np.concatenate([inputs.uniform_positions(c["n"], c["box"], c["seed"]) for c in cl])
        pos = preshear(args, S, cfg, pos, stream, name)
        if name == "batch_16x5e5":
            batch_state = (cl[0], pos[:cl[0]["n"]].copy())
        runs = {f: time_form(args, S, [cfg], [pos], f, theta, stream, torch, np,
                             label=f"{name} ") for f in forms}
        out[name] = dict(forms={f: form_summary(r, np) for f, r in runs.items()}, runs=runs)
        if "learned" in runs and "plain" in runs:
            out[name]["learned_vs_plain"] = round(runs["learned"]["value"] /
                                                  runs["plain"]["value"], 4)
    return out, batch_state


def run_small(args, S, inputs, theta, stream, torch, np):
    """The N = 1000, L = 10 small case (100 steps, tol 1e-10) and the paper's
    own box (four replicas of C = 20060 at shear 0, 0.005, 0.05, 0.5, its
    noise form), both bound by launch and reduction latency: particle-steps/s
    and the time of one CG iteration."""
    from paper_1808_06381_amd import paper_runs
    case = inputs.small_case(seed=1)
    c1 = case["params"]
    p1 = inputs.uniform_positions(c1["n"], c1["box"], c1["seed"])
    out = {}
    res = {}
    for form in ("plain", "learned"):
        r = time_form(args, S, [c1], [p1], form, theta, stream, torch, np, steps=case["steps"],
                      warmup=5, probe_every=4, tol=case["tol"], label="small ")
        res[form] = form_summary(r, np)
        it = r["kernels"].get("cg_iteration")
        res[form]["us_per_cg_iteration"] = None if not it else round(it["mean_us"], 2)
    out["small_n1000"] = dict(
        workload="N=1000, L=10, shear 0.05, Jacobi or learned PCG to 1e-10, 100 steps",
        forms=res)
    pcfgs, ppos = paper_runs.make_batch("paper", 11, paper_runs.SHEARS)
    res = {}
    for form in ("plain", "learned"):
        r = time_form(args, S, [pcfgs], [ppos], form, theta, stream, torch, np, steps=100,
                      warmup=5, probe_every=4, label="paper box ")
        res[form] = form_summary(r, np)
        it = r["kernels"].get("cg_iteration")
        res[form]["us_per_cg_iteration"] = None if not it else round(it["mean_us"], 2)
    out["paper_box"] = dict(
        workload=f"the paper's box 87.6 x 43.6 x 22, C={pcfgs[0]['n']} per replica, four replicas "
                 f"at shear {list(paper_runs.SHEARS)}, Gaussian weight and core, gamma0 1, "
                 f"alpha 4, the paper's noise form, tol {args.tol}, 100 steps",
        forms=res)
    return out


def cpu_small(np):
    """The oracle on the N = 1000 small case, all 100 steps, 1 core and all."""
    import oracle
    from paper_1808_06381_amd import inputs
    case = inputs.small_case(seed=1)
    cfg = case["params"]
    pos = inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"])
    out = {}
    for th in (1, os.cpu_count() or 1):
        used = oracle.set_threads(th)
        t0 = time.perf_counter()
        oracle.run(cfg, pos, case["steps"], tol=case["tol"])
        dt = time.perf_counter() - t0
        out[f"threads_{used}"] = dict(value=round(cfg["n"] * case["steps"] / dt, 1),
                                      seconds=round(dt, 3))
    return out


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
    # achievable HBM bandwidth: a plain 1 GiB device copy (read + write)
    nbytes = 1 << 30
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    copy_ms = S.copy_probe(src, dst, reps=10, stream=stream)
    copy_gbs = 2 * nbytes / (copy_ms * 1e-3) / 1e9
    # what a launch-bound event pair adds per timed launch: the same copy
    # (64 MB, a CG kernel's duration) timed in a chain and one by one
    ev_chain, ev_each = S.event_probe(src[:8 << 20], dst[:8 << 20], reps=64, stream=stream)
    args.event_over_us = max(0.0, (ev_each - ev_chain) * 1e3)
    log(f"copy probe {copy_gbs:.0f} GB/s; event probe: copy {ev_chain * 1e3:.2f} us in a chain, "
        f"{ev_each * 1e3:.2f} us timed one by one: {args.event_over_us:.2f} us per timed launch")
    del src, dst
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    theta = None
    if "learned" in forms:
        if not os.path.exists(args.weights):
            log(f"no weights at {args.weights}: skipping the learned form")
            forms = [f for f in forms if f != "learned"]
        else:
            from paper_1808_06381_amd import precond
            theta = precond.load(args.weights)
    head = "learned" if "learned" in forms else forms[0]
    if args.only == "small":
        # the latency-bound small workloads alone (not the metric's line)
        print(json.dumps(run_small(args, S, inputs, theta, stream, torch, np)), flush=True)
        return
    if args.only == "c2":
        # the N = 1e6 boxes with S(q) and the velocity correlation alone
        print(json.dumps(run_c2(args, S, inputs, theta, forms, head, stream, torch, np, copy_gbs)),
              flush=True)
        return
    if args.only == "aniso":
        # the anisotropic-friction box alone (FP64 and FP32-valued block products)
        print(json.dumps({"anisotropic": measure_aniso(args, S, inputs, np)}), flush=True)
        return

    c5, batch_state = run_c5(args, S, inputs, theta, forms, stream, torch, np, copy_gbs)
    hr = c5["single_n8e6"]["runs"][head]
    traffic = read_traffic("c5_single_n8e6", head)
    roofline = iteration_roofline(hr, copy_gbs, traffic)
    out = {
        "metric": METRIC,
        "value": round(hr["value"], 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hr["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-spmv/f64" if args.fp32_spmv else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"one box N=8000000, L=200, density 1, shear 0.5, r_c=1, (1-r/r_c)^2 "
                        f"weight, soft potential eps=1kT, gamma0=0.1, alpha=1, kT=1, dt=0.01, FDT "
                        f"noise, pre-sheared {args.c5_preshear} plain steps from uniform "
                        f"positions; {head}-preconditioned CG to a true relative residual "
                        f"{args.tol} per component; one bench step = one time step of the box",
            "precond": head,
            "cg_tol": args.tol,
            "particles_per_step": hr["particles"],
            "mean_cg_iters": round(float(np.mean(hr["iters"])), 2),
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": None,
        "forms": c5["single_n8e6"]["forms"],
        "graph_steps": not args.no_graph,
    }
    if "learned_vs_plain" in c5["single_n8e6"]:
        out["learned_vs_plain"] = c5["single_n8e6"]["learned_vs_plain"]
    if "batch_16x5e5" in c5:
        b = c5["batch_16x5e5"]
        out["batch_16x5e5"] = dict(
            workload=f"16 replicas N=500000 (L=79.37) in one handle, shear 0.5, same physics, "
                     f"pre-sheared {args.c5_preshear} plain steps; one bench step = one time step "
                     f"of every replica", forms=b["forms"],
            learned_vs_plain=b.get("learned_vs_plain"),
            roofline=iteration_roofline(b["runs"][head], copy_gbs, None))
    out["event_overhead_us"] = round(args.event_over_us, 2)

    if not args.only:
        out.update(run_c2(args, S, inputs, theta, forms, head, stream, torch, np, copy_gbs))
        # 64 replicas of uneven size in one handle
        bcfgs = inputs.batch_replicas(count=64, seed=7)
        bpos = np.concatenate([inputs.uniform_positions(c["n"], c["box"], c["seed"]) for c in bcfgs])
        bruns = {form: time_form(args, S, [bcfgs], [bpos], form, theta, stream, torch, np,
                                 steps=args.batch_steps, label="batch64 ")
                 for form in forms}
        out["batch_64_uneven"] = dict(
            workload=f"64 replicas in one handle, N log-uniform in [1e4, 2e5] (sum "
                     f"{bruns[forms[0]]['particles']}), density 1, shear log-uniform in "
                     f"[0.005, 1], same physics; one bench step = one time step of every replica",
            forms={f: form_summary(r, np) for f, r in bruns.items()})
        if "learned" in bruns and "plain" in bruns:
            out["batch_64_uneven"]["learned_vs_plain"] = round(bruns["learned"]["value"] /
                                                               bruns["plain"]["value"], 4)
        out.update(run_small(args, S, inputs, theta, stream, torch, np))
        out["anisotropic"] = measure_aniso(args, S, inputs, np)

    if not args.no_cpu_baseline and batch_state is not None:
        log("timing the CPU oracle on a bounded sample")
        cfg0, pos0 = batch_state
        out["cpu_baseline"] = cpu_baseline(cfg0, pos0, args.c5_preshear, args.tol)
        if not args.only:
            out["cpu_baseline"]["small_n1000_100_steps"] = cpu_small(np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
