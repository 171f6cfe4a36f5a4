"""Benchmark of the dual-time EDAC SPH hot path on one MI355X.

A step is one real time step of Algorithm 2 (cell build, wall pass, rate pass
and predictor, cell rebuild or list filter, pseudo-time loop until the stop
test, corrector; particle shifting where the workload uses it) over the whole
workload. Default workload: the batch of 64 independent 2D Taylor-Green and
lid-driven-cavity simulations (2.57M particles), FP32 pair sums with float64
positions, pressure accumulation and residuals, inputs resident in HBM before
the timed region. The value is neighbour-pair evaluations of the pseudo-time
iterations per second (pairs of the exact neighbour lists times iterations run,
per sim); the batch's instance-steps per second are reported beside it.

Also reported: the same workload on the plain FP64 path, the dam break (the
largest single simulation) as a second leg, the roofline of the pseudo-iteration
pair pass and of the cell build (HIP events on the library's stream around
sampled launches of the timed region), and the CPU oracle timed on a bounded
sample of the same workload on the host cores (all threads and one).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C4]
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of the pair pass per unit (one ordered neighbour pair in one
# pseudo-iteration): 70 FLOP (FMA = 2) counted from the pressure-rate and
# momentum sums with artificial viscosity; the kernels as built execute 50 (2D)
# and 60 (3D) FLOP on the workloads without artificial viscosity.
FLOP_PER_PAIR = 70
FLOP_PER_PAIR_IMPL = {2: 50, 3: 60}
FLOP_PER_PAIR_CONV = {2: 62, 3: 78}  # with the convective sum (steady solve)
# algorithmic bytes per fluid particle per pseudo-iteration: positions, cell,
# velocity, pressure and BDF2 constant read, velocity and pressure written
PASS_BYTES = {("f32", 2): 60, ("f32", 3): 76, ("f64", 2): 84, ("f64", 3): 116}
# MI355X peaks: FP32 vector 157.3 TFLOP/s (packed instructions; 78.6 without),
# FP64 vector 78.6 TFLOP/s, HBM3E 8 TB/s
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
PEAK_NONPACKED_F32 = 78.6
HBM_GBPS = 8000.0

WORKLOADS = {
    "C0": "2D Taylor-Green vortex, periodic unit square, 50x50 particles, Re=100",
    "C1": "2D Taylor-Green vortex, periodic unit square, 400x400 particles, Re=100",
    "C2": "3D Taylor-Green vortex, periodic unit cube, 64^3 particles, Re=1600",
    "C3": "2D dam break, 1x2 column in a 4x4 tank, dx=0.002, 3 wall layers",
    "C4": "batch of 64 periodic TGV / lid-driven cavity instances, 2.5k-160k particles",
}


def build_bytes_per_particle(dtype, dim, exact_entries, cand_entries):
    """Algorithmic bytes of one full build per particle: the keys read the
    positions (8 dim); the reorder reads and writes the state once (S: caller
    index, sim index, float64 positions and r^n, V^n, V^n - V^{n-1}, V^k - V^n,
    V^(0) - V^n in the pass type, float64 pressure and p^n, the pressure rate);
    the lists write their entries (exact and candidate, 4 B each) and counts
    (8); the records written are the packed float64 positions (8 dim), the
    pass's position record (4 dim FP32, 8 dim FP64) and the {V, p} record."""
    t = 4 if dtype == "f32" else 8
    state = 4 + 4 + 2 * 8 * dim + 4 * t * dim + 8 + 8 + t
    records = 8 * dim + t * dim + 4 * t
    return 8 * dim + 2 * state + 4 * (exact_entries + cand_entries) + 8 + records


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pair_evals(reports):
    return sum(r["pairs"] * r["iters"] for step in reports for r in step)


def _pass_src_hash():
    """sha256 of the source that holds the pair-pass kernel."""
    src = os.path.join(ROOT, "paper_1904_00861_amd", "csrc", "dtsph_pass_dev.h")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def traffic_from_profile(cfg, dtype):
    """HBM bytes per full-batch pseudo-iteration pair-pass launch from the committed
    counter summary of this workload (FETCH_SIZE and WRITE_SIZE runs, calibrated by
    a copy kernel), with the algorithmic bytes of the same launch; None if there is
    no summary or the pass kernel changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"counters_{cfg}_{'fp32' if dtype == 'f32' else 'fp64'}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"source sha256: ([0-9a-f]{64})", txt)
    m_tr = re.search(r"traffic per launch: ([0-9.eE+]+) bytes; algorithmic: ([0-9.eE+]+) bytes", txt)
    if not m_hash or not m_tr or m_hash.group(1) != _pass_src_hash():
        return None
    return float(m_tr.group(1)), float(m_tr.group(2))


def apply_shape(sim, shape):
    """Fixed launch shape (L, B, G, M): pair-pass lanes per particle, workgroup
    size, neighbour-build lanes per particle (0: the staged-tile kernel), cell
    subdivision."""
    from paper_1904_00861_amd import dtsph as D

    lanes, block, nbr_lanes, cell_div = shape
    sim.set_option(D.OPT_LANES, lanes)
    sim.set_option(D.OPT_BLOCK, block)
    sim.set_option(D.OPT_NBR_TILES, 1 if nbr_lanes == 0 else 0)
    if nbr_lanes:
        sim.set_option(D.OPT_NBR_LANES, nbr_lanes)
    sim.set_option(D.OPT_CELL_DIV, cell_div)


def run_leg(problems, precision, steps, warmup, timing_every, shape=None, pair_cache=0, graphs=0, schedule=None):
    import torch
    from paper_1904_00861_amd import dtsph as D

    sim = D.Sim(problems, precision=precision)
    if pair_cache:
        sim.set_option(D.OPT_PAIR_CACHE, pair_cache)
    if graphs:
        sim.set_option(D.OPT_GRAPHS, 1)
    if schedule is not None:
        sim.set_option(D.OPT_TAIL_LOOP, schedule)
    if shape:  # fixed launch configuration instead of the autotuner
        lanes, block, nbr_lanes, cell_div = shape
        apply_shape(sim, shape)
        tune = dict(lanes=lanes, block=block, nbr_lanes=nbr_lanes, nbr_tiles=int(nbr_lanes == 0),
                    cell_div=cell_div, fixed=True)
        log(f"fixed launch shape: pass lanes {lanes} block {block}, neighbour-build lanes {nbr_lanes} "
            f"(0: staged tiles), cell subdivision {cell_div}")
    else:
        tune = sim.autotune()
        log(f"autotune: pass lanes {tune['lanes']} block {tune['block']} ({tune['us']:.2f} us); " +
            " ".join(f"{e['lanes']}x{e['block']}:{e['us']:.1f}" for e in tune["entries"]) +
            f"; cell subdivision {tune['cell_div']} (full build {tune['build_us']:.1f} us)"
            f"; neighbour build {'staged tiles' if tune['nbr_tiles'] else 'lanes ' + str(tune['nbr_lanes'])} "
            f"({tune['nbr_us']:.1f} us), "
            f"filter lanes {tune['filter_lanes']} ({tune['filter_us']:.1f} us)")
    if warmup:
        sim.step(warmup)
    sim.set_option(D.OPT_TIMING, timing_every)
    sim.set_option(D.OPT_RESET_TIMING, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, reps = sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = sim.timing()
    info = dict(sim.info)
    sim.close()
    return dict(seconds=t1 - t0, reports=reps, timing=tm, status=st, info=info, tune=tune)


def leg_summary(problems, leg, dtype, steps, cfg=None, timing_every=-1):
    """Throughput and rooflines of one timed leg."""
    dim = problems[0].params["dim"]
    evals = pair_evals(leg["reports"])
    secs = leg["seconds"]
    iters = [r["iters"] for step in leg["reports"] for r in step]
    tm = leg["timing"]
    out = dict(value=evals / secs, unit="pair-evals/s", ms_per_step=secs * 1e3 / steps,
               instance_steps_per_s=len(problems) * steps / secs,
               iterations_per_step_mean=sum(iters) / len(iters),
               iterations_per_step_max=max(max(r["iters"] for r in step) for step in leg["reports"]))
    if tm["pass_launches"] > 0 and tm["pass_ms"] > 0:
        t_s = tm["pass_ms"] * 1e-3
        achieved = FLOP_PER_PAIR * tm["pass_pairs"] / t_s / 1e12
        peak = PEAK_TFLOPS[dtype]
        byts = PASS_BYTES[(dtype, dim)] * tm["pass_particles"]
        gbps = byts / t_s / 1e9
        tr = traffic_from_profile(cfg, dtype) if cfg else None
        rf = dict(bound="alu", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                  frac=round(achieved / peak, 4),
                  traffic=tr[0] if tr else None,
                  kernel="k_pass (pseudo-time pair pass: EDAC pressure rate, momentum, update, residual partials)",
                  flop_per_pair=FLOP_PER_PAIR, flop_per_pair_as_built=FLOP_PER_PAIR_IMPL[dim],
                  bytes_per_particle=PASS_BYTES[(dtype, dim)],
                  hbm=dict(achieved_GBps=round(gbps, 1), peak_GBps=HBM_GBPS, frac=round(gbps / HBM_GBPS, 4)),
                  launches=tm["pass_launches"],
                  timed_launches=("the first pseudo-iteration pair pass of every step of the timed region "
                                  "(every sim takes part), HIP events on the library's stream"
                                  if timing_every == -1 else
                                  f"every {timing_every}-th pair-pass launch of the timed region that had "
                                  f"work (HIP events on the library's stream)"),
                  avg_launch_us=round(tm["pass_ms"] * 1e3 / tm["pass_launches"], 3),
                  pairs_per_launch=round(tm["pass_pairs"] / tm["pass_launches"], 1),
                  particles_per_launch=round(tm["pass_particles"] / tm["pass_launches"], 1),
                  launch_shape=dict(lanes_per_particle=leg["tune"]["lanes"], block=leg["tune"]["block"],
                                    nbr_lanes=leg["tune"]["nbr_lanes"], nbr_tiles=leg["tune"]["nbr_tiles"],
                                    cell_div=leg["tune"]["cell_div"],
                                    autotuned=not leg["tune"].get("fixed", False)))
        if dtype == "f32":
            rf["frac_of_nonpacked_peak"] = round(achieved / PEAK_NONPACKED_F32, 4)
        if tr:
            rf["traffic_note"] = ("HBM bytes per full-batch launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                  "calibrated), from the committed counter summary of this kernel source")
            rf["traffic_over_algorithmic"] = round(tr[0] / tr[1], 3)
        out["roofline"] = rf
        # the time every pair evaluation of the timed region would take at the
        # rate of the timed full-batch launches, as a share of that region
        s_per_pair = tm["pass_ms"] * 1e-3 / tm["pass_pairs"]
        out["pass_share_of_step_time"] = round(evals * s_per_pair / secs, 4)
    if tm["build_launches"] > 0 and tm["build_ms"] > 0:
        n_all = sum(p.n for p in problems)
        exact = sum(r["pairs"] for r in leg["reports"][-1]) / n_all  # fluid rows; walls add few
        p0 = problems[0].params
        skin = (0.25 if p0.get("shift", 0) else 0.3) * p0["h"]
        kh = p0["kappa"] * p0["h"]
        cand = exact * ((kh + skin) / kh) ** dim
        bpp = build_bytes_per_particle(dtype, dim, exact, cand)
        t_s = tm["build_ms"] * 1e-3
        gbps = bpp * tm["build_particles"] / t_s / 1e9
        out["roofline_build"] = dict(
            bound="hbm", achieved=round(gbps, 1), peak=HBM_GBPS, unit="GB/s", frac=round(gbps / HBM_GBPS, 4),
            traffic=None, kernel="full cell build (k_keys, scans, k_scatter, k_rank_gather, k_nbr)",
            bytes_per_particle=round(bpp, 1), exact_entries_per_particle=round(exact, 2),
            candidate_entries_per_particle_est=round(cand, 2), launches=tm["build_launches"],
            avg_build_us=round(tm["build_ms"] * 1e3 / tm["build_launches"], 2),
            builds_per_step=round(tm["full_builds"] / steps, 3))
    return out


def steady_leg(n=150, segments=5, iters=100, timing_every=4, pair_cache=0):
    """Steady lid-driven cavity (sections 2.3, 3.3; Re 100, n x n particles):
    segments of a fixed number of pseudo-iterations, particles fixed."""
    import torch
    from paper_1904_00861_amd import dtsph as D
    from paper_1904_00861_amd import inputs as I

    prob = I.cavity(n, re=100.0, steady=True)
    sim = D.Sim(prob, precision=D.FP32)
    tune = sim.autotune()
    if pair_cache:
        sim.set_option(D.OPT_PAIR_CACHE, pair_cache)
    sim.predict()
    sim.pseudo_iterate(iters)  # warm-up segment
    sim.correct()
    sim.set_option(D.OPT_TIMING, timing_every)
    sim.set_option(D.OPT_RESET_TIMING, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = 0
    for _ in range(segments):
        sim.predict()
        _, rep = sim.pseudo_iterate(iters)
        sim.correct()
        evals += rep[0]["pairs"] * rep[0]["iters"]
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    tm = sim.timing()
    sim.close()
    out = dict(workload=f"steady lid-driven cavity, Re 100, {n}x{n} particles, FP32 sums, "
                        f"{segments} segments of {iters} pseudo-iterations" +
                        (", cached pair coefficients" if pair_cache else ""),
               value=evals / secs, unit="pair-evals/s", ms_per_iteration=secs * 1e3 / (segments * iters),
               launch_shape=dict(lanes=tune["lanes"], block=tune["block"]))
    if tm["pass_launches"]:
        us = tm["pass_ms"] * 1e3 / tm["pass_launches"]
        achieved = FLOP_PER_PAIR_CONV[2] * tm["pass_pairs"] / (tm["pass_ms"] * 1e-3) / 1e12
        out["pass"] = dict(kernel="k_pass (pseudo-time pair pass with the convective sum)",
                           avg_launch_us=round(us, 3), flop_per_pair_as_built=FLOP_PER_PAIR_CONV[2],
                           achieved_tflops=round(achieved, 3))
    return out


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(problems, budget_s=12.0, single_s=4.0):
    """The FP64 oracle on the host: real steps of the sims in batch order (each
    from its state after its previous step, the first from the initial state),
    round after round, until the budget is spent (all OpenMP threads); then the
    same with one thread on a shorter budget."""
    import oracle as O

    def sample(budget):
        t0 = time.perf_counter()
        evals, done = 0, 0
        state = [(p.x, p.v, p.v_prev, p.p) for p in problems]
        while True:
            for s, prob in enumerate(problems):
                x, v, vp, p = state[s]
                x, v, vp, p, reps, st = O.step(prob.params, prob.n_fluid, prob.n_wall, x, v, vp, p, 1)
                state[s] = (x, v, vp, p)
                evals += sum(r["pairs"] * r["iters"] for r in reps)
                done += 1
                if time.perf_counter() - t0 >= budget:
                    return evals, done, time.perf_counter() - t0

    threads = O.num_threads()
    ev, k, dt = sample(budget_s)
    O.set_num_threads(1)
    try:
        ev1, k1, dt1 = sample(single_s)
    finally:
        O.set_num_threads(threads)
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(value=ev / dt, unit="pair-evals/s", cores=threads, kind="oracle",
                sample=f"{k} real sim-steps of the workload, sims in batch order, round after round from the "
                       f"initial states ({dt:.1f} s, FP64 C oracle, OpenMP, {threads} threads)",
                instance_steps_per_s=k / dt, nproc=aff, cpu_model=_cpu_model(),
                single_thread=dict(value=ev1 / dt1, unit="pair-evals/s",
                                   sample=f"{k1} sim-steps, the same order ({dt1:.1f} s, 1 thread)"))


def counter_run(problems, prec, steps, warmup, fixed, shape):
    """Fixed-iteration steps for a hardware-counter run of the profiler: every
    pseudo-iteration pair pass covers the whole workload, so each launch's
    counters compare with the same algorithmic bytes."""
    import torch
    from paper_1904_00861_amd import dtsph as D

    sim = D.Sim(problems, precision=prec)
    if shape:
        apply_shape(sim, shape)
    pairs = 0
    for k in range(warmup + steps):
        sim.predict()
        _, reps = sim.pseudo_iterate(fixed)
        sim.correct()
        pairs = sum(r["pairs"] for r in reps)
    torch.cuda.synchronize()
    info = sim.info
    sim.close()
    print(json.dumps({"counter_run": dict(steps=warmup + steps, fixed_iterations=fixed, particles=info["n"],
                                          fluid=info["n_fluid"], pairs_per_iteration=pairs, shape=shape,
                                          pass_source_sha256=_pass_src_hash())}), flush=True)


def summarize_counters(dirs):
    """Per-dispatch averages of every counter found in rocprofv3 counter CSVs
    under dirs, grouped by kernel name (one JSON line per kernel). Values of one
    counter reported over several rows of a dispatch are summed."""
    per = {}
    for d in dirs:
        for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            for row in csv.DictReader(open(path)):
                key = (path, row.get("Dispatch_Id"))
                ent = per.setdefault(key, dict(kernel=row.get("Kernel_Name", ""), ctr={}))
                ctr = row.get("Counter_Name", "")
                ent["ctr"][ctr] = ent["ctr"].get(ctr, 0.0) + float(row.get("Counter_Value", "nan"))
    groups = {}
    for ent in per.values():
        g = groups.setdefault(ent["kernel"], {})
        for k, v in ent["ctr"].items():
            g.setdefault(k, []).append(v)
    out = []
    for name, g in sorted(groups.items()):
        rec = dict(kernel=name, dispatches=max(len(v) for v in g.values()),
                   avg={k: sum(v) / len(v) for k, v in sorted(g.items())})
        out.append(rec)
        print(json.dumps(rec))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=47)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C4", choices=["C0", "C1", "C2", "C3", "C4"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64 and second-workload legs")
    ap.add_argument("--all-legs", action="store_true",
                    help="also the legs with shifting, particles moving in pseudo-time and the steady solve")
    ap.add_argument("--second", default="C3", choices=["C0", "C1", "C2", "C3", "C4"],
                    help="workload of the second leg")
    ap.add_argument("--second-steps", type=int, default=20)
    ap.add_argument("--no-timing", action="store_true", help="no HIP events in the timed region")
    ap.add_argument("--schedule", type=int, default=None, choices=[0, 1, 2],
                    help="loop schedule of the main leg (DTSPH_OPT_TAIL_LOOP): 0 plain chunks, 1 cut first chunk "
                         "and a persistent tail launch (the library's default), 2 cut first chunk, plain chunks")
    ap.add_argument("--graphs", type=int, default=0, choices=[0, 1],
                    help="1: record each step's segment up to the first chunk of pseudo-iterations as a HIP "
                         "graph and replay it (main leg)")
    ap.add_argument("--shape", default=None, metavar="L,B,G,M",
                    help="fixed launch shape instead of the autotuner: pair-pass lanes per particle, "
                         "workgroup size, neighbour-build lanes (0: the staged-tile kernel), cell subdivision "
                         "(for profiling runs)")
    ap.add_argument("--timing-every", type=int, default=-1, metavar="N",
                    help="HIP events around every N-th pair-pass and build launch in the timed region; -1 "
                         "(default): the first pair pass of every step (the whole workload takes part and the "
                         "launch is queued behind the build, so its events hold the kernel alone) and every "
                         "build (each event record costs host time; sampling keeps it off the step time)")
    ap.add_argument("--shift", type=int, default=None, choices=[0, 1],
                    help="override the workload's particle shifting (section 3.5)")
    ap.add_argument("--pair-cache", type=int, default=0, choices=[0, 1, 2],
                    help="cached pair coefficients in the main leg: 0 off, 1 on, 2 automatic")
    ap.add_argument("--counter-run", type=int, default=0, metavar="K",
                    help="only run --steps steps of K fixed pseudo-iterations each (after --warmup), "
                         "for the hardware counters of a profiler")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise copy of MIB MiB (float32) five times, for "
                         "scaling the HBM byte counters of a profiler; prints its bytes")
    ap.add_argument("--summarize-counters", nargs="+", default=None, metavar="DIR",
                    help="only print per-kernel averages of the counters in rocprofv3 counter CSVs under "
                         "DIR(s) (no GPU needed)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the batched workload shards whole simulations across GPUs without "
              "communication, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return

    import torch
    from paper_1904_00861_amd import dtsph as D
    from paper_1904_00861_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.rand(n, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.add(src, 0.0, out=dst)  # reads 4n bytes, writes 4n bytes
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "elementwise copy", "read_bytes_per_launch": 4 * n,
                          "write_bytes_per_launch": 4 * n, "launches": 5}))
        return
    D.lib()
    prec = D.FP32 if args.precision == "fp32" else D.FP64
    dtype = "f32" if args.precision == "fp32" else "f64"

    def problems_of(cfg):
        prob = I.config(cfg)
        probs = prob if isinstance(prob, list) else [prob]
        if args.shift is not None:
            for p in probs:
                p.params = dict(p.params, shift=args.shift)
        return probs

    problems = problems_of(args.config)
    n_particles = sum(p.n for p in problems)
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    log(f"main leg {args.config} {args.precision}: {len(problems)} sims, {n_particles} particles, "
        f"{args.warmup} warmup + {args.steps} timed steps")
    if args.counter_run:
        counter_run(problems, prec, args.steps, args.warmup, args.counter_run, shape)
        return
    every = 0 if args.no_timing else args.timing_every
    main_leg = run_leg(problems, prec, args.steps, args.warmup, every, shape, args.pair_cache, args.graphs,
                       args.schedule)
    main = leg_summary(problems, main_leg, dtype, args.steps, args.config, args.timing_every)
    log(f"main leg: {main_leg['seconds'] * 1e3:.2f} ms, {main['value']:.3e} pair-evals/s, "
        f"{main['ms_per_step']:.3f} ms/step, iterations/step mean {main['iterations_per_step_mean']:.2f}")

    legs, extras = {}, {}
    if not args.no_extras:
        other = D.FP64 if prec == D.FP32 else D.FP32
        oname, odt = ("fp64", "f64") if other == D.FP64 else ("fp32", "f32")
        log(f"{oname} leg on the same workload")
        leg = run_leg(problems, other, args.steps, args.warmup, every)
        legs[oname] = leg_summary(problems, leg, odt, args.steps, args.config, args.timing_every)
        legs[oname]["workload"] = f"{args.config}, {oname} pair sums"
        extras[f"speedup_{args.precision}_over_{oname}"] = main["value"] / legs[oname]["value"]
        if args.second != args.config:
            sp = problems_of(args.second)
            log(f"second leg {args.second}: {sum(p.n for p in sp)} particles, {args.second_steps} steps")
            leg = run_leg(sp, prec, args.second_steps, args.warmup, every)
            legs[args.second] = leg_summary(sp, leg, dtype, args.second_steps, args.second, args.timing_every)
            legs[args.second]["workload"] = f"{args.second}: {WORKLOADS[args.second]}, {args.precision} sums"
    if args.all_legs:
        for key, upd in (("with_shifting", dict(shift=1)), ("moving", dict(move=1)),
                         ("moving_list_updates", dict(move=2))):
            mod = []
            for p in problems:
                q = p.copy()
                q.params = dict(p.params, **upd)
                mod.append(q)
            log(f"leg {key}")
            ml = run_leg(mod, prec, args.steps, args.warmup, 0)
            extras[f"{key}_value"] = pair_evals(ml["reports"]) / ml["seconds"]
            extras[f"{key}_ms_per_step"] = ml["seconds"] * 1e3 / args.steps
        log("steady-state legs (lid-driven cavity)")
        extras["steady"] = steady_leg()
        extras["steady_pair_cache"] = steady_leg(pair_cache=1)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(problems)

    out = {
        "metric": "pseudo-iteration neighbour-pair evaluations per second (FP32 sums; batched sims/s beside it)",
        "value": main["value"],
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "sims": len(problems),
                   "particles": n_particles,
                   "particle_shifting": bool(any(p.params.get("shift", 0) for p in problems)),
                   "pair_sums": args.precision, "pair_cache": args.pair_cache, "graphs": args.graphs,
                   "loop_schedule": 1 if args.schedule is None else args.schedule,
                   "positions_pressure_residuals": "f64",
                   "instance_steps_per_s": main["instance_steps_per_s"],
                   "iterations_per_step_mean": main["iterations_per_step_mean"],
                   "iterations_per_step_max": main["iterations_per_step_max"]},
        "roofline": main.get("roofline"),
        "roofline_build": main.get("roofline_build"),
        "cpu_baseline": cpu,
        "legs": legs,
        "extras": dict(extras, pass_share_of_step_time=main.get("pass_share_of_step_time")),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
