"""Benchmark of the dual-time EDAC SPH hot path on one MI355X.

A step is one real time step of Algorithm 2 (cell build, wall pass, rate pass
and predictor, cell rebuild, pseudo-time loop until the stop test, corrector)
over the whole workload. Default workload: 2D Taylor-Green vortex, 400 x 400
particles, FP32 pair sums with float64 positions, pressure accumulation and
residuals. The metric is neighbour-pair evaluations of the pseudo-time
iterations per second (pairs of the exact neighbour lists times iterations run,
per sim), inputs resident in HBM before the timed region.

Also reported: the same workload on the plain FP64 path, the 64-instance
batched workload in instance-steps/s, the roofline of the pseudo-iteration pair
pass (HIP events on the library's stream around each launch in the timed
region) and the CPU oracle timed on a bounded sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C1]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic floating-point work of one neighbour pair in the pass kernel
# (FMA = 2): 50 in 2D, 60 in 3D (count in the pass kernel's formula).
FLOP_PER_PAIR = {2: 50, 3: 60}
# with the convective sum of the steady-state solve: + 12 in 2D, + 18 in 3D
FLOP_PER_PAIR_CONV = {2: 62, 3: 78}
# FP32 vector peak without packed instructions: 256 CU x 4 SIMD x 16 lanes x
# 2.4 GHz x 2 (FMA) = 78.6 TFLOP/s; FP64 vector: 78.6 TFLOP/s.
PEAK_TFLOPS = {"f32": 78.6, "f64": 78.6}
PEAK_PACKED_F32 = 157.3

WORKLOADS = {
    "C0": "2D Taylor-Green vortex, periodic unit square, 50x50 particles, Re=100",
    "C1": "2D Taylor-Green vortex, periodic unit square, 400x400 particles, Re=100",
    "C2": "3D Taylor-Green vortex, periodic unit cube, 64^3 particles, Re=1600",
    "C3": "2D dam break, 1x2 column in a 4x4 tank, dx=0.002, 3 wall layers",
    "C4": "batch of 64 periodic TGV / lid-driven cavity instances, 2.5k-160k particles",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pair_evals(reports):
    return sum(r["pairs"] * r["iters"] for step in reports for r in step)


def run_leg(problems, precision, steps, warmup, timing_every, shape=None, pair_cache=0):
    import torch
    from paper_1904_00861_amd import dtsph as D

    sim = D.Sim(problems, precision=precision)
    if pair_cache:
        sim.set_option(D.OPT_PAIR_CACHE, pair_cache)
    if shape:  # fixed launch configuration instead of the autotuner
        lanes, block, nbr_lanes, cell_div = shape
        sim.set_option(D.OPT_LANES, lanes)
        sim.set_option(D.OPT_BLOCK, block)
        sim.set_option(D.OPT_NBR_LANES, nbr_lanes)
        sim.set_option(D.OPT_CELL_DIV, cell_div)
        tune = dict(lanes=lanes, block=block, nbr_lanes=nbr_lanes, cell_div=cell_div, fixed=True)
        log(f"fixed launch shape: pass lanes {lanes} block {block}, neighbour-build lanes {nbr_lanes}, "
            f"cell subdivision {cell_div}")
    else:
        tune = sim.autotune()
    if not shape:
        log(f"autotune: pass lanes {tune['lanes']} block {tune['block']} ({tune['us']:.2f} us); " +
        " ".join(f"{e['lanes']}x{e['block']}:{e['us']:.1f}" for e in tune["entries"]) +
        f"; cell subdivision {tune['cell_div']} (full build {tune['build_us']:.1f} us)"
        f"; neighbour build lanes {tune['nbr_lanes']} ({tune['nbr_us']:.1f} us), "
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


def traffic_from_profile(kernel_src, shape):
    """HBM bytes per pair-pass launch from the committed counter summary for the
    launch shape (lanes, block, cell subdivision), or None if the summary is
    missing, has no row for that shape or the pass kernel changed since it was
    taken."""
    path = os.path.join(ROOT, "profiles", "k_pass_C1_fp32_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"source sha256: ([0-9a-f]{64})", txt)
    if not m_hash:
        return None
    digest = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if digest != m_hash.group(1):
        return None  # counters were taken for an older kernel
    for m in re.finditer(r"traffic: lanes (\d+) block (\d+) cell_div (\d+) bytes ([0-9.eE+]+)", txt):
        if tuple(int(m.group(k)) for k in (1, 2, 3)) == shape:
            return float(m.group(4))
    return None


# launch shapes whose pass traffic the counter sweep measures: cell subdivision
# outermost, then lanes, then workgroup size (the order the summary relies on)
SWEEP_SHAPES = [(lanes, block, 2, cell_div) for cell_div in (1, 2, 3)
                for lanes in (1, 2, 4) for block in (64, 128, 256)]


def traffic_sweep(problems, prec):
    """Run the workload briefly in every launch shape of SWEEP_SHAPES, one after
    the other in one process, for a hardware-counter run of the profiler."""
    for i, shape in enumerate(SWEEP_SHAPES):
        log(f"sweep leg {i}: lanes {shape[0]} block {shape[1]} cell_div {shape[3]}")
        run_leg(problems, prec, 10, 3, 0, shape)
    print(json.dumps({"traffic_sweep": [dict(lanes=s[0], block=s[1], cell_div=s[3]) for s in SWEEP_SHAPES]}))


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
               launch_shape=dict(lanes_per_particle=tune["lanes"], block=tune["block"]))
    if tm["pass_launches"]:
        us = tm["pass_ms"] * 1e3 / tm["pass_launches"]
        achieved = FLOP_PER_PAIR_CONV[2] * tm["pass_pairs"] / (tm["pass_ms"] * 1e-3) / 1e12
        out["pass"] = dict(kernel="k_pass (pseudo-time pair pass with the convective sum)",
                           avg_launch_us=round(us, 3), flop_per_pair=FLOP_PER_PAIR_CONV[2],
                           achieved_tflops=round(achieved, 3), frac=round(achieved / PEAK_TFLOPS["f32"], 4))
    return out


def cpu_baseline(prob, budget_s=12.0, max_steps=400):
    import oracle as O

    x, v, vp, p = prob.x, prob.v, prob.v_prev, prob.p
    t0 = time.perf_counter()
    evals, steps = 0, 0
    while steps < max_steps and time.perf_counter() - t0 < budget_s:
        x, v, vp, p, reps, st = O.step(prob.params, prob.n_fluid, prob.n_wall, x, v, vp, p, 1)
        evals += sum(r["pairs"] * r["iters"] for r in reps)
        steps += 1
    dt = time.perf_counter() - t0
    return dict(value=evals / dt, unit="pair-evals/s", cores=O.num_threads(), kind="oracle",
                sample=f"{steps} real steps of the same workload from its initial state "
                       f"({dt:.1f} s, FP64 C oracle, OpenMP)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C1", choices=["C0", "C1", "C2", "C3", "C4"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64 and batched legs")
    ap.add_argument("--no-timing", action="store_true", help="no HIP events in the timed region")
    ap.add_argument("--shape", default=None, metavar="L,B,G,M",
                    help="fixed launch shape instead of the autotuner: pair-pass lanes per particle, "
                         "workgroup size, neighbour-build lanes, cell subdivision (for profiling runs)")
    ap.add_argument("--timing-every", type=int, default=8, metavar="N",
                    help="HIP events around every N-th pair-pass launch in the timed region (each "
                         "event record costs host time; sampling keeps it off the step time)")
    ap.add_argument("--shift", type=int, default=None, choices=[0, 1],
                    help="override the workload's particle shifting (section 3.5)")
    ap.add_argument("--pair-cache", type=int, default=0, choices=[0, 1, 2],
                    help="cached pair coefficients in the main leg: 0 off, 1 on, 2 automatic")
    ap.add_argument("--traffic-sweep", action="store_true",
                    help="only run the workload for 3+10 steps in each launch shape of a fixed list, "
                         "for the HBM byte counters of a profiler")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise copy of MIB MiB (float32) five times, for "
                         "scaling the HBM byte counters of a profiler; prints its bytes")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the batched workload shards whole simulations across GPUs without "
              "communication, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

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
    prob = I.config(args.config)
    problems = prob if isinstance(prob, list) else [prob]
    if args.shift is not None:
        for p in problems:
            p.params = dict(p.params, shift=args.shift)
    dim = problems[0].params["dim"]
    n_particles = sum(p.n for p in problems)

    log(f"main leg {args.config} {args.precision}: {n_particles} particles, "
        f"{args.warmup} warmup + {args.steps} timed steps")
    if args.traffic_sweep:
        traffic_sweep(problems, prec)
        return
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    main_leg = run_leg(problems, prec, args.steps, args.warmup, 0 if args.no_timing else args.timing_every, shape,
                       args.pair_cache)
    evals = pair_evals(main_leg["reports"])
    secs = main_leg["seconds"]
    value = evals / secs
    iters = [r["iters"] for step in main_leg["reports"] for r in step]
    tm = main_leg["timing"]
    log(f"main leg: {secs * 1e3:.2f} ms, {evals:.3e} pair evals, iterations/step "
        f"mean {sum(iters) / len(iters):.2f}, pair-pass {tm['pass_launches']} launches "
        f"{tm['pass_ms']:.3f} ms")

    roofline = None
    if tm["pass_launches"] > 0 and tm["pass_ms"] > 0:
        flop = FLOP_PER_PAIR[dim] * tm["pass_pairs"]
        achieved = flop / (tm["pass_ms"] * 1e-3) / 1e12
        peak = PEAK_TFLOPS[dtype]
        src = os.path.join(ROOT, "paper_1904_00861_amd", "csrc", "dtsph_pass.hip")
        tr = traffic_from_profile(src, (main_leg["tune"]["lanes"], main_leg["tune"]["block"],
                                        main_leg["tune"]["cell_div"])) \
            if (args.config == "C1" and dtype == "f32") else None
        roofline = dict(bound="alu", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                        frac=round(achieved / peak, 4), traffic=tr,
                        kernel="k_pass (pseudo-time pair pass)",
                        launches=tm["pass_launches"],
                        timed_launches="every %d-th pair-pass launch of the timed region" % args.timing_every,
                        avg_launch_us=round(tm["pass_ms"] * 1e3 / tm["pass_launches"], 3),
                        pairs_per_launch=round(tm["pass_pairs"] / tm["pass_launches"], 1),
                        flop_per_pair=FLOP_PER_PAIR[dim],
                        launch_shape=dict(lanes_per_particle=main_leg["tune"]["lanes"],
                                          block=main_leg["tune"]["block"],
                                          nbr_lanes=main_leg["tune"]["nbr_lanes"],
                                          cell_div=main_leg["tune"]["cell_div"],
                                          autotuned=not shape),
                        frac_of_packed_peak=round(achieved / PEAK_PACKED_F32, 4) if dtype == "f32" else None)

    extras = {}
    if not args.no_extras:
        other = D.FP64 if prec == D.FP32 else D.FP32
        oname = "fp64" if other == D.FP64 else "fp32"
        log(f"{oname} leg on the same workload")
        leg = run_leg(problems, other, args.steps, args.warmup, 0)
        ov = pair_evals(leg["reports"]) / leg["seconds"]
        extras[f"{oname}_value"] = ov
        extras[f"speedup_{args.precision}_over_{oname}"] = value / ov
        if args.config != "C4":
            batch = I.config("C4")
            bsteps = 5
            log(f"batched leg C4: {len(batch)} sims, {sum(p.n for p in batch)} particles, {bsteps} steps")
            bl = run_leg(batch, D.FP32, bsteps, 1, 0)
            extras["batched_instance_steps_per_s"] = len(batch) * bsteps / bl["seconds"]
            extras["batched_pair_evals_per_s"] = pair_evals(bl["reports"]) / bl["seconds"]
            extras["batched_workload"] = WORKLOADS["C4"] + ", FP32 sums, 5 steps"
        if not any(p.params.get("shift", 0) for p in problems):
            # the same workload with the paper's particle shifting after each step
            shifted = []
            for p in problems:
                q = p.copy()
                q.params = dict(p.params, shift=1)
                shifted.append(q)
            log("leg with particle shifting")
            sl = run_leg(shifted, prec, args.steps, args.warmup, 0)
            extras["with_shifting_value"] = pair_evals(sl["reports"]) / sl["seconds"]
            extras["with_shifting_ms_per_step"] = sl["seconds"] * 1e3 / args.steps
        for mv, key in ((1, "moving"), (2, "moving_list_updates")):
            # Algorithm 1 on the same workload: particles advected in pseudo-time,
            # with the lists of r^(0) or recomputed every iteration
            moved = []
            for p in problems:
                q = p.copy()
                q.params = dict(p.params, move=mv)
                moved.append(q)
            log(f"leg with particles moving in pseudo-time (move={mv})")
            ml = run_leg(moved, prec, args.steps, args.warmup, 0)
            extras[f"{key}_value"] = pair_evals(ml["reports"]) / ml["seconds"]
            extras[f"{key}_ms_per_step"] = ml["seconds"] * 1e3 / args.steps
            extras[f"{key}_step_time_over_frozen"] = (ml["seconds"] / args.steps) / (secs / args.steps)
        log("steady-state leg (lid-driven cavity)")
        extras["steady"] = steady_leg()
        extras["steady_pair_cache"] = steady_leg(pair_cache=1)
    extras["iterations_per_step_mean"] = sum(iters) / len(iters)
    if tm["pass_launches"]:
        launches_all = sum(max(r["iters"] for r in step) for step in main_leg["reports"])
        extras["pass_share_of_step_time"] = tm["pass_ms"] / tm["pass_launches"] * launches_all * 1e-3 / secs

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(problems[0] if len(problems) == 1 else problems[0])

    out = {
        "metric": "pseudo-iteration neighbour-pair evaluations per second",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "particles": n_particles,
                   "particle_shifting": bool(any(p.params.get("shift", 0) for p in problems)),
                   "pair_sums": args.precision, "pair_cache": args.pair_cache,
                   "positions_pressure_residuals": "f64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
