"""Benchmark: lattice-point updates/s of the DP-AVF2 hot path on one MI355X.

Default workload: 3-D KGS on [-8,8)^3, n = 256, float64 state, tau = 0.002,
psi0 = e^{-|x|^2} e^{i(x + 0.5y)}, u0 = 0.5 e^{-|x|^2/2}, v0 = 0, all
parameters 1.  One benchmark "step" is one DP-AVF2 time step of the whole
grid (both colour sweeps); the timed region runs exactly --steps of them
followed by one energy evaluation (the drift report), with the state already
resident in HBM.  Prints one JSON line.

    python bench.py [--steps 200] [--warmup 200] [--precision fp64|fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import statistics
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_3d256.json")
KERNEL_SOURCES = ("kgs_stream3d.hip", "kgs_sweep.hip", "kgs_sweep_body.h", "kgs_point.h",
                  "kgs_internal.h", "kgs_layout.h")
ALGO_BYTES = {"fp64": 64, "fp32": 32}  # read + write (P, Q, U, V) once per point-step
METRIC = "lattice-point updates/s + % HBM roofline (3D 256³ FP64); served p50/p99"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["3d", "batched", "batched3d", "serving", "1d", "2d", "paper2d",
                                           "paper3d"], default="3d",
                    help="3d: the headline line (default); batched: 64 uneven 2-D instances; "
                         "serving: Poisson request stream; 1d/2d: the 1-D and 2-D configurations; "
                         "paper2d/paper3d: the paper's own GPU timing examples (t = 1, tau = 0.01)")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed DP-AVF2 steps (default: the workload's own count)")
    # the GPU needs tens of milliseconds of load to reach its steady clock:
    # 200 steps of the 3-D grid take about 50 ms
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=None,
                    help="points per axis (3d, paper3d: 256; paper2d: 2048)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--kernel", choices=["auto", "sweep", "stream"], default="auto")
    ap.add_argument("--tile", type=str, default=None,
                    help="stream kernel shape tile_x,tile_y,chunk,steps_per_launch")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch configuration with kgs_autotune before timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also time a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="3-D: repetitions of the K-step call after the timed one (median reported)")
    ap.add_argument("--requests", type=int, default=120, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=50.0, help="serving: mean arrivals per second")
    ap.add_argument("--budget-gb", type=int, default=64, help="serving: device memory budget")
    ap.add_argument("--round-steps", type=int, default=100, help="serving: steps per round")
    ap.add_argument("--round-work", type=int, default=0,
                    help="serving: point-steps per big-grid round (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true",
                    help="3d: skip the served-latency run (p50/p99 of the serving mix)")
    ap.add_argument("--cpu-steps", type=int, default=4,
                    help="oracle steps on the full grid for the CPU baseline")
    return ap.parse_args()


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_09537_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (each scaled by what the counter reads for a
    plain copy of known size), or None if the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    e = data.get(key)
    if not e or e.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return (e["fetch_kib_per_launch"] * e["fetch_scale"] +
            e["write_kib_per_launch"] * e["write_scale"]) * 1024.0


def host_threads() -> int:
    """Threads the all-cores oracle leg uses: the OpenMP setting if there is
    one, else the CPUs this process may run on, at most 16 (a one-GPU
    share of the host)."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return min(int(env), 16)
    try:
        return min(len(os.sched_getaffinity(0)), 16)
    except AttributeError:
        return min(os.cpu_count() or 1, 16)


def cpu_baseline(problem, steps):
    """The float64 oracle on `steps` steps of the same grid and initial data,
    once on all host threads (OpenMP over the points of each colour pass) and
    once on one thread; the two final states must be bitwise equal."""
    import numpy as np

    import oracle

    g = oracle.Grid(problem.dim, problem.n, problem.lo, problem.hi, problem.kappa1,
                    problem.kappa2, problem.mu, problem.gamma)
    threads = host_threads()
    runs = {}
    for nt in (threads, 1):
        s = oracle.State.from_fields(problem.psi, problem.u, problem.v)
        t0 = time.perf_counter()
        oracle.step_passes(g, problem.tau, s, steps, storage_bits=64, threads=nt)
        runs[nt] = (time.perf_counter() - t0, s)
    dt, s_all = runs[threads]
    dt1, s_one = runs[1]
    same = all(np.array_equal(a, b) for a, b in zip(s_all.arrays(), s_one.arrays()))
    return {"value": problem.points * steps / dt, "unit": "lattice-point updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{problem.dim}-D n={problem.n} same initial data, {steps} DP-AVF2 steps "
                      f"of the full grid, float64, {dt:.1f} s on {threads} threads "
                      f"(one thread: {dt1:.1f} s)",
            "single_core": {"value": problem.points * steps / dt1, "cores": 1},
            "bitwise_equal_to_single_core": same,
            "host_cpu": host_cpu(), "host_threads": os.cpu_count()}


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_errors(got, ref):
    """Max-norm relative errors (psi, u, v) of a state against a reference
    state (numpy arrays or torch tensors), each field against its own
    largest magnitude; v also against the larger of the v and u scales."""
    def mx(a):
        return float(abs(a).max())
    (gp, gu, gv), (rp, ru, rv) = got, ref
    return {"psi": mx(gp - rp) / max(mx(rp), 1e-300), "u": mx(gu - ru) / max(mx(ru), 1e-300),
            "v": mx(gv - rv) / max(mx(rv), 1e-300),
            "v_uv_scale": mx(gv - rv) / max(mx(rv), mx(ru), 1e-300)}


def fp32_vs_fp64(kgs, problems, states, steps):
    """Errors of float32-state results against the float64 path on the same
    problems (the float64 path matches the float64 oracle to 1e-12)."""
    worst = {"psi": 0.0, "u": 0.0, "v": 0.0, "v_uv_scale": 0.0}
    for p, got in zip(problems, states):
        p64 = p.with_(precision=0)
        sim = kgs.simulation_from_problem(p64)
        sim.step(steps)
        ref = sim.read_state(as_torch=type(got[1]).__module__.startswith("torch"))
        sim.close()
        e = rel_errors(got, ref)
        worst = {k: max(worst[k], e[k]) for k in worst}
    return worst


def device_copy_gbs(torch, stream, mib):
    """Bytes read plus written per second by a plain device-to-device copy of
    `mib` MiB (best of 5)."""
    a = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 1e30
    for _ in range(5):
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        b.copy_(a)
        s1.record(stream)
        torch.cuda.synchronize()
        best = min(best, s0.elapsed_time(s1) / 1e3)
    n = a.numel() * 8
    del a, b
    return 2 * n / best / 1e9


def settle_clock(torch, stream, call, min_s=0.5, max_calls=1000, tol=0.02):
    """Untimed repetitions of `call` (one K-step call) until the GPU runs at
    its steady clock: at least `min_s` seconds of calls, and the last two
    within `tol` of each other.  Returns what it ran."""
    times = []
    t0 = time.perf_counter()
    while len(times) < max_calls:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        call()
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
        if (time.perf_counter() - t0 >= min_s and len(times) >= 2 and
                abs(times[-1] - times[-2]) <= tol * times[-1]):
            break
    return {"calls": len(times), "first_ms": times[0], "last_ms": times[-1],
            "s": time.perf_counter() - t0}


def _timed_ms(torch, stream, fn):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b), (time.perf_counter() - t0) * 1e3


def bench_batched(args):
    """64 uneven 2-D instances (n uniform in {128, 192, ..., 1024}), 500 steps
    each, or (--workload batched3d) 16 uneven 3-D instances (n uniform in
    {64, 96, ..., 256}), 40 steps each: one launch sequence per instance vs
    batched launches vs batched launches replayed from a hipGraph; all three
    end bitwise equal.  Each mode is timed on its second run from the
    initial state."""
    import numpy as np
    import torch

    from paper_2502_09537_amd import kgs, workloads

    prec = workloads.FP32 if args.precision == "fp32" else workloads.FP64
    three = args.workload == "batched3d"
    steps = args.steps or (40 if three else 500)
    if three:
        probs = workloads.batched3d_instances(count=16, steps=steps, precision=prec)
    else:
        probs = workloads.batched_instances(count=64, steps=steps, precision=prec)
    pick = (0, 7, 15) if three else (0, 17, 63)
    points = sum(p.points for p in probs)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    results = {}
    finals = {}
    for mode in ("per_instance", "batched", "batched_graph", "batched_tuned"):
        sims = [kgs.simulation_from_problem(p) for p in probs]
        if mode == "per_instance":
            # each handle completes its steps (kgs_sync applies the closing
            # sweep that kgs_step leaves pending), as a batched run does
            run = lambda: [s.step(steps) for s in sims] + [s.sync() for s in sims]
        else:
            b = kgs.Batch(sims, graph=(mode != "batched"))
            if mode == "batched_tuned":
                # untimed: the batch tuner times each group's launch
                # configurations on the initial states (left unchanged)
                b.autotune(steps=4, use_cache=False)
            run = lambda: b.step(steps)
        # every mode: one untimed run (first launches, the GPU's clock ramp,
        # and in graph mode the capture), then the timed run from the
        # initial state again
        run()
        torch.cuda.synchronize()
        for s, p in zip(sims, probs):
            s.write_state(p.psi, p.u, p.v)
        ms, wall = _timed_ms(torch, stream, run)
        results[mode] = {"ms": ms, "updates_per_s": points * steps / (wall / 1e3)}
        finals[mode] = [sims[i].read_state() for i in pick]
        if mode != "per_instance":
            b.close()
        for s in sims:
            s.close()
    identical = all(np.array_equal(x, y) for m in ("batched", "batched_graph", "batched_tuned")
                    for a, b2 in zip(finals["per_instance"], finals[m]) for x, y in zip(a, b2))
    best = max(results, key=lambda m: results[m]["updates_per_s"])
    what = ("16 3-D instances n in {64..256 step 32}, box [-8,8)^3, tau=0.002" if three else
            "64 2-D instances n in {128..1024 step 64}")
    out = {"metric": f"lattice-point updates/s (batched {'3-D' if three else '2-D'} instances)",
           "value": results[best]["updates_per_s"], "unit": "lattice-point updates/s",
           "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": results[best]["ms"] / steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"batched: {what}, params U[0.5,2], {steps} steps, "
                                  f"{args.precision}",
                      "points": points, "state": args.precision, "best_mode": best},
           "modes": results, "bitwise_identical_across_modes": identical,
           "speedup_vs_per_instance": results[best]["updates_per_s"] /
           results["per_instance"]["updates_per_s"]}
    if prec == workloads.FP32:
        sample = [probs[i] for i in pick]
        out["fp32_max_rel_err_vs_fp64"] = fp32_vs_fp64(kgs, sample, finals["batched"], steps)
        out["fp32_error_sample"] = (f"instances {', '.join(map(str, pick))} after the run, "
                                    "against float64 runs")
    print(json.dumps(out), flush=True)


def bench_serving(args, only=None, emit=True):
    """Poisson request stream (mean --rate per second; 1-D n in [256, 8192],
    2-D n in [128, 1024], 3-D n in [64, 256], steps in [100, 2000], fp32 or
    fp64 at random), replayed in real time against the continuous-batching
    server and against one request at a time (max_active = 1).  Latency is
    measured from each request's arrival to its retirement.  Each server is
    warmed first (untimed) with the first requests of the mix, a few steps
    each."""
    import numpy as np
    import torch

    from paper_2502_09537_amd import kgs, workloads

    torch.cuda.set_device(0)
    reqs = workloads.serving_requests(count=args.requests, rate=args.rate, seed=1, arrays=False)
    work = sum(r.problem.points * r.problem.steps for r in reqs)
    out = {"metric": "served solves/s with p50/p99 latency", "unit": "solves/s", "n_gpus": 1,
           "steps": None, "warmup": 0, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"serving: {args.requests} Poisson requests at {args.rate}/s, "
                                  "1-D/2-D/3-D mix, fp32/fp64, steps U[100,2000]",
                      "state": "fp64 and fp32 requests",
                      "budget_gb": args.budget_gb, "steps_per_round": args.round_steps,
                      "round_work": args.round_work,
                      "lattice_updates_total": work}}
    # "saturated" submits every request at once: its makespan gives the
    # continuous server's capacity on this mix, and the offered load is
    # rho = offered updates/s / that capacity
    modes = {"continuous": dict(max_active=0, steps_per_round=args.round_steps,
                                round_work=args.round_work),
             "one_at_a_time": dict(max_active=1, steps_per_round=0),
             "saturated": dict(max_active=0, steps_per_round=args.round_steps,
                               round_work=args.round_work)}
    if only:  # these modes, in this order
        modes = {m: modes[m] for m in only}
    offered = work / (reqs[-1].arrival - reqs[0].arrival)
    check_ids = []

    def warm_up(srv, count=32, steps=4):
        # untimed: the first requests of the mix, a few steps each, run to
        # completion on this server, so that the timed run meets a warm
        # server (every kernel it launches loaded, its memory pool grown)
        wid = []
        for r in reqs[:count]:
            f = workloads.gaussian_fields_torch(r.problem)
            wid.append(srv.submit_device(kgs.config_of(r.problem), *f, steps))
        while True:
            nr, nq = srv.run(1)
            if nr == 0 and nq == 0:
                break
        for rid in wid:
            srv.release(rid)
        torch.cuda.synchronize()
        return srv.stats().rounds

    for mode, kw in modes.items():
        burst = mode == "saturated"
        srv = kgs.Server(budget_bytes=args.budget_gb << 30, **kw)
        warm_rounds = warm_up(srv)
        keep = []
        ids = []
        i = 0
        t_start = time.perf_counter()
        offset = srv.stats().now  # server clock at t_start
        while True:
            now = time.perf_counter() - t_start
            while i < len(reqs) and (burst or reqs[i].arrival <= now):
                p = reqs[i].problem
                f = workloads.gaussian_fields_torch(p)
                rid = srv.submit_device(kgs.config_of(p), *f, p.steps)
                keep.append(f)
                ids.append((rid, i))
                i += 1
            st = srv.stats()
            if st.running == 0 and st.queued == 0:
                if i == len(reqs):
                    break
                time.sleep(max(0.0, reqs[i].arrival - (time.perf_counter() - t_start)))
                continue
            srv.run(1)
            keep.clear()
        t_end = time.perf_counter() - t_start
        lat, done_t = [], []
        for rid, j in ids:
            info = srv.poll(rid)
            assert info.state == kgs.KGS_REQ_DONE, (mode, j, info.state, info.status)
            lat.append(info.t_done - ((0.0 if burst else reqs[j].arrival) + offset))
            done_t.append(info.t_done - offset)
        lat = np.array(lat)
        span = max(done_t) - (0.0 if burst else reqs[0].arrival)
        if burst:
            out[mode] = {"makespan_s": span, "capacity_updates_per_s": work / span,
                         "solves_per_s": len(reqs) / span}
            out["offered_load_rho"] = offered / (work / span)
            srv.close()
            continue
        out[mode] = {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                     "mean_s": float(lat.mean()), "solves_per_s": len(reqs) / span,
                     "lattice_updates_per_s": work / span, "makespan_s": span,
                     "offered_updates_per_s": offered,
                     "rounds": int(srv.stats().rounds - warm_rounds)}
        if mode == "continuous":
            # results in the mix equal results alone (a sample of small requests)
            small = [(rid, j) for rid, j in ids if reqs[j].problem.points <= 1 << 16][:6]
            ok = True
            fp32_err = {"psi": 0.0, "u": 0.0, "v": 0.0, "v_uv_scale": 0.0}
            for rid, j in small:
                p = reqs[j].problem
                got = srv.result(rid)
                f = workloads.gaussian_fields_torch(p)
                sim = kgs.Simulation(kgs.config_of(p), torch.complex(f[0], f[1]), f[2], f[3])
                sim.step(p.steps)
                ref = sim.read_state()
                sim.close()
                ok &= all(np.array_equal(a, b) for a, b in zip(got, ref))
                if p.precision == workloads.FP32:
                    p64 = p.with_(precision=workloads.FP64)
                    s64 = kgs.Simulation(kgs.config_of(p64), torch.complex(f[0], f[1]), f[2], f[3])
                    s64.step(p.steps)
                    e = rel_errors(got, s64.read_state())
                    s64.close()
                    fp32_err = {k: max(fp32_err[k], e[k]) for k in fp32_err}
            out["mix_equals_alone_bitwise"] = {"checked": len(small), "identical": bool(ok)}
            out["fp32_max_rel_err_vs_fp64"] = fp32_err
        srv.close()
    best = out["continuous"]
    out["value"] = best["solves_per_s"]
    out["ms_per_step"] = None
    out["p50_s"], out["p99_s"] = best["p50_s"], best["p99_s"]
    if emit:
        print(json.dumps(out), flush=True)
    return out


def bench_small_dims(args):
    """The 1-D (n = 256, 1000 steps) and 2-D (n = 1024^2, 1000 steps) float64
    configurations: updates/s of the library's default kernel for the grid,
    energy drift over the run, and the oracle on the same grid."""
    import torch

    from paper_2502_09537_amd import kgs, workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.workload == "1d":
        p = workloads.config_1d()
    else:
        p = workloads.config_2d()
    steps = args.steps if args.steps is not None else p.steps
    sim = kgs.simulation_from_problem(p)
    info = sim.info()
    sim.step(args.warmup)
    e0 = sim.energy()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(steps)
    stop.record(stream)
    e1 = sim.energy()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    names = {kgs.KGS_KERNEL_SWEEP: "sweep", kgs.KGS_KERNEL_STREAM: "stream",
             kgs.KGS_KERNEL_RESIDENT: "resident", kgs.KGS_KERNEL_TILE: "tile"}
    out = {"metric": "lattice-point updates/s", "value": p.points * steps / wall,
           "unit": "lattice-point updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{p.name} n={p.n}^{p.dim} box [{p.lo},{p.hi}) tau={p.tau} "
                                  f"float64, {steps} DP-AVF2 steps",
                      "points": p.points, "kernel": names.get(info.kernel, str(info.kernel)),
                      "parallelism": "1 GPU"},
           "kernel_ms": start.elapsed_time(stop),
           "energy_rel_drift": abs(e1 - e0) / abs(e0)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, steps if p.dim == 1 else 2)
    print(json.dumps(out), flush=True)


# The paper's GPU times (one NVIDIA A40, precision not stated, t = 1 with
# tau = 0.01, i.e. 100 steps) for its timing examples: Tab. time-2d (2-D four
# solitons) and Tab. gpu3d_list (3-D example of sec. 5.2), by points per axis.
PAPER_A40_S = {
    "paper2d": {512: 2.29e-2, 768: 5.25e-2, 1024: 9.34e-2, 1280: 1.28e-1, 1536: 1.96e-1,
                1792: 2.76e-1, 2048: 3.70e-1},
    "paper3d": {128: 1.72e-1, 192: 6.25e-1, 256: 1.61, 320: 3.30, 384: 6.03, 448: 9.96,
                512: 15.6},
}


def bench_paper(args):
    """One of the paper's own GPU timing examples at its own size and step
    count: the run of 100 steps with the state resident on the GPU (value),
    repeated, and the same run with the state copied from and back to host
    memory around it (as the paper's GPU algorithm does), against the paper's
    A40 time for the same grid."""
    import numpy as np
    import torch

    from paper_2502_09537_amd import kgs, workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    prec = workloads.FP32 if args.precision == "fp32" else workloads.FP64
    n = args.n or (2048 if args.workload == "paper2d" else 256)
    p = (workloads.timing_2d if args.workload == "paper2d" else workloads.timing_3d)(n, prec)
    steps = args.steps if args.steps is not None else p.steps
    sim = kgs.simulation_from_problem(p)
    info = sim.info()
    sim.step(args.warmup)
    sim.sync()
    e0 = sim.energy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    wall = time.perf_counter() - t0
    e1 = sim.energy()
    reps = []
    for _ in range(args.repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(steps)
        b.record(stream)
        torch.cuda.synchronize()
        reps.append(a.elapsed_time(b) / 1e3)
    sim.close()

    # The KGS_HOST boundary: the four float64 fields in host memory, as a
    # caller holds them, copied in by kgs_init and out by kgs_read_state.
    # The arrays are prepared outside the timed region.
    cfg = kgs.config_of(p)
    fields = [np.ascontiguousarray(a, dtype=np.float64) for a in (p.psi.real, p.psi.imag, p.u, p.v)]
    outs = [np.ones_like(a) for a in fields]

    def host_run():
        t = [time.perf_counter()]
        h = kgs.kgs_init(cfg, *[a.ctypes.data for a in fields], kgs.KGS_HOST, 0)
        t.append(time.perf_counter())
        kgs.kgs_step(h, steps)
        kgs.kgs_sync(h)
        t.append(time.perf_counter())
        kgs.kgs_read_state(h, *[a.ctypes.data for a in outs], kgs.KGS_HOST)
        t.append(time.perf_counter())
        kgs.kgs_free(h)
        t.append(time.perf_counter())
        return t[-1] - t[0], {k: t[i + 1] - t[i] for i, k in enumerate(("init", "steps", "read", "free"))}
    host_run()
    host_s, host_parts = host_run()

    names = {kgs.KGS_KERNEL_SWEEP: "sweep", kgs.KGS_KERNEL_STREAM: "stream",
             kgs.KGS_KERNEL_RESIDENT: "resident", kgs.KGS_KERNEL_TILE: "tile"}
    updates = p.points * steps
    paper_s = PAPER_A40_S[args.workload].get(n) if steps == 100 else None
    out = {"metric": "lattice-point updates/s", "value": updates / wall,
           "unit": "lattice-point updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": (updates / wall) / (updates / paper_s) if paper_s else None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{p.name} n={n}^{p.dim} box [{p.lo},{p.hi}) tau={p.tau} "
                                  f"kappa1={p.kappa1} kappa2={p.kappa2} mu={p.mu} "
                                  f"gamma={p.gamma}, {args.precision} state, {steps} DP-AVF2 steps",
                      "points": p.points, "state": args.precision,
                      "kernel": names.get(info.kernel, str(info.kernel)), "parallelism": "1 GPU"},
           "run_s": wall,
           "repeats_s": reps,
           "host_inclusive_s": host_s,
           "host_inclusive_parts_s": host_parts,
           "host_state_bytes_each_way": 4 * 8 * p.points,
           "paper_a40_s": paper_s,
           "speedup_vs_paper_a40": paper_s / wall if paper_s else None,
           "host_inclusive_speedup_vs_paper_a40": paper_s / host_s if paper_s else None,
           "energy_rel_drift": abs(e1 - e0) / abs(e0)}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the library runs one simulation on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload in ("batched", "batched3d"):
        return bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload in ("1d", "2d"):
        return bench_small_dims(args)
    if args.workload in ("paper2d", "paper3d"):
        return bench_paper(args)
    if args.n is None:
        args.n = 256
    if args.steps is None:
        args.steps = 200
    import torch

    from paper_2502_09537_amd import kgs, workloads

    prec = workloads.FP32 if args.precision == "fp32" else workloads.FP64
    p = workloads.config_3d(n=args.n, steps=args.steps, precision=prec)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    sim = kgs.simulation_from_problem(p)
    if args.kernel != "auto" or args.tile:
        t = sim.tuning
        if args.kernel != "auto":
            t.kernel = {"sweep": kgs.KGS_KERNEL_SWEEP, "stream": kgs.KGS_KERNEL_STREAM}[args.kernel]
        if args.tile:
            t.tile_x, t.tile_y, t.chunk, t.steps_per_launch = (int(v) for v in args.tile.split(","))
        sim.tuning = t
    if args.autotune:
        sim.autotune(steps=16, use_cache=False)
    info = sim.info()
    tun = sim.tuning
    sim.step(args.warmup)
    sim.sync()
    settle = settle_clock(torch, stream, lambda: sim.step(args.steps))
    e0 = sim.energy()

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(args.steps)
    stop.record(stream)
    e1 = sim.energy()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kernel_ms = start.elapsed_time(stop)

    # the same K-step call repeated: the spread of the timed region
    reps = []
    for _ in range(args.repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(args.steps)
        b.record(stream)
        torch.cuda.synchronize()
        reps.append(a.elapsed_time(b))

    # the dominant kernel's own average duration: a kgs_step call of K steps
    # is K/spl streaming launches (or 2K sweeps); the sweep closing its last
    # step is left pending and fused into the next call's first launch, and
    # whatever fixed cost a call has besides cancels in the difference of
    # 2- and 4-step calls
    def timed(k):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(k)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)
    spl = tun.steps_per_launch if info.kernel == kgs.KGS_KERNEL_STREAM else 1
    per = 1 if info.kernel == kgs.KGS_KERNEL_STREAM else 2  # launches per spl steps
    t_small = min(timed(2 * spl) for _ in range(3))
    t_big = min(timed(4 * spl) for _ in range(3))
    unit_ms = (t_big - t_small) / (2 * per)           # one dominant-kernel launch
    closing_ms = max(t_small - 2 * per * unit_ms, 0.0)  # a call's fixed cost
    sim.close()

    updates = p.points * args.steps
    value = updates / wall
    n_dom = int(round(args.steps / spl * per))
    avg_launch_s = max(kernel_ms - closing_ms, 1e-9) / 1e3 / n_dom
    # algorithmic bytes of one launch at 64/K bytes per point-step (float64;
    # 32/K in float32) for K steps fused in the launch: a streaming launch
    # reads and writes every point's four values once, whatever its K; a
    # sweep launch does so for the half of the points of its colour
    algo_per_launch = ALGO_BYTES[args.precision] * p.points * (1.0 if per == 1 else 0.5)
    achieved = algo_per_launch / avg_launch_s / 1e9
    # the same launch priced as if each of its steps moved the state once
    # (one step per launch); above the peak whenever K > 1 pays off
    effective = algo_per_launch * (spl if per == 1 else 1) / avg_launch_s / 1e9
    key = f"{args.precision}:" + ("stream%d" % spl if per == 1 else "sweep")
    traffic = measured_traffic(key) if args.n == 256 else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "lattice-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",  # the arithmetic; the state precision is in config
        "data": "synthetic",
        "config": {"workload": f"kgs3d n={p.n}^3 box [-8,8)^3 tau={p.tau} "
                               f"{args.precision} state, {args.steps} DP-AVF2 steps",
                   "points": p.points, "state": args.precision, "kernel": int(info.kernel),
                   "tile": [tun.tile_x, tun.tile_y, tun.chunk, tun.steps_per_launch]
                   if info.kernel == kgs.KGS_KERNEL_STREAM else None,
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": key, "avg_launch_us": avg_launch_s * 1e6,
                     "algorithmic_bytes_per_launch": algo_per_launch,
                     "steps_per_launch": spl if per == 1 else 0.5,
                     "effective_GBs": effective, "effective_frac": effective / HBM_PEAK_GBS},
        "settle": settle,
        "energy_rel_drift": abs(e1 - e0) / abs(e0),
        "kernel_ms": kernel_ms,
        "repeats_ms": reps,
        "median_updates_per_s": updates / (statistics.median(reps) / 1e3) if reps else None,
    }
    if args.precision == "fp32":
        # the float32 state's error after the timed number of steps, against
        # the float64 path from the same initial data
        s32 = kgs.simulation_from_problem(p)
        s32.step(args.steps)
        got = s32.read_state(as_torch=True)
        s32.close()
        out["fp32_max_rel_err_vs_fp64"] = fp32_vs_fp64(kgs, [p], [got], args.steps)
        del got
    if traffic:
        # actual HBM traffic rate of the dominant kernel, against the peak and
        # against what a plain device copy reaches on this GPU
        out["roofline"]["traffic_GBs"] = traffic / avg_launch_s / 1e9
        # measured HBM bytes per lattice-point update (algorithmic: 64 / 32)
        out["roofline"]["traffic_bytes_per_update"] = traffic / (
            p.points * (spl if per == 1 else 0.5))
        copy_gbs = device_copy_gbs(torch, stream, 1024)
        out["roofline"]["copy_GBs"] = copy_gbs
        out["roofline"]["traffic_frac_of_peak"] = traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS
        out["roofline"]["traffic_frac_of_copy"] = traffic / avg_launch_s / 1e9 / copy_gbs
    if args.calibrate_copy:
        a = torch.empty(args.calibrate_copy << 17, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(10):
            b.copy_(a)
        s1.record(stream)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": a.numel() * 8, "bytes_written": a.numel() * 8,
                                   "ms": s0.elapsed_time(s1) / 10,
                                   "GBs": 2 * a.numel() * 8 / (s0.elapsed_time(s1) / 10 / 1e3) / 1e9}
    if not args.no_served:
        # the metric's served latencies: the continuous-batching server on the
        # serving mix (Poisson arrivals, 1-/2-/3-D requests), replayed in real
        # time, and the same requests submitted at once for the capacity and
        # the offered load
        sv = bench_serving(args, only=("continuous", "saturated"), emit=False)
        out["served"] = {"workload": sv["config"]["workload"], "p50_s": sv["p50_s"],
                         "p99_s": sv["p99_s"], "solves_per_s": sv["value"],
                         "lattice_updates_per_s": sv["continuous"]["lattice_updates_per_s"],
                         "capacity_updates_per_s": sv["saturated"]["capacity_updates_per_s"],
                         "offered_load_rho": sv["offered_load_rho"],
                         "mix_equals_alone_bitwise": sv["mix_equals_alone_bitwise"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(workloads.config_3d(n=args.n), args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
