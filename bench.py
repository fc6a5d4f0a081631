#!/usr/bin/env python
"""Throughput of the split-step Crank-Nicolson spin-1 step on one MI355X.

Headline workload: 512 x 512 real-time run (Dresselhaus gamma = 1, Rabi 0.2,
Omega = 0.9, c0 = 200, c2 = +5, dx = 0.05, dt = 1e-4) started from the
imaginary-time state of the same parameters plus seeded complex noise of 1e-3;
a step is one whole SSCN step (local substep, x sweep, y sweep).  Timed in
FP64 (the headline value) and in FP32 bulk.  Also timed: 4096 x 4096
imaginary-time steps (Rashba gamma = 0.75, Omega = 0.95, c0 = 1000, c2 = -20,
dx = 0.02), the grid whose state (805 MB in FP64) does not fit in the caches,
which gives the honest HBM roofline fraction.  All inputs are seeded and
synthetic.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_BPS = 8.0e12  # MI355X HBM3E, vendor figure
METRIC = "3-comp grid-point-steps/s FP64 vs FP32 (%HBM roofline); p50/p99 solve latency"
UNIT = "3-comp grid-point-steps/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_complex(prec):
    return 16 if prec == "fp64" else 8


def kernel_roofline(timing, npts, prec):
    """Roofline of the dominant sweep kernel: algorithmic bytes per launch
    (read + write of the 3 components, 6 s bytes per point) / mean launch time."""
    per_launch = 6 * bytes_per_complex(prec) * npts
    rows = {}
    for kind in ("x_sweep", "y_sweep"):
        t = timing[kind]
        if t["launches"]:
            avg_s = t["ms"] / t["launches"] / 1e3
            rows[kind] = {"avg_us": avg_s * 1e6, "achieved_GBps": per_launch / avg_s / 1e9,
                          "frac": per_launch / avg_s / HBM_PEAK_BPS, "total_ms": t["ms"]}
    dom = max(rows, key=lambda k: rows[k]["total_ms"])
    d = rows[dom]
    return {"bound": "hbm", "kernel": dom, "achieved": round(d["achieved_GBps"], 1), "peak": HBM_PEAK_BPS / 1e9,
            "unit": "GB/s", "frac": round(d["frac"], 4), "traffic": None,
            "bytes_per_launch": per_launch,
            "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in rows.items()}}


TILES = {"fp64": [(8, 2), (8, 4), (4, 4), (4, 8)], "fp32": [(8, 4), (4, 8), (4, 4), (8, 8)]}


def tile_args(prec, tile):
    """Template arguments (points per lane, waves, lines one at a time) of window tile 1..8."""
    kk, nw = TILES[prec][(tile - 1) & 3]
    return f"{kk}, {nw}, {'true' if (tile - 1) & 4 else 'false'}, "


def traffic_for(roof, prec, imag, plan, workload):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when there is none for these kernel sources."""
    from paper_2105_10517_amd import profile_summary
    t = profile_summary.read_traffic(os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.md"))
    T = "double" if prec == "fp64" else "float"
    im = "true" if imag else "false"
    if roof["kernel"] == "x_sweep":
        if plan["x_solver"] == 2:
            prefix = f"gp::k_x_window<{T}, {im}, " + tile_args(prec, plan["x_tile"])
        else:
            prefix = f"gp::k_x_scan<{T}, {im}, {plan['x_points_per_thread']}, "
    else:
        prefix = f"gp::k_y_window<{T}, {im}, " + tile_args(prec, plan["y_tile"])
    for k, v in t.items():
        if k.startswith(prefix):
            return v
    return None


def time_steps(solver, t, nsteps, imag, torch):
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    (solver.step_imag if imag else solver.step_real)(t, nsteps)
    e1.record(st)
    torch.cuda.synchronize()
    solver.sync()
    return e0.elapsed_time(e1)


def kernel_timing(solver, t, nsteps, imag):
    solver.timing(True)
    (solver.step_imag if imag else solver.step_real)(t, nsteps)
    res = solver.timing_read()
    solver.timing(False)
    return res


def c2_initial_state(torch, binding, inputs):
    """Imaginary-time state of the headline parameters (dt = 0.1 dx^2, stop at
    |dE|/E < 1e-10 over 100 steps or 20000 steps), plus 1e-3 noise (seed 3)."""
    p = inputs.config_c2()
    q = dict(p, dt=0.1 * p["dx"] * p["dx"])
    psi = inputs.gaussian(p["nx"], p["ny"], p["dx"], p["dy"], seed=2, phase_noise=0.1)
    s = binding.Solver(q, "fp64")
    t = torch.from_numpy(psi).to("cuda")
    e_prev, steps = None, 0
    while steps < 20000:
        s.step_imag(t, 100)
        steps += 100
        e = s.observables(t)["energy"]
        if e_prev is not None and abs(e - e_prev) < 1e-10 * abs(e):
            break
        e_prev = e
    log(f"[bench] C2 initial state: {steps} imaginary-time steps, E = {e:.10f}")
    out = inputs.add_noise(t.cpu().numpy(), p["dx"], p["dy"], 1e-3, seed=3)
    s.close()
    return p, out


def cpu_baseline(p, psi0, seconds):
    """The oracle on all host threads for about `seconds`, and on one thread
    for a fifth of that."""
    import oracle
    threads = oracle.get_threads()

    def rate(budget):
        t0 = time.perf_counter()
        psi = oracle.step(p, psi0, 1, False)
        t1 = time.perf_counter() - t0
        n = max(1, int(budget / max(t1, 1e-6)))
        t0 = time.perf_counter()
        oracle.step(p, psi, n, False)
        dt = time.perf_counter() - t0
        return p["nx"] * p["ny"] * n / dt, n, dt

    v, n, dt = rate(seconds)
    oracle.set_threads(1)
    v1, n1, dt1 = rate(seconds / 5)
    oracle.set_threads(threads)
    return {"value": v, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{n} real-time FP64 steps of the {p['nx']}x{p['ny']} workload (block-Thomas oracle, "
                      f"{dt:.1f} s)",
            "value_1_core": v1, "sample_1_core": f"{n1} steps on one thread ({dt1:.1f} s)"}


def copy_rate(torch, nbytes, reps=50):
    """Bytes moved per second by a plain device copy of nbytes (read + write),
    the practical ceiling beside the 8 TB/s peak."""
    a = torch.ones(nbytes // 16, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
        a.copy_(b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
        a.copy_(b)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / (2 * reps)
    del a, b
    return 2 * nbytes / sec


def batch_c4(torch, binding, inputs, nsteps):
    """256 condensates of the parameter scan (FP32 bulk, imaginary time) in
    batched launches, against the same solves one at a time in FP64."""
    ps = inputs.batch_scan(256, seed=5)
    psi0 = [inputs.gaussian(p["nx"], p["ny"], p["dx"], p["dy"], x0=p["x0"], y0=p["y0"], seed=1000 + k)
            for k, p in enumerate(ps)]
    pts = sum(p["nx"] * p["ny"] for p in ps) * nsteps
    b = binding.Batch(ps, "fp32")
    ts = [torch.from_numpy(a).to(torch.complex64).to("cuda") for a in psi0]
    b.step(ts, [5] * len(ps), ["imag"] * len(ps))  # warm-up
    b.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    b.step(ts, [nsteps] * len(ps), ["imag"] * len(ps))
    e1.record()
    b.sync()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    info = b.info()
    b.close()
    del ts
    # the same solves one at a time, FP64
    t64 = [torch.from_numpy(a).to("cuda") for a in psi0]
    solvers = [binding.Solver(p, "fp64") for p in ps]
    for s_, t in zip(solvers, t64):
        s_.step_imag(t, 5)
    torch.cuda.synchronize()
    e0.record()
    for s_, t in zip(solvers, t64):
        s_.step_imag(t, nsteps)
    e1.record()
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1)
    for s_ in solvers:
        s_.close()
    del t64
    torch.cuda.empty_cache()
    out = {"workload": f"256 condensates, N = 32 k (k ~ U{{4..16}}), {nsteps} imaginary-time steps each",
           "value_fp32_batched": pts / (ms_b / 1e3), "value_fp64_one_at_a_time": pts / (ms_s / 1e3),
           "ms_batched": ms_b, "ms_one_at_a_time": ms_s, "unit": UNIT, "grouped": info["grouped"],
           "individual": info["individual"], "x_points": info["x_points"][0], "y_tile": info["y_tile"][0]}
    log(f"[bench] C4 batch: FP32 batched {out['value_fp32_batched']:.3e} pt-steps/s vs FP64 one at a time "
        f"{out['value_fp64_one_at_a_time']:.3e} ({ms_b:.1f} ms vs {ms_s:.1f} ms)")
    return out


def serving_c5(torch, binding, inputs, n, rate):
    """The serving trace (Poisson arrivals, N in {128..1024}, 500-5000 steps,
    imaginary or real time, FP32) replayed in real time."""
    trace = inputs.serving_trace(n, rate, seed=6)
    reqs = []
    for r in trace:
        p = r["params"]
        a = inputs.gaussian(p["nx"], p["ny"], p["dx"], p["dy"], x0=p["x0"], y0=p["y0"], seed=r["seed"])
        reqs.append(dict(r, psi=torch.from_numpy(a).to(torch.complex64).to("cuda")))
    torch.cuda.synchronize()
    res, st = binding.serve(reqs, "fp32", max_slots=256, hbm_budget_bytes=200e9, chunk_steps=250, time_scale=1.0)
    out = {"workload": f"{n} requests, Poisson {rate:g}/s, N in {{128,256,512,1024}} (p .4/.3/.2/.1), "
                       f"500-5000 steps, imaginary or real time, FP32, 200 GB budget",
           "p50_latency_s": st["p50_latency"], "p99_latency_s": st["p99_latency"],
           "mean_latency_s": st["mean_latency"], "served_rate": st["served_rate"],
           "offered_rate": st["offered_rate"], "wall_s": st["wall_s"], "rounds": st["rounds"],
           "mean_in_flight": st["mean_active"], "max_in_flight": st["max_active"], "unit_rate": UNIT}
    log(f"[bench] C5 serving: p50 {st['p50_latency']:.3f} s, p99 {st['p99_latency']:.3f} s, served "
        f"{st['served_rate']:.3e} vs offered {st['offered_rate']:.3e} pt-steps/s, {st['mean_active']:.1f} in flight")
    del reqs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000, help="timed SSCN steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--c3-steps", type=int, default=100, help="timed steps of the 4096^2 grid (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-baseline sample length (0 = skip)")
    ap.add_argument("--timing-steps", type=int, default=500, help="steps of the per-kernel timing pass")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="imaginary-time steps of the 256-condensate batch (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=64, help="requests of the serving trace (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=25.0, help="arrival rate of the serving trace (1/s)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (each condensate runs on "
              f"one device and this build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2105_10517_amd import binding, inputs
    binding.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    p, psi0 = c2_initial_state(torch, binding, inputs)
    npts = p["nx"] * p["ny"]
    results = {}
    for prec in ("fp64", "fp32"):
        s = binding.Solver(p, prec, autotune=True)
        t = torch.from_numpy(psi0).to("cuda").to(s.dtype)
        s.step_real(t, args.warmup)
        ms = time_steps(s, t, args.steps, False, torch)
        norm = s.observables(t)["norm_total"]
        tim = kernel_timing(s, t, args.timing_steps, False)
        roof = kernel_roofline(tim, npts, prec)
        roof["traffic"] = traffic_for(roof, prec, False, s.plan(False), "c2_512")
        cp = copy_rate(torch, 3 * npts * bytes_per_complex(prec))
        roof["copy_GBps"] = round(cp / 1e9, 1)
        roof["frac_of_copy"] = round(roof["achieved"] * 1e9 / cp, 4)
        val = npts * args.steps / (ms / 1e3)
        step_bytes = 12 * bytes_per_complex(prec) * npts
        results[prec] = {"value": val, "ms_per_step": ms / args.steps, "roofline": roof,
                         "step_frac": step_bytes / (ms / args.steps / 1e3) / HBM_PEAK_BPS,
                         "norm_drift": norm - 1.0, "plan": s.plan(False)}
        log(f"[bench] 512^2 real {prec}: {val:.3e} pt-steps/s, {ms / args.steps * 1e3:.2f} us/step, "
            f"dominant {roof['kernel']} {roof['achieved']:.0f} GB/s ({roof['frac'] * 100:.1f}% of HBM peak), "
            f"norm drift {norm - 1:.2e}")
        s.close()
        del t
        torch.cuda.empty_cache()

    c3 = {}
    if args.c3_steps > 0:
        q = inputs.config_c3(4096)
        psi3 = inputs.gaussian(4096, 4096, q["dx"], q["dy"], seed=4, full_phase=True)
        n3 = 4096 * 4096
        for prec in ("fp64", "fp32"):
            s = binding.Solver(q, prec, autotune=True)
            t = torch.from_numpy(psi3).to("cuda").to(s.dtype)
            s.step_imag(t, 5)
            ms = time_steps(s, t, args.c3_steps, True, torch)
            tim = kernel_timing(s, t, max(10, args.c3_steps // 5), True)
            roof = kernel_roofline(tim, n3, prec)
            roof["traffic"] = traffic_for(roof, prec, True, s.plan(True), "c3_4096")
            cp = copy_rate(torch, 3 * n3 * bytes_per_complex(prec), reps=10)
            roof["copy_GBps"] = round(cp / 1e9, 1)
            roof["frac_of_copy"] = round(roof["achieved"] * 1e9 / cp, 4)
            val = n3 * args.c3_steps / (ms / 1e3)
            step_bytes = 12 * bytes_per_complex(prec) * n3
            c3[prec] = {"value": val, "ms_per_step": ms / args.c3_steps, "roofline": roof,
                        "step_frac": step_bytes / (ms / args.c3_steps / 1e3) / HBM_PEAK_BPS}
            log(f"[bench] 4096^2 imag {prec}: {val:.3e} pt-steps/s, {ms / args.c3_steps:.3f} ms/step, "
                f"step {c3[prec]['step_frac'] * 100:.1f}% of the 12 s B/pt-step roofline, dominant "
                f"{roof['kernel']} {roof['frac'] * 100:.1f}%")
            s.close()
            del t
            torch.cuda.empty_cache()
        del psi3

    c4 = batch_c4(torch, binding, inputs, args.batch_steps) if args.batch_steps > 0 else None
    c5 = serving_c5(torch, binding, inputs, args.serve_requests, args.serve_rate) if args.serve_requests > 0 else None

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(p, psi0, args.cpu_seconds)
        log(f"[bench] CPU oracle baseline: {cpu['value']:.3e} pt-steps/s on {cpu['cores']} threads, "
            f"{cpu['value_1_core']:.3e} on one")

    r = results["fp64"]
    line = {
        "metric": METRIC, "value": r["value"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "512x512 real-time SSCN step, Dresselhaus gamma=1, Rabi=0.2, Omega=0.9, c0=200, "
                               "c2=+5, dx=0.05, dt=1e-4, from the imaginary-time state + 1e-3 noise",
                   "nx": 512, "ny": 512, "mode": "real", "precision": "fp64"},
        "roofline": r["roofline"],
        "step_roofline_frac": round(r["step_frac"], 4),
        "cpu_baseline": cpu,
        "fp32": {"value": results["fp32"]["value"], "ms_per_step": results["fp32"]["ms_per_step"],
                 "dtype": "f32 bulk, f64 reductions", "roofline": results["fp32"]["roofline"],
                 "step_roofline_frac": round(results["fp32"]["step_frac"], 4),
                 "norm_drift": results["fp32"]["norm_drift"]},
        "norm_drift_fp64": r["norm_drift"],
        "c3_4096": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"], "roofline": v["roofline"],
                        "step_roofline_frac": round(v["step_frac"], 4)} for k, v in c3.items()},
        "plan": {"x_points_per_thread": r["plan"]["x_points_per_thread"], "y_solver": r["plan"]["y_solver"],
                 "y_halo": r["plan"]["y_halo"]},
        "batch_c4": c4,
        "serving_c5": c5,
    }
    if c5 is not None:
        line["p50_latency_s"] = c5["p50_latency_s"]
        line["p99_latency_s"] = c5["p99_latency_s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
