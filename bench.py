#!/usr/bin/env python
"""Throughput of the split-step Crank-Nicolson spin-1 step on one MI355X.

Headline workload (``value``): the 4096 x 4096 imaginary-time run (Rashba
gamma = 0.75, Omega = 0.95, c0 = 1000, c2 = -20, Rabi 0, dx = 0.02,
dt = 0.1 dx^2) from a seeded random-phase Gaussian, in FP64; a step is one
whole SSCN step (local substep, x sweep, y sweep, renormalisation).  Its
state (805 MB in FP64) does not fit in the caches, so the roofline fraction
is an HBM figure.  Beside it: the same grid in FP32 bulk (FP64 reductions),
with its error against the FP64 oracle; the same parameters on 2048^2; the
128^2 ground-state run (200
imaginary-time steps, timed in full); the 512^2 real-time run from the
imaginary-time state of its parameters plus 1e-3 noise; the 256-condensate
parameter scan (batched FP32 against one-at-a-time FP32 and FP64); and the
serving trace (Poisson arrivals, 200 per second, 2000 requests).  All inputs
are seeded and synthetic, resident in device memory before any timed region.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
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
    (read + write of the 3 components, 6 s bytes per point) / mean launch
    duration, from event pairs that the kernel dispatches themselves stamp on
    the solver's stream."""
    per_launch = 6 * bytes_per_complex(prec) * npts
    rows = {}
    for kind in ("x_sweep", "y_sweep"):
        t = timing[kind]
        if t["launches"]:
            avg_s = t["ms"] / t["launches"] / 1e3
            rows[kind] = {"avg_us": avg_s * 1e6, "achieved_GBps": per_launch / avg_s / 1e9,
                          "frac": per_launch / avg_s / HBM_PEAK_BPS, "total_ms": t["ms"]}
    other = {k: round(v["ms"] / v["launches"] * 1e3, 2) for k, v in timing.items()
             if k not in rows and v["launches"]}
    dom = max(rows, key=lambda k: rows[k]["total_ms"])
    d = rows[dom]
    return {"bound": "hbm", "kernel": dom, "achieved": round(d["achieved_GBps"], 1), "peak": HBM_PEAK_BPS / 1e9,
            "unit": "GB/s", "frac": round(d["frac"], 4), "traffic": None,
            "bytes_per_launch": per_launch,
            "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in rows.items()},
            "other_kernels_avg_us": other}


XTILES = {"fp64": [(4, 4), (8, 2), (2, 4), (4, 2)], "fp32": [(4, 4), (8, 4), (8, 2), (16, 2)]}
YCTILES = {"fp64": [(8, 2), (8, 4), (4, 4), (7, 4)], "fp32": [(8, 4), (8, 8), (4, 4), (16, 2)]}
# stacked y windows: (rows per lane, segments, one line at a time) of tiles 1..6
STACK = {"fp64": [(8, 16, False), (6, 16, False), (8, 16, True), (6, 16, True), (8, 32, True), (6, 32, True)],
         "fp32": [(8, 16, False), (16, 16, False), (8, 16, True), (16, 16, True), (8, 32, True), (16, 32, True)]}
WTILES = {"fp64": [(8, 2), (8, 4), (4, 4), (4, 8)], "fp32": [(8, 4), (4, 8), (4, 4), (8, 8)]}


def tile_args(table, prec, tile):
    """Template arguments (points per lane, waves, lines one at a time) of tile 1..8."""
    kk, nw = table[prec][(tile - 1) & 3]
    return f"{kk}, {nw}, {'true' if (tile - 1) & 4 else 'false'}, "


def kernel_prefix(kind, prec, imag, plan):
    """Name prefix of the kernel a plan launches for one sweep."""
    T = "double" if prec == "fp64" else "float"
    im = "true" if imag else "false"
    if kind == "x_sweep":
        if plan["x_solver"] == 3:
            return f"gp::k_x_chain<{T}, {im}, " + tile_args(XTILES, prec, plan["x_tile"])
        if plan["x_solver"] == 2:
            return f"gp::k_x_window<{T}, {im}, " + tile_args(WTILES, prec, plan["x_tile"])
        return f"gp::k_x_scan<{T}, {im}, {plan['x_points_per_thread']}, "
    if plan["y_solver"] == 4:
        kk, ns, seq = STACK[prec][plan["y_tile"] - 1]
        return f"gp::k_y_stack<{T}, {im}, {kk}, {ns}, {'true' if seq else 'false'}, "
    if plan["y_solver"] == 3:
        return f"gp::k_y_chain<{T}, {im}, " + tile_args(YCTILES, prec, plan["y_tile"])
    if plan["y_solver"] == 2:
        return f"gp::k_y_thomas<{T}, {im}, "
    return f"gp::k_y_window<{T}, {im}, " + tile_args(WTILES, prec, plan["y_tile"])


def traffic_for(roof, prec, imag, plan, workload):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when there is none for these kernel sources."""
    from paper_2105_10517_amd import profile_summary
    t = profile_summary.read_traffic(os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.md"))
    prefix = kernel_prefix(roof["kernel"], prec, imag, plan)
    for k, v in t.items():
        if k.startswith(prefix):
            return v
    return None


def time_steps(solver, t, nsteps, imag, torch):
    """Wall time in ms of nsteps on the solver's stream (events on that stream)."""
    st = solver.stream
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


def errors_vs_oracle(np, got, obs, want, o, prec):
    """FP64: relative L2 on psi; FP32 (and FP64): density error relative to
    the peak density, relative errors of mu_total and of each mu_m."""
    rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
    out = {"psi_rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
           "density_err": float(np.abs(rho_g - rho_w).max() / rho_w.max()),
           "mu_err": abs(obs["mu_total"] - o["mu_total"]) / abs(o["mu_total"]),
           "mu_m_err": max(abs(obs["mu"][m] - o["mu"][m]) / abs(o["mu"][m]) for m in range(3) if o["mu"][m] != 0)}
    return {k: float(f"{v:.3e}") for k, v in out.items()}


def gpu_state(torch, np, binding, p, psi0, prec, nsteps, imag, **kw):
    """psi after nsteps on a fresh solver (with the given launch options), and its observables."""
    s = binding.Solver(p, prec, **kw)
    t = torch.from_numpy(psi0).to("cuda").to(s.dtype)
    (s.step_imag if imag else s.step_real)(t, nsteps)
    s.sync()
    obs = s.observables(t)
    out = t.cpu().numpy().astype(np.complex128)
    s.close()
    del t
    return out, obs


def single_solve(torch, binding, p, psi0, prec, imag, steps, warmup, timing_steps, autotune=True):
    """Steps/s of one condensate: autotuned launch shapes, warm-up, timed steps,
    then a separate pass with per-kernel timing."""
    s = binding.Solver(p, prec, autotune=autotune)
    t = torch.from_numpy(psi0).to("cuda").to(s.dtype)
    if warmup:
        (s.step_imag if imag else s.step_real)(t, warmup)
    ms = time_steps(s, t, steps, imag, torch)
    tim = kernel_timing(s, t, timing_steps, imag)
    plan = s.plan(imag)
    norm = s.observables(t)["norm_total"]
    s.close()
    del t
    torch.cuda.empty_cache()
    return ms, tim, plan, norm


def c2_initial_state(torch, binding, inputs):
    """Imaginary-time state of the 512^2 real-time parameters (dt = 0.1 dx^2,
    stop at |dE|/E < 1e-10 over 100 steps or 20000 steps), plus 1e-3 noise (seed 3)."""
    p = inputs.config_c2()
    q = dict(p, dt=0.1 * p["dx"] * p["dx"])
    psi = inputs.gaussian(p["nx"], p["ny"], p["dx"], p["dy"], seed=2, phase_noise=0.1)
    s = binding.Solver(q, "fp64")
    t = torch.from_numpy(psi).to("cuda")
    e_prev, steps, e = None, 0, 0.0
    while steps < 20000:
        s.step_imag(t, 100)
        steps += 100
        e = s.observables(t)["energy"]
        if e_prev is not None and abs(e - e_prev) < 1e-10 * abs(e):
            break
        e_prev = e
    log(f"[bench] 512^2 initial state: {steps} imaginary-time steps, E = {e:.10f}")
    out = inputs.add_noise(t.cpu().numpy(), p["dx"], p["dy"], 1e-3, seed=3)
    s.close()
    return p, out


def oracle_run(p, psi0, nsteps, imag, seconds=None):
    """The oracle (all host threads): nsteps, or as many as fit `seconds`
    after a one-step probe.  Returns (state, steps, wall seconds)."""
    import oracle
    if seconds is not None:
        t0 = time.perf_counter()
        oracle.step(p, psi0, 1, imag)
        t1 = time.perf_counter() - t0
        nsteps = max(2, int(round(seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    out = oracle.step(p, psi0, nsteps, imag)
    return out, nsteps, time.perf_counter() - t0


def batch_c4(torch, binding, inputs, nsteps):
    """256 condensates of the parameter scan (imaginary time) in batched FP32
    launches, against the same solves one at a time in FP32 and in FP64."""
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
    e0.record(b.stream)
    b.step(ts, [nsteps] * len(ps), ["imag"] * len(ps))
    e1.record(b.stream)
    b.sync()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    info = b.info()
    b.close()
    del ts

    def one_at_a_time(prec):
        dt = torch.complex128 if prec == "fp64" else torch.complex64
        tt = [torch.from_numpy(a).to(dt).to("cuda") for a in psi0]
        solvers = [binding.Solver(p, prec) for p in ps]
        for s_, t in zip(solvers, tt):
            s_.step_imag(t, 5)
        st = solvers[0].stream
        torch.cuda.synchronize()
        e0.record(st)
        for s_, t in zip(solvers, tt):
            s_.step_imag(t, nsteps)
        e1.record(st)
        torch.cuda.synchronize()
        for s_ in solvers:
            s_.close()
        del tt
        torch.cuda.empty_cache()
        return e0.elapsed_time(e1)

    ms_32 = one_at_a_time("fp32")
    ms_64 = one_at_a_time("fp64")
    bps = 96 * pts / (ms_b / 1e3)  # 12 s bytes per point-step, s = 8
    out = {"workload": f"256 condensates, N = 32 k (k ~ U{{4..16}}), {nsteps} imaginary-time steps each",
           "value_fp32_batched": pts / (ms_b / 1e3), "value_fp32_one_at_a_time": pts / (ms_32 / 1e3),
           "value_fp64_one_at_a_time": pts / (ms_64 / 1e3),
           "ms_batched": ms_b, "ms_fp32_one_at_a_time": ms_32, "ms_fp64_one_at_a_time": ms_64, "unit": UNIT,
           "roofline_batched": {"bound": "hbm", "achieved": round(bps / 1e9, 1), "peak": HBM_PEAK_BPS / 1e9,
                                "unit": "GB/s", "frac": round(bps / HBM_PEAK_BPS, 4),
                                "basis": "12 s = 96 B per 3-comp point-step over the whole batched step"},
           "grouped": info["grouped"], "individual": info["individual"], "x_points": info["x_points"][0],
           "y_tile": info["y_tile"][0],
           "shape": {"x": {1: "whole-row scans", 3: "chain windows"}.get(info["x_solver"][0], info["x_solver"][0]),
                     "x_tile": info["x_tile"][0],
                     "y": {1: "scanned windows", 4: "stacked chain windows"}.get(info["y_solver"][0],
                                                                                 info["y_solver"][0])}}
    log(f"[bench] C4 batch: FP32 batched {out['value_fp32_batched']:.3e} pt-steps/s ({bps / 1e12:.2f} TB/s), "
        f"FP32 one at a time {out['value_fp32_one_at_a_time']:.3e}, FP64 one at a time "
        f"{out['value_fp64_one_at_a_time']:.3e} ({ms_b:.1f} / {ms_32:.1f} / {ms_64:.1f} ms)")
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
    for k in ("gpu_busy", "admit_ms"):
        if k in st:
            out[k] = st[k]
    log(f"[bench] C5 serving {rate:g}/s x {n}: p50 {st['p50_latency']:.3f} s, p99 {st['p99_latency']:.3f} s, served "
        f"{st['served_rate']:.3e} vs offered {st['offered_rate']:.3e} pt-steps/s, {st['mean_active']:.1f} in flight, "
        f"GPU busy {st.get('gpu_busy', 0.0):.3f}, admission {st.get('admit_ms', 0.0):.0f} ms")
    del reqs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed SSCN steps of the 4096^2 headline workload")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--timing-steps", type=int, default=40, help="steps of each per-kernel timing pass")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle sample on the 4096^2 grid (also the FP32/FP64 error check; 0 = skip)")
    ap.add_argument("--c1", type=int, default=1, help="time the 128^2 200-step ground-state run (0 = skip)")
    ap.add_argument("--c2-steps", type=int, default=2000, help="timed steps of the 512^2 real-time run (0 = skip)")
    ap.add_argument("--c2-check-steps", type=int, default=300, help="steps of the 512^2 error check against the oracle")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="imaginary-time steps of the 256-condensate batch (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests of the serving trace (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="arrival rate of the serving trace (1/s)")
    ap.add_argument("--serve-sweep", default="", help="extra arrival rates to replay (comma list), 10 s of trace each")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (each condensate runs on "
              f"one device and the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2105_10517_amd import binding, inputs
    binding.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    # ---- headline: 4096^2 imaginary time, FP64 and FP32 ----
    q = inputs.config_c3(4096)
    psi3 = inputs.gaussian(4096, 4096, q["dx"], q["dy"], seed=4, full_phase=True)
    n3 = 4096 * 4096
    c3 = {}
    for prec in ("fp64", "fp32"):
        ms, tim, plan, norm = single_solve(torch, binding, q, psi3, prec, True, args.steps, args.warmup,
                                           args.timing_steps)
        roof = kernel_roofline(tim, n3, prec)
        roof["traffic"] = traffic_for(roof, prec, True, plan, "c3_4096")
        cp = copy_rate(torch, 3 * n3 * bytes_per_complex(prec), reps=10)
        roof["copy_GBps"] = round(cp / 1e9, 1)
        roof["frac_of_copy"] = round(roof["achieved"] * 1e9 / cp, 4)
        val = n3 * args.steps / (ms / 1e3)
        step_bytes = 12 * bytes_per_complex(prec) * n3
        c3[prec] = {"value": val, "ms_per_step": ms / args.steps, "roofline": roof,
                    "step_frac": step_bytes / (ms / args.steps / 1e3) / HBM_PEAK_BPS, "plan": plan,
                    "norm_after": norm}
        log(f"[bench] 4096^2 imag {prec}: {val:.3e} pt-steps/s, {ms / args.steps:.3f} ms/step, step "
            f"{c3[prec]['step_frac'] * 100:.1f}% of the 12 s B/pt-step roofline; x {roof['kernels']['x_sweep']['avg_us']:.1f} us, "
            f"y {roof['kernels']['y_sweep']['avg_us']:.1f} us; dominant {roof['kernel']} {roof['frac'] * 100:.1f}%")

    # the oracle on the same grid: CPU baseline sample, and the reference for the error of both precisions
    cpu = None
    if args.cpu_seconds > 0:
        want, n_or, sec = oracle_run(q, psi3, None, True, seconds=args.cpu_seconds)
        import oracle
        o = oracle.observables(q, want)
        cpu = {"value": n3 * n_or / sec, "unit": UNIT, "cores": oracle.get_threads(), "kind": "oracle",
               "sample": f"{n_or} imaginary-time FP64 steps of the 4096x4096 workload from its initial state "
                         f"(block-Thomas oracle, {sec:.1f} s)"}
        for prec in ("fp64", "fp32"):
            got, obs = gpu_state(torch, np, binding, q, psi3, prec, n_or, True, autotune=True)
            c3[prec]["err_vs_oracle"] = dict(errors_vs_oracle(np, got, obs, want, o, prec), steps=n_or)
            log(f"[bench] 4096^2 {prec} after {n_or} steps vs oracle: {c3[prec]['err_vs_oracle']}")
        del want, got
        log(f"[bench] CPU oracle 4096^2: {cpu['value']:.3e} pt-steps/s on {cpu['cores']} threads")
    del psi3

    # ---- 2048^2, the large-grid run's other size (same parameters), timed like the headline ----
    c3b = {"workload": "2048x2048 imaginary-time steps, the 4096^2 parameters (dx=0.02)"}
    q2 = inputs.config_c3(2048)
    psi2 = inputs.gaussian(2048, 2048, q2["dx"], q2["dy"], seed=4, full_phase=True)
    for prec in ("fp64", "fp32"):
        ms, tim, plan, norm = single_solve(torch, binding, q2, psi2, prec, True, args.steps, args.warmup,
                                           args.timing_steps)
        n2 = 2048 * 2048
        c3b[prec] = {"value": n2 * args.steps / (ms / 1e3), "ms_per_step": ms / args.steps,
                     "step_frac": 12 * bytes_per_complex(prec) * n2 / (ms / args.steps / 1e3) / HBM_PEAK_BPS,
                     "kernels_us": {k: round(v["ms"] / v["launches"] * 1e3, 2) for k, v in tim.items() if v["launches"]},
                     "plan": {k: plan[k] for k in ("x_solver", "x_tile", "y_solver", "y_tile")}}
        log(f"[bench] 2048^2 imag {prec}: {c3b[prec]['value']:.3e} pt-steps/s, {ms / args.steps:.3f} ms/step, "
            f"step {100 * c3b[prec]['step_frac']:.1f}% of the 12 s B/pt-step roofline")
    del psi2
    torch.cuda.empty_cache()

    # ---- 128^2 ground state, 200 imaginary-time steps, timed in full ----
    c1 = None
    if args.c1:
        import oracle
        p1 = inputs.config_c1()
        psi1 = inputs.gaussian(128, 128, 0.1, 0.1, seed=1, phase_noise=0.1)
        c1 = {"workload": "128x128, dx=0.1, dt=5e-4, 200 imaginary-time steps, c0=50, c2=-1, Rashba gamma=0.5, "
                          "Omega=0.5; Gaussian with +-0.1 rad phase noise (seed 1)"}
        want1, _, sec1 = oracle_run(p1, psi1, 200, True)
        o1 = oracle.observables(p1, want1)
        threads = oracle.get_threads()
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.step(p1, psi1, 40, True)
        sec_one = time.perf_counter() - t0
        oracle.set_threads(threads)
        c1["cpu_baseline"] = {"value": 128 * 128 * 200 / sec1, "unit": UNIT, "cores": threads, "kind": "oracle",
                              "sample": f"the whole 200-step run ({sec1:.2f} s)",
                              "value_1_core": 128 * 128 * 40 / sec_one, "sample_1_core": f"40 steps ({sec_one:.2f} s)"}
        for prec in ("fp64", "fp32"):
            s = binding.Solver(p1, prec, autotune=True)
            t = torch.from_numpy(psi1).to("cuda").to(s.dtype)
            s.step_imag(t, 200)  # warm-up run (then a fresh state)
            t.copy_(torch.from_numpy(psi1).to(s.dtype))
            ms = time_steps(s, t, 200, True, torch)
            obs = s.observables(t)
            got = t.cpu().numpy().astype(np.complex128)
            t.copy_(torch.from_numpy(psi1).to(s.dtype))
            tim = kernel_timing(s, t, 200, True)
            ktot = sum(v["ms"] for v in tim.values())
            # the same 200 steps replayed from a captured HIP graph (captured by the first call)
            t.copy_(torch.from_numpy(psi1).to(s.dtype))
            s.step_graph(t, 200, True)
            s.sync()
            t.copy_(torch.from_numpy(psi1).to(s.dtype))
            torch.cuda.synchronize()
            g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            g0.record(s.stream)
            s.step_graph(t, 200, True)
            g1.record(s.stream)
            torch.cuda.synchronize()
            s.sync()
            ms_graph = g0.elapsed_time(g1)
            same = bool(np.array_equal(t.cpu().numpy().astype(np.complex128), got))
            c1[prec] = {"value": 128 * 128 * 200 / (ms / 1e3), "ms_run": ms, "us_per_step": ms / 200 * 1e3,
                        "kernel_us_per_step": ktot / 200 * 1e3, "plan": s.plan(True),
                        "graph": {"value": 128 * 128 * 200 / (ms_graph / 1e3), "ms_run": ms_graph,
                                  "us_per_step": ms_graph / 200 * 1e3, "equals_eager": same},
                        "err_vs_oracle": dict(errors_vs_oracle(np, got, obs, want1, o1, prec), steps=200)}
            log(f"[bench] 128^2 imag {prec}: 200 steps in {ms:.2f} ms ({c1[prec]['value']:.3e} pt-steps/s, "
                f"{c1[prec]['us_per_step']:.2f} us/step, kernels {c1[prec]['kernel_us_per_step']:.2f} us/step; "
                f"HIP graph {ms_graph:.2f} ms, {c1[prec]['graph']['us_per_step']:.2f} us/step, equal {same}); "
                f"vs oracle {c1[prec]['err_vs_oracle']}")
            s.close()

    # ---- 512^2 real time from the imaginary-time state ----
    c2 = None
    if args.c2_steps > 0:
        import oracle
        p, psi0 = c2_initial_state(torch, binding, inputs)
        npts = p["nx"] * p["ny"]
        want2, n2, sec2 = oracle_run(p, psi0, args.c2_check_steps, False)
        o2 = oracle.observables(p, want2)
        c2 = {"workload": "512x512 real-time SSCN step, Dresselhaus gamma=1, Rabi=0.2, Omega=0.9, c0=200, c2=+5, "
                          "dx=0.05, dt=1e-4, from the imaginary-time state + 1e-3 noise; 12.6 MB of FP64 state, "
                          "resident in the caches (no HBM roofline)",
              "cpu_baseline": {"value": npts * n2 / sec2, "unit": UNIT, "cores": oracle.get_threads(),
                               "kind": "oracle", "sample": f"{n2} real-time steps ({sec2:.1f} s)"}}
        for prec in ("fp64", "fp32"):
            ms, tim, plan, norm = single_solve(torch, binding, p, psi0, prec, False, args.c2_steps, 200,
                                               min(500, args.c2_steps))
            roof = kernel_roofline(tim, npts, prec)
            got, obs = gpu_state(torch, np, binding, p, psi0, prec, n2, False, autotune=True)
            c2[prec] = {"value": npts * args.c2_steps / (ms / 1e3), "ms_per_step": ms / args.c2_steps,
                        "roofline": roof, "norm_drift": norm - 1.0, "plan": plan,
                        "err_vs_oracle": dict(errors_vs_oracle(np, got, obs, want2, o2, prec), steps=n2)}
            log(f"[bench] 512^2 real {prec}: {c2[prec]['value']:.3e} pt-steps/s, {ms / args.c2_steps * 1e3:.2f} "
                f"us/step, norm drift {norm - 1:.2e}, vs oracle after {n2} steps {c2[prec]['err_vs_oracle']}")

    c4 = batch_c4(torch, binding, inputs, args.batch_steps) if args.batch_steps > 0 else None
    c5 = serving_c5(torch, binding, inputs, args.serve_requests, args.serve_rate) if args.serve_requests > 0 else None
    sweep = []
    for r in [float(x) for x in args.serve_sweep.split(",") if x.strip()]:
        sweep.append(serving_c5(torch, binding, inputs, max(1, int(round(10 * r))), r))

    r = c3["fp64"]
    line = {
        "metric": METRIC, "value": r["value"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "4096x4096 imaginary-time SSCN step (local substep, x and y Crank-Nicolson sweeps, "
                               "renormalisation): Rashba gamma=0.75, Omega=0.95, c0=1000, c2=-20, Rabi=0, dx=0.02, "
                               "dt=4e-5, from a seeded random-phase Gaussian",
                   "nx": 4096, "ny": 4096, "mode": "imag", "precision": "fp64"},
        "roofline": r["roofline"],
        "step_roofline_frac": round(r["step_frac"], 4),
        "cpu_baseline": cpu,
        "err_vs_oracle_fp64": r.get("err_vs_oracle"),
        "plan_fp64": r["plan"],
        "fp32": {"value": c3["fp32"]["value"], "ms_per_step": c3["fp32"]["ms_per_step"],
                 "dtype": "f32 bulk, f64 reductions", "roofline": c3["fp32"]["roofline"],
                 "step_roofline_frac": round(c3["fp32"]["step_frac"], 4),
                 "err_vs_oracle": c3["fp32"].get("err_vs_oracle"), "plan": c3["fp32"]["plan"]},
        "c3_2048": c3b,
        "c1_128": c1,
        "c2_512": c2,
        "batch_c4": c4,
        "serving_c5": c5,
    }
    if sweep:
        line["serving_c5_sweep"] = sweep
    if c5 is not None:
        line["p50_latency_s"] = c5["p50_latency_s"]
        line["p99_latency_s"] = c5["p99_latency_s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
