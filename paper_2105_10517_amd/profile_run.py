"""Short, profiler-friendly runs of the SSCN step (for rocprofv3 counters).

    python3 paper_2105_10517_amd/profile_run.py --workload c2 --precision fp64 --steps 50
    python3 paper_2105_10517_amd/profile_run.py --copy-mib 512

The first form builds one solver for a named workload and advances a seeded
state by ``--steps`` steps (launch shapes from the autotuner, from the
``--x-*`` / ``--y-tile`` / ``--block-order`` options, or the defaults): ``c2`` is the 512 x 512 real-time workload
(Dresselhaus, Rabi 0.2, Omega 0.9), ``c3_<n>`` the n x n imaginary-time
workload (Rashba, Omega 0.95).  The second form times nothing: it launches a
plain device-to-device copy of a known size, whose FETCH_SIZE / WRITE_SIZE
readings calibrate the counters against known traffic.
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="c2", help="c2 or c3_<n>")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--copy-mib", type=int, default=0, help="run a plain copy of this many MiB instead")
    ap.add_argument("--autotune", action="store_true", help="tune the launch shapes first (as bench.py does)")
    ap.add_argument("--x-solver", default="auto", choices=("auto", "scan", "window", "chain"))
    ap.add_argument("--y-solver", default="auto", choices=("auto", "window", "thomas", "chain", "stack"))
    ap.add_argument("--x-tile", type=int, default=0, help="x window tile (1..8, with --x-solver window)")
    ap.add_argument("--x-points", type=int, default=0, help="points per thread of the whole-row x sweep")
    ap.add_argument("--y-tile", type=int, default=0, help="y window tile (1..8)")
    ap.add_argument("--block-order", default="auto", choices=("auto", "hardware", "xcd", "bands", "rows"))
    args = ap.parse_args()

    import torch
    from paper_2105_10517_amd import binding, inputs
    assert torch.cuda.is_available(), "profile_run needs a GPU"
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 16
        a = torch.ones(n, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy: 5 x {args.copy_mib} MiB read + {args.copy_mib} MiB written", flush=True)
        return
    if args.workload == "c2":
        p, imag = inputs.config_c2(), False
    elif args.workload.startswith("c3_"):
        p, imag = inputs.config_c3(int(args.workload.split("_")[1])), True
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    s = binding.Solver(p, args.precision, args.y_solver, autotune=args.autotune, x_solver=args.x_solver, x_tile=args.x_tile,
                       x_points=args.x_points, y_tile=args.y_tile, block_order=args.block_order)
    psi = inputs.gaussian(p["nx"], p["ny"], p["dx"], p["dy"], seed=4, full_phase=imag)
    t = torch.from_numpy(psi).to("cuda").to(s.dtype)
    (s.step_imag if imag else s.step_real)(t, args.steps)
    s.sync()
    pl = s.plan(imag)
    print(f"{args.workload} {args.precision}: {args.steps} steps, plan {pl}", flush=True)
    s.close()


if __name__ == "__main__":
    main()
