"""Benchmark of the relativistic lattice Boltzmann step on one MI355X.

Workload (default): the large Sod tube -- N_x = 2^20 cells, Q = 64 x 4
quadrature points, tau = 1e-2, synthetic Sod initial states -- advanced by
full SSP-RK3 steps.  The headline is the FP32 form (FP32 stencil and
relaxation, Kahan-compensated FP32 moment sums, FP64 Landau matching); the
FP64 form is timed beside it.

Prints ONE JSON line: metric, value (cell x quadrature-point updates per
second), the roofline of the stage kernel (algorithmic bytes per launch over
its average duration, timed with HIP events on the launch stream), the CPU
oracle timed on a bounded sample of the same workload, and the FP64 figures.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def stage_bytes_per_step(nx, Q, rsize):
    """Algorithmic HBM bytes of one SSP-RK3 step (three stage launches).

    Stage 1 reads f^n and writes f1; stages 2 and 3 read their input and f^n
    and write their output: 8 accesses per point.  Each stage also reads and
    writes the five FP64 moments of every cell (80 bytes per cell).
    """
    return 8 * nx * Q * rsize + 3 * 80 * nx


def time_path(precision, params, steps, warmup, schedule=None):
    import torch
    from paper_1608_03004_amd import Lattice, Tube
    lat = Lattice([Tube(**params)], precision=precision)
    if schedule:
        lat.set_schedule(**schedule)
    lat.set_initial_state((1.0, 1.0, 0.0), (0.1, 0.125, 0.0))
    lat.step(warmup)
    lat.check()
    stream = lat.stream
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    lat.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(stop)
    lat.check()
    fields = lat.moments(0)
    Q = params["q_xi"] * params["q_p"]
    nx = params["nx"]
    rsize = 4 if precision == "fp32" else 8
    launch_ms = ev_ms / (3 * steps)
    bytes_launch = stage_bytes_per_step(nx, Q, rsize) / 3
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    out = dict(
        value=nx * Q * steps / wall,
        ms_per_step=1e3 * wall / steps,
        event_ms_per_step=ev_ms / steps,
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                      bytes_per_launch=int(bytes_launch), launch_us=round(launch_ms * 1e3, 2)),
        e_min=float(fields[5].min()),
    )
    del lat
    torch.cuda.empty_cache()
    return out


def cpu_baseline(params, target_s=10.0):
    """The CPU FP64 oracle on a bounded sample: the same Q and tau on a
    2^16-cell sub-tube, timed over whole steps (about 10 s of CPU work)."""
    from oracle import oracle as O
    nx = 1 << 16
    t = O.Tube(nx=nx, q_xi=params["q_xi"], q_p=params["q_p"], tau=params["tau"])
    F = O.init(t, (1.0, 1.0, 0.0), (0.1, 0.125, 0.0))
    t0 = time.perf_counter()
    F = O.step(t, F, 1)
    one = time.perf_counter() - t0
    extra = max(0, min(4, int(target_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    if extra:
        F = O.step(t, F, extra)
    el = time.perf_counter() - t0
    steps, secs = (extra, el) if extra else (1, one)
    pts = nx * t.Q * steps
    return dict(value=pts / secs, unit="cell*quad-point updates/s", cores=O.num_threads(), kind="oracle",
                sample=f"FP64 oracle, {nx} cells x Q={t.Q} ({params['q_xi']}x{params['q_p']}), "
                       f"tau={params['tau']}, {steps} step(s), {secs:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--fp64", type=int, default=1, help="also time the FP64 path")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    params = dict(nx=args.nx, q_xi=64, q_p=4, tau=1e-2)
    r32 = time_path("fp32", params, args.steps, args.warmup)
    r64 = time_path("fp64", params, args.steps, args.warmup) if args.fp64 else None
    line = {
        "metric": "cell*quad-point updates/s (FP32 vs FP64) + % HBM roofline; adjoint steps/s",
        "value": r32["value"],
        "unit": "cell*quad-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "sod_large: Sod tube, N_x=2^20, Q=64x4 (Gauss-Legendre x Gauss-Laguerre), "
                               "tau=1e-2, FP32 with Kahan moments and FP64 Landau",
                   "nx": params["nx"], "q_xi": 64, "q_p": 4, "tau": 1e-2},
        "roofline": r32["roofline"],
    }
    if r64:
        line["fp64"] = dict(value=r64["value"], ms_per_step=r64["ms_per_step"], roofline=r64["roofline"],
                            speedup_fp32_over_fp64=r32["value"] / r64["value"])
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(params)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
