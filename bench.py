"""Benchmark of the relativistic lattice Boltzmann step on one MI355X.

Headline workload: the large Sod tube -- N_x = 2^20 cells, Q = 64 x 4
quadrature points, tau = 1e-2, synthetic Sod initial states (the paper's
left/right states) -- advanced by full SSP-RK3 steps in the FP32 form (FP32
stencil and relaxation, Kahan-compensated FP32 moment sums, FP64 Landau
matching).  A "step" is one full time step (three stage launches) of the
whole tube.  Beside it, on the same line:
  fp64        the FP64 form on the same tube, and the FP32-vs-FP64 error table
              (max and L2 relative errors of e, v, T^{mu nu}) after the run;
  batched     4096 seeded tubes of uneven size, order and tau in one launch
              per stage, schedule chosen by the autotuner, replayed from a
              hipGraph;
  adjoint     gradient of the profile loss of the 4096-cell, Q = 32 x 3 tube
              over 2000 steps (forward + sqrt(N)-checkpointed backward);
  ballistic   the 2^22-cell, Q = 256 x 4 tube at tau = 1e3 (FP32);
  high        the headline tube with the high-order equilibrium (N_v = 63),
              FP32 and FP64, with the matrix-core roofline of its pre-pass;
  plane       the multi-dimensional model on a 1024 x 1024 plane (Q = 120),
              FP32 and FP64;
  roofline    of the stage kernel: algorithmic bytes per launch over its mean
              duration, timed with HIP events on the launch stream;
  cpu_baseline the CPU FP64 oracle on a bounded sample of the headline tube.

Prints ONE JSON line.  Inputs are resident in HBM before every timed region.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
SOD_L, SOD_R = (1.0, 1.0, 0.0), (0.1, 0.125, 0.0)


def step_bytes(tubes, rsize):
    """Algorithmic HBM bytes of one SSP-RK3 step (three stage launches).

    Per point: stage 1 reads f^n and writes f1; stages 2 and 3 read their input
    and f^n and write their output: 8 accesses.  Per cell and stage the five
    FP64 moments are read and written (80 bytes).
    """
    return sum(8 * t.nx * t.Q * rsize + 3 * 80 * t.nx for t in tubes)


def timed_steps(lat, steps):
    import torch
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(lat.stream)
    lat.step(steps)
    stop.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, start.elapsed_time(stop) * 1e-3


KERNEL_SOURCES = {"stage_kernel": "rlb_kernels.hip", "feq_kernel": "rlb_feq.hip", "plane_stage_kernel": "rlb_plane.hip"}
TRAFFIC_FILES = {"stage_kernel": "stage_kernel_traffic.json", "feq_kernel": "feq_kernel_traffic.json",
                 "plane_stage_kernel": "plane_stage_kernel_traffic.json"}


def kernel_source_sha1(kernel="stage_kernel"):
    """SHA-1 of the sources a kernel is built from (its own file and the two
    shared headers)."""
    import hashlib
    h = hashlib.sha1()
    for f in (KERNEL_SOURCES[kernel], "rlb_device.h", "rlb_internal.h"):
        with open(os.path.join(ROOT, "paper_1608_03004_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision, kernel="stage_kernel"):
    """HBM bytes per launch of a kernel on its benchmark workload from the
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs (calibrated on the copy
    kernel), or None when the kernel's sources changed since those counters
    were taken."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[kernel])
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha1") != kernel_source_sha1(kernel) or precision not in t:
        return None
    return int(t[precision]["traffic_bytes_per_launch"])


def roofline(tubes, rsize, steps, event_s, traffic=None):
    launch_s = event_s / (3 * steps)
    bytes_launch = step_bytes(tubes, rsize) / 3
    achieved = bytes_launch / launch_s / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                bytes_per_launch=int(bytes_launch), launch_us=round(launch_s * 1e6, 2))


def leg_single(precision, params, steps, warmup, schedule=None):
    from paper_1608_03004_amd import Lattice, Tube
    tube = Tube(**params)
    lat = Lattice([tube], precision=precision)
    if schedule:
        lat.set_schedule(**schedule)
    lat.set_initial_state(SOD_L, SOD_R)
    lat.step(warmup)
    lat.check()
    wall, ev = timed_steps(lat, steps)
    fields = lat.moments(0)
    rsize = 4 if precision == "fp32" else 8
    traffic = measured_traffic(precision) if (tube.nx, tube.q_xi, tube.q_p) == (1 << 20, 64, 4) else None
    out = dict(value=tube.nx * tube.Q * steps / wall, ms_per_step=1e3 * wall / steps,
               roofline=roofline([tube], rsize, steps, ev, traffic), schedule=lat.get_schedule())
    return out, fields, lat


def error_table(f32, f64):
    """Max and L2 relative errors (normwise per field) of FP32 against FP64."""
    import numpy as np
    names = dict(e=5, v=7, T00=2, T0z=3, Tzz=4, N0=0, n=6)
    out = {}
    for name, k in names.items():
        d = f32[k] - f64[k]
        s = max(np.abs(f64[k]).max(), 1e-300)
        out[name] = dict(max=float(np.abs(d).max() / s), l2=float(np.sqrt(np.mean(d * d)) / s))
    return out


def leg_batched(steps, tune=True):
    import torch
    import workloads
    from paper_1608_03004_amd import Lattice, Tube
    from paper_1608_03004_amd import autotune
    w = workloads.sod_batched()
    tubes = [Tube(**t) for t in w["tubes"]]
    lat = Lattice(tubes, precision="fp32")
    lat.set_initial_states(w["left"], w["right"])
    lat.step(1)
    sched, timings = (autotune.tune(lat, steps=3, use_cache=False) if tune else (None, {}))
    lat.set_initial_states(w["left"], w["right"])
    lat.step(2)
    lat.check()
    wall, ev = timed_steps(lat, steps)
    lat.check()
    pts = sum(t.nx * t.Q for t in tubes)
    best = sorted(timings.values())[:1]
    out = dict(value=pts * steps / wall, unit="cell*quad-point updates/s", ms_per_step=1e3 * wall / steps,
               steps=steps, tubes=len(tubes), points_per_step=pts, schedule=lat.get_schedule(),
               roofline=roofline(tubes, 4, steps, ev),
               autotune_candidates=len(timings),
               workload="sod_batched: 4096 tubes, numpy default_rng(0): N_x~U{256..8192}, "
                        "Q_xi~U{8,16,32,64,128}, Q_p=3, log tau~U[ln1e-4,ln10], "
                        "log(P_L/P_R)~U[ln2,ln100], n_L/n_R~U[1,10], FP32")
    del lat
    torch.cuda.empty_cache()
    return out


def leg_adjoint(precision, nsteps=2000):
    import torch
    import workloads
    from paper_1608_03004_amd import Lattice, Tube
    from paper_1608_03004_amd.autograd import SodProfile
    w = workloads.sod_adjoint()
    p = dict(w["tubes"][0])
    p["dt"] = 0.5 / p["nx"]
    lat = Lattice([Tube(**p)], precision=precision, adjoint=True)
    f64, dev = torch.float64, lat.device
    tg = w["target"]
    # target profile from the forward at (tau, P_L) = (0.05, 1.5)
    with torch.no_grad():
        target = SodProfile.apply(torch.tensor(tg["tau"], dtype=f64), torch.tensor(tg["P_L"], dtype=f64),
                                  torch.tensor(tg["n_L"], dtype=f64), torch.tensor(0.1, dtype=f64),
                                  torch.tensor(0.125, dtype=f64), lat, nsteps, 0).clone()
    st = w["start"]
    P_R, n_R = torch.tensor(0.1, dtype=f64, device=dev), torch.tensor(0.125, dtype=f64, device=dev)
    # two gradient evaluations, the second one timed (as in an optimisation
    # loop, the first backward pays the segment scratch allocation and the
    # autograd set-up)
    for _ in range(2):
        theta = [torch.tensor(v, dtype=f64, device=dev, requires_grad=True) for v in (st["tau"], st["P_L"], st["n_L"])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = SodProfile.apply(*theta, P_R, n_R, lat, nsteps, 0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = torch.sum((e - target) ** 2) / p["nx"]
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    grads = [float(x.grad) for x in theta]
    out = dict(adjoint_steps_per_s=nsteps / (t2 - t1), forward_steps_per_s=nsteps / (t1 - t0),
               backward_s=t2 - t1, steps=nsteps, checkpoint_every=math.ceil(math.sqrt(nsteps)),
               grad_tau=grads[0], grad_P_L=grads[1], grad_n_L=grads[2], loss=float(loss.detach()),
               workload="sod_adjoint: N_x=4096, Q=32x3, 2000 steps, dt=0.5 dz, start (tau,P_L,n_L)=(0.02,1,1), "
                        "target from (0.05,1.5,1)")
    del lat
    torch.cuda.empty_cache()
    return out


def leg_ballistic(steps, warmup=2):
    import numpy as np
    import torch
    from paper_1608_03004_amd import Lattice, Tube
    tube = Tube(nx=1 << 22, q_xi=256, q_p=4, tau=1e3)
    lat = Lattice([tube], precision="fp32")
    lat.set_initial_state(SOD_L, SOD_R)
    lat.step(warmup)
    wall, ev = timed_steps(lat, steps)
    lat.check()
    out = dict(value=tube.nx * tube.Q * steps / wall, ms_per_step=1e3 * wall / steps, steps=steps,
               roofline=roofline([tube], 4, steps, ev),
               workload="sod_ballistic: N_x=2^22, Q=256x4, tau=1e3, FP32")
    del lat
    torch.cuda.empty_cache()
    return out


MFMA_F64_PEAK_TFS = 78.6  # MI355X dense FP64 matrix


def high_order_flops(tube):
    """Algorithmic flops of one equilibrium pre-pass over a high-order tube:
    per cell and radial node the two even/odd products, ceil(q_xi/2) rows by
    B auxiliary pairs, one multiply and one add each."""
    B = 4 * ((tube.n_v + 89 + 15) // 16)
    return 4 * ((tube.q_xi + 1) // 2) * B * tube.nx * tube.q_p


def leg_high_order(precision, steps, warmup=2, reps=10):
    """The large Sod tube with the high-order equilibrium (N_v = 63 = Q_xi - 1):
    every stage runs the matrix-core pre-pass and then the stage kernel that
    streams its output."""
    import torch
    from paper_1608_03004_amd import Lattice, Tube
    tube = Tube(nx=1 << 20, q_xi=64, q_p=4, n_v=63, tau=1e-2)
    lat = Lattice([tube], precision=precision)
    lat.set_initial_state(SOD_L, SOD_R)
    lat.step(warmup)
    lat.check()
    wall, ev = timed_steps(lat, steps)
    lat.check()
    fields = lat.moments(0)
    # the pre-pass alone on the lattice's stream (same launch as inside a
    # stage), one launch per timing: inside a step each pre-pass alternates
    # with the memory-bound stage kernel, while back-to-back launches of the
    # matrix-core kernel run measurably slower (clock management); median
    out = lat.new_state()
    lat.equilibrium(out)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        start.record(lat.stream)
        lat.equilibrium(out)
        stop.record(lat.stream)
        torch.cuda.synchronize()
        times.append(start.elapsed_time(stop) * 1e-3)
    feq_s = sorted(times)[reps // 2]
    rsize = 4 if precision == "fp32" else 8
    flops = high_order_flops(tube)
    stage_s = ev / steps / 3 - feq_s
    # stage kernel bytes: the low-order stage's streams plus the equilibrium read
    stage_bytes = step_bytes([tube], rsize) / 3 + tube.nx * tube.Q * rsize
    res = dict(value=tube.nx * tube.Q * steps / wall, unit="cell*quad-point updates/s",
               ms_per_step=1e3 * wall / steps, steps=steps,
               roofline=dict(bound="mfma", achieved=round(flops / feq_s / 1e12, 2), peak=MFMA_F64_PEAK_TFS,
                             unit="TFLOP/s", frac=round(flops / feq_s / 1e12 / MFMA_F64_PEAK_TFS, 4),
                             traffic=measured_traffic(precision, "feq_kernel"),
                             kernel="feq_kernel", flops_per_launch=flops, launch_us=round(feq_s * 1e6, 2)),
               stage_roofline=dict(bound="hbm", achieved=round(stage_bytes / stage_s / 1e9, 1), peak=HBM_PEAK_GBS,
                                   unit="GB/s", frac=round(stage_bytes / stage_s / 1e9 / HBM_PEAK_GBS, 4),
                                   bytes_per_launch=int(stage_bytes), launch_us=round(stage_s * 1e6, 2)),
               workload=f"sod_large_high_order: N_x=2^20, Q=64x4, N_v=63, N_p=2, tau=1e-2, {precision.upper()}")
    del lat, out
    torch.cuda.empty_cache()
    return res, fields


def plane_quadrants(nx, nz):
    """Per-cell (P, n, u^x, u^z) of a 2D Riemann problem: four constant states
    meeting at the centre of [-0.5, 0.5]^2."""
    import numpy as np
    x = -0.5 + (np.arange(nx) + 0.5) / nx
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    X, Z = np.meshgrid(x, z)
    states = {(0, 0): (1.0, 1.0, 0.0, 0.0), (1, 0): (0.3, 0.5, 0.2, 0.0),
              (0, 1): (0.4, 0.6, 0.0, -0.3), (1, 1): (0.1, 0.125, 0.1, 0.1)}
    f = np.zeros((4, nz, nx))
    for (a, b), st in states.items():
        m = ((X >= 0) == bool(a)) & ((Z >= 0) == bool(b))
        for c in range(4):
            f[c][m] = st[c]
    return f


def plane_step_bytes(spec, rsize):
    """Algorithmic HBM bytes of one plane step: 8 accesses per point (as for a
    tube) and per cell and stage the nine FP64 records read and written."""
    return 8 * spec.nx * spec.nz * spec.Q * rsize + 3 * 144 * spec.nx * spec.nz


# Vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one lane
# operation per lane and cycle (FP32 without packed math, which the build
# disables, and FP64 alike): 39.3 T operations/s, i.e. 78.6 TFLOP/s of FMAs.
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4


def plane_point_ops(spec):
    """Algorithmic vector operations per point and stage of the plane update:
    two WENO5 faces of 37 operations each (difference form, one reciprocal),
    the equilibrium polynomial in c = v . u_hat (2 + N_v), advection and
    relaxation (8), the RK combination (3) and the six moment FMAs.  Per-cell
    work (Landau frame, projection) and the tile's extra faces are excluded."""
    return 2 * 37 + (2 + spec.n_v) + 8 + 3 + 6


def leg_plane(precision, steps, warmup=2):
    """The multi-dimensional model: a 1024 x 1024 plane, Q = 3 x 8 x 5 evolved
    points (Q_phi = 8), a 2D Riemann problem."""
    import torch
    from paper_1608_03004_amd import Plane, PlaneSpec
    spec = PlaneSpec(nx=1024, nz=1024, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gp = Plane(spec, precision=precision)
    gp.set_initial_fields(plane_quadrants(spec.nx, spec.nz))
    gp.step(warmup)
    gp.check()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(gp.stream)
    gp.step(steps)
    stop.record(gp.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gp.check()
    fields = gp.moments()
    ev = start.elapsed_time(stop) * 1e-3
    rsize = 4 if precision == "fp32" else 8
    launch_s = ev / (3 * steps)
    bytes_launch = plane_step_bytes(spec, rsize) / 3
    pts = spec.nx * spec.nz * spec.Q
    ops_launch = plane_point_ops(spec) * pts
    res = dict(value=pts * steps / wall, unit="cell*quad-point updates/s", ms_per_step=1e3 * wall / steps,
               steps=steps,
               roofline=dict(bound="hbm", achieved=round(bytes_launch / launch_s / 1e9, 1), peak=HBM_PEAK_GBS,
                             unit="GB/s", frac=round(bytes_launch / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                             traffic=measured_traffic(precision, "plane_stage_kernel"), kernel="plane_stage_kernel",
                             bytes_per_launch=int(bytes_launch),
                             launch_us=round(launch_s * 1e6, 2)),
               roofline_alu=dict(bound="alu", achieved=round(ops_launch / launch_s / 1e9, 1), peak=VALU_PEAK_GOPS,
                                 unit="Gop/s", frac=round(ops_launch / launch_s / 1e9 / VALU_PEAK_GOPS, 4),
                                 kernel="plane_stage_kernel", ops_per_point=plane_point_ops(spec)),
               workload=f"plane_quadrants: 1024 x 1024 cells, Q = 3 x 8 x (8/2+1) = 120, N_v = 5, tau = 1e-2, "
                        f"2D Riemann problem, {precision.upper()}")
    del gp
    torch.cuda.empty_cache()
    return res, fields


def plane_error_table(f32, f64):
    """Max and L2 relative errors (normwise per field) of the FP32 plane
    against the FP64 plane after the same steps."""
    import numpy as np
    names = dict(e=9, vx=11, vz=12, T00=3, T0x=4, T0z=5, Txx=6, Txz=7, Tzz=8, N0=0, n=10)
    out = {}
    for name, k in names.items():
        d = f32[k] - f64[k]
        s = max(np.abs(f64[k]).max(), 1e-300)
        out[name] = dict(max=float(np.abs(d).max() / s), l2=float(np.sqrt(np.mean(d * d)) / s))
    return out


def leg_copy(nbytes=1 << 30, reps=5):
    """Plain device-to-device copy through the library's copy kernel: the
    practical HBM ceiling, and the calibration of the HBM byte counters."""
    import torch
    from paper_1608_03004_amd import rlb
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    rlb.device_copy(dst, src, nbytes)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    start.record(stream)
    for _ in range(reps):
        rlb.device_copy(dst, src, nbytes)
    stop.record(stream)
    torch.cuda.synchronize()
    s = start.elapsed_time(stop) * 1e-3 / reps
    ok = bool(torch.equal(dst, src))
    del src, dst
    torch.cuda.empty_cache()
    return dict(bytes_read=nbytes, bytes_written=nbytes, us_per_copy=round(s * 1e6, 2),
                achieved_GBs=round(2 * nbytes / s / 1e9, 1), frac_of_peak=round(2 * nbytes / s / 1e9 / HBM_PEAK_GBS, 4),
                verified=ok)


def cpu_baseline(params, target_s=12.0):
    """The CPU FP64 oracle on a bounded sample: the headline tube's Q and tau on
    a sub-tube of 2^16 cells, timed over whole steps (12 to about 25 s of CPU
    work)."""
    from oracle import oracle as O
    nx = 1 << 16
    t = O.Tube(nx=nx, q_xi=params["q_xi"], q_p=params["q_p"], tau=params["tau"], dt=0.5 / params["nx"])
    F = O.init(t, SOD_L, SOD_R)
    F = O.step(t, F, 1)  # warm-up (thread pool, first touch of the arrays)
    # batches of 1, 2, 4, ... steps until target_s of stepping is timed (the
    # first steps run slower than the steady state, so no single-step estimate)
    n, secs, k = 0, 0.0, 1
    while secs < target_s and n < 400:
        t0 = time.perf_counter()
        F = O.step(t, F, k)
        secs += time.perf_counter() - t0
        n += k
        k = min(2 * k, 400 - n)
    return dict(value=nx * t.Q * n / secs, unit="cell*quad-point updates/s", cores=O.num_threads(), kind="oracle",
                sample=f"FP64 oracle on {nx} cells x Q={t.Q} ({params['q_xi']}x{params['q_p']}), tau={params['tau']}, "
                       f"{n} steps in {secs:.1f} s (the headline tube's per-point work on 1/16 of its cells)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=1 << 20)
    ap.add_argument("--tile", type=int, default=256)
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64"),
                    help="form of the headline tube (fp64 is for profiling runs; the headline is fp32)")
    ap.add_argument("--legs", default="fp64,batched,adjoint,ballistic,high,plane,copy,cpu",
                    help="comma-separated extra legs (fp64, batched, adjoint, ballistic, high, plane, copy, "
                         "cpu) or 'none'")
    ap.add_argument("--plane-steps", type=int, default=20)
    ap.add_argument("--high-steps", type=int, default=20)
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--ballistic-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (--gpus 1); the multi-GPU "
                                   "slab decomposition is a design, not built"}))
        sys.exit(2)
    legs = set() if args.legs == "none" else set(args.legs.split(","))
    import torch
    torch.cuda.set_device(0)
    params = dict(nx=args.nx, q_xi=64, q_p=4, tau=1e-2)
    sched = dict(tile=args.tile)
    r32, f32, lat = leg_single(args.precision, params, args.steps, args.warmup, sched)
    del lat
    torch.cuda.empty_cache()
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
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "sod_large: Sod tube, N_x=2^20, Q=64x4 (Gauss-Legendre x Gauss-Laguerre), "
                               "tau=1e-2, FP32 stencil/relaxation, Kahan FP32 moments, FP64 Landau",
                   "nx": params["nx"], "q_xi": 64, "q_p": 4, "tau": 1e-2, "schedule": r32["schedule"]},
        "roofline": r32["roofline"],
    }
    if "fp64" in legs:
        r64, f64, lat = leg_single("fp64", params, args.steps, args.warmup, sched)
        del lat
        torch.cuda.empty_cache()
        line["fp64"] = dict(value=r64["value"], ms_per_step=r64["ms_per_step"], roofline=r64["roofline"],
                            speedup_fp32_over_fp64=r32["value"] / r64["value"])
        line["fp32_vs_fp64_error"] = dict(after_steps=args.steps + args.warmup, fields=error_table(f32, f64))
    if "batched" in legs:
        line["batched"] = leg_batched(args.batched_steps)
    if "adjoint" in legs:
        line["adjoint"] = dict(fp64=leg_adjoint("fp64"), fp32=leg_adjoint("fp32"))
    if "ballistic" in legs:
        line["ballistic"] = leg_ballistic(args.ballistic_steps)
    if "high" in legs:
        h32, hf32 = leg_high_order("fp32", args.high_steps)
        h64, hf64 = leg_high_order("fp64", args.high_steps)
        line["high_order"] = dict(fp32=h32, fp64=h64, fp32_vs_fp64_error=dict(
            after_steps=args.high_steps + 2, fields=error_table(hf32, hf64)))
    if "plane" in legs:
        p32, pf32 = leg_plane("fp32", args.plane_steps)
        p64, pf64 = leg_plane("fp64", args.plane_steps)
        line["plane"] = dict(fp32=p32, fp64=p64, fp32_vs_fp64_error=dict(
            after_steps=args.plane_steps + 2, fields=plane_error_table(pf32, pf64)))
    if "copy" in legs:
        line["copy"] = leg_copy()
    if "cpu" in legs:
        line["cpu_baseline"] = cpu_baseline(params)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
