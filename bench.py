"""Benchmark of the relativistic lattice Boltzmann step on one MI355X.

Headline workload: the large Sod tube -- N_x = 2^20 cells, Q = 64 x 4
quadrature points, tau = 1e-2, synthetic Sod initial states (the paper's
left/right states) -- advanced by full SSP-RK3 steps in the FP32 form (FP32
stencil and relaxation, Kahan-compensated FP32 moment sums, FP64 Landau
matching).  A "step" is one full time step (three stage launches) of the
whole tube.  Beside it, on the same line:
  fp64        the FP64 form on the same tube;
  tau_sweep   the large tube for its 2000 steps at tau = 1e-4, 1e-2, 1, 100 in
              FP32 and FP64: throughput, FP32-vs-FP64 max/L2 errors of e, u,
              T^{mu nu} over the whole tube, and at tau = 100 the error
              against the free-streaming profile of eq. ballistic;
  batched     4096 seeded tubes of uneven size, order and tau in one launch
              per stage, schedule chosen by the autotuner, replayed from a
              hipGraph;
  adjoint     gradient of the profile loss of the 4096-cell, Q = 32 x 3 tube
              over 2000 steps (forward + sqrt(N)-checkpointed backward), with
              central differences (h = 1e-6) at full size;
  ballistic   the 2^22-cell, Q = 256 x 4 tube at tau = 1e3 (FP32): a short
              timed run, and the full 4000-step run against eq. ballistic;
  high        the headline tube with the high-order equilibrium (N_v = 63),
              FP32 and FP64, with the matrix-core roofline of its pre-pass;
  plane       the multi-dimensional model on a 1024 x 1024 plane (Q = 120),
              FP32 and FP64;
  copy, stream the practical HBM ceilings: a plain copy, and the stage
              kernel's own memory pattern with no arithmetic;
  roofline    of the stage kernel: algorithmic bytes per launch over its mean
              duration, timed with HIP events on the launch stream;
  cpu_baseline the CPU FP64 oracle on a bounded sample of the headline tube,
              and on the windows of every leg's result that it can follow
              (the max and L2 errors of e, u and T^{mu nu} against the FP64
              oracle are attached to each leg as oracle_error).

Prints ONE JSON line (progress lines go to stderr).  Inputs are resident in
HBM before every timed region.
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


KERNEL_SOURCES = {"stage_kernel": "rlb_kernels.hip", "feq_kernel": "rlb_feq.hip", "plane_stage_kernel": "rlb_plane.hip",
                  "box_stage_kernel": "rlb_box.hip"}
TRAFFIC_FILES = {"stage_kernel": "stage_kernel_traffic.json", "feq_kernel": "feq_kernel_traffic.json",
                 "plane_stage_kernel": "plane_stage_kernel_traffic.json",
                 "box_stage_kernel": "box_stage_kernel_traffic.json"}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha1(kernel="stage_kernel"):
    """SHA-1 of the sources a kernel is built from (its own file and the two
    shared headers)."""
    import hashlib
    h = hashlib.sha1()
    for f in (KERNEL_SOURCES[kernel], "rlb_device.h", "rlb_internal.h"):
        with open(os.path.join(ROOT, "paper_1608_03004_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel="stage_kernel"):
    """HBM bytes per launch of a kernel on a benchmark workload (e.g.
    "sod_large/fp32") from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs
    (calibrated on the copy kernel), or None when the kernel's sources changed
    since those counters were taken."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[kernel])
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha1") != kernel_source_sha1(kernel):
        return None
    w = t.get("workloads", {}).get(workload)
    return int(w["traffic_bytes_per_launch"]) if w else None


def roofline(tubes, rsize, steps, event_s, traffic=None):
    launch_s = event_s / (3 * steps)
    bytes_launch = step_bytes(tubes, rsize) / 3
    achieved = bytes_launch / launch_s / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                bytes_per_launch=int(bytes_launch), launch_us=round(launch_s * 1e6, 2))


# ---------------------------------------------------------------------------
# Reference profiles the benchmark checks against (closed forms of the paper)
# ---------------------------------------------------------------------------
DN = SOD_L[1] - SOD_R[1]  # the normalisation of the paper's error measure


def n_ballistic(z, t, nL=1.0, nR=0.125):
    """Density of free streaming from the Sod states (eq. ballistic): with
    s = z/t, |N| = sqrt(((nL+nR)/2 - (nL-nR) s/2)^2 - ((nL-nR)/4)^2 (1-s^2)^2)."""
    import numpy as np
    s = np.clip(np.asarray(z, dtype=np.float64) / t, -1.0, 1.0)
    return np.sqrt(((nL + nR) / 2 - (nL - nR) / 2 * s) ** 2 - ((nL - nR) / 4) ** 2 * (1 - s * s) ** 2)


def staircase_bound(xi, w, nL=1.0, nR=0.125):
    """Largest deviation (in units of nL - nR) of the discrete-velocity free
    streaming, every polar node xi_j moving exactly, from eq. ballistic: the
    error of the quadrature itself, which the lattice run approaches."""
    import numpy as np
    s = np.linspace(-0.999999, 0.999999, 200001)[None, :]
    left = (s < np.asarray(xi)[:, None])  # node j at z = s t came from the left iff xi_j > s
    n = np.where(left, nL, nR)
    wj = np.asarray(w)[:, None] / 2
    N0, Nz = (wj * n).sum(0), (wj * n * np.asarray(xi)[:, None]).sum(0)
    return float(np.abs(np.sqrt(N0 * N0 - Nz * Nz) - n_ballistic(s[0], 1.0, nL, nR)).max() / (nL - nR))


FIELD_ROWS = dict(e=5, T00=2, T0z=3, Tzz=4, N0=0, n=6)


def error_table(a, b):
    """Max and L2 relative errors (normwise per field) of fields a against b:
    e, u = gamma v, T^{mu nu}, N^0 and n."""
    import numpy as np
    out = {}
    for name, k in FIELD_ROWS.items():
        d = a[k] - b[k]
        s = max(np.abs(b[k]).max(), 1e-300)
        out[name] = dict(max=float(np.abs(d).max() / s), l2=float(np.sqrt(np.mean(d * d)) / s))
    ua, ub = a[7] / np.sqrt(1 - a[7] ** 2), b[7] / np.sqrt(1 - b[7] ** 2)
    s = max(np.abs(ub).max(), 1e-300)
    out["u"] = dict(max=float(np.abs(ua - ub).max() / s), l2=float(np.sqrt(np.mean((ua - ub) ** 2)) / s))
    return out


def window_request(name, params, left, right, nsteps, dt, fields, half=256):
    """A centre window of a full-tube result that the oracle can follow: the
    initial state of cells [c - half - 9 n, c + half + 9 n) evolves exactly
    like the full tube on its inner 2 half cells (three stages of three-cell
    stencils per step); whole tubes when they are short."""
    nx = params["nx"]
    pad = 9 * nsteps
    c = nx // 2
    a, b = max(0, c - half - pad), min(nx, c + half + pad)
    lo, hi = (0, nx) if (a == 0 or b == nx) else (c - half, c + half)
    if lo == 0 and hi == nx:
        a, b = 0, nx
    return dict(name=name, params=dict(params), left=left, right=right, nsteps=nsteps, dt=dt, a=a, b=b, lo=lo,
                hi=hi, gpu=fields[:, lo:hi].copy())


# ---------------------------------------------------------------------------
# Legs
# ---------------------------------------------------------------------------
def head_schedule(precision, tile=0):
    """Schedule of the headline tube, from an autotune.tune sweep over it on MI355X: FP32 keeps
    256-cell tiles (within 0.5 % of the best candidate), FP64 runs 64-cell tiles (3.57 against 3.64
    ms per step).  Both launch stage by stage: graph replay gains at most 0.8 % here, and its
    capture would fall inside a short timed run."""
    if tile:
        return dict(tile=tile)
    return dict(tile=256 if precision == "fp32" else 64)


def leg_single(precision, params, steps, warmup, schedule=None, traffic_key=None):
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
    traffic = measured_traffic(traffic_key) if traffic_key else None
    out = dict(value=tube.nx * tube.Q * steps / wall, ms_per_step=1e3 * wall / steps,
               roofline=roofline([tube], rsize, steps, ev, traffic), schedule=lat.get_schedule())
    win = window_request(f"sod_large/{precision}", params, SOD_L, SOD_R, steps + warmup, lat.info(0)["dt"], fields)
    return out, fields, lat, win


def leg_tau_sweep(nsteps=2000, taus=(1e-4, 1e-2, 1.0, 100.0)):
    """The large tube for its stated 2000 steps at each tau, FP32 and FP64, in the headline
    schedules."""
    import numpy as np
    import torch
    from paper_1608_03004_amd import Lattice, Tube
    res = {}
    for tau in taus:
        r, f = {}, {}
        for prec in ("fp32", "fp64"):
            tube = Tube(nx=1 << 20, q_xi=64, q_p=4, tau=tau)
            lat = Lattice([tube], precision=prec)
            lat.set_schedule(**head_schedule(prec))
            lat.set_initial_state(SOD_L, SOD_R)
            tot0 = lat.totals(0)
            wall, ev = timed_steps(lat, nsteps)
            f[prec] = lat.moments(0)
            tot = lat.totals(0)
            t = lat.info(0)["time"]
            flags = lat.flags()
            rsize = 4 if prec == "fp32" else 8
            # conservation (A19): N0, T00 constant; T0z grows by (P_L - P_R) t
            drift = (tot - tot0 - np.array([0.0, 0.0, (SOD_L[0] - SOD_R[0]) * t])) / tot0[1]
            r[prec] = dict(value=tube.nx * tube.Q * nsteps / wall, ms_per_step=1e3 * wall / nsteps,
                           roofline=roofline([tube], rsize, nsteps, ev), conservation_drift=drift.tolist(),
                           fast_flow=flags["fast_flow"])
            if tau == 100.0:
                xi, w, _, _ = lat.tables(0)
                z = -0.5 + (np.arange(tube.nx) + 0.5) / tube.nx
                r[prec]["ballistic_error"] = float(np.abs(f[prec][9] - n_ballistic(z, t)).max() / DN)
                r["staircase_bound"] = staircase_bound(xi, w)
            del lat
            torch.cuda.empty_cache()
        r["fp32_vs_fp64_error"] = error_table(f["fp32"], f["fp64"])
        r["speedup_fp32_over_fp64"] = r["fp32"]["value"] / r["fp64"]["value"]
        r["t_end"] = t
        res[f"tau={tau:g}"] = r
        progress(f"tau sweep: tau = {tau:g} done")
    res["workload"] = "sod_large: N_x=2^20, Q=64x4, 2000 steps, tau in {1e-4, 1e-2, 1, 100}, FP32 and FP64"
    return res


def batched_selection(w):
    """Tubes of the seeded draw whose results are checked against the oracle:
    the first of every polar order, the stiffest and the shortest."""
    import numpy as np
    tubes = w["tubes"]
    sel = [next(k for k, t in enumerate(tubes) if t["q_xi"] == q) for q in (8, 16, 32, 64, 128)]
    sel += [int(np.argmin([t["tau"] for t in tubes])), int(np.argmin([t["nx"] for t in tubes]))]
    return sorted(set(sel))


def leg_batched(steps, schedule=None, full_steps=500):
    import torch
    import workloads
    from paper_1608_03004_amd import Lattice, Tube
    from paper_1608_03004_amd import autotune
    w = workloads.sod_batched()
    tubes = [Tube(**t) for t in w["tubes"]]
    lat = Lattice(tubes, precision="fp32")
    lat.set_initial_states(w["left"], w["right"])
    lat.step(1)
    if schedule:  # a fixed schedule (profiling runs), no autotuning
        lat.set_schedule(**schedule)
        timings = {}
    else:
        _, timings = autotune.tune(lat, steps=3, use_cache=False)
    lat.set_initial_states(w["left"], w["right"])
    warm = 2
    lat.step(warm)
    lat.check()
    wall, ev = timed_steps(lat, steps)
    lat.check()
    pts = sum(t.nx * t.Q for t in tubes)
    wins = []
    for k in batched_selection(w):
        wins.append(window_request(f"sod_batched/tube{k}", w["tubes"][k], w["left"][k], w["right"][k],
                                   warm + steps, lat.info(k)["dt"], lat.moments(k)))
    full = None
    if full_steps and not schedule:
        # the configuration's whole run (not in profiling runs): full_steps
        # steps of every tube from its initial states, timed as one; no
        # non-physical state may occur and e, n stay positive in every cell
        import numpy as np
        lat.set_initial_states(w["left"], w["right"])
        wall_full, _ = timed_steps(lat, full_steps)
        lat.check()
        fl = lat.flags()
        mins = np.array([lat.moments(k)[5:7].min(axis=1) for k in range(len(tubes))])
        full = dict(steps=full_steps, value=pts * full_steps / wall_full, ms_per_step=1e3 * wall_full / full_steps,
                    min_e=float(mins[:, 0].min()), min_n=float(mins[:, 1].min()), fast_flow=fl["fast_flow"])
        progress(f"batched full run: {full_steps} steps in {wall_full:.2f} s")
    out = dict(value=pts * steps / wall, unit="cell*quad-point updates/s", ms_per_step=1e3 * wall / steps,
               steps=steps, tubes=len(tubes), points_per_step=pts, schedule=lat.get_schedule(), full_run=full,
               roofline=roofline(tubes, 4, steps, ev, measured_traffic("sod_batched/fp32")),
               autotune_candidates=len(timings),
               autotune_top=[dict(json.loads(k), ms_per_step=round(v * 1e3, 3))
                             for k, v in sorted(timings.items(), key=lambda kv: kv[1])[:3]],
               workload="sod_batched: 4096 tubes, numpy default_rng(0): N_x~U{256..8192}, "
                        "Q_xi~U{8,16,32,64,128}, Q_p=3, log tau~U[ln1e-4,ln10], "
                        "log(P_L/P_R)~U[ln2,ln100], n_L/n_R~U[1,10], FP32")
    del lat
    torch.cuda.empty_cache()
    return out, wins


def leg_adjoint(precision, nsteps=2000, fd=False):
    import numpy as np
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
    if fd:
        # central differences of the forward at h = 1e-6 (FP64), dt fixed
        tgt = target.cpu().numpy()

        def loss_at(tau, PL):
            plat = Lattice([Tube(**p)], precision="fp64")
            plat.set_tau(tau)
            plat.set_initial_state((PL, st["n_L"], 0.0), SOD_R)
            plat.step(nsteps)
            return float(np.sum((plat.moments(0)[5] - tgt) ** 2) / p["nx"])

        h = 1e-6
        fd_tau = (loss_at(st["tau"] + h, st["P_L"]) - loss_at(st["tau"] - h, st["P_L"])) / (2 * h)
        fd_PL = (loss_at(st["tau"], st["P_L"] + h) - loss_at(st["tau"], st["P_L"] - h)) / (2 * h)
        out["fd_h"] = h
        out["fd_grad_tau"], out["fd_grad_P_L"] = fd_tau, fd_PL
        out["fd_rel_err"] = dict(tau=abs(fd_tau - grads[0]) / abs(fd_tau), P_L=abs(fd_PL - grads[1]) / abs(fd_PL))
    del lat
    torch.cuda.empty_cache()
    return out


def leg_ballistic(steps, warmup=2, full_steps=4000):
    """The ballistic stress tube: a short timed run (throughput, and a window
    the oracle can follow) and the stated 4000-step run against eq. ballistic."""
    import numpy as np
    import torch
    from paper_1608_03004_amd import Lattice, Tube
    params = dict(nx=1 << 22, q_xi=256, q_p=4, tau=1e3)
    tube = Tube(**params)
    lat = Lattice([tube], precision="fp32")
    lat.set_initial_state(SOD_L, SOD_R)
    lat.step(warmup)
    wall, ev = timed_steps(lat, steps)
    lat.check()
    win = window_request("sod_ballistic/fp32", params, SOD_L, SOD_R, steps + warmup, lat.info(0)["dt"],
                         lat.moments(0))
    out = dict(value=tube.nx * tube.Q * steps / wall, ms_per_step=1e3 * wall / steps, steps=steps,
               roofline=roofline([tube], 4, steps, ev, measured_traffic("sod_ballistic/fp32")),
               workload="sod_ballistic: N_x=2^22, Q=256x4, tau=1e3, FP32")
    progress("ballistic: short run done")
    if full_steps:
        lat.set_initial_state(SOD_L, SOD_R)
        wall, ev = timed_steps(lat, full_steps)
        f = lat.moments(0)
        t = lat.info(0)["time"]
        xi, w, _, _ = lat.tables(0)
        z = -0.5 + (np.arange(tube.nx) + 0.5) / tube.nx
        out["full_run"] = dict(steps=full_steps, t_end=t, value=tube.nx * tube.Q * full_steps / wall,
                               ms_per_step=1e3 * wall / full_steps,
                               roofline=roofline([tube], 4, full_steps, ev),
                               ballistic_error=float(np.abs(f[9] - n_ballistic(z, t)).max() / DN),
                               staircase_bound=staircase_bound(xi, w), flags=lat.flags())
        progress("ballistic: 4000-step run done")
    del lat
    torch.cuda.empty_cache()
    return out, win


MFMA_F64_PEAK_TFS = 78.6  # MI355X dense FP64 matrix


def high_order_flops(tube):
    """Algorithmic flops of one equilibrium pre-pass over a high-order tube:
    per cell and radial node the two even/odd products, ceil(q_xi/2) rows by
    B auxiliary pairs, one multiply and one add each."""
    B = 4 * ((tube.n_v + 89 + 15) // 16)
    return 4 * ((tube.q_xi + 1) // 2) * B * tube.nx * tube.q_p


def leg_high_order(precision, steps, warmup=2, reps=10, q_xi=64):
    """The large Sod tube with the high-order equilibrium (N_v = Q_xi - 1):
    every stage runs the matrix-core pre-pass and then the stage kernel that
    streams its output.  Q_xi = 64 on 2^20 cells, or Q_xi = 128 on 2^19 cells
    (the same number of points)."""
    import torch
    from paper_1608_03004_amd import Lattice, Tube
    nx = (1 << 20) * 64 // q_xi
    params = dict(nx=nx, q_xi=q_xi, q_p=4, n_v=q_xi - 1, tau=1e-2)
    name = "sod_large_high_order" if q_xi == 64 else f"sod_large_high_order_q{q_xi}"
    tube = Tube(**params)
    lat = Lattice([tube], precision=precision)
    lat.set_initial_state(SOD_L, SOD_R)
    lat.step(warmup)
    lat.check()
    wall, ev = timed_steps(lat, steps)
    lat.check()
    fields = lat.moments(0)
    win = window_request(f"{name}/{precision}", params, SOD_L, SOD_R, steps + warmup,
                         lat.info(0)["dt"], fields, half=64)
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
                             traffic=measured_traffic(f"{name}/{precision}", "feq_kernel"),
                             kernel="feq_kernel", flops_per_launch=flops, launch_us=round(feq_s * 1e6, 2)),
               stage_roofline=dict(bound="hbm", achieved=round(stage_bytes / stage_s / 1e9, 1), peak=HBM_PEAK_GBS,
                                   unit="GB/s", frac=round(stage_bytes / stage_s / 1e9 / HBM_PEAK_GBS, 4),
                                   bytes_per_launch=int(stage_bytes), launch_us=round(stage_s * 1e6, 2)),
               workload=f"{name}: N_x=2^{nx.bit_length() - 1}, Q={q_xi}x4, N_v={q_xi - 1}, N_p=2, tau=1e-2, "
                        f"{precision.upper()}")
    del lat, out
    torch.cuda.empty_cache()
    return res, fields, win


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


def leg_plane(precision, steps, warmup=2, window_steps=5, window_half=8):
    """The multi-dimensional model: a 1024 x 1024 plane, Q = 3 x 8 x 5 evolved
    points (Q_phi = 8), a 2D Riemann problem; a separate short run gives a
    centre window the oracle can follow."""
    import torch
    from paper_1608_03004_amd import Plane, PlaneSpec
    spec = PlaneSpec(nx=1024, nz=1024, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gp = Plane(spec, precision=precision)
    init = plane_quadrants(spec.nx, spec.nz)
    gp.set_initial_fields(init)
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
                             traffic=measured_traffic(f"plane_quadrants/{precision}", "plane_stage_kernel"),
                             kernel="plane_stage_kernel", bytes_per_launch=int(bytes_launch),
                             launch_us=round(launch_s * 1e6, 2)),
               roofline_alu=dict(bound="alu", achieved=round(ops_launch / launch_s / 1e9, 1), peak=VALU_PEAK_GOPS,
                                 unit="Gop/s", frac=round(ops_launch / launch_s / 1e9 / VALU_PEAK_GOPS, 4),
                                 kernel="plane_stage_kernel", ops_per_point=plane_point_ops(spec)),
               workload=f"plane_quadrants: 1024 x 1024 cells, Q = 3 x 8 x (8/2+1) = 120, N_v = 5, tau = 1e-2, "
                        f"2D Riemann problem, {precision.upper()}")
    # the window: a short run from the same initial state
    gp.set_initial_fields(init)
    gp.step(window_steps)
    short = gp.moments()
    pad = 9 * window_steps
    c = spec.nx // 2
    a, b = c - window_half - pad, c + window_half + pad
    win = dict(name=f"plane_quadrants/{precision}", plane=True,
               spec=dict(nx=b - a, nz=b - a, q_xi=8, q_phi=8, q_p=3, tau=1e-2, x_min=-0.5 + a / spec.nx,
                         x_max=-0.5 + b / spec.nx, z_min=-0.5 + a / spec.nz, z_max=-0.5 + b / spec.nz,
                         dt=gp.info()["dt"]),
               init=init[:, a:b, a:b].copy(), nsteps=window_steps, pad=pad, half=window_half,
               gpu=short[:, c - window_half:c + window_half, c - window_half:c + window_half].copy())
    del gp
    torch.cuda.empty_cache()
    return res, fields, win


def plane_error_table(a, b):
    """Max and L2 relative errors (normwise per field) of plane fields."""
    import numpy as np
    names = dict(e=9, vx=11, vz=12, T00=3, T0x=4, T0z=5, Txx=6, Txz=7, Tzz=8, N0=0, n=10)
    out = {}
    for name, k in names.items():
        d = a[k] - b[k]
        s = max(np.abs(b[k]).max(), 1e-300)
        out[name] = dict(max=float(np.abs(d).max() / s), l2=float(np.sqrt(np.mean(d * d)) / s))
    return out


def box_octants(nx, ny, nz):
    """Per-cell (P, n, u^x, u^y, u^z) of a 3D Riemann problem on [-0.5, 0.5]^3:
    eight constant states meeting at the centre, with flows along all three
    axes (so every azimuthal node carries its own values)."""
    import numpy as np
    x = -0.5 + (np.arange(nx) + 0.5) / nx
    y = -0.5 + (np.arange(ny) + 0.5) / ny
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    f = np.zeros((5, nz, ny, nx))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                m = ((X >= 0) == bool(a)) & ((Y >= 0) == bool(b)) & ((Z >= 0) == bool(c))
                hi = (a + b + c) % 2 == 0
                st = ((1.0 if hi else 0.2) * (1 + 0.2 * a), 1.0 if hi else 0.3, 0.1 * (a - b), 0.15 * (b - c),
                      0.12 * (c - a))
                for k in range(5):
                    f[k][m] = st[k]
    return f


def box_step_bytes(spec, rsize):
    """Algorithmic HBM bytes of one box step: 8 accesses per point (as for a
    tube) and per cell and stage the 14 FP64 records read and written."""
    return 8 * spec.cells * spec.Q * rsize + 3 * 224 * spec.cells


def box_point_ops(spec):
    """Algorithmic vector operations per point and stage of the box update:
    three WENO5 faces of 37 operations each (one per direction: a face is
    shared by the two cells beside it), the equilibrium polynomial in
    c = v . u_hat (2 + N_v), advection and relaxation (11), the RK combination
    (3) and the ten moment FMAs.  Per-cell work (Landau frame, projection) and
    the faces a tile computes twice are excluded."""
    return 3 * 37 + (2 + spec.n_v) + 11 + 3 + 10


def leg_box(precision, steps, warmup=2, window_steps=2, window_half=4, n=128):
    """The three-dimensional model: a 128^3 box, Q = 3 x 8 x 8 = 192 evolved
    points (every azimuthal node), a 3D Riemann problem; a separate short run
    gives a centre window the oracle can follow."""
    import torch
    from paper_1608_03004_amd import Box, BoxSpec
    spec = BoxSpec(nx=n, ny=n, nz=n, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gb = Box(spec, precision=precision)
    init = box_octants(n, n, n)
    gb.set_initial_fields(init)
    gb.step(warmup)
    gb.check()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(gb.stream)
    gb.step(steps)
    stop.record(gb.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gb.check()
    fields = gb.moments()
    ev = start.elapsed_time(stop) * 1e-3
    rsize = 4 if precision == "fp32" else 8
    launch_s = ev / (3 * steps)
    bytes_launch = box_step_bytes(spec, rsize) / 3
    pts = spec.cells * spec.Q
    ops_launch = box_point_ops(spec) * pts
    res = dict(value=pts * steps / wall, unit="cell*quad-point updates/s", ms_per_step=1e3 * wall / steps,
               steps=steps,
               roofline_alu=dict(bound="alu", achieved=round(ops_launch / launch_s / 1e9, 1), peak=VALU_PEAK_GOPS,
                                 unit="Gop/s", frac=round(ops_launch / launch_s / 1e9 / VALU_PEAK_GOPS, 4),
                                 kernel="box_stage_kernel", ops_per_point=box_point_ops(spec),
                                 launch_us=round(launch_s * 1e6, 2)),
               roofline_hbm=dict(bound="hbm", achieved=round(bytes_launch / launch_s / 1e9, 1), peak=HBM_PEAK_GBS,
                                 unit="GB/s", frac=round(bytes_launch / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                                 traffic=measured_traffic(f"box_octants/{precision}", "box_stage_kernel"),
                                 kernel="box_stage_kernel", bytes_per_launch=int(bytes_launch)),
               workload=f"box_octants: {n}^3 cells, Q = 3 x 8 x 8 = 192 (every azimuthal node), N_v = 5, "
                        f"tau = 1e-2, 3D Riemann problem, {precision.upper()}")
    gb.set_initial_fields(init)
    gb.step(window_steps)
    pad = 9 * window_steps
    c = n // 2
    short = gb.fields()[:, c - window_half:c + window_half, c - window_half:c + window_half,
                        c - window_half:c + window_half].cpu().numpy()
    a, b = c - window_half - pad, c + window_half + pad
    lo, hi = -0.5 + a / n, -0.5 + b / n
    win = dict(name=f"box_octants/{precision}", box=True,
               spec=dict(nx=b - a, ny=b - a, nz=b - a, q_xi=8, q_phi=8, q_p=3, tau=1e-2, x_min=lo, x_max=hi,
                         y_min=lo, y_max=hi, z_min=lo, z_max=hi, dt=gb.info()["dt"]),
               init=init[:, a:b, a:b, a:b].copy(), nsteps=window_steps, pad=pad, half=window_half, gpu=short)
    del gb
    torch.cuda.empty_cache()
    return res, fields, win


def box_error_table(a, b):
    """Max and L2 relative errors (normwise per field) of box fields."""
    import numpy as np
    names = dict(N0=0, T00=4, T0x=5, T0y=6, T0z=7, Txx=8, Txy=9, Tyy=11, Tzz=13, e=14, n=15, vx=16, vy=17, vz=18)
    out = {}
    for name, k in names.items():
        d = a[k] - b[k]
        s = max(np.abs(b[k]).max(), 1e-300)
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


def leg_stream(rows=256, cols=1 << 20, reps=10):
    """The stage kernel's memory pattern with no arithmetic (rlb_device_stream)
    on the headline tube's array shape, FP32 and FP64: one read and one write
    per point (stage 1), two reads and one write (stages 2, 3)."""
    import torch
    from paper_1608_03004_amd import rlb
    res = {}
    for prec, dtype in (("fp32", torch.float32), ("fp64", torch.float64)):
        a = torch.rand(rows * cols, dtype=dtype, device="cuda")
        b = torch.rand(rows * cols, dtype=dtype, device="cuda")
        out = torch.empty_like(a)
        r = {}
        for name, bb, nacc in (("read1_write1", None, 2), ("read2_write1", b, 3)):
            rlb.device_stream(out, a, bb, rows, cols, cols)
            torch.cuda.synchronize()
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            stream = torch.cuda.current_stream()
            start.record(stream)
            for _ in range(reps):
                rlb.device_stream(out, a, bb, rows, cols, cols)
            stop.record(stream)
            torch.cuda.synchronize()
            s = start.elapsed_time(stop) * 1e-3 / reps
            byts = nacc * rows * cols * a.element_size()
            ok = bool(torch.equal(out, a + b if bb is not None else a))
            r[name] = dict(bytes=byts, us=round(s * 1e6, 2), achieved_GBs=round(byts / s / 1e9, 1),
                           frac_of_peak=round(byts / s / 1e9 / HBM_PEAK_GBS, 4), verified=ok)
        # a step moves one read1/write1 and two read2/write1 passes
        step_s = (r["read1_write1"]["us"] + 2 * r["read2_write1"]["us"]) * 1e-6
        r["step_us"] = round(step_s * 1e6, 2)
        r["step_GBs"] = round(8 * rows * cols * a.element_size() / step_s / 1e9, 1)
        res[prec] = r
        del a, b, out
        torch.cuda.empty_cache()
    res["shape"] = f"[{rows}][{cols}] rows of the headline tube's state"
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(params, windows, target_s=12.0):
    """The CPU FP64 oracle: (1) on a bounded sample of the headline workload --
    the headline tube's Q and tau on a sub-tube of 2^16 cells, timed over
    whole steps (12 to about 25 s of CPU work); (2) on the windows of the GPU
    results that it can follow, which gives every leg's max and L2 errors
    against the oracle (its time is counted in the sample too)."""
    import numpy as np
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
    sample_updates = nx * t.Q * n
    errors, win_updates, win_secs = {}, 0, 0.0
    for w in windows:
        t0 = time.perf_counter()
        if w.get("box"):
            bx = O.Box(**w["spec"])
            ref = O.box_fields(bx, O.box_run(bx, w["init"], w["nsteps"]))
            p, h = w["pad"], w["half"]
            ref = ref[:, p:p + 2 * h, p:p + 2 * h, p:p + 2 * h]
            win_updates += bx.cells * bx.Q * w["nsteps"]
            errors[w["name"]] = box_error_table(w["gpu"], ref)
        elif w.get("plane"):
            pl = O.Plane(**w["spec"])
            Fp = O.plane_run(pl, w["init"], w["nsteps"])
            ref = O.plane_fields(pl, Fp)
            p, h = w["pad"], w["half"]
            ref = ref[:, p:p + 2 * h, p:p + 2 * h]
            win_updates += pl.nx * pl.nz * pl.Q * w["nsteps"]
            errors[w["name"]] = plane_error_table(w["gpu"], ref)
        else:
            nxf = w["params"]["nx"]
            dz = 1.0 / nxf
            wp = dict(w["params"], nx=w["b"] - w["a"], z_min=-0.5 + w["a"] * dz, z_max=-0.5 + w["b"] * dz, dt=w["dt"])
            ot = O.Tube(**wp)
            ref = O.fields(ot, O.run(ot, w["left"], w["right"], w["nsteps"]))
            ref = ref[:, w["lo"] - w["a"]:w["hi"] - w["a"]]
            win_updates += ot.nx * ot.Q * w["nsteps"]
            errors[w["name"]] = error_table(w["gpu"], ref)
            errors[w["name"]]["cells"] = [w["lo"], w["hi"]]
            errors[w["name"]]["after_steps"] = w["nsteps"]
        win_secs += time.perf_counter() - t0
    base = dict(value=sample_updates / secs, unit="cell*quad-point updates/s", cores=O.num_threads(), kind="oracle",
                cpu=cpu_model(), affinity_cpus=len(os.sched_getaffinity(0)),
                sample=f"FP64 oracle on {nx} cells x Q={t.Q} ({params['q_xi']}x{params['q_p']}), tau={params['tau']}, "
                       f"{n} steps in {secs:.1f} s (the headline tube's per-point work on 1/16 of its cells); plus "
                       f"{len(windows)} windows of the legs' results ({win_updates:.3g} point updates in "
                       f"{win_secs:.1f} s) for their oracle errors")
    return base, errors


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nx", type=int, default=1 << 20)
    ap.add_argument("--tile", type=int, default=0,
                    help="tile of the headline tube (0: the schedule of head_schedule)")
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64"),
                    help="form of the headline tube (fp64 is for profiling runs; the headline is fp32)")
    ap.add_argument("--legs", default="fp64,tau,batched,adjoint,ballistic,high,plane,box,copy,stream,cpu",
                    help="comma-separated extra legs (fp64, tau, batched, adjoint, ballistic, high, plane, box, copy, "
                         "stream, cpu) or 'none'")
    ap.add_argument("--plane-steps", type=int, default=20)
    ap.add_argument("--box-steps", type=int, default=10)
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="steps of the adjoint configuration (2000 is the benchmarked workload)")
    ap.add_argument("--adjoint-fd", type=int, default=1, help="central-difference check of the FP64 gradients")
    ap.add_argument("--high-steps", type=int, default=20)
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--batched-full-steps", type=int, default=500,
                    help="the batched configuration's whole run after the timed steps (0: none)")
    ap.add_argument("--ballistic-steps", type=int, default=20)
    ap.add_argument("--ballistic-full-steps", type=int, default=4000,
                    help="steps of the ballistic run checked against eq. ballistic (0: skip)")
    ap.add_argument("--tau-steps", type=int, default=2000)
    ap.add_argument("--batched-schedule", default="",
                    help="tile,persistent,blocks_per_cu,graph_steps[,chunk,split_below] for the batched leg "
                         "instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (--gpus 1); the multi-GPU "
                                   "slab decomposition is a design, not built"}))
        sys.exit(2)
    legs = set() if args.legs == "none" else set(args.legs.split(","))
    import torch
    torch.cuda.set_device(0)
    params = dict(nx=args.nx, q_xi=64, q_p=4, tau=1e-2)
    key = f"sod_large/{args.precision}" if args.nx == 1 << 20 else None
    r32, f32, lat, win32 = leg_single(args.precision, params, args.steps, args.warmup,
                                      head_schedule(args.precision, args.tile), key)
    del lat
    torch.cuda.empty_cache()
    progress("headline done")
    windows = [win32]
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
    legs_out = {}
    if "fp64" in legs:
        r64, f64, lat, win64 = leg_single("fp64", params, args.steps, args.warmup, head_schedule("fp64", args.tile),
                                          "sod_large/fp64" if args.nx == 1 << 20 else None)
        del lat
        torch.cuda.empty_cache()
        windows.append(win64)
        line["fp64"] = dict(value=r64["value"], ms_per_step=r64["ms_per_step"], roofline=r64["roofline"],
                            speedup_fp32_over_fp64=r32["value"] / r64["value"])
        line["fp32_vs_fp64_error"] = dict(after_steps=args.steps + args.warmup, fields=error_table(f32, f64))
        progress("fp64 done")
    if "tau" in legs:
        line["tau_sweep"] = leg_tau_sweep(args.tau_steps)
    if "batched" in legs:
        bs = None
        if args.batched_schedule:
            v = [int(x) for x in args.batched_schedule.split(",")]
            bs = dict(zip(("tile", "persistent", "blocks_per_cu", "graph_steps", "chunk", "split_below"), v))
        line["batched"], wins = leg_batched(args.batched_steps, bs, args.batched_full_steps)
        windows += wins
        progress("batched done")
    if "adjoint" in legs:
        line["adjoint"] = dict(fp64=leg_adjoint("fp64", nsteps=args.adjoint_steps, fd=bool(args.adjoint_fd)),
                               fp32=leg_adjoint("fp32", nsteps=args.adjoint_steps))
        g64, g32 = line["adjoint"]["fp64"], line["adjoint"]["fp32"]
        line["adjoint"]["fp32_vs_fp64_rel"] = dict(tau=abs(g32["grad_tau"] - g64["grad_tau"]) / abs(g64["grad_tau"]),
                                                   P_L=abs(g32["grad_P_L"] - g64["grad_P_L"]) / abs(g64["grad_P_L"]))
        progress("adjoint done")
    if "ballistic" in legs:
        line["ballistic"], win = leg_ballistic(args.ballistic_steps, full_steps=args.ballistic_full_steps)
        windows.append(win)
    if "high" in legs:
        h32, hf32, w32 = leg_high_order("fp32", args.high_steps)
        h64, hf64, w64 = leg_high_order("fp64", args.high_steps)
        windows += [w32, w64]
        line["high_order"] = dict(fp32=h32, fp64=h64, fp32_vs_fp64_error=dict(
            after_steps=args.high_steps + 2, fields=error_table(hf32, hf64)))
        g32, _, wg32 = leg_high_order("fp32", args.high_steps, q_xi=128)
        g64, _, wg64 = leg_high_order("fp64", args.high_steps, q_xi=128)
        windows += [wg32, wg64]
        line["high_order_q128"] = dict(fp32=g32, fp64=g64)
        progress("high-order done")
    if "plane" in legs:
        p32, pf32, w32 = leg_plane("fp32", args.plane_steps)
        p64, pf64, w64 = leg_plane("fp64", args.plane_steps)
        windows += [w32, w64]
        line["plane"] = dict(fp32=p32, fp64=p64, fp32_vs_fp64_error=dict(
            after_steps=args.plane_steps + 2, fields=plane_error_table(pf32, pf64)))
        progress("plane done")
    if "box" in legs:
        b32, bf32, w32 = leg_box("fp32", args.box_steps)
        b64, bf64, w64 = leg_box("fp64", args.box_steps)
        windows += [w32, w64]
        line["box"] = dict(fp32=b32, fp64=b64, fp32_vs_fp64_error=dict(
            after_steps=args.box_steps + 2, fields=box_error_table(bf32, bf64)))
        progress("box done")
    if "copy" in legs:
        line["copy"] = leg_copy()
    if "stream" in legs:
        line["stream"] = leg_stream()
        # the stage kernel against its own memory pattern with no arithmetic
        st = line["stream"][args.precision]
        line["roofline"]["stream_step_us"] = st["step_us"]
        line["roofline"]["frac_of_stream"] = round(st["step_us"] / (3 * line["roofline"]["launch_us"]), 4)
        if "fp64" in line:
            line["fp64"]["roofline"]["frac_of_stream"] = round(
                line["stream"]["fp64"]["step_us"] / (3 * line["fp64"]["roofline"]["launch_us"]), 4)
        progress("copy/stream done")
    if "cpu" in legs:
        line["cpu_baseline"], errors = cpu_baseline(params, windows)
        # every result's max and L2 errors against the FP64 oracle
        for name, err in errors.items():
            leg, form = name.split("/")
            if leg == "sod_large" and form == args.precision:
                line["oracle_error"] = err
            elif leg == "sod_large":
                line.setdefault("fp64", {})["oracle_error"] = err
            elif leg == "sod_batched":
                line.setdefault("batched", {}).setdefault("oracle_error", {})[form] = err
            elif leg == "sod_ballistic":
                line.setdefault("ballistic", {})["oracle_error"] = err
            elif leg == "sod_large_high_order":
                line.setdefault("high_order", {}).setdefault(form, {})["oracle_error"] = err
            elif leg == "sod_large_high_order_q128":
                line.setdefault("high_order_q128", {}).setdefault(form, {})["oracle_error"] = err
            elif leg == "plane_quadrants":
                line.setdefault("plane", {}).setdefault(form, {})["oracle_error"] = err
            elif leg == "box_octants":
                line.setdefault("box", {}).setdefault(form, {})["oracle_error"] = err
        progress("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
