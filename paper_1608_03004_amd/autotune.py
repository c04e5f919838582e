"""Launch-schedule autotuner for the stage kernels.

For a lattice it times a few time steps under each candidate schedule
(cells per workgroup, plain or persistent grid with a number of resident
workgroups per CU, hipGraph replay of several steps, quadrature points per
LDS chunk, the threshold below which a stage is spread over the radial nodes)
and keeps the fastest.
The lattice state and the tubes' clocks are saved before the sweep and
restored afterwards.  Results
are cached in a JSON file keyed by the device name, the precision and a
signature of the tube set, so a later run with the same workload reuses the
choice without timing.
"""
import hashlib
import json
import os
import time

DEFAULT_CACHE = os.environ.get("RLB_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "rlb_autotune.json"))

def candidates_for(precision: str):
    """The searched schedules: tile (64, 128, 256 cells), plain or persistent grid
    (2, 4, 8 resident workgroups per CU), graph replay of 8 steps or none, the
    default or doubled chunk of quadrature points, and the radial-node split
    of small groups at its default threshold (the CU count), never, or always."""
    ch2 = 16 if precision == "fp32" else 8
    out = [dict(tile=t, persistent=0, blocks_per_cu=4, graph_steps=g, chunk=0, split_below=-1)
           for t in (64, 128, 256) for g in (0, 8)]
    out += [dict(tile=t, persistent=1, blocks_per_cu=b, graph_steps=g, chunk=0, split_below=-1)
            for t in (64, 128, 256) for b in (2, 4, 8) for g in (0, 8)]
    out += [dict(tile=t, persistent=0, blocks_per_cu=4, graph_steps=g, chunk=ch2, split_below=-1)
            for t in (64, 128, 256) for g in (0, 8)]
    out += [dict(tile=t, persistent=0, blocks_per_cu=4, graph_steps=8, chunk=0, split_below=s)
            for t in (64, 128) for s in (0, 1 << 30)]
    return out


CANDIDATES = None  # per precision: candidates_for(lattice.precision)


def signature(lat) -> str:
    h = hashlib.sha1()
    for t in lat.tubes:
        h.update(repr((t.nx, t.q_xi, t.q_p, t.n_v, t.n_p)).encode())
    return f"{lat.precision}:{len(lat.tubes)}:{h.hexdigest()[:16]}"


def _device_name():
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(lat, steps: int = 4, candidates=None, cache_path: str = DEFAULT_CACHE, use_cache: bool = True,
         verbose: bool = False):
    """Returns (best schedule dict, {schedule key: seconds per step}) and applies the best."""
    import torch
    if candidates is None:
        candidates = candidates_for(lat.precision)
    key = f"{_device_name()}|{signature(lat)}"
    cache = _load(cache_path) if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["schedule"]
        lat.set_schedule(**best)
        return best, cache[key].get("timings", {})
    saved = lat.get_state().clone()
    clocks = [lat.info(t)["time"] for t in range(len(lat.tubes))]
    timings = {}
    from .rlb import RLBError
    for cand in candidates:
        try:
            lat.set_schedule(**cand)
        except RLBError:  # not valid for this lattice (e.g. a doubled chunk on the longest tubes)
            continue
        lat.set_state(saved)
        g = cand["graph_steps"]
        n = max(steps, g) if g else steps
        lat.step(max(1, g or 1))  # warm-up, graph capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(n)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / n
        timings[json.dumps(cand, sort_keys=True)] = sec
        if verbose:
            print(f"autotune {cand}: {sec * 1e3:.3f} ms/step", flush=True)
    best_key = min(timings, key=timings.get)
    best = json.loads(best_key)
    lat.set_schedule(**best)
    lat.set_state(saved)
    for t, clock in enumerate(clocks):
        lat.set_time(clock, t)
    lat.check()
    if use_cache:
        cache = _load(cache_path)
        cache[key] = dict(schedule=best, timings=timings)
        os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, timings
