"""CPU checks of the benchmark's contract and of the algorithmic byte, flop
and operation models its rooflines divide by (no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1608_03004_amd import PlaneSpec, Tube  # noqa: E402


def test_more_than_one_gpu_is_refused_before_touching_a_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_tube_step_bytes_are_eight_accesses_per_point_and_240_bytes_per_cell():
    t = Tube(nx=1 << 20, q_xi=64, q_p=4, tau=1e-2)
    assert bench.step_bytes([t], 4) == (1 << 20) * 256 * 32 + (1 << 20) * 240   # FP32: 32 B per point-step
    assert bench.step_bytes([t], 8) == (1 << 20) * 256 * 64 + (1 << 20) * 240   # FP64: 64 B
    # batched tubes add up
    u = Tube(nx=300, q_xi=8, q_p=3, tau=1e-2)
    assert bench.step_bytes([t, u], 4) == bench.step_bytes([t], 4) + bench.step_bytes([u], 4)


def test_plane_models():
    spec = PlaneSpec(nx=1024, nz=1024, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    assert spec.Q == 3 * 8 * 5
    cells = 1024 * 1024
    # 8 accesses per point and step, nine FP64 records in and out per cell and stage
    assert bench.plane_step_bytes(spec, 4) == 8 * cells * 120 * 4 + 3 * 144 * cells
    # two WENO5 faces of 37 operations, 2 + N_v for the equilibrium, 17 for the rest
    assert bench.plane_point_ops(spec) == 2 * 37 + 7 + 17 == 98


@pytest.mark.parametrize("q_xi,n_v,pairs", [(64, 63, 40), (33, 20, 28), (16, 15, 28), (9, 8, 28)])
def test_high_order_flops(q_xi, n_v, pairs):
    # B = 4 ceil((n_v + 89) / 16) auxiliary pairs; two [ceil(q_xi/2) x B] x [B x cells]
    # products per radial node, a multiply and an add each
    t = Tube(nx=1000, q_xi=q_xi, q_p=4, n_v=n_v, tau=1e-2)
    assert bench.high_order_flops(t) == 4 * ((q_xi + 1) // 2) * pairs * 1000 * 4


def test_cpu_baseline_record_and_oracle_windows():
    # a window request whose "GPU" result is the oracle's own full-tube run:
    # the window evolves exactly like the full tube, so the errors vanish
    import numpy as np
    from oracle import oracle as O
    params = dict(nx=640, q_xi=8, q_p=3, tau=1e-2)
    t = O.Tube(**params)
    full = O.fields(t, O.run(t, bench.SOD_L, bench.SOD_R, 6))
    win = bench.window_request("sod_large/fp64", params, bench.SOD_L, bench.SOD_R, 6, t.step_dt, full, half=32)
    assert (win["a"], win["b"], win["lo"], win["hi"]) == (320 - 32 - 54, 320 + 32 + 54, 288, 352)
    r, errs = bench.cpu_baseline(dict(nx=1 << 20, q_xi=8, q_p=3, tau=1e-2), [win], target_s=0.05)
    assert r["kind"] == "oracle" and r["cores"] >= 1 and r["value"] > 0 and r["cpu"]
    assert r["unit"] == "cell*quad-point updates/s" and "steps in" in r["sample"]
    e = errs["sod_large/fp64"]
    assert max(v["max"] for k, v in e.items() if isinstance(v, dict)) < 1e-14
    # a short tube is taken whole
    short = dict(nx=100, q_xi=8, q_p=3, tau=1e-2)
    w2 = bench.window_request("x/fp32", short, bench.SOD_L, bench.SOD_R, 6, 0.005, np.zeros((10, 100)))
    assert (w2["a"], w2["b"], w2["lo"], w2["hi"]) == (0, 100, 0, 100)


def test_ballistic_profile_and_staircase_bound():
    # worked values of eq. ballistic (n_L = 1, n_R = 0.125) and the quadrature
    # staircase bound of a 64-node Gauss-Legendre rule
    import numpy as np
    nb = bench.n_ballistic(np.array([0.0, 0.5, -0.5]), 1.0)
    assert np.allclose(nb, [0.518222623493031, 0.302072108268456, 0.763829207738058], rtol=0, atol=1e-14)
    assert bench.n_ballistic(np.array([-2.0, 2.0]), 1.0).tolist() == [1.0, 0.125]
    xi, w = np.polynomial.legendre.leggauss(64)
    assert abs(bench.staircase_bound(xi, w) - 0.01346) < 2e-4
    xi, w = np.polynomial.legendre.leggauss(256)
    assert abs(bench.staircase_bound(xi, w) - 0.00338) < 1e-4


def test_error_table_fields():
    import numpy as np
    b = np.ones((10, 50))
    b[7] = 0.5  # v
    a = b.copy()
    a[5, 3] += 1e-6
    e = bench.error_table(a, b)
    assert abs(e["e"]["max"] - 1e-6) < 1e-12 and e["T00"]["max"] == 0 and e["u"]["max"] == 0
    assert set(e) == {"e", "u", "T00", "T0z", "Tzz", "N0", "n"}


def test_box_models_and_oracle_window():
    # 8 accesses per point, 14 FP64 records in and out per cell and stage;
    # three WENO5 faces per point (one per direction)
    import numpy as np
    from oracle import oracle as O
    from paper_1608_03004_amd import BoxSpec
    spec = BoxSpec(nx=128, ny=128, nz=128, q_xi=8, q_phi=8, q_p=3)
    assert spec.Q == 192 and spec.cells == 1 << 21
    assert bench.box_step_bytes(spec, 4) == 8 * (1 << 21) * 192 * 4 + 3 * 224 * (1 << 21)
    assert bench.box_point_ops(spec) == 3 * 37 + 7 + 11 + 3 + 10 == 142
    # the octant problem: eight states, flows along all three axes
    f = bench.box_octants(6, 4, 2)
    assert f.shape == (5, 2, 4, 6)
    assert len({tuple(f[:, k, j, i]) for k in range(2) for j in range(4) for i in range(6)}) == 8
    assert all(np.abs(f[c]).max() > 0 for c in (2, 3, 4))
    # a window whose "GPU" result is the oracle's own run has no error
    spec_w = dict(nx=10, ny=10, nz=10, q_xi=4, q_phi=8, q_p=3, tau=1e-2)
    ob = O.Box(**spec_w)
    init = bench.box_octants(10, 10, 10)
    ref = O.box_fields(ob, O.box_run(ob, init, 1))
    win = dict(name="box_octants/fp64", box=True, spec=spec_w, init=init, nsteps=1, pad=3, half=2,
               gpu=ref[:, 3:7, 3:7, 3:7].copy())
    _, errs = bench.cpu_baseline(dict(nx=1 << 20, q_xi=8, q_p=3, tau=1e-2), [win], target_s=0.05)
    e = errs["box_octants/fp64"]
    assert set(e) >= {"e", "n", "vx", "vy", "vz", "T00", "Txy"} and max(v["max"] for v in e.values()) == 0.0
