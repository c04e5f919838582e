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


def test_cpu_baseline_record():
    r = bench.cpu_baseline(dict(nx=1 << 20, q_xi=8, q_p=3, tau=1e-2), target_s=0.05)
    assert r["kind"] == "oracle" and r["cores"] >= 1 and r["value"] > 0
    assert r["unit"] == "cell*quad-point updates/s" and "steps in" in r["sample"]
