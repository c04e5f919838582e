"""Parity of the plane (x, z) HIP path with the oracle's multi-dimensional model.

Bars as for the tubes: FP64 within 1e-12 normwise relative per field and per
quadrature row, FP32 within 1e-5.
"""
import math

import numpy as np
import pytest

from tests.helpers import normwise

pytestmark = pytest.mark.gpu

NAMES = ("N0", "Nx", "Nz", "T00", "T0x", "T0z", "Txx", "Txz", "Tzz", "e", "n", "vx", "vz", "T")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def _specs(params):
    from oracle import oracle as O
    from paper_1608_03004_amd import PlaneSpec
    return PlaneSpec(**params), O.Plane(**params)


def _blob(pl, ux=0.0, uz=0.0):
    x, z = pl.centres()
    r2 = (x[None, :] - 0.1) ** 2 + (z[:, None] + 0.05) ** 2
    f = np.zeros((4, pl.nz, pl.nx))
    f[0] = 0.2 + np.exp(-r2 / 0.02)
    f[1] = 0.4 + 0.6 * np.exp(-r2 / 0.05)
    f[2] = ux + 0.3 * np.sin(2 * math.pi * x)[None, :] * np.exp(-r2 / 0.05)
    f[3] = uz
    return f


def _quadrants(pl):
    # a 2D Riemann problem: four constant states meeting at the origin
    x, z = pl.centres()
    X, Z = np.meshgrid(x, z)
    st = {(0, 0): (1.0, 1.0, 0.0, 0.0), (1, 0): (0.3, 0.5, 0.2, 0.0),
          (0, 1): (0.4, 0.6, 0.0, -0.3), (1, 1): (0.1, 0.125, 0.1, 0.1)}
    f = np.zeros((4, pl.nz, pl.nx))
    for (a, b), s in st.items():
        m = ((X >= 0) == bool(a)) & ((Z >= 0) == bool(b))
        for c in range(4):
            f[c][m] = s[c]
    return f


def _waves(pl):
    # smooth variations everywhere, so that every window (edges included) has
    # structure
    x, z = pl.centres()
    X, Z = np.meshgrid(x, z)
    f = np.zeros((4, pl.nz, pl.nx))
    f[0] = 0.6 + 0.3 * np.sin(6 * math.pi * X) * np.cos(4 * math.pi * Z)
    f[1] = 0.7 + 0.2 * np.cos(6 * math.pi * X + 1.0) * np.sin(4 * math.pi * Z)
    f[2] = 0.2 * np.sin(2 * math.pi * (X + Z))
    f[3] = 0.15 * np.cos(2 * math.pi * (X - Z))
    return f


def _fields_err_tensor_scale(gpu, ref):
    # error of each component relative to its tensor's scale (N^mu to N^0,
    # T^{mu nu} and e to T^00, v to the speed of light), for windows where a
    # component passes through zero
    scale = {k: np.abs(ref[NAMES.index(k)]).max() for k in ("N0", "T00", "n", "T")}
    ref_of = {"N0": "N0", "Nx": "N0", "Nz": "N0", "n": "n", "T": "T"}
    out = {}
    for k, name in enumerate(NAMES):
        s = 1.0 if name in ("vx", "vz") else scale[ref_of.get(name, "T00")]
        out[name] = np.abs(gpu[k] - ref[k]).max() / s
    return out


def _fields_err(gpu, ref):
    out = {}
    for k, name in enumerate(NAMES):
        out[name] = np.abs(gpu[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300)
    return out


CASES = [
    (dict(nx=40, nz=36, q_xi=8, q_phi=8, q_p=3, tau=1e-2), "blob"),
    (dict(nx=70, nz=13, q_xi=6, q_phi=9, q_p=3, tau=3e-2), "quadrants"),     # ragged tiles, odd q_phi
    (dict(nx=24, nz=24, q_xi=8, q_phi=10, q_p=4, tau=5e-2), "quadrants"),    # Q_p = 4 group
    (dict(nx=16, nz=20, q_xi=7, q_phi=10, q_p=5, n_p=3, n_v=7, tau=1e-1), "blob"),  # generic group
    (dict(nx=20, nz=18, q_xi=8, q_phi=8, q_p=3, tau=math.inf), "blob"),      # collisionless
    (dict(nx=8, nz=8, q_xi=6, q_phi=8, q_p=3, tau=1e-2), "quadrants"),       # the smallest plane
    (dict(nx=9, nz=67, q_xi=7, q_phi=8, q_p=3, tau=2e-2), "blob"),           # thin, odd q_xi, ragged tile rows
    (dict(nx=130, nz=9, q_xi=6, q_phi=9, q_p=4, tau=5e-3), "quadrants"),     # three tile columns, one row
    (dict(nx=12, nz=10, q_xi=64, q_phi=64, q_p=8, n_p=3, n_v=7, tau=1e-2), "blob"),  # Q = 8 x 64 x 33
]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_plane_against_oracle(torch_cuda, case, precision, tol):
    from oracle import oracle as O
    from paper_1608_03004_amd import Plane
    params, init = CASES[case]
    spec, opl = _specs(params)
    f0 = _blob(opl, 0.2, -0.1) if init == "blob" else _quadrants(opl)
    gp = Plane(spec, precision=precision)
    gp.set_initial_fields(f0)
    F0 = O.plane_init(opl, f0)
    assert normwise(gp.state_array().reshape(spec.Q, -1), F0.reshape(spec.Q, -1)).max() < tol
    nsteps = 10
    gp.step(nsteps)
    F = O.plane_step(opl, F0, nsteps)
    errs = _fields_err(gp.moments(), O.plane_fields(opl, F))
    print(f"[plane case {case} {precision}] " + " ".join(f"{k}:{v:.1e}" for k, v in errs.items()), flush=True)
    assert max(errs.values()) < tol, errs
    assert normwise(gp.state_array().reshape(spec.Q, -1), F.reshape(spec.Q, -1)).max() < tol
    assert abs(gp.info()["time"] - nsteps * opl.step_dt) < 1e-15


def test_plane_without_x_dependence_matches_the_tube_lattice(torch_cuda):
    # the GPU plane with a z-Sod tube in every column against the GPU 1D path
    from paper_1608_03004_amd import Lattice, Plane, PlaneSpec, Tube
    spec = PlaneSpec(nx=8, nz=256, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gp = Plane(spec, precision="fp64")
    z = -0.5 + (np.arange(256) + 0.5) / 256
    f = np.zeros((4, 256, 8))
    f[0] = np.where(z < 0, 1.0, 0.1)[:, None]
    f[1] = np.where(z < 0, 1.0, 0.125)[:, None]
    f[3] = 0.2
    gp.set_initial_fields(f)
    gp.step(30)
    pf = gp.moments()
    lat = Lattice([Tube(nx=256, q_xi=8, q_p=3, tau=1e-2, dt=gp.info()["dt"])], precision="fp64")
    lat.set_initial_state((1.0, 1.0, 0.2), (0.1, 0.125, 0.2))
    lat.step(30)
    tf = lat.moments(0)
    for a2, a1 in ((0, 0), (2, 1), (3, 2), (5, 3), (8, 4), (9, 5), (10, 6), (12, 7), (13, 8)):
        assert np.abs(pf[a2] - tf[a1][:, None]).max() < 1e-12 * np.abs(tf[a1]).max(), a2
    assert np.abs(pf[1]).max() < 1e-14 and np.abs(pf[4]).max() < 1e-14


def test_plane_state_round_trip_and_zero_steps(torch_cuda):
    from oracle import oracle as O
    from paper_1608_03004_amd import Plane
    params = dict(nx=33, nz=21, q_xi=6, q_phi=8, q_p=3, tau=2e-2)
    spec, opl = _specs(params)
    gp = Plane(spec, precision="fp64")
    gp.set_initial_fields(_quadrants(opl))
    gp.step(0)
    gp.step(4)
    snap = gp.get_state().clone()
    gp.step(4)
    direct = gp.state_array()
    gp.set_state(snap)
    gp.step(4)
    assert np.array_equal(gp.state_array(), direct)
    # a host state written through load_array evolves like the oracle
    F0 = O.plane_run(opl, _blob(opl), 3)
    gp.set_state(gp.load_array(F0))
    gp.step(3)
    assert normwise(gp.state_array().reshape(spec.Q, -1), O.plane_step(opl, F0, 3).reshape(spec.Q, -1)).max() < 1e-12


def test_plane_full_size_window(torch_cuda):
    # 1024 x 1024 cells, Q = 3 x 8 x 5: the centre of a quadrant problem follows
    # the oracle on a window widened by 9 cells per step in x and z
    from oracle import oracle as O
    from paper_1608_03004_amd import Plane, PlaneSpec
    n, nsteps, half = 1024, 2, 16
    spec = PlaneSpec(nx=n, nz=n, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gp = Plane(spec, precision="fp32")
    opl_full = O.Plane(nx=n, nz=n, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gp.set_initial_fields(_quadrants(opl_full))
    gp.step(nsteps)
    full = gp.fields()[:, n // 2 - half: n // 2 + half, n // 2 - half: n // 2 + half].cpu().numpy()
    pad = 9 * nsteps
    a, b = n // 2 - half - pad, n // 2 + half + pad
    d = 1.0 / n
    w = O.Plane(nx=b - a, nz=b - a, q_xi=8, q_phi=8, q_p=3, tau=1e-2, x_min=-0.5 + a * d, x_max=-0.5 + b * d,
                z_min=-0.5 + a * d, z_max=-0.5 + b * d, dt=gp.info()["dt"])
    ref = O.plane_fields(w, O.plane_run(w, _quadrants(w), nsteps))[:, pad:pad + 2 * half, pad:pad + 2 * half]
    errs = _fields_err(full, ref)
    print("[plane 1024^2 fp32 window] " + " ".join(f"{k}:{v:.1e}" for k, v in errs.items()), flush=True)
    assert max(errs.values()) < 1e-5, errs


def test_plane_max_size_windows(torch_cuda):
    # the largest plane the library accepts, 8192 x 8192 = 2^26 cells, Q = 120,
    # FP32 (three states of 32 GB), smooth data: a window at the centre and
    # one at the upper corner (outflow edges, largest indices) follow the
    # oracle on windows widened by 9 cells per step inward
    from oracle import oracle as O
    from paper_1608_03004_amd import Plane, PlaneSpec
    n, nsteps, w = 8192, 2, 24
    pad = 9 * nsteps
    spec = PlaneSpec(nx=n, nz=n, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gp = Plane(spec, precision="fp32")
    gp.set_initial_fields(_waves(O.Plane(nx=n, nz=n, q_xi=8, q_phi=8, q_p=3, tau=1e-2)))
    gp.step(nsteps)
    d = 1.0 / n
    for name, (a, b) in (("centre", (n // 2 - w, n // 2 + w)), ("corner", (n - 2 * w, n))):
        lo, hi = a - pad, min(b + pad, n)
        full = gp.fields()[:, a:b, a:b].cpu().numpy()
        win = O.Plane(nx=hi - lo, nz=hi - lo, q_xi=8, q_phi=8, q_p=3, tau=1e-2, x_min=-0.5 + lo * d,
                      x_max=-0.5 + hi * d, z_min=-0.5 + lo * d, z_max=-0.5 + hi * d, dt=gp.info()["dt"])
        ref = O.plane_fields(win, O.plane_run(win, _waves(win), nsteps))[:, a - lo:b - lo, a - lo:b - lo]
        errs = _fields_err_tensor_scale(full, ref)
        print(f"[plane 8192^2 fp32 {name} window] " + " ".join(f"{k}:{v:.1e}" for k, v in errs.items()), flush=True)
        assert max(errs.values()) < 1e-5, (name, errs)


def test_plane_nonphysical_state_raises_sticky_flag(torch_cuda):
    from paper_1608_03004_amd import Plane, RLBError
    spec, opl = _specs(dict(nx=16, nz=16, q_xi=6, q_phi=8, q_p=3, tau=1e-2))
    gp = Plane(spec)
    f = _blob(opl)
    gp.set_initial_fields(f)
    bad = gp.get_state().clone()
    bad.mul_(-1.0)  # a negative distribution: e < 0 in every cell
    gp.set_state(bad)
    gp.step(1)
    with pytest.raises(RLBError) as ei:
        gp.check()
    assert ei.value.status == -2
    gp.set_initial_fields(f)  # a fresh initial state clears the flag
    gp.step(1)
    gp.check()
