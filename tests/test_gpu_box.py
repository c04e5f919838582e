"""Parity of the box (x, y, z) HIP path with the oracle's three-dimensional model.

Bars as for the tubes and planes: FP64 within 1e-12 normwise relative per field
and per quadrature row, FP32 within 1e-5.  Flows point in every direction
(u^x, u^y, u^z all non-zero), so every azimuthal node carries its own values.
"""
import math

import numpy as np
import pytest

from tests.helpers import normwise

pytestmark = pytest.mark.gpu

NAMES = ("N0", "Nx", "Ny", "Nz", "T00", "T0x", "T0y", "T0z", "Txx", "Txy", "Txz", "Tyy", "Tyz", "Tzz",
         "e", "n", "vx", "vy", "vz", "T")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def _specs(params):
    from oracle import oracle as O
    from paper_1608_03004_amd import BoxSpec
    return BoxSpec(**params), O.Box(**params)


def _grid(b):
    # Z, Y, X of shape [nz, ny, nx]
    x, y, z = b.centres()
    return np.meshgrid(z, y, x, indexing="ij")


def _blob(b, u=(0.2, -0.15, 0.1)):
    Z, Y, X = _grid(b)
    r2 = (X - 0.1) ** 2 + (Y + 0.05) ** 2 + (Z - 0.02) ** 2
    f = np.zeros((5, b.nz, b.ny, b.nx))
    f[0] = 0.2 + np.exp(-r2 / 0.02)
    f[1] = 0.4 + 0.6 * np.exp(-r2 / 0.05)
    f[2] = u[0] + 0.3 * np.sin(2 * math.pi * X) * np.exp(-r2 / 0.05)
    f[3] = u[1] + 0.2 * np.cos(2 * math.pi * Z) * np.exp(-r2 / 0.05)
    f[4] = u[2]
    return f


def _octants(b):
    # a 3D Riemann problem: eight constant states meeting at the origin
    Z, Y, X = _grid(b)
    f = np.zeros((5, b.nz, b.ny, b.nx))
    for a in (0, 1):
        for c in (0, 1):
            for d in (0, 1):
                m = ((X >= 0) == bool(a)) & ((Y >= 0) == bool(c)) & ((Z >= 0) == bool(d))
                P = 1.0 if (a + c + d) % 2 == 0 else 0.2
                n = 1.0 if (a + c + d) % 2 == 0 else 0.3
                st = (P * (1 + 0.2 * a), n, 0.1 * (a - c), 0.15 * (c - d), 0.12 * (d - a))
                for k in range(5):
                    f[k][m] = st[k]
    return f


def _waves(b):
    Z, Y, X = _grid(b)
    f = np.zeros((5, b.nz, b.ny, b.nx))
    f[0] = 0.6 + 0.3 * np.sin(6 * math.pi * X) * np.cos(4 * math.pi * Z) * np.cos(2 * math.pi * Y)
    f[1] = 0.7 + 0.2 * np.cos(6 * math.pi * X + 1.0) * np.sin(4 * math.pi * Z)
    f[2] = 0.2 * np.sin(2 * math.pi * (X + Z))
    f[3] = 0.15 * np.cos(2 * math.pi * (Y - X))
    f[4] = 0.15 * np.cos(2 * math.pi * (X - Z + Y))
    return f


def _fields_err(gpu, ref):
    out = {}
    for k, name in enumerate(NAMES):
        out[name] = np.abs(gpu[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300)
    return out


def _fields_err_tensor_scale(gpu, ref):
    # error of each component relative to its tensor's scale (N^mu to N^0,
    # T^{mu nu} and e to T^00, v to the speed of light)
    scale = {k: np.abs(ref[NAMES.index(k)]).max() for k in ("N0", "T00", "n", "T")}
    ref_of = {"N0": "N0", "Nx": "N0", "Ny": "N0", "Nz": "N0", "n": "n", "T": "T"}
    out = {}
    for k, name in enumerate(NAMES):
        s = 1.0 if name in ("vx", "vy", "vz") else scale[ref_of.get(name, "T00")]
        out[name] = np.abs(gpu[k] - ref[k]).max() / s
    return out


CASES = [
    (dict(nx=20, ny=12, nz=10, q_xi=6, q_phi=8, q_p=3, tau=1e-2), "blob"),
    (dict(nx=70, ny=6, nz=5, q_xi=6, q_phi=9, q_p=3, tau=3e-2), "octants"),     # ragged x and y tiles, odd q_phi
    (dict(nx=10, ny=9, nz=8, q_xi=6, q_phi=10, q_p=4, tau=5e-2), "octants"),    # Q_p = 4 group
    (dict(nx=8, ny=7, nz=6, q_xi=7, q_phi=10, q_p=5, n_p=3, n_v=7, tau=1e-1), "blob"),  # generic group
    (dict(nx=12, ny=10, nz=8, q_xi=6, q_phi=8, q_p=3, tau=math.inf), "blob"),   # collisionless
    (dict(nx=5, ny=1, nz=3, q_xi=4, q_phi=8, q_p=3, tau=1e-2), "octants"),      # degenerate extents
    (dict(nx=9, ny=13, nz=11, q_xi=5, q_phi=11, q_p=3, tau=2e-2), "blob"),      # odd everything
    (dict(nx=6, ny=5, nz=4, q_xi=16, q_phi=64, q_p=8, n_p=3, n_v=7, tau=1e-2), "blob"),  # Q = 8 x 16 x 64
]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_box_against_oracle(torch_cuda, case, precision, tol):
    from oracle import oracle as O
    from paper_1608_03004_amd import Box
    params, init = CASES[case]
    spec, ob = _specs(params)
    f0 = _blob(ob) if init == "blob" else _octants(ob)
    gb = Box(spec, precision=precision)
    gb.set_initial_fields(f0)
    F0 = O.box_init(ob, f0)
    assert normwise(gb.state_array().reshape(spec.Q, -1), F0.reshape(spec.Q, -1)).max() < tol
    assert max(_fields_err(gb.moments(), O.box_fields(ob, F0)).values()) < tol
    nsteps = 6
    gb.step(nsteps)
    F = O.box_step(ob, F0, nsteps)
    errs = _fields_err(gb.moments(), O.box_fields(ob, F))
    print(f"[box case {case} {precision}] " + " ".join(f"{k}:{v:.1e}" for k, v in errs.items()), flush=True)
    assert max(errs.values()) < tol, errs
    assert normwise(gb.state_array().reshape(spec.Q, -1), F.reshape(spec.Q, -1)).max() < tol
    assert abs(gb.info()["time"] - nsteps * ob.step_dt) < 1e-15
    assert gb.info()["Q"] == spec.Q


def test_box_with_one_y_cell_and_no_y_flow_matches_the_plane(torch_cuda):
    # ny = 1 and u^y = 0: the box (every azimuthal node evolved) against the
    # GPU plane (mirrored nodes folded)
    from oracle import oracle as O
    from paper_1608_03004_amd import Box, BoxSpec, Plane, PlaneSpec
    q = dict(q_xi=8, q_phi=8, q_p=3, tau=2e-2)
    pl = Plane(PlaneSpec(nx=24, nz=20, **q), precision="fp64")
    opl = O.Plane(nx=24, nz=20, **q)
    x, z = opl.centres()
    X, Z = np.meshgrid(x, z)
    f2 = np.zeros((4, 20, 24))
    f2[0] = 0.3 + np.exp(-((X - 0.1) ** 2 + Z ** 2) / 0.03)
    f2[1] = 0.5 + 0.4 * np.exp(-(X ** 2 + (Z + 0.1) ** 2) / 0.05)
    f2[2] = 0.2 * np.sin(2 * math.pi * X)
    f2[3] = -0.15 + 0.1 * np.cos(2 * math.pi * Z)
    pl.set_initial_fields(f2)
    bx = Box(BoxSpec(nx=24, ny=1, nz=20, dt=pl.info()["dt"], **q), precision="fp64")
    f3 = np.zeros((5, 20, 1, 24))
    f3[0, :, 0], f3[1, :, 0], f3[2, :, 0], f3[4, :, 0] = f2[0], f2[1], f2[2], f2[3]
    bx.set_initial_fields(f3)
    pl.step(8)
    bx.step(8)
    pf, bf = pl.moments(), bx.moments()[:, :, 0, :]
    # plane order N0 Nx Nz T00 T0x T0z Txx Txz Tzz e n vx vz T
    pairs = ((0, 0), (1, 1), (2, 3), (3, 4), (4, 5), (5, 7), (6, 8), (7, 10), (8, 13), (9, 14), (10, 15),
             (11, 16), (12, 18), (13, 19))
    for a2, a3 in pairs:
        assert np.abs(bf[a3] - pf[a2]).max() <= 1e-12 * max(np.abs(pf[a2]).max(), 1e-300), (a2, a3)
    # the y components vanish by symmetry (to rounding)
    for a3 in (2, 6, 9, 12, 17):
        assert np.abs(bf[a3]).max() < 1e-14, a3


def test_box_varying_along_z_only_matches_the_tube_lattice(torch_cuda):
    # a z-Sod tube in every (x, y) column with u along z, against the GPU 1D path
    from paper_1608_03004_amd import Box, BoxSpec, Lattice, Tube
    bx = Box(BoxSpec(nx=3, ny=5, nz=128, q_xi=8, q_phi=8, q_p=3, tau=1e-2), precision="fp64")
    z = -0.5 + (np.arange(128) + 0.5) / 128
    f = np.zeros((5, 128, 5, 3))
    f[0] = np.where(z < 0, 1.0, 0.1)[:, None, None]
    f[1] = np.where(z < 0, 1.0, 0.125)[:, None, None]
    f[4] = 0.2
    bx.set_initial_fields(f)
    bx.step(20)
    bf = bx.moments()
    lat = Lattice([Tube(nx=128, q_xi=8, q_p=3, tau=1e-2, dt=bx.info()["dt"])], precision="fp64")
    lat.set_initial_state((1.0, 1.0, 0.2), (0.1, 0.125, 0.2))
    lat.step(20)
    tf = lat.moments(0)
    # tube order N0 Nz T00 T0z Tzz e n v T
    for a3, a1 in ((0, 0), (3, 1), (4, 2), (7, 3), (13, 4), (14, 5), (15, 6), (18, 7), (19, 8)):
        assert np.abs(bf[a3] - tf[a1][:, None, None]).max() < 1e-12 * np.abs(tf[a1]).max(), a3
    for a3 in (1, 2, 5, 6, 9, 10, 12, 16, 17):
        assert np.abs(bf[a3]).max() < 1e-14, a3
    # T^xx = T^yy (isotropy about z)
    assert np.abs(bf[8] - bf[11]).max() < 1e-13 * np.abs(bf[8]).max()


def test_box_quarter_turn_about_z(torch_cuda):
    # q_phi divisible by 4: the node set is invariant under the quarter turn
    # (x, y) -> (-y, x), so a rotated initial state gives the rotated fields
    from paper_1608_03004_amd import Box, BoxSpec
    spec = BoxSpec(nx=16, ny=16, nz=6, q_xi=6, q_phi=8, q_p=3, tau=2e-2)
    x = -0.5 + (np.arange(16) + 0.5) / 16
    z = -0.5 + (np.arange(6) + 0.5) / 6
    Z, Y, X = np.meshgrid(z, x, x, indexing="ij")
    f = np.zeros((5, 6, 16, 16))
    f[0] = 0.3 + np.exp(-((X - 0.12) ** 2 + (Y + 0.2) ** 2 + Z ** 2) / 0.03)
    f[1] = 0.5 + 0.3 * np.exp(-((X + 0.1) ** 2 + Y ** 2) / 0.05)
    f[2] = 0.2 * np.sin(2 * math.pi * X) * np.cos(math.pi * Y)
    f[3] = -0.1 + 0.1 * np.cos(2 * math.pi * Y)
    f[4] = 0.05 * np.sin(2 * math.pi * Z)
    # the rotated scalar g(x, y) = f(y, -x); on the symmetric grid, g[.., j, i]
    # = f[.., n-1-i, j] (axes y, x)
    def rot(a):
        return np.rot90(a, k=-1, axes=(1, 2))
    g = np.zeros_like(f)
    g[0], g[1], g[4] = rot(f[0]), rot(f[1]), rot(f[4])
    g[2], g[3] = -rot(f[3]), rot(f[2])   # u' = (-u^y, u^x)
    a = Box(spec, precision="fp64")
    a.set_initial_fields(f)
    b = Box(spec, precision="fp64")
    b.set_initial_fields(g)
    a.step(5)
    b.step(5)
    fa, fb = a.moments(), b.moments()
    N = {n: k for k, n in enumerate(NAMES)}
    expect = {"N0": rot(fa[N["N0"]]), "Nx": -rot(fa[N["Ny"]]), "Ny": rot(fa[N["Nx"]]), "Nz": rot(fa[N["Nz"]]),
              "T00": rot(fa[N["T00"]]), "Txx": rot(fa[N["Tyy"]]), "Tyy": rot(fa[N["Txx"]]),
              "Txy": -rot(fa[N["Txy"]]), "Tzz": rot(fa[N["Tzz"]]), "vx": -rot(fa[N["vy"]]), "vy": rot(fa[N["vx"]]),
              "n": rot(fa[N["n"]]), "T": rot(fa[N["T"]])}
    for name, e in expect.items():
        assert np.abs(fb[N[name]] - e).max() < 1e-12 * max(np.abs(e).max(), 1e-3), name


def test_box_state_round_trip_and_zero_steps(torch_cuda):
    from oracle import oracle as O
    from paper_1608_03004_amd import Box
    params = dict(nx=33, ny=7, nz=9, q_xi=6, q_phi=8, q_p=3, tau=2e-2)
    spec, ob = _specs(params)
    gb = Box(spec, precision="fp64")
    gb.set_initial_fields(_octants(ob))
    gb.step(0)
    gb.step(3)
    snap = gb.get_state().clone()
    gb.step(3)
    direct = gb.state_array()
    gb.set_state(snap)
    gb.step(3)
    assert np.array_equal(gb.state_array(), direct)
    # a host state written through load_array evolves like the oracle
    F0 = O.box_run(ob, _blob(ob), 2)
    gb.set_state(gb.load_array(F0))
    gb.step(2)
    assert normwise(gb.state_array().reshape(spec.Q, -1), O.box_step(ob, F0, 2).reshape(spec.Q, -1)).max() < 1e-12


def test_box_nonphysical_state_raises_sticky_flag(torch_cuda):
    from paper_1608_03004_amd import Box, RLBError
    spec, ob = _specs(dict(nx=10, ny=6, nz=5, q_xi=6, q_phi=8, q_p=3, tau=1e-2))
    gb = Box(spec)
    f = _blob(ob)
    gb.set_initial_fields(f)
    bad = gb.get_state().clone()
    bad.mul_(-1.0)  # a negative distribution: e < 0 in every cell
    gb.set_state(bad)
    gb.step(1)
    with pytest.raises(RLBError) as ei:
        gb.check()
    assert ei.value.status == -2
    assert gb.flags()["nonphysical"]
    gb.set_initial_fields(f)  # a fresh initial state clears the flag
    gb.step(1)
    gb.check()


def test_box_full_size_windows(torch_cuda):
    # 128^3 cells, Q = 3 x 8 x 8 = 192, FP32 (the benchmarked box): a window at
    # the centre and one at the upper corner (outflow faces, largest indices)
    # follow the oracle on windows widened by 9 cells per step inward
    from oracle import oracle as O
    from paper_1608_03004_amd import Box, BoxSpec
    n, nsteps, w = 128, 2, 4
    pad = 9 * nsteps
    q = dict(q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gb = Box(BoxSpec(nx=n, ny=n, nz=n, **q), precision="fp32")
    gb.set_initial_fields(_waves(O.Box(nx=n, ny=n, nz=n, **q)))
    gb.step(nsteps)
    d = 1.0 / n
    for name, (a, b) in (("centre", (n // 2 - w, n // 2 + w)), ("corner", (n - 2 * w, n))):
        lo, hi = a - pad, min(b + pad, n)
        full = gb.fields()[:, a:b, a:b, a:b].cpu().numpy()
        win = O.Box(nx=hi - lo, ny=hi - lo, nz=hi - lo, x_min=-0.5 + lo * d, x_max=-0.5 + hi * d,
                    y_min=-0.5 + lo * d, y_max=-0.5 + hi * d, z_min=-0.5 + lo * d, z_max=-0.5 + hi * d,
                    dt=gb.info()["dt"], **q)
        ref = O.box_fields(win, O.box_run(win, _waves(win), nsteps))[:, a - lo:b - lo, a - lo:b - lo, a - lo:b - lo]
        errs = _fields_err_tensor_scale(full, ref)
        print(f"[box 128^3 fp32 {name} window] " + " ".join(f"{k}:{v:.1e}" for k, v in errs.items()), flush=True)
        assert max(errs.values()) < 1e-5, (name, errs)


def test_box_max_size_windows(torch_cuda):
    # the largest box the library accepts, 512 x 512 x 256 = 2^26 cells with
    # Q = 192, FP32 (three states of 52 GB): a window at the centre and one at
    # the upper corner (outflow faces, largest indices) follow the oracle on
    # windows widened by 9 cells per step inward
    from oracle import oracle as O
    from paper_1608_03004_amd import Box, BoxSpec
    nx, ny, nz, nsteps, w = 512, 512, 256, 2, 4
    pad = 9 * nsteps
    q = dict(q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gb = Box(BoxSpec(nx=nx, ny=ny, nz=nz, **q), precision="fp32")
    gb.set_initial_fields(_waves(O.Box(nx=nx, ny=ny, nz=nz, **q)))
    gb.step(nsteps)
    d = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    for name, c in (("centre", (nx // 2, ny // 2, nz // 2)), ("corner", (nx - w, ny - w, nz - w))):
        a = [ci - w for ci in c]
        b = [ci + w for ci in c]
        lo = [ai - pad for ai in a]
        hi = [min(bi + pad, n) for bi, n in zip(b, (nx, ny, nz))]
        full = gb.fields()[:, a[2]:b[2], a[1]:b[1], a[0]:b[0]].cpu().numpy()
        win = O.Box(nx=hi[0] - lo[0], ny=hi[1] - lo[1], nz=hi[2] - lo[2],
                    x_min=-0.5 + lo[0] * d[0], x_max=-0.5 + hi[0] * d[0], y_min=-0.5 + lo[1] * d[1],
                    y_max=-0.5 + hi[1] * d[1], z_min=-0.5 + lo[2] * d[2], z_max=-0.5 + hi[2] * d[2],
                    dt=gb.info()["dt"], **q)
        ref = O.box_fields(win, O.box_run(win, _waves(win), nsteps))
        ref = ref[:, a[2] - lo[2]:b[2] - lo[2], a[1] - lo[1]:b[1] - lo[1], a[0] - lo[0]:b[0] - lo[0]]
        errs = _fields_err_tensor_scale(full, ref)
        print(f"[box 2^26 fp32 {name} window] " + " ".join(f"{k}:{v:.1e}" for k, v in errs.items()), flush=True)
        assert max(errs.values()) < 1e-5, (name, errs)
    del gb
    torch_cuda.cuda.empty_cache()


def test_box_full_size_fp64_window(torch_cuda):
    # the benchmarked 128^3 box in FP64 on a centre window, to the FP64 bar
    from oracle import oracle as O
    from paper_1608_03004_amd import Box, BoxSpec
    n, nsteps, w = 128, 2, 4
    pad = 9 * nsteps
    q = dict(q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    gb = Box(BoxSpec(nx=n, ny=n, nz=n, **q), precision="fp64")
    gb.set_initial_fields(_octants(O.Box(nx=n, ny=n, nz=n, **q)))
    gb.step(nsteps)
    a, b = n // 2 - w, n // 2 + w
    lo, hi = a - pad, b + pad
    d = 1.0 / n
    full = gb.fields()[:, a:b, a:b, a:b].cpu().numpy()
    win = O.Box(nx=hi - lo, ny=hi - lo, nz=hi - lo, x_min=-0.5 + lo * d, x_max=-0.5 + hi * d,
                y_min=-0.5 + lo * d, y_max=-0.5 + hi * d, z_min=-0.5 + lo * d, z_max=-0.5 + hi * d,
                dt=gb.info()["dt"], **q)
    ref = O.box_fields(win, O.box_run(win, _octants(win), nsteps))[:, a - lo:b - lo, a - lo:b - lo, a - lo:b - lo]
    errs = _fields_err_tensor_scale(full, ref)
    print("[box 128^3 fp64 centre window] " + " ".join(f"{k}:{v:.1e}" for k, v in errs.items()), flush=True)
    assert max(errs.values()) < 1e-12, errs
