"""Pins of the oracle's three-dimensional model (every azimuthal node, any flow
direction) against what the paper and the mathematics fix: the perfect-fluid
moments of the truncated equilibrium (eq. mom_feq) for any 3D velocity, the
Landau frame as the timelike eigenvector of T^mu_nu (section Relativistic LB
equation) with its rotation covariance, the reductions to the plane (u^y = 0,
no y dependence) and to the tube (z dependence only), the symmetries of the
node set (x <-> y exchange, y reflection) and conservation of N^0 and
T^{0 mu}."""
import math

import numpy as np
import pytest

from oracle import oracle as O

RNG = np.random.default_rng(20240611)


def perfect_fluid(n, T, u):
    """N^mu and T^{mu nu} of a perfect massless fluid (e = 3P = 3nT) as the 14
    moments N0, N^i, T00, T^{0i}, T^{ij} (i <= j); metric (-, +, +, +)."""
    u = np.asarray(u, dtype=np.float64)
    g = math.sqrt(1.0 + u @ u)
    P, e = n * T, 3 * n * T
    m = [n * g] + list(n * u) + [(e + P) * g * g - P] + list((e + P) * g * u)
    for a in range(3):
        for b in range(a, 3):
            m.append((e + P) * u[a] * u[b] + (P if a == b else 0.0))
    return np.array(m)


def random_u(vmax):
    d = RNG.standard_normal(3)
    d /= np.linalg.norm(d)
    v = RNG.uniform(0.0, vmax)
    return d * v / math.sqrt(1 - v * v)


@pytest.mark.parametrize("q_xi,q_phi,q_p,n_v", [(6, 8, 3, 5), (8, 8, 4, 5), (7, 11, 3, 6), (9, 10, 5, 7)])
def test_equilibrium_moments_are_perfect_fluid_in_any_direction(q_xi, q_phi, q_p, n_v):
    box = O.Box(nx=1, ny=1, nz=1, q_xi=q_xi, q_phi=q_phi, q_p=q_p, n_v=n_v, n_p=min(2, q_p - 1))
    B = O.box_moments_weights(box)
    for _ in range(6):
        n, T, u = RNG.uniform(0.2, 3.0), RNG.uniform(0.3, 2.0), random_u(0.85)
        got = B @ O.box_feq_nodes(box, n, T, *u)
        ref = perfect_fluid(n, T, u)
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max(), (u, got - ref)


def test_too_few_azimuthal_nodes_break_the_moments():
    # Q_phi = N_v + 2 no longer integrates the degree N_v + 2 terms of T^{ij}
    box = O.Box(nx=1, ny=1, nz=1, q_xi=8, q_phi=7, q_p=3, n_v=5)
    B = O.box_moments_weights(box)
    u = np.array([0.8, 0.5, 0.1])
    err = np.abs(B @ O.box_feq_nodes(box, 1.0, 1.0, *u) - perfect_fluid(1.0, 1.0, u)).max()
    assert err > 1e-6


def test_landau_frame_round_trip_and_eigen_residual():
    for _ in range(8):
        n, T, u = RNG.uniform(0.2, 3.0), RNG.uniform(0.3, 2.0), random_u(0.95)
        r = O.landau3d(perfect_fluid(n, T, u))
        g = math.sqrt(1 + u @ u)
        assert abs(r[0] - 3 * n * T) < 1e-13 * 3 * n * T
        assert np.abs(r[1:4] - u / g).max() < 1e-13
        assert abs(r[5] - n) < 1e-13 * n and abs(r[6] - T) < 1e-13 * T
    # non-equilibrium moments of random positive distributions on the box
    # quadrature: T^mu_nu u^nu = -e u^mu
    box = O.Box(nx=1, ny=1, nz=1, q_xi=6, q_phi=8, q_p=3)
    B = O.box_moments_weights(box)
    for _ in range(8):
        m = B @ RNG.uniform(0.05, 1.0, box.Q)
        e, vx, vy, vz, gamma = O.landau3d(m)[:5]
        U = gamma * np.array([1.0, vx, vy, vz])
        T00, T0, Tij = m[4], m[5:8], np.zeros((3, 3))
        q = 8
        for a in range(3):
            for b in range(a, 3):
                Tij[a, b] = Tij[b, a] = m[q]
                q += 1
        Tup = np.zeros((4, 4))
        Tup[0, 0], Tup[0, 1:], Tup[1:, 0], Tup[1:, 1:] = T00, T0, T0, Tij
        Tmix = Tup @ np.diag([-1.0, 1.0, 1.0, 1.0])  # T^mu_nu
        res = Tmix @ U + e * U
        assert np.abs(res).max() < 1e-12 * T00


def test_landau_frame_is_rotation_covariant():
    box = O.Box(nx=1, ny=1, nz=1, q_xi=6, q_phi=8, q_p=3)
    B = O.box_moments_weights(box)
    for _ in range(6):
        m = B @ RNG.uniform(0.05, 1.0, box.Q)
        Rm, _ = np.linalg.qr(RNG.standard_normal((3, 3)))
        N, T0 = m[1:4], m[5:8]
        Tij = np.zeros((3, 3))
        q = 8
        for a in range(3):
            for b in range(a, 3):
                Tij[a, b] = Tij[b, a] = m[q]
                q += 1
        T2 = Rm @ Tij @ Rm.T
        m2 = np.concatenate([[m[0]], Rm @ N, [m[4]], Rm @ T0, [T2[a, b] for a in range(3) for b in range(a, 3)]])
        r1, r2 = O.landau3d(m), O.landau3d(m2)
        assert abs(r1[0] - r2[0]) < 1e-13 * r1[0] and abs(r1[5] - r2[5]) < 1e-13 * r1[5]
        assert np.abs(Rm @ r1[1:4] - r2[1:4]).max() < 1e-13


def _quadrant_fields(nx, nz, ny=1):
    x = -0.5 + (np.arange(nx) + 0.5) / nx
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    X, Z = np.meshgrid(x, z)
    f = np.zeros((5, nz, ny, nx))
    states = {(0, 0): (1.0, 1.0, 0.0, 0.0), (1, 0): (0.3, 0.5, 0.2, 0.0),
              (0, 1): (0.4, 0.6, 0.0, -0.3), (1, 1): (0.1, 0.125, 0.1, 0.1)}
    for (a, b), st in states.items():
        mk = ((X >= 0) == bool(a)) & ((Z >= 0) == bool(b))
        for y in range(ny):
            f[0, :, y][mk], f[1, :, y][mk], f[2, :, y][mk], f[4, :, y][mk] = st
    return f


def test_box_without_y_dependence_reduces_to_the_plane():
    nx, nz, steps = 14, 12, 4
    kw = dict(q_xi=6, q_phi=8, q_p=3, tau=1e-2)
    dt = 0.5 / (nx + nz)
    box = O.Box(nx=nx, ny=1, nz=nz, dt=dt, **kw)
    pl = O.Plane(nx=nx, nz=nz, dt=dt, **kw)
    f = _quadrant_fields(nx, nz)
    fb = O.box_fields(box, O.box_run(box, f, steps))[:, :, 0, :]
    fp = O.plane_fields(pl, O.plane_run(pl, f[[0, 1, 2, 4], :, 0, :], steps))
    # plane rows N0, Nx, Nz, T00, T0x, T0z, Txx, Txz, Tzz, e, n, vx, vz, T
    pairs = [(0, 0), (1, 1), (3, 2), (4, 3), (5, 4), (7, 5), (8, 6), (10, 7), (13, 8), (14, 9), (15, 10), (16, 11),
             (18, 12), (19, 13)]
    for kb, kp in pairs:
        scale = max(np.abs(fp[kp]).max(), 1e-3)
        assert np.abs(fb[kb] - fp[kp]).max() < 1e-13 * scale, (kb, kp)
    # y components vanish (mirror-symmetric nodes carry equal values)
    for kb in (2, 6, 9, 12, 17):
        assert np.abs(fb[kb]).max() < 1e-14 * np.abs(fb[4]).max()


def test_box_varying_along_z_only_reduces_to_the_tube():
    nz, steps = 60, 6
    box = O.Box(nx=1, ny=1, nz=nz, q_xi=8, q_phi=8, q_p=3, tau=1e-2, dt=0.5 / nz)
    t = O.Tube(nx=nz, q_xi=8, q_p=3, tau=1e-2, dt=0.5 / nz)
    z = box.centres()[2]
    f = np.zeros((5, nz, 1, 1))
    left = z < 0
    f[0, :, 0, 0] = np.where(left, 1.0, 0.1)
    f[1, :, 0, 0] = np.where(left, 1.0, 0.125)
    f[4, :, 0, 0] = np.where(left, 0.3, -0.2)
    fb = O.box_fields(box, O.box_run(box, f, steps))[:, :, 0, 0]
    ft = O.fields(t, O.run(t, (1.0, 1.0, 0.3), (0.1, 0.125, -0.2), steps))
    for kb, kt in ((0, 0), (3, 1), (4, 2), (7, 3), (13, 4), (14, 5), (15, 6), (18, 7), (19, 8)):
        assert np.abs(fb[kb] - ft[kt]).max() < 1e-13 * np.abs(ft[kt]).max(), (kb, kt)


def _smooth_fields(nx, ny, nz):
    x = -0.5 + (np.arange(nx) + 0.5) / nx
    y = -0.5 + (np.arange(ny) + 0.5) / ny
    z = -0.5 + (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    blob = np.exp(-((X - 0.1) ** 2 + (Y + 0.05) ** 2 + Z ** 2) / 0.02)
    f = np.zeros((5, nz, ny, nx))
    f[0] = 1.0 + 0.5 * blob
    f[1] = 1.0 + 0.3 * blob
    f[2] = 0.2 + 0.1 * blob
    f[3] = -0.3 + 0.2 * blob * X
    f[4] = 0.05
    return f


def test_x_and_y_exchange_symmetry():
    # Q_phi = 8: phi -> pi/2 - phi maps the node set onto itself, so the
    # problem with x and y exchanged evolves into the exchanged solution
    box = O.Box(nx=10, ny=10, nz=4, q_xi=6, q_phi=8, q_p=3, tau=5e-3)
    f = _smooth_fields(10, 10, 4)
    g = f.transpose(0, 1, 3, 2)[[0, 1, 3, 2, 4]].copy()
    a = O.box_fields(box, O.box_run(box, f, 3))
    b = O.box_fields(box, O.box_run(box, g, 3))
    perm = [0, 2, 1, 3, 4, 6, 5, 7, 11, 9, 12, 8, 10, 13, 14, 15, 17, 16, 18, 19]
    bt = b[perm].transpose(0, 1, 3, 2)
    scale = np.abs(a).max(axis=(1, 2, 3))
    assert (np.abs(a - bt).max(axis=(1, 2, 3)) <= 1e-13 * np.maximum(scale, 1e-3)).all()


def test_y_reflection_symmetry():
    box = O.Box(nx=6, ny=9, nz=5, q_xi=6, q_phi=10, q_p=3, tau=5e-3)
    f = _smooth_fields(6, 9, 5)
    g = f[:, :, ::-1, :].copy()
    g[3] *= -1
    a = O.box_fields(box, O.box_run(box, f, 3))
    b = O.box_fields(box, O.box_run(box, g, 3))[:, :, ::-1, :]
    sign = np.ones(20)
    sign[[2, 6, 9, 12, 17]] = -1  # Ny, T0y, Txy, Tyz, v_y
    scale = np.abs(a).max(axis=(1, 2, 3))
    assert (np.abs(a - sign[:, None, None, None] * b).max(axis=(1, 2, 3)) <= 1e-13 * np.maximum(scale, 1e-3)).all()


def test_conservation_with_flow_in_every_direction():
    # a narrow blob on a uniform background moving with u^x, u^y, u^z != 0;
    # over one step (three stages of three-cell stencils) the outflow edges
    # stay uniform to 1e-10 and the boundary fluxes cancel pairwise
    n = 24
    box = O.Box(nx=n, ny=n, nz=n, q_xi=6, q_phi=8, q_p=3, tau=2e-2)
    f = np.zeros((5, n, n, n))
    x = -0.5 + (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    blob = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 0.003)
    f[0], f[1] = 0.5 + blob, 0.6 + 0.5 * blob
    f[2], f[3], f[4] = 0.1, -0.15, 0.05
    F0 = O.box_init(box, f)
    B = O.box_moments_weights(box)
    tot0 = np.tensordot(B, F0, axes=(1, 0)).sum(axis=(1, 2, 3))
    F = O.box_step(box, F0, 1)
    tot = np.tensordot(B, F, axes=(1, 0)).sum(axis=(1, 2, 3))
    for k in (0, 4, 5, 6, 7):  # N0, T00, T0x, T0y, T0z
        assert abs(tot[k] - tot0[k]) < 5e-14 * abs(tot0[4]), (k, tot[k] - tot0[k])
