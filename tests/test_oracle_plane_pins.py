"""Pins of the oracle's multi-dimensional (plane) model against what the paper
and the mathematics fix, independently of the oracle's own formulas:
perfect-fluid moments of the equilibrium for any flow direction (and their
failure when the azimuthal rule is too coarse), the moment-recovery property
(eq. mom_feq) against the exact Maxwell-Juettner distribution on independent
high-order rules, the Landau frame as the timelike eigenvector of T^mu_nu
(eigen-residual, rotation covariance, the 1D closed form), reduction of a
plane without x dependence to the 1D tube, mirror symmetry and conservation."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O


def _perfect_fluid9(n, T, ux, uz):
    g = math.sqrt(1 + ux * ux + uz * uz)
    e, P = 3 * n * T, n * T
    u = (g, ux, uz)
    eta = (-1.0, 1.0, 1.0)

    def t(a, b):
        return (e + P) * u[a] * u[b] + (P * eta[a] if a == b else 0.0)
    return np.array([n * g, n * ux, n * uz, t(0, 0), t(0, 1), t(0, 2), t(1, 1), t(1, 2), t(2, 2)])


@pytest.mark.parametrize("qx,qphi,qp,nv", [(8, 8, 3, 5), (5, 9, 3, 5), (16, 12, 4, 5), (4, 5, 3, 2)])
def test_plane_equilibrium_moments_are_perfect_fluid(qx, qphi, qp, nv):
    # N^mu = n u^mu, T^{mu nu} = (e+P) u^mu u^nu + P g^{mu nu} for any direction of u in the plane
    pl = O.Plane(nx=4, nz=4, q_xi=qx, q_phi=qphi, q_p=qp, n_v=nv)
    B = O.plane_moments_weights(pl)
    rng = np.random.default_rng(7)
    for _ in range(20):
        n, T = rng.uniform(0.1, 2.0), rng.uniform(0.2, 2.0)
        v, ang = rng.uniform(0.0, 0.9), rng.uniform(0, 2 * math.pi)
        g = 1 / math.sqrt(1 - v * v)
        ux, uz = g * v * math.cos(ang), g * v * math.sin(ang)
        m = B @ O.plane_feq_nodes(pl, n, T, ux, uz)
        ref = _perfect_fluid9(n, T, ux, uz)
        assert np.abs(m - ref).max() <= 3e-14 * np.abs(ref).max()


def test_plane_azimuthal_rule_needs_more_than_nv_plus_2_nodes():
    # T^{xx} of the truncated equilibrium holds cos^2(phi) P_k(c) terms of
    # trigonometric degree N_v + 2: Q_phi = N_v + 2 nodes miss it, N_v + 3 recover it
    n, T, ux, uz = 0.8, 1.1, 0.7, 0.2
    errs = []
    for qphi in (7, 8):
        pl = O.Plane(nx=4, nz=4, q_xi=8, q_phi=qphi, q_p=3, n_v=5)
        m = O.plane_moments_weights(pl) @ O.plane_feq_nodes(pl, n, T, ux, uz)
        ref = _perfect_fluid9(n, T, ux, uz)
        errs.append(np.abs(m - ref).max() / np.abs(ref).max())
    assert errs[0] > 1e-6 and errs[1] < 3e-14


def test_plane_truncation_recovers_the_moments_of_the_exact_distribution():
    # eq. mom_feq: for every L_l(p) v_x^a v_z^b with l <= N_p, a + b <= N_v the
    # quadrature of the truncated equilibrium equals the integral of the exact
    # Maxwell-Juettner F = n/(4T^3) exp(p (1 - (gamma - v.u)/T)) under
    # p e^{-p} dp dOmega/(2 pi), done on independent high-order rules
    # (Q_phi = 12 > 2 N_v and 2 Q_xi > 2 N_v make the nodal sums exact).
    pl = O.Plane(nx=4, nz=4, q_xi=8, q_phi=12, q_p=3, n_v=5, n_p=2)
    n, T, ux, uz = 0.9, 1.2, 0.5, -0.4
    g = math.sqrt(1 + ux * ux + uz * uz)
    xi, wxi, p, wp = O.tables(O.Tube(nx=8, q_xi=8, q_p=3))
    cphi, om = O.plane_tables(pl)
    F = O.plane_feq_nodes(pl, n, T, ux, uz).reshape(3, 8, pl.q_h)
    sth = np.sqrt(1 - xi ** 2)
    VX = sth[:, None] * cphi[None, :]
    VZ = np.broadcast_to(xi[:, None], VX.shape)
    W = wxi[:, None] * om[None, :]
    # independent rules: 80-point Gauss-Laguerre (alpha = 1), 48 x 96 sphere rule
    pr, wr = sp.roots_genlaguerre(80, 1)
    xa, wa = np.polynomial.legendre.leggauss(48)
    phi = 2 * np.pi * np.arange(96) / 96
    vxa = np.sqrt(1 - xa ** 2)[:, None] * np.cos(phi)[None, :]
    vza = np.broadcast_to(xa[:, None], vxa.shape)
    wa2 = wa[:, None] * np.full(96, 1 / 96)[None, :]
    beta = (g - vxa * ux - vza * uz) / T
    for l in range(3):
        Lp = sp.eval_genlaguerre(l, 1, p)
        Lr = sp.eval_genlaguerre(l, 1, pr)
        for a in range(6):
            for b in range(6 - a):
                quad = np.sum(wp[:, None, None] * Lp[:, None, None] * W[None] * VX[None] ** a * VZ[None] ** b * F)
                ang = wa2 * vxa ** a * vza ** b
                exact = sum(wr[q] * Lr[q] * np.sum(ang * n / (4 * T ** 3) * np.exp(pr[q] * (1 - beta)))
                            for q in range(80))
                assert abs(quad - exact) < 1e-12 * max(1.0, abs(exact)), (l, a, b)


def _random_moments(rng):
    # moments of a random positive distribution on a fine product rule
    pl = O.Plane(nx=4, nz=4, q_xi=12, q_phi=16, q_p=4)
    B = O.plane_moments_weights(pl)
    return B @ rng.uniform(0.05, 1.0, pl.Q)


def test_landau2d_is_the_timelike_eigenvector():
    rng = np.random.default_rng(3)
    g = np.diag([-1.0, 1.0, 1.0])
    for _ in range(20):
        m = _random_moments(rng)
        M = O.landau2d(m)
        Tm = np.array([[m[3], m[4], m[5]], [m[4], m[6], m[7]], [m[5], m[7], m[8]]])
        u = M["gamma"] * np.array([1.0, M["vx"], M["vz"]])
        res = Tm @ g @ u + M["e"] * u
        assert np.abs(res).max() < 1e-13 * np.abs(Tm).max()
        assert abs(M["vx"] ** 2 + M["vz"] ** 2) < 1
        assert abs(M["n"] - M["gamma"] * (m[0] - M["vx"] * m[1] - M["vz"] * m[2])) < 1e-14 * m[0]


def test_landau2d_rotation_covariance_and_1d_limit():
    rng = np.random.default_rng(5)
    m = _random_moments(rng)
    M = O.landau2d(m)
    for alpha in (0.3, 1.9, -2.4):
        c, s = math.cos(alpha), math.sin(alpha)
        R = np.array([[c, -s], [s, c]])
        N = R @ m[1:3]
        T0 = R @ m[4:6]
        Ts = R @ np.array([[m[6], m[7]], [m[7], m[8]]]) @ R.T
        Mr = O.landau2d([m[0], N[0], N[1], m[3], T0[0], T0[1], Ts[0, 0], Ts[0, 1], Ts[1, 1]])
        vr = R @ np.array([M["vx"], M["vz"]])
        assert abs(Mr["vx"] - vr[0]) < 1e-14 and abs(Mr["vz"] - vr[1]) < 1e-14
        assert abs(Mr["e"] - M["e"]) < 1e-14 * M["e"] and abs(Mr["n"] - M["n"]) < 1e-14 * M["n"]
    # no x components: the closed-form 1D root
    m1 = np.array([m[0], m[2], m[3], m[5], m[8]])
    M1 = O.landau(m1)
    Mz = O.landau2d([m[0], 0.0, m[2], m[3], 0.0, m[5], m[6], 0.0, m[8]])
    assert abs(Mz["vx"]) == 0.0 and abs(Mz["vz"] - M1["v"]) < 1e-14
    assert abs(Mz["e"] - M1["e"]) < 1e-14 * M1["e"] and abs(Mz["T"] - M1["T"]) < 1e-14 * M1["T"]


def _sod_fields(pl, along="z", left=(1.0, 1.0), right=(0.1, 0.125), u=(0.0, 0.0)):
    x, z = pl.centres()
    c = np.broadcast_to((z[:, None] if along == "z" else x[None, :]) < 0, (pl.nz, pl.nx))
    f = np.zeros((4, pl.nz, pl.nx))
    f[0] = np.where(c, left[0], right[0])
    f[1] = np.where(c, left[1], right[1])
    f[2], f[3] = u
    return f


def test_plane_without_x_dependence_is_the_tube():
    # u^x = 0 and no x dependence: every azimuthal node carries the 1D value
    pl = O.Plane(nx=6, nz=40, q_xi=8, q_phi=8, q_p=3, tau=1e-2)
    for u in ((0.0, 0.0), (0.0, 0.3)):
        F = O.plane_run(pl, _sod_fields(pl, u=u), 12)
        fl = O.plane_fields(pl, F)
        t = O.Tube(nx=40, q_xi=8, q_p=3, dt=pl.step_dt, tau=1e-2)
        ref = O.fields(t, O.run(t, (1.0, 1.0, u[1]), (0.1, 0.125, u[1]), 12))
        for a2, a1 in ((0, 0), (2, 1), (3, 2), (5, 3), (8, 4), (9, 5), (10, 6), (12, 7), (13, 8)):
            assert np.abs(fl[a2] - ref[a1][:, None]).max() < 1e-13 * np.abs(ref[a1]).max(), (u, a2)
        assert np.abs(fl[1]).max() < 1e-15 and np.abs(fl[4]).max() < 1e-15


def test_plane_mirror_symmetry():
    # data even in x (u^x odd) stay so: phi_k -> pi - phi_k maps v_x -> -v_x
    pl = O.Plane(nx=16, nz=12, q_xi=6, q_phi=8, q_p=3, tau=3e-2)
    x, z = pl.centres()
    r2 = x[None, :] ** 2 + (z[:, None] - 0.1) ** 2
    f = np.zeros((4, pl.nz, pl.nx))
    f[0] = 0.2 + np.exp(-r2 / 0.02)
    f[1] = 0.5 + 0.5 * np.exp(-r2 / 0.05)
    f[2] = 0.3 * x[None, :] * np.exp(-r2 / 0.05)
    f[3] = 0.1
    fl = O.plane_fields(pl, O.plane_run(pl, f, 8))
    for a, sgn in ((0, 1), (1, -1), (2, 1), (3, 1), (4, -1), (5, 1), (6, 1), (7, -1), (8, 1)):
        assert np.abs(fl[a] - sgn * fl[a][:, ::-1]).max() < 1e-14 * np.abs(fl[a]).max(), a


def test_plane_conservation():
    # a pressure blob in a uniform gas at rest: N^0, T^{00}, T^{0x}, T^{0z}
    # totals are constant while the disturbance (numerically, 9 cells per
    # step) has not reached the outflow edges
    pl = O.Plane(nx=48, nz=48, q_xi=6, q_phi=8, q_p=3, tau=1e-2)
    x, z = pl.centres()
    r2 = x[None, :] ** 2 + z[:, None] ** 2
    f = np.zeros((4, pl.nz, pl.nx))
    f[0] = 0.1 + 0.9 * np.exp(-r2 / 0.004)
    f[1] = 0.125 + 0.3 * np.exp(-r2 / 0.004)
    F = O.plane_init(pl, f)
    tot0 = O.plane_fields(pl, F)[[0, 3, 4, 5]].sum(axis=(1, 2))
    fl = O.plane_fields(pl, O.plane_step(pl, F, 5))
    tot = fl[[0, 3, 4, 5]].sum(axis=(1, 2))
    assert np.abs(tot - tot0).max() < 2e-14 * np.abs(tot0).max()
    # the edges still hold the undisturbed state
    assert np.abs(fl[10][0] - 0.125).max() < 1e-13
