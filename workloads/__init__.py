"""Synthetic Sod-tube workloads (shared input recipes; no lattice Boltzmann arithmetic).

Every workload is a list of tube parameter dicts plus left/right states
(P, n, u).  The Sod states are the paper's (section Riemann problem,
eq. condinit); the sizes are those of the benchmark configurations:

  sod_small     N_x = 800, Q = 8 x 3, tau = 1e-2, to t = 0.2 (320 steps)
  sod_large     N_x = 2^20, Q = 64 x 4, tau in {1e-4, 1e-2, 1, 100}, 2000 steps
  sod_batched   4096 tubes drawn with numpy's default_rng(0) (see below), 500 steps
  sod_adjoint   N_x = 4096, Q = 32 x 3, 2000 steps, target (tau 0.05, P_L 1.5)
  sod_ballistic N_x = 2^22, Q = 256 x 4, tau = 1e3, 4000 steps
"""
import math

import numpy as np

SOD_LEFT = (1.0, 1.0, 0.0)
SOD_RIGHT = (0.1, 0.125, 0.0)


def tube(nx, q_xi, q_p=3, tau=1e-2, **kw):
    d = dict(nx=int(nx), q_xi=int(q_xi), q_p=int(q_p), n_v=5, n_p=2, tau=float(tau))
    d.update(kw)
    return d


def sod_small():
    return dict(tubes=[tube(800, 8, 3, 1e-2)], left=SOD_LEFT, right=SOD_RIGHT, steps=320)


def sod_large(tau=1e-2, nx=1 << 20):
    return dict(tubes=[tube(nx, 64, 4, tau)], left=SOD_LEFT, right=SOD_RIGHT, steps=2000)


def sod_ballistic(nx=1 << 22):
    return dict(tubes=[tube(nx, 256, 4, 1e3)], left=SOD_LEFT, right=SOD_RIGHT, steps=4000)


def sod_adjoint():
    return dict(tubes=[tube(4096, 32, 3, 0.02)], left=(1.0, 1.0, 0.0), right=SOD_RIGHT, steps=2000,
                target=dict(tau=0.05, P_L=1.5, n_L=1.0), start=dict(tau=0.02, P_L=1.0, n_L=1.0))


def sod_batched(ntubes=4096, seed=0):
    """4096 independent tubes, seeded draw:

    N_x ~ U{256..8192}; q_xi ~ U{8, 16, 32, 64, 128}; q_p = 3;
    log tau ~ U[ln 1e-4, ln 10]; log(P_L/P_R) ~ U[ln 2, ln 100] with P_R = 0.1;
    n_L/n_R ~ U[1, 10] with n_R = 0.125; fluid at rest.
    The time step is min(0.5 dz, 0.5 tau) per tube.
    """
    rng = np.random.default_rng(seed)
    nx = rng.integers(256, 8192, size=ntubes, endpoint=True)
    qxi = rng.choice(np.array([8, 16, 32, 64, 128]), size=ntubes)
    tau = np.exp(rng.uniform(math.log(1e-4), math.log(10.0), size=ntubes))
    pratio = np.exp(rng.uniform(math.log(2.0), math.log(100.0), size=ntubes))
    nratio = rng.uniform(1.0, 10.0, size=ntubes)
    tubes, lefts, rights = [], [], []
    for k in range(ntubes):
        tubes.append(tube(nx[k], qxi[k], 3, tau[k]))
        lefts.append((0.1 * pratio[k], 0.125 * nratio[k], 0.0))
        rights.append((0.1, 0.125, 0.0))
    return dict(tubes=tubes, left=lefts, right=rights, steps=500)


def points(tubes):
    """Cell x quadrature points advanced per step."""
    return sum(t["nx"] * t["q_xi"] * t["q_p"] for t in tubes)
