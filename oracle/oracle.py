"""Python front end of the CPU FP64 oracle (test infrastructure only).

Thin ctypes wrappers around ``liboracle.so`` (built from ``rlb_oracle.cpp`` by
``oracle/build.py``) returning numpy arrays.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark import this module; the GPU
product path never does.

Arrays of the distribution use the layout ``F[s, x]`` with ``s = i*q_xi + j``
(radial node ``i`` outer, polar node ``j`` inner) and hold the weight-free
values ``F = 2*pi*exp(p)*f`` at the nodes.
"""
import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Tube(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("z_min", ctypes.c_double), ("z_max", ctypes.c_double),
                ("q_xi", ctypes.c_int32), ("q_p", ctypes.c_int32),
                ("n_v", ctypes.c_int32), ("n_p", ctypes.c_int32),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("T0", ctypes.c_double),
                ("weno_eps", ctypes.c_double)]


class _State(ctypes.Structure):
    _fields_ = [("P", ctypes.c_double), ("n", ctypes.c_double), ("u", ctypes.c_double)]


@dataclass
class Tube:
    """One shock tube, in the paper's problem-statement terms.

    ``dt`` defaults to ``min(cfl*dz, dt_tau_max*tau)``: the CFL condition with
    the speed of light as the largest speed, capped by the relaxation time.
    """
    nx: int = 800
    q_xi: int = 8
    q_p: int = 3
    n_v: int = 5
    n_p: int = 2
    tau: float = 1e-2
    z_min: float = -0.5
    z_max: float = 0.5
    cfl: float = 0.5
    dt_tau_max: float = 0.5
    dt: float = 0.0
    T0: float = 1.0
    weno_eps: float = 1e-6

    @property
    def dz(self) -> float:
        return (self.z_max - self.z_min) / self.nx

    @property
    def step_dt(self) -> float:
        if self.dt > 0:
            return self.dt
        return min(self.cfl * self.dz, self.dt_tau_max * self.tau)

    @property
    def Q(self) -> int:
        return self.q_xi * self.q_p

    def z(self) -> np.ndarray:
        return self.z_min + (np.arange(self.nx) + 0.5) * self.dz

    def _c(self) -> _Tube:
        return _Tube(self.nx, self.z_min, self.z_max, self.q_xi, self.q_p, self.n_v, self.n_p,
                     self.tau, self.step_dt, self.T0, self.weno_eps)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build as _build
            _build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        tp = ctypes.POINTER(_Tube)
        lib.oracle_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        lib.oracle_gauss_laguerre1.argtypes = [ctypes.c_int, dp, dp]
        lib.oracle_legendre.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.oracle_legendre.restype = ctypes.c_double
        lib.oracle_laguerre1.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.oracle_laguerre1.restype = ctypes.c_double
        lib.oracle_weno5.argtypes = [ctypes.c_double] * 6
        lib.oracle_weno5.restype = ctypes.c_double
        lib.oracle_landau.argtypes = [dp, dp]
        lib.oracle_feq_coefficients.argtypes = [tp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        lib.oracle_feq_nodes.argtypes = [tp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        lib.oracle_tables.argtypes = [tp, dp, dp, dp, dp]
        lib.oracle_init.argtypes = [tp, _State, _State, dp]
        lib.oracle_step.argtypes = [tp, dp, ctypes.c_int64]
        lib.oracle_rhs.argtypes = [tp, dp, dp]
        lib.oracle_fields.argtypes = [tp, dp, dp]
        lib.oracle_step_tangent.argtypes = [tp, dp, dp, ctypes.c_double, ctypes.c_int64]
        lib.oracle_init_tangent.argtypes = [tp, _State, _State, _State, _State, dp, dp]
        lib.oracle_fields_tangent.argtypes = [tp, dp, dp, dp, dp]
        lib.oracle_num_threads.restype = ctypes.c_int
        pp = ctypes.POINTER(_Plane)
        lib.oracle_plane_tables.argtypes = [pp, dp, dp]
        lib.oracle_landau2d.argtypes = [dp, dp]
        lib.oracle_plane_feq_nodes.argtypes = [pp] + [ctypes.c_double] * 4 + [dp]
        lib.oracle_plane_init.argtypes = [pp, dp, dp]
        lib.oracle_plane_step.argtypes = [pp, dp, ctypes.c_int64]
        lib.oracle_plane_rhs.argtypes = [pp, dp, dp]
        lib.oracle_plane_fields.argtypes = [pp, dp, dp]
        bp = ctypes.POINTER(_Box)
        lib.oracle_box_tables.argtypes = [bp, dp, dp]
        lib.oracle_landau3d.argtypes = [dp, dp]
        lib.oracle_box_feq_nodes.argtypes = [bp] + [ctypes.c_double] * 5 + [dp]
        lib.oracle_box_init.argtypes = [bp, dp, dp]
        lib.oracle_box_step.argtypes = [bp, dp, ctypes.c_int64]
        lib.oracle_box_rhs.argtypes = [bp, dp, dp]
        lib.oracle_box_fields.argtypes = [bp, dp, dp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc):
    if rc != 0:
        raise ValueError("oracle call rejected its arguments")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def gauss_legendre(q: int):
    x = np.zeros(q); w = np.zeros(q)
    _check(_load().oracle_gauss_legendre(q, _ptr(x), _ptr(w)))
    return x, w


def gauss_laguerre1(q: int):
    x = np.zeros(q); w = np.zeros(q)
    _check(_load().oracle_gauss_laguerre1(q, _ptr(x), _ptr(w)))
    return x, w


def legendre(n: int, x: float) -> float:
    return _load().oracle_legendre(n, x)


def laguerre1(n: int, x: float) -> float:
    return _load().oracle_laguerre1(n, x)


def weno5(v, eps=1e-6) -> float:
    return _load().oracle_weno5(*[float(a) for a in v], float(eps))


def landau(m):
    """(N0, Nz, T00, T0z, Tzz) -> dict(e, v, gamma, u, n, T)."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    out = np.zeros(6)
    _load().oracle_landau(_ptr(m), _ptr(out))
    return dict(zip(("e", "v", "gamma", "u", "n", "T"), out))


def feq_coefficients(tube: Tube, n: float, T: float, u: float) -> np.ndarray:
    """Projection coefficients C[k, l] (k <= n_v, l <= n_p)."""
    C = np.zeros((tube.n_v + 1) * (tube.n_p + 1))
    _check(_load().oracle_feq_coefficients(ctypes.byref(tube._c()), n, T, u, _ptr(C)))
    return C.reshape(tube.n_v + 1, tube.n_p + 1)


def feq_nodes(tube: Tube, n: float, T: float, u: float) -> np.ndarray:
    """Weight-free truncated equilibrium at the Q nodes, shape [Q]."""
    F = np.zeros(tube.Q)
    _check(_load().oracle_feq_nodes(ctypes.byref(tube._c()), n, T, u, _ptr(F)))
    return F


def tables(tube: Tube):
    """(xi, w_xi, p, w_p) quadrature tables of the tube."""
    xi = np.zeros(tube.q_xi); wxi = np.zeros(tube.q_xi)
    p = np.zeros(tube.q_p); wp = np.zeros(tube.q_p)
    _check(_load().oracle_tables(ctypes.byref(tube._c()), _ptr(xi), _ptr(wxi), _ptr(p), _ptr(wp)))
    return xi, wxi, p, wp


def init(tube: Tube, left, right) -> np.ndarray:
    """Initial distribution F[Q, nx] for left/right states (P, n, u)."""
    F = np.zeros((tube.Q, tube.nx))
    _check(_load().oracle_init(ctypes.byref(tube._c()), _State(*left), _State(*right), _ptr(F)))
    return F


def step(tube: Tube, F: np.ndarray, nsteps: int) -> np.ndarray:
    """Returns F advanced by ``nsteps`` SSP-RK3 steps (input untouched)."""
    G = np.array(F, dtype=np.float64, order="C", copy=True)
    _check(_load().oracle_step(ctypes.byref(tube._c()), _ptr(G), int(nsteps)))
    return G


def rhs(tube: Tube, F: np.ndarray) -> np.ndarray:
    G = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros_like(G)
    _check(_load().oracle_rhs(ctypes.byref(tube._c()), _ptr(G), _ptr(out)))
    return out


FIELD_NAMES = ("N0", "Nz", "T00", "T0z", "Tzz", "e", "n", "v", "T", "Nabs")


def fields(tube: Tube, F: np.ndarray) -> np.ndarray:
    """Per-cell fields [10, nx]: N0, Nz, T00, T0z, Tzz, e, n, v, T, |N|."""
    G = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros((10, tube.nx))
    _check(_load().oracle_fields(ctypes.byref(tube._c()), _ptr(G), _ptr(out)))
    return out


def step_tangent(tube: Tube, F: np.ndarray, dF: np.ndarray, dtau: float, nsteps: int):
    """Tangent-linear model: (F, dF) advanced by ``nsteps`` with tau moving by dtau."""
    G = np.array(F, dtype=np.float64, order="C", copy=True)
    dG = np.array(dF, dtype=np.float64, order="C", copy=True)
    _check(_load().oracle_step_tangent(ctypes.byref(tube._c()), _ptr(G), _ptr(dG), float(dtau), int(nsteps)))
    return G, dG


def init_tangent(tube: Tube, left, right, dleft, dright):
    F = np.zeros((tube.Q, tube.nx)); dF = np.zeros((tube.Q, tube.nx))
    _check(_load().oracle_init_tangent(ctypes.byref(tube._c()), _State(*left), _State(*right),
                                       _State(*dleft), _State(*dright), _ptr(F), _ptr(dF)))
    return F, dF


def fields_tangent(tube: Tube, F: np.ndarray, dF: np.ndarray):
    G = np.ascontiguousarray(F, dtype=np.float64)
    dG = np.ascontiguousarray(dF, dtype=np.float64)
    out = np.zeros((10, tube.nx)); dout = np.zeros((10, tube.nx))
    _check(_load().oracle_fields_tangent(ctypes.byref(tube._c()), _ptr(G), _ptr(dG), _ptr(out), _ptr(dout)))
    return out, dout


def run(tube: Tube, left, right, nsteps: int) -> np.ndarray:
    """Initial state then ``nsteps`` steps; returns F[Q, nx]."""
    return step(tube, init(tube, left, right), nsteps)


def moments_weights(tube: Tube) -> np.ndarray:
    """Moment basis B[5, Q]: N0..Tzz = B @ F[:, x]."""
    xi, wxi, p, wp = tables(tube)
    B = np.zeros((5, tube.Q))
    t3, t4 = tube.T0 ** 3, tube.T0 ** 4
    for i in range(tube.q_p):
        for j in range(tube.q_xi):
            w = wp[i] * wxi[j]
            s = i * tube.q_xi + j
            B[:, s] = w * np.array([t3 * p[i], t3 * p[i] * xi[j], t4 * p[i] ** 2,
                                    t4 * p[i] ** 2 * xi[j], t4 * p[i] ** 2 * xi[j] ** 2])
    return B


SOD_LEFT = (1.0, 1.0, 0.0)
SOD_RIGHT = (0.1, 0.125, 0.0)
PI = math.pi


# ---------------------------------------------------------------------------
# Multi-dimensional model on a plane (x, z)
# ---------------------------------------------------------------------------
class _Plane(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
                ("z_min", ctypes.c_double), ("z_max", ctypes.c_double),
                ("q_xi", ctypes.c_int32), ("q_phi", ctypes.c_int32), ("q_p", ctypes.c_int32),
                ("n_v", ctypes.c_int32), ("n_p", ctypes.c_int32),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("T0", ctypes.c_double),
                ("weno_eps", ctypes.c_double)]


@dataclass
class Plane:
    """A 2D (x, z) domain with the full momentum quadrature (Q_p x Q_xi x Q_phi;
    the evolved azimuthal nodes are k = 0 .. Q_phi // 2).

    ``dt`` defaults to ``min(cfl / (1/dx + 1/dz), dt_tau_max * tau)``.
    """
    nx: int = 32
    nz: int = 32
    q_xi: int = 8
    q_phi: int = 8
    q_p: int = 3
    n_v: int = 5
    n_p: int = 2
    tau: float = 1e-2
    x_min: float = -0.5
    x_max: float = 0.5
    z_min: float = -0.5
    z_max: float = 0.5
    cfl: float = 0.5
    dt_tau_max: float = 0.5
    dt: float = 0.0
    T0: float = 1.0
    weno_eps: float = 1e-6

    @property
    def dx(self) -> float:
        return (self.x_max - self.x_min) / self.nx

    @property
    def dz(self) -> float:
        return (self.z_max - self.z_min) / self.nz

    @property
    def step_dt(self) -> float:
        if self.dt > 0:
            return self.dt
        return min(self.cfl / (1.0 / self.dx + 1.0 / self.dz), self.dt_tau_max * self.tau)

    @property
    def q_h(self) -> int:
        return self.q_phi // 2 + 1

    @property
    def Q(self) -> int:
        return self.q_p * self.q_xi * self.q_h

    def centres(self):
        x = self.x_min + (np.arange(self.nx) + 0.5) * self.dx
        z = self.z_min + (np.arange(self.nz) + 0.5) * self.dz
        return x, z

    def _c(self) -> _Plane:
        return _Plane(self.nx, self.nz, self.x_min, self.x_max, self.z_min, self.z_max, self.q_xi, self.q_phi,
                      self.q_p, self.n_v, self.n_p, self.tau, self.step_dt, self.T0, self.weno_eps)


def plane_tables(plane: Plane):
    """(cos phi_k, omega_k) of the evolved azimuthal nodes."""
    c = np.zeros(plane.q_h); w = np.zeros(plane.q_h)
    _check(_load().oracle_plane_tables(ctypes.byref(plane._c()), _ptr(c), _ptr(w)))
    return c, w


def landau2d(m):
    """(N0, Nx, Nz, T00, T0x, T0z, Txx, Txz, Tzz) -> dict(e, vx, vz, gamma, n, T)."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    out = np.zeros(6)
    _load().oracle_landau2d(_ptr(m), _ptr(out))
    return dict(zip(("e", "vx", "vz", "gamma", "n", "T"), out))


def plane_feq_nodes(plane: Plane, n: float, T: float, ux: float, uz: float) -> np.ndarray:
    F = np.zeros(plane.Q)
    _check(_load().oracle_plane_feq_nodes(ctypes.byref(plane._c()), n, T, ux, uz, _ptr(F)))
    return F


def plane_init(plane: Plane, fields: np.ndarray) -> np.ndarray:
    """F[Q, nz, nx] from per-cell states fields[4, nz, nx] = (P, n, u^x, u^z)."""
    f = np.ascontiguousarray(fields, dtype=np.float64)
    assert f.shape == (4, plane.nz, plane.nx)
    F = np.zeros((plane.Q, plane.nz, plane.nx))
    _check(_load().oracle_plane_init(ctypes.byref(plane._c()), _ptr(f), _ptr(F)))
    return F


def plane_step(plane: Plane, F: np.ndarray, nsteps: int) -> np.ndarray:
    G = np.array(F, dtype=np.float64, order="C", copy=True)
    _check(_load().oracle_plane_step(ctypes.byref(plane._c()), _ptr(G), int(nsteps)))
    return G


def plane_rhs(plane: Plane, F: np.ndarray) -> np.ndarray:
    G = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros_like(G)
    _check(_load().oracle_plane_rhs(ctypes.byref(plane._c()), _ptr(G), _ptr(out)))
    return out


def plane_fields(plane: Plane, F: np.ndarray) -> np.ndarray:
    """Per-cell fields [14, nz, nx]: N0, Nx, Nz, T00, T0x, T0z, Txx, Txz, Tzz, e, n, vx, vz, T."""
    G = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros((14, plane.nz, plane.nx))
    _check(_load().oracle_plane_fields(ctypes.byref(plane._c()), _ptr(G), _ptr(out)))
    return out


def plane_moments_weights(plane: Plane) -> np.ndarray:
    """Moment basis B[9, Q]: the 9 moments of a cell = B @ F[:, z, x]."""
    xi, wxi, p, wp = tables(Tube(nx=8, q_xi=plane.q_xi, q_p=plane.q_p, n_v=plane.n_v, n_p=plane.n_p,
                                 T0=plane.T0))
    cphi, om = plane_tables(plane)
    B = np.zeros((9, plane.Q))
    t3, t4 = plane.T0 ** 3, plane.T0 ** 4
    for i in range(plane.q_p):
        for j in range(plane.q_xi):
            for k in range(plane.q_h):
                s = (i * plane.q_xi + j) * plane.q_h + k
                w = wp[i] * wxi[j] * om[k]
                vx, vz = math.sqrt(1 - xi[j] ** 2) * cphi[k], xi[j]
                a3, a4 = t3 * p[i] * w, t4 * p[i] ** 2 * w
                B[:, s] = [a3, a3 * vx, a3 * vz, a4, a4 * vx, a4 * vz, a4 * vx * vx, a4 * vx * vz, a4 * vz * vz]
    return B


def plane_run(plane: Plane, fields: np.ndarray, nsteps: int) -> np.ndarray:
    return plane_step(plane, plane_init(plane, fields), nsteps)


# ---------------------------------------------------------------------------
# Three-dimensional box, any flow direction (full azimuthal node set)
# ---------------------------------------------------------------------------
class _Box(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
                ("y_min", ctypes.c_double), ("y_max", ctypes.c_double),
                ("z_min", ctypes.c_double), ("z_max", ctypes.c_double),
                ("q_xi", ctypes.c_int32), ("q_phi", ctypes.c_int32), ("q_p", ctypes.c_int32),
                ("n_v", ctypes.c_int32), ("n_p", ctypes.c_int32),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("T0", ctypes.c_double),
                ("weno_eps", ctypes.c_double)]


BOX_FIELDS = ("N0", "Nx", "Ny", "Nz", "T00", "T0x", "T0y", "T0z", "Txx", "Txy", "Txz", "Tyy", "Tyz", "Tzz",
              "e", "n", "vx", "vy", "vz", "T")


@dataclass
class Box:
    """An (x, y, z) box with the full momentum quadrature Q_p x Q_xi x Q_phi
    (every azimuthal node evolved).

    ``dt`` defaults to ``min(cfl / (1/dx + 1/dy + 1/dz), dt_tau_max * tau)``.
    """
    nx: int = 8
    ny: int = 8
    nz: int = 8
    q_xi: int = 6
    q_phi: int = 8
    q_p: int = 3
    n_v: int = 5
    n_p: int = 2
    tau: float = 1e-2
    x_min: float = -0.5
    x_max: float = 0.5
    y_min: float = -0.5
    y_max: float = 0.5
    z_min: float = -0.5
    z_max: float = 0.5
    cfl: float = 0.5
    dt_tau_max: float = 0.5
    dt: float = 0.0
    T0: float = 1.0
    weno_eps: float = 1e-6

    @property
    def dx(self) -> float:
        return (self.x_max - self.x_min) / self.nx

    @property
    def dy(self) -> float:
        return (self.y_max - self.y_min) / self.ny

    @property
    def dz(self) -> float:
        return (self.z_max - self.z_min) / self.nz

    @property
    def step_dt(self) -> float:
        if self.dt > 0:
            return self.dt
        return min(self.cfl / (1.0 / self.dx + 1.0 / self.dy + 1.0 / self.dz), self.dt_tau_max * self.tau)

    @property
    def Q(self) -> int:
        return self.q_p * self.q_xi * self.q_phi

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def centres(self):
        x = self.x_min + (np.arange(self.nx) + 0.5) * self.dx
        y = self.y_min + (np.arange(self.ny) + 0.5) * self.dy
        z = self.z_min + (np.arange(self.nz) + 0.5) * self.dz
        return x, y, z

    def _c(self) -> _Box:
        return _Box(self.nx, self.ny, self.nz, self.x_min, self.x_max, self.y_min, self.y_max, self.z_min, self.z_max,
                    self.q_xi, self.q_phi, self.q_p, self.n_v, self.n_p, self.tau, self.step_dt, self.T0,
                    self.weno_eps)


def box_tables(box: Box):
    """(cos phi_k, sin phi_k) of the azimuthal nodes."""
    c = np.zeros(box.q_phi); s = np.zeros(box.q_phi)
    _check(_load().oracle_box_tables(ctypes.byref(box._c()), _ptr(c), _ptr(s)))
    return c, s


def landau3d(m):
    """Landau frame of the 14 moments -> (e, v_x, v_y, v_z, gamma, n, T)."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    out = np.zeros(7)
    _load().oracle_landau3d(_ptr(m), _ptr(out))
    return out


def box_feq_nodes(box: Box, n: float, T: float, ux: float, uy: float, uz: float) -> np.ndarray:
    F = np.zeros(box.Q)
    _check(_load().oracle_box_feq_nodes(ctypes.byref(box._c()), n, T, ux, uy, uz, _ptr(F)))
    return F


def box_init(box: Box, fields: np.ndarray) -> np.ndarray:
    """F[Q, nz, ny, nx] from per-cell states fields[5, nz, ny, nx] = P, n, u^x, u^y, u^z."""
    f = np.ascontiguousarray(fields, dtype=np.float64)
    assert f.shape == (5, box.nz, box.ny, box.nx)
    F = np.zeros((box.Q, box.nz, box.ny, box.nx))
    _check(_load().oracle_box_init(ctypes.byref(box._c()), _ptr(f), _ptr(F)))
    return F


def box_step(box: Box, F: np.ndarray, nsteps: int) -> np.ndarray:
    G = np.array(F, dtype=np.float64, order="C", copy=True)
    _check(_load().oracle_box_step(ctypes.byref(box._c()), _ptr(G), int(nsteps)))
    return G


def box_rhs(box: Box, F: np.ndarray) -> np.ndarray:
    G = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros_like(G)
    _check(_load().oracle_box_rhs(ctypes.byref(box._c()), _ptr(G), _ptr(out)))
    return out


def box_fields(box: Box, F: np.ndarray) -> np.ndarray:
    """Fields [20, nz, ny, nx]: the 14 moments, e, n, v_x, v_y, v_z, T."""
    G = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros((20, box.nz, box.ny, box.nx))
    _check(_load().oracle_box_fields(ctypes.byref(box._c()), _ptr(G), _ptr(out)))
    return out


def box_run(box: Box, fields: np.ndarray, nsteps: int) -> np.ndarray:
    return box_step(box, box_init(box, fields), nsteps)


def box_moments_weights(box: Box) -> np.ndarray:
    """Moment basis B[14, Q]: the 14 moments of a cell = B @ F[:, cell]."""
    xi, wxi, p, wp = tables(Tube(nx=1, q_xi=box.q_xi, q_p=box.q_p, n_v=box.n_v, n_p=box.n_p, T0=box.T0))
    cphi, sphi = box_tables(box)
    B = np.zeros((14, box.Q))
    t3, t4 = box.T0 ** 3, box.T0 ** 4
    for i in range(box.q_p):
        for j in range(box.q_xi):
            st = math.sqrt(1.0 - xi[j] ** 2)
            for k in range(box.q_phi):
                s = (i * box.q_xi + j) * box.q_phi + k
                w = wp[i] * wxi[j] / box.q_phi
                v = (st * cphi[k], st * sphi[k], xi[j])
                row = [t3 * p[i]] + [t3 * p[i] * v[a] for a in range(3)] + [t4 * p[i] ** 2] + \
                      [t4 * p[i] ** 2 * v[a] for a in range(3)] + \
                      [t4 * p[i] ** 2 * v[a] * v[b] for a in range(3) for b in range(a, 3)]
                B[:, s] = w * np.array(row)
    return B
