"""Python binding of ``librlb.so`` (the C interface of include/rlb.h).

Argument marshalling only: every step of the lattice Boltzmann update runs in
the HIP kernels of the library.  PyTorch supplies device memory (the
workspace, state and adjoint buffers) and the HIP stream.  Import fails loudly
if the library has not been built; there is no fallback path.
"""
import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlb.so")

RLB_OK = 0
RLB_ERR_INVALID_ARG = -1
RLB_ERR_NONPHYSICAL = -2
RLB_ERR_HIP = -3
RLB_ERR_STATE = -4
RLB_ERR_UNSTABLE_DT = -5

RLB_FP64 = 0
RLB_FP32 = 1
RLB_WITH_ADJOINT = 1
RLB_FLAG_NONPHYSICAL = 1
RLB_FLAG_FAST_FLOW = 2

FIELD_NAMES = ("N0", "Nz", "T00", "T0z", "Tzz", "e", "n", "v", "T", "Nabs")


class TubeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("q_xi", ctypes.c_int32), ("q_p", ctypes.c_int32),
                ("n_v", ctypes.c_int32), ("n_p", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("z_min", ctypes.c_double), ("z_max", ctypes.c_double), ("tau", ctypes.c_double),
                ("cfl", ctypes.c_double), ("dt_tau_max", ctypes.c_double), ("dt", ctypes.c_double),
                ("T0", ctypes.c_double), ("weno_eps", ctypes.c_double)]


class State(ctypes.Structure):
    _fields_ = [("P", ctypes.c_double), ("n", ctypes.c_double), ("u", ctypes.c_double)]


class Schedule(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("split_below", ctypes.c_int32)]


class RLBError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None

# name -> (restype, argtypes); every symbol the header declares
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
class PlaneDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("q_xi", ctypes.c_int32),
                ("q_phi", ctypes.c_int32), ("q_p", ctypes.c_int32), ("n_v", ctypes.c_int32),
                ("n_p", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("x_min", ctypes.c_double), ("x_max", ctypes.c_double), ("z_min", ctypes.c_double),
                ("z_max", ctypes.c_double), ("tau", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dt_tau_max", ctypes.c_double), ("dt", ctypes.c_double), ("T0", ctypes.c_double),
                ("weno_eps", ctypes.c_double)]


class BoxDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("q_xi", ctypes.c_int32), ("q_phi", ctypes.c_int32), ("q_p", ctypes.c_int32),
                ("n_v", ctypes.c_int32), ("n_p", ctypes.c_int32),
                ("x_min", ctypes.c_double), ("x_max", ctypes.c_double), ("y_min", ctypes.c_double),
                ("y_max", ctypes.c_double), ("z_min", ctypes.c_double), ("z_max", ctypes.c_double),
                ("tau", ctypes.c_double), ("cfl", ctypes.c_double), ("dt_tau_max", ctypes.c_double),
                ("dt", ctypes.c_double), ("T0", ctypes.c_double), ("weno_eps", ctypes.c_double)]


_SIGNATURES = {
    "rlb_tube_defaults": [ctypes.POINTER(TubeDesc)],
    "rlb_create": [ctypes.POINTER(TubeDesc), ctypes.c_int32, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_VP)],
    "rlb_destroy": [_VP],
    "rlb_workspace_size": [_VP, ctypes.POINTER(ctypes.c_size_t)],
    "rlb_bind": [_VP, _VP, ctypes.c_size_t, _VP],
    "rlb_set_stream": [_VP, _VP],
    "rlb_set_schedule": [_VP, ctypes.POINTER(Schedule)],
    "rlb_get_schedule": [_VP, ctypes.POINTER(Schedule)],
    "rlb_set_initial_state": [_VP, ctypes.c_int32, State, State],
    "rlb_set_initial_states": [_VP, ctypes.c_int32, ctypes.POINTER(State), ctypes.POINTER(State)],
    "rlb_step": [_VP, ctypes.c_int64],
    "rlb_fields": [_VP, ctypes.c_int32, _VP, ctypes.c_int64],
    "rlb_moments": [_VP, ctypes.c_int32, _DP, ctypes.c_int64],
    "rlb_totals": [_VP, ctypes.c_int32, _DP],
    "rlb_check": [_VP],
    "rlb_state_elems": [_VP, ctypes.POINTER(ctypes.c_int64)],
    "rlb_state_layout": [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "rlb_get_state": [_VP, _VP],
    "rlb_set_state": [_VP, _VP],
    "rlb_equilibrium": [_VP, _VP],
    "rlb_set_tau": [_VP, ctypes.c_int32, ctypes.c_double],
    "rlb_tube_info": [_VP, ctypes.c_int32, _DP, _DP, ctypes.POINTER(ctypes.c_int32)],
    "rlb_tables": [_VP, ctypes.c_int32, _DP, _DP, _DP, _DP],
    "rlb_device_copy": [_VP, _VP, ctypes.c_size_t, _VP],
    "rlb_device_stream": [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _VP],
    "rlb_adjoint_step": [_VP, _VP, _VP, _VP],
    "rlb_adjoint_segment_size": [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "rlb_adjoint_segment": [_VP, _VP, ctypes.c_int32, _VP, ctypes.c_size_t, _VP, _VP],
    "rlb_adjoint_segment_forward": [_VP, _VP, ctypes.c_int32, _VP, ctypes.c_size_t, _VP],
    "rlb_adjoint_segment_reverse": [_VP, ctypes.c_int32, _VP, ctypes.c_size_t, _VP, _VP],
    "rlb_fields_adjoint": [_VP, ctypes.c_int32, _VP, _VP, ctypes.c_int64, _VP],
    "rlb_initial_state_adjoint": [_VP, ctypes.c_int32, _VP, _DP, _DP],
    "rlb_step_noalloc": [_VP, _VP, ctypes.c_int64, _VP, _VP],
    "rlb_flags": [_VP, ctypes.POINTER(ctypes.c_uint32)],
    "rlb_set_time": [_VP, ctypes.c_int32, ctypes.c_double],
}
_SIGNATURES.update({
    "rlb_plane_defaults": [ctypes.POINTER(PlaneDesc)],
    "rlb_plane_create": [ctypes.POINTER(PlaneDesc), ctypes.c_int, ctypes.POINTER(_VP)],
    "rlb_plane_destroy": [_VP],
    "rlb_plane_workspace_size": [_VP, ctypes.POINTER(ctypes.c_size_t)],
    "rlb_plane_bind": [_VP, _VP, ctypes.c_size_t, _VP],
    "rlb_plane_set_initial_fields": [_VP, _VP],
    "rlb_plane_step": [_VP, ctypes.c_int64],
    "rlb_plane_fields": [_VP, _VP],
    "rlb_plane_layout": [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "rlb_plane_get_state": [_VP, _VP],
    "rlb_plane_set_state": [_VP, _VP],
    "rlb_plane_info": [_VP, _DP, _DP, ctypes.POINTER(ctypes.c_int32)],
    "rlb_plane_check": [_VP],
    "rlb_plane_flags": [_VP, ctypes.POINTER(ctypes.c_uint32)],
    "rlb_box_defaults": [ctypes.POINTER(BoxDesc)],
    "rlb_box_create": [ctypes.POINTER(BoxDesc), ctypes.c_int, ctypes.POINTER(_VP)],
    "rlb_box_destroy": [_VP],
    "rlb_box_workspace_size": [_VP, ctypes.POINTER(ctypes.c_size_t)],
    "rlb_box_bind": [_VP, _VP, ctypes.c_size_t, _VP],
    "rlb_box_set_initial_fields": [_VP, _VP],
    "rlb_box_step": [_VP, ctypes.c_int64],
    "rlb_box_fields": [_VP, _VP],
    "rlb_box_layout": [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "rlb_box_get_state": [_VP, _VP],
    "rlb_box_set_state": [_VP, _VP],
    "rlb_box_info": [_VP, _DP, _DP, ctypes.POINTER(ctypes.c_int32)],
    "rlb_box_check": [_VP],
    "rlb_box_flags": [_VP, ctypes.POINTER(ctypes.c_uint32)],
})
_STRING_FUNCS = {"rlb_status_string": [ctypes.c_int], "rlb_last_error": [_VP], "rlb_plane_last_error": [_VP],
                 "rlb_box_last_error": [_VP]}


def load_library():
    """Loads librlb.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1608_03004_amd/build.py "
                              "(or __graft_entry__.build()); there is no non-HIP fallback")
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        for name, args in _STRING_FUNCS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def declared_symbols(header: Optional[str] = None) -> List[str]:
    """Entry points declared in include/rlb.h."""
    import re
    header = header or os.path.join(os.path.dirname(_HERE), "include", "rlb.h")
    text = open(header).read()
    return sorted(set(re.findall(r"\b(rlb_[a-z0-9_]+)\s*\(", text)))


@dataclass
class Tube:
    """One shock tube; fields mirror ``rlb_tube_desc``."""
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

    def c(self) -> TubeDesc:
        return TubeDesc(self.nx, self.q_xi, self.q_p, self.n_v, self.n_p, 0, self.z_min, self.z_max,
                        self.tau, self.cfl, self.dt_tau_max, self.dt, self.T0, self.weno_eps)

    @property
    def Q(self) -> int:
        return self.q_xi * self.q_p


def _torch():
    import torch
    return torch


class Lattice:
    """A set of shock tubes advanced together on one GPU.

    The workspace is a torch uint8 tensor on the current device; work is queued
    on ``stream`` (default: torch's current stream).
    """

    def __init__(self, tubes: Sequence[Tube], precision: str = "fp64", adjoint: bool = False,
                 stream=None, device=None, bind: bool = True):
        torch = _torch()
        self.lib = load_library()
        self.tubes = list(tubes)
        self.precision = precision
        prec = {"fp64": RLB_FP64, "fp32": RLB_FP32}[precision]
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        arr = (TubeDesc * len(self.tubes))(*[t.c() for t in self.tubes])
        h = _VP()
        st = self.lib.rlb_create(arr, len(self.tubes), prec, RLB_WITH_ADJOINT if adjoint else 0, ctypes.byref(h))
        if st != RLB_OK:
            raise RLBError(st, self.lib.rlb_last_error(None).decode())
        self.h = h
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if bind:
            size = ctypes.c_size_t()
            self._check(self.lib.rlb_workspace_size(self.h, ctypes.byref(size)))
            # +256 so that the base can be aligned
            self._ws = torch.empty(size.value + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            self._check(self.lib.rlb_bind(self.h, _VP(self._ws_ptr), size.value, _VP(self.stream.cuda_stream)))
        n = ctypes.c_int64()
        self._check(self.lib.rlb_state_elems(self.h, ctypes.byref(n)))
        self.state_elems = n.value

    # -- helpers ---------------------------------------------------------
    def _check(self, st: int):
        if st != RLB_OK:
            raise RLBError(st, self.lib.rlb_last_error(self.h).decode() or self.lib.rlb_status_string(st).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.rlb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API -------------------------------------------------------------
    def set_schedule(self, tile=256, persistent=0, blocks_per_cu=4, graph_steps=0, chunk=0, split_below=-1):
        s = Schedule(tile, persistent, blocks_per_cu, graph_steps, chunk, split_below)
        self._check(self.lib.rlb_set_schedule(self.h, ctypes.byref(s)))

    def get_schedule(self) -> dict:
        s = Schedule()
        self._check(self.lib.rlb_get_schedule(self.h, ctypes.byref(s)))
        return dict(tile=s.tile, persistent=s.persistent, blocks_per_cu=s.blocks_per_cu, graph_steps=s.graph_steps,
                    chunk=s.chunk, split_below=s.split_below)

    def set_initial_state(self, left, right, tube: int = -1):
        self._check(self.lib.rlb_set_initial_state(self.h, tube, State(*left), State(*right)))

    def set_initial_states(self, lefts, rights):
        n = len(self.tubes)
        L = (State * n)(*[State(*s) for s in lefts])
        R = (State * n)(*[State(*s) for s in rights])
        self._check(self.lib.rlb_set_initial_states(self.h, n, L, R))

    def step(self, nsteps: int = 1):
        self._check(self.lib.rlb_step(self.h, int(nsteps)))

    def fields(self, tube: int = 0):
        """Device tensor [10, nx] (FP64), queued on the stream."""
        torch = _torch()
        nx = self.tubes[tube].nx
        out = torch.empty((10, nx), dtype=torch.float64, device=self.device)
        self._check(self.lib.rlb_fields(self.h, tube, _VP(out.data_ptr()), nx))
        return out

    def moments(self, tube: int = 0) -> np.ndarray:
        """Host array [10, nx]; synchronizes and reports the sticky flag."""
        nx = self.tubes[tube].nx
        out = np.zeros((10, nx))
        self._check(self.lib.rlb_moments(self.h, tube, out.ctypes.data_as(_DP), nx))
        return out

    def totals(self, tube: int = 0) -> np.ndarray:
        out = np.zeros(3)
        self._check(self.lib.rlb_totals(self.h, tube, out.ctypes.data_as(_DP)))
        return out

    def check(self):
        self._check(self.lib.rlb_check(self.h))

    def flags(self) -> dict:
        """Sticky flag bits since the last initial state (synchronizes)."""
        f = ctypes.c_uint32()
        self._check(self.lib.rlb_flags(self.h, ctypes.byref(f)))
        return dict(nonphysical=bool(f.value & RLB_FLAG_NONPHYSICAL), fast_flow=bool(f.value & RLB_FLAG_FAST_FLOW))

    def layout(self, tube: int):
        off, ld = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.rlb_state_layout(self.h, tube, ctypes.byref(off), ctypes.byref(ld)))
        return off.value, ld.value

    def new_state(self):
        torch = _torch()
        return torch.empty(self.state_elems, dtype=self.dtype, device=self.device)

    def get_state(self, out=None):
        out = self.new_state() if out is None else out
        assert out.numel() >= self.state_elems and out.dtype == self.dtype and out.is_contiguous()
        self._check(self.lib.rlb_get_state(self.h, _VP(out.data_ptr())))
        return out

    def set_state(self, src):
        assert src.numel() >= self.state_elems and src.dtype == self.dtype and src.is_contiguous()
        self._check(self.lib.rlb_set_state(self.h, _VP(src.data_ptr())))

    def equilibrium(self, out=None):
        """Truncated equilibrium of the current state for the tubes with
        n_v > 7 (flat state layout; other tubes' entries of ``out`` are left
        as they are, zeros for a new tensor)."""
        if out is None:
            torch = _torch()
            with torch.cuda.stream(self.stream):
                out = torch.zeros(self.state_elems, dtype=self.dtype, device=self.device)
        assert out.numel() >= self.state_elems and out.dtype == self.dtype and out.is_contiguous()
        self._check(self.lib.rlb_equilibrium(self.h, _VP(out.data_ptr())))
        return out

    def tube_view(self, state, tube: int = 0):
        """View [Q, nx] of one tube inside a flat state tensor."""
        off, ld = self.layout(tube)
        t = self.tubes[tube]
        return state[off: off + t.Q * ld].view(t.Q, ld)[:, : t.nx]

    def state_array(self, tube: int = 0) -> np.ndarray:
        """Host FP64 copy [Q, nx] of a tube's current state (synchronizes)."""
        s = self.get_state()
        self.stream.synchronize()
        return self.tube_view(s, tube).double().cpu().numpy()

    def load_array(self, F: np.ndarray, tube: int = 0, state=None):
        """Writes a host [Q, nx] array into a (new) state tensor for set_state."""
        torch = _torch()
        state = torch.zeros(self.state_elems, dtype=self.dtype, device=self.device) if state is None else state
        self.tube_view(state, tube).copy_(torch.as_tensor(F, dtype=self.dtype))
        return state

    def step_noalloc(self, state, nsteps: int = 1, flags=None, stream=None):
        """Advances a caller-owned state tensor in place by nsteps steps with no
        allocation (rlb_step_noalloc); works on a lattice created with
        bind=False.  flags: None or a device int32 tensor of one element that
        receives the sticky flag bits raised during the call."""
        assert state.dtype == self.dtype and state.is_contiguous() and state.numel() >= self.state_elems
        fp = _VP(flags.data_ptr()) if flags is not None else None
        if flags is not None:
            assert flags.element_size() == 4 and flags.numel() >= 1 and flags.device == state.device
        s = stream if stream is not None else self.stream
        self._check(self.lib.rlb_step_noalloc(self.h, _VP(state.data_ptr()), int(nsteps), fp, _VP(s.cuda_stream)))

    def set_tau(self, tau: float, tube: int = 0):
        self._check(self.lib.rlb_set_tau(self.h, tube, float(tau)))

    def info(self, tube: int = 0):
        dt, time, Q = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        self._check(self.lib.rlb_tube_info(self.h, tube, ctypes.byref(dt), ctypes.byref(time), ctypes.byref(Q)))
        return dict(dt=dt.value, time=time.value, Q=Q.value)

    def set_time(self, time: float, tube: int = -1):
        self._check(self.lib.rlb_set_time(self.h, int(tube), float(time)))

    def tables(self, tube: int = 0):
        t = self.tubes[tube]
        xi, wxi, p, wp = (np.zeros(t.q_xi), np.zeros(t.q_xi), np.zeros(t.q_p), np.zeros(t.q_p))
        self._check(self.lib.rlb_tables(self.h, tube, *(a.ctypes.data_as(_DP) for a in (xi, wxi, p, wp))))
        return xi, wxi, p, wp


def _lattice_adjoint_methods():
    def adjoint_step(self, state_n, lam, dL_dtau):
        """lam: dL/df^{n+1} -> dL/df^n (in place); dL_dtau (device FP64, one per tube) is incremented."""
        for t in (state_n, lam):
            assert t.dtype == self.dtype and t.is_contiguous() and t.numel() >= self.state_elems
        assert dL_dtau.dtype.is_floating_point and dL_dtau.element_size() == 8 and dL_dtau.numel() >= len(self.tubes)
        self._check(self.lib.rlb_adjoint_step(self.h, _VP(state_n.data_ptr()), _VP(lam.data_ptr()),
                                              _VP(dL_dtau.data_ptr())))

    def adjoint_segment_size(self, nsteps: int) -> int:
        n = ctypes.c_size_t(0)
        self._check(self.lib.rlb_adjoint_segment_size(self.h, int(nsteps), ctypes.byref(n)))
        return n.value

    def adjoint_segment(self, state0, nsteps: int, scratch, lam, dL_dtau):
        """Reverse sweep over the nsteps steps that start from state0: lam goes from
        dL/df^{n+nsteps} to dL/df^n in place, dL_dtau is incremented.  scratch: a
        device uint8 tensor of at least adjoint_segment_size(nsteps) bytes."""
        for t in (state0, lam):
            assert t.dtype == self.dtype and t.is_contiguous() and t.numel() >= self.state_elems
        assert scratch.is_contiguous() and scratch.element_size() == 1
        assert dL_dtau.dtype.is_floating_point and dL_dtau.element_size() == 8 and dL_dtau.numel() >= len(self.tubes)
        self._check(self.lib.rlb_adjoint_segment(self.h, _VP(state0.data_ptr()), int(nsteps), _VP(scratch.data_ptr()),
                                                 scratch.numel(), _VP(lam.data_ptr()), _VP(dL_dtau.data_ptr())))

    def adjoint_segment_forward(self, state0, nsteps: int, scratch, stream=None):
        """Forward half of adjoint_segment: the segment's states into scratch, on
        `stream` (a torch stream; default: the lattice's)."""
        assert state0.dtype == self.dtype and state0.is_contiguous() and state0.numel() >= self.state_elems
        assert scratch.is_contiguous() and scratch.element_size() == 1
        s = _VP(stream.cuda_stream) if stream is not None else _VP(None)
        self._check(self.lib.rlb_adjoint_segment_forward(self.h, _VP(state0.data_ptr()), int(nsteps),
                                                         _VP(scratch.data_ptr()), scratch.numel(), s))

    def adjoint_segment_reverse(self, nsteps: int, scratch, lam, dL_dtau):
        """Reverse half of adjoint_segment on the lattice's stream."""
        assert lam.dtype == self.dtype and lam.is_contiguous() and lam.numel() >= self.state_elems
        assert scratch.is_contiguous() and scratch.element_size() == 1
        assert dL_dtau.dtype.is_floating_point and dL_dtau.element_size() == 8 and dL_dtau.numel() >= len(self.tubes)
        self._check(self.lib.rlb_adjoint_segment_reverse(self.h, int(nsteps), _VP(scratch.data_ptr()),
                                                         scratch.numel(), _VP(lam.data_ptr()),
                                                         _VP(dL_dtau.data_ptr())))

    def fields_adjoint(self, tube, state, dfields, lam):
        """Writes dL/df of a loss on the fields of `state` into tube's rows of lam."""
        assert dfields.element_size() == 8 and dfields.is_contiguous() and dfields.shape[0] == 10
        self._check(self.lib.rlb_fields_adjoint(self.h, tube, _VP(state.data_ptr()), _VP(dfields.data_ptr()),
                                                dfields.shape[1], _VP(lam.data_ptr())))

    def initial_state_adjoint(self, tube, lam0):
        gl, gr = np.zeros(3), np.zeros(3)
        self._check(self.lib.rlb_initial_state_adjoint(self.h, tube, _VP(lam0.data_ptr()), gl.ctypes.data_as(_DP),
                                                       gr.ctypes.data_as(_DP)))
        return gl, gr

    Lattice.adjoint_step = adjoint_step
    Lattice.adjoint_segment_size = adjoint_segment_size
    Lattice.adjoint_segment = adjoint_segment
    Lattice.adjoint_segment_forward = adjoint_segment_forward
    Lattice.adjoint_segment_reverse = adjoint_segment_reverse
    Lattice.fields_adjoint = fields_adjoint
    Lattice.initial_state_adjoint = initial_state_adjoint


_lattice_adjoint_methods()


def device_copy(dst, src, nbytes: int, stream=None):
    torch = _torch()
    lib = load_library()
    stream = stream if stream is not None else torch.cuda.current_stream()
    st = lib.rlb_device_copy(_VP(dst.data_ptr()), _VP(src.data_ptr()), nbytes, _VP(stream.cuda_stream))
    if st != RLB_OK:
        raise RLBError(st, "device copy failed")


def device_stream(out, a, b, rows: int, ld: int, cols: int, stream=None):
    """out = a (+ b) over [rows][ld] matrices with the stage kernel's memory
    pattern (rlb_device_stream); b may be None."""
    torch = _torch()
    lib = load_library()
    stream = stream if stream is not None else torch.cuda.current_stream()
    st = lib.rlb_device_stream(_VP(out.data_ptr()), _VP(a.data_ptr()), _VP(b.data_ptr()) if b is not None else None,
                               int(rows), int(ld), int(cols), out.element_size(), _VP(stream.cuda_stream))
    if st != RLB_OK:
        raise RLBError(st, "device stream failed")


PLANE_FIELDS = ("N0", "Nx", "Nz", "T00", "T0x", "T0z", "Txx", "Txz", "Tzz", "e", "n", "vx", "vz", "T")


@dataclass
class PlaneSpec:
    """An (x, z) plane; fields mirror ``rlb_plane_desc``."""
    nx: int = 64
    nz: int = 64
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

    def c(self) -> PlaneDesc:
        return PlaneDesc(self.nx, self.nz, self.q_xi, self.q_phi, self.q_p, self.n_v, self.n_p, 0, self.x_min,
                         self.x_max, self.z_min, self.z_max, self.tau, self.cfl, self.dt_tau_max, self.dt,
                         self.T0, self.weno_eps)

    @property
    def Q(self) -> int:
        return self.q_p * self.q_xi * (self.q_phi // 2 + 1)


class Plane:
    """The multi-dimensional model on one (x, z) plane (workspace and stream
    as for a Lattice)."""

    def __init__(self, spec: PlaneSpec, precision: str = "fp64", stream=None, device=None):
        torch = _torch()
        self.lib = load_library()
        self.spec = spec
        self.precision = precision
        prec = {"fp64": RLB_FP64, "fp32": RLB_FP32}[precision]
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        h = _VP()
        st = self.lib.rlb_plane_create(ctypes.byref(spec.c()), prec, ctypes.byref(h))
        if st != RLB_OK:
            raise RLBError(st, self.lib.rlb_plane_last_error(None).decode())
        self.h = h
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        size = ctypes.c_size_t()
        self._check(self.lib.rlb_plane_workspace_size(self.h, ctypes.byref(size)))
        self._ws = torch.empty(size.value + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.lib.rlb_plane_bind(self.h, _VP(self._ws_ptr), size.value, _VP(self.stream.cuda_stream)))
        n, ld = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.rlb_plane_layout(self.h, ctypes.byref(n), ctypes.byref(ld)))
        self.state_elems, self.ldx = n.value, ld.value

    def _check(self, st: int):
        if st != RLB_OK:
            raise RLBError(st, self.lib.rlb_plane_last_error(self.h).decode() or self.lib.rlb_status_string(st).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.rlb_plane_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_initial_fields(self, fields):
        """fields: [4, nz, nx] (P, n, u^x, u^z), numpy array or tensor."""
        torch = _torch()
        with torch.cuda.stream(self.stream):
            f = torch.as_tensor(fields, dtype=torch.float64).to(self.device).contiguous()
        assert tuple(f.shape) == (4, self.spec.nz, self.spec.nx)
        self._check(self.lib.rlb_plane_set_initial_fields(self.h, _VP(f.data_ptr())))
        self.stream.synchronize()  # f may be freed after this call returns

    def step(self, nsteps: int = 1):
        self._check(self.lib.rlb_plane_step(self.h, int(nsteps)))

    def fields(self, out=None):
        """Device tensor [14, nz, nx] (FP64), queued on the stream."""
        torch = _torch()
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty((14, self.spec.nz, self.spec.nx), dtype=torch.float64, device=self.device)
        self._check(self.lib.rlb_plane_fields(self.h, _VP(out.data_ptr())))
        return out

    def moments(self) -> np.ndarray:
        """Host copy [14, nz, nx] of the fields; checks the sticky flag."""
        f = self.fields()
        self.stream.synchronize()
        out = f.cpu().numpy()
        self.check()
        return out

    def new_state(self):
        torch = _torch()
        return torch.empty(self.state_elems, dtype=self.dtype, device=self.device)

    def get_state(self, out=None):
        out = self.new_state() if out is None else out
        self._check(self.lib.rlb_plane_get_state(self.h, _VP(out.data_ptr())))
        return out

    def set_state(self, src):
        assert src.numel() >= self.state_elems and src.dtype == self.dtype and src.is_contiguous()
        self._check(self.lib.rlb_plane_set_state(self.h, _VP(src.data_ptr())))

    def state_array(self) -> np.ndarray:
        """Host FP64 copy [Q, nz, nx] of the current state (synchronizes)."""
        s = self.get_state()
        self.stream.synchronize()
        Q = self.spec.Q
        return s.view(Q, self.spec.nz, self.ldx)[:, :, :self.spec.nx].double().cpu().numpy()

    def load_array(self, F: np.ndarray):
        """A state tensor holding the host array F[Q, nz, nx]."""
        torch = _torch()
        Q = self.spec.Q
        s = torch.zeros((Q, self.spec.nz, self.ldx), dtype=self.dtype)
        s[:, :, :self.spec.nx] = torch.as_tensor(F, dtype=self.dtype)
        return s.reshape(-1).to(self.device)

    def info(self):
        dt, t, Q = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        self._check(self.lib.rlb_plane_info(self.h, ctypes.byref(dt), ctypes.byref(t), ctypes.byref(Q)))
        return dict(dt=dt.value, time=t.value, Q=Q.value)

    def check(self):
        self._check(self.lib.rlb_plane_check(self.h))

    def flags(self) -> dict:
        f = ctypes.c_uint32()
        self._check(self.lib.rlb_plane_flags(self.h, ctypes.byref(f)))
        return dict(nonphysical=bool(f.value & RLB_FLAG_NONPHYSICAL), fast_flow=bool(f.value & RLB_FLAG_FAST_FLOW))


BOX_FIELDS = ("N0", "Nx", "Ny", "Nz", "T00", "T0x", "T0y", "T0z", "Txx", "Txy", "Txz", "Tyy", "Tyz", "Tzz",
              "e", "n", "vx", "vy", "vz", "T")


@dataclass
class BoxSpec:
    """An (x, y, z) box; fields mirror ``rlb_box_desc``."""
    nx: int = 32
    ny: int = 32
    nz: int = 32
    q_xi: int = 8
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

    def c(self) -> BoxDesc:
        return BoxDesc(self.nx, self.ny, self.nz, self.q_xi, self.q_phi, self.q_p, self.n_v, self.n_p, self.x_min,
                       self.x_max, self.y_min, self.y_max, self.z_min, self.z_max, self.tau, self.cfl,
                       self.dt_tau_max, self.dt, self.T0, self.weno_eps)

    @property
    def Q(self) -> int:
        return self.q_p * self.q_xi * self.q_phi

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


class Box:
    """The multi-dimensional model on an (x, y, z) box (workspace and stream
    as for a Lattice)."""

    def __init__(self, spec: BoxSpec, precision: str = "fp64", stream=None, device=None):
        torch = _torch()
        self.lib = load_library()
        self.spec = spec
        self.precision = precision
        prec = {"fp64": RLB_FP64, "fp32": RLB_FP32}[precision]
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        h = _VP()
        st = self.lib.rlb_box_create(ctypes.byref(spec.c()), prec, ctypes.byref(h))
        if st != RLB_OK:
            raise RLBError(st, self.lib.rlb_box_last_error(None).decode())
        self.h = h
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        size = ctypes.c_size_t()
        self._check(self.lib.rlb_box_workspace_size(self.h, ctypes.byref(size)))
        self._ws = torch.empty(size.value + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.lib.rlb_box_bind(self.h, _VP(self._ws_ptr), size.value, _VP(self.stream.cuda_stream)))
        n, ld = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.rlb_box_layout(self.h, ctypes.byref(n), ctypes.byref(ld)))
        self.state_elems, self.ldx = n.value, ld.value

    def _check(self, st: int):
        if st != RLB_OK:
            raise RLBError(st, self.lib.rlb_box_last_error(self.h).decode() or self.lib.rlb_status_string(st).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.rlb_box_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.spec.nz, self.spec.ny, self.spec.nx)

    def set_initial_fields(self, fields):
        """fields: [5, nz, ny, nx] (P, n, u^x, u^y, u^z), numpy array or tensor."""
        torch = _torch()
        with torch.cuda.stream(self.stream):
            f = torch.as_tensor(fields, dtype=torch.float64).to(self.device).contiguous()
        assert tuple(f.shape) == (5,) + self.shape
        self._check(self.lib.rlb_box_set_initial_fields(self.h, _VP(f.data_ptr())))
        self.stream.synchronize()  # f may be freed after this call returns

    def step(self, nsteps: int = 1):
        self._check(self.lib.rlb_box_step(self.h, int(nsteps)))

    def fields(self, out=None):
        """Device tensor [20, nz, ny, nx] (FP64), queued on the stream."""
        torch = _torch()
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty((20,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.rlb_box_fields(self.h, _VP(out.data_ptr())))
        return out

    def moments(self) -> np.ndarray:
        """Host copy [20, nz, ny, nx] of the fields; checks the sticky flag."""
        f = self.fields()
        self.stream.synchronize()
        out = f.cpu().numpy()
        self.check()
        return out

    def new_state(self):
        torch = _torch()
        return torch.empty(self.state_elems, dtype=self.dtype, device=self.device)

    def get_state(self, out=None):
        out = self.new_state() if out is None else out
        self._check(self.lib.rlb_box_get_state(self.h, _VP(out.data_ptr())))
        return out

    def set_state(self, src):
        assert src.numel() >= self.state_elems and src.dtype == self.dtype and src.is_contiguous()
        self._check(self.lib.rlb_box_set_state(self.h, _VP(src.data_ptr())))

    def state_array(self) -> np.ndarray:
        """Host FP64 copy [Q, nz, ny, nx] of the current state (synchronizes)."""
        s = self.get_state()
        self.stream.synchronize()
        return s.view((self.spec.Q,) + self.shape[:2] + (self.ldx,))[..., :self.spec.nx].double().cpu().numpy()

    def load_array(self, F: np.ndarray):
        """A state tensor holding the host array F[Q, nz, ny, nx]."""
        torch = _torch()
        s = torch.zeros((self.spec.Q,) + self.shape[:2] + (self.ldx,), dtype=self.dtype)
        s[..., :self.spec.nx] = torch.as_tensor(F, dtype=self.dtype)
        return s.reshape(-1).to(self.device)

    def info(self):
        dt, t, Q = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        self._check(self.lib.rlb_box_info(self.h, ctypes.byref(dt), ctypes.byref(t), ctypes.byref(Q)))
        return dict(dt=dt.value, time=t.value, Q=Q.value)

    def check(self):
        self._check(self.lib.rlb_box_check(self.h))

    def flags(self) -> dict:
        f = ctypes.c_uint32()
        self._check(self.lib.rlb_box_flags(self.h, ctypes.byref(f)))
        return dict(nonphysical=bool(f.value & RLB_FLAG_NONPHYSICAL), fast_flow=bool(f.value & RLB_FLAG_FAST_FLOW))
