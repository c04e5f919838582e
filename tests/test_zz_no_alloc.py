"""The allocation-free step (rlb_step_noalloc) against rlb_step on a bound
lattice, through the C interface.

Both run the same kernels in the same order on the same state (the records
are recomputed from the state in both), so the states must agree to the bit.
Two calls in a row, the second on a smaller lattice, check that the shared
scratch array's leftover contents from the first call do not leak into the
second; a third call repeats the first lattice after the smaller one.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SOD_L, SOD_R = (1.0, 1.0, 0.0), (0.1, 0.125, 0.0)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def _reference(tubes, precision, lefts, rights, warm, nsteps):
    """(state after `warm` steps, state after warm + nsteps) of a bound lattice."""
    from paper_1608_03004_amd import Lattice
    lat = Lattice(tubes, precision=precision)
    lat.set_initial_states(lefts, rights)
    lat.step(warm)
    s0 = lat.get_state().clone()
    lat.step(nsteps)
    ref = lat.get_state().clone()
    lat.check()
    lat.stream.synchronize()
    return s0, ref


def _noalloc(torch, tubes, precision, s0, nsteps):
    from paper_1608_03004_amd import Lattice
    lat = Lattice(tubes, precision=precision, bind=False)
    state = s0.clone()
    flags = torch.full((1,), -1, dtype=torch.int32, device=state.device)
    lat.step_noalloc(state, nsteps, flags)
    lat.stream.synchronize()
    return state, int(flags.item())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_step_on_two_calls(torch_cuda, precision):
    torch = torch_cuda
    from paper_1608_03004_amd import Tube
    big = [Tube(nx=700, q_xi=8, q_p=3, tau=1e-2), Tube(nx=333, q_xi=16, q_p=4, tau=1e-1),
           Tube(nx=200, q_xi=16, q_p=3, n_v=15, tau=5e-3)]          # low- and high-order groups
    small = [Tube(nx=90, q_xi=6, q_p=3, tau=2e-2)]                   # one ragged tile, node-split launch
    lb, rb = [SOD_L, (2.0, 1.5, 0.2), (1.0, 1.0, 0.3)], [SOD_R, (0.1, 0.125, 0.0), (0.3, 0.5, -0.4)]
    s0_big, ref_big = _reference(big, precision, lb, rb, 3, 9)
    s0_small, ref_small = _reference(small, precision, [SOD_L], [SOD_R], 2, 5)
    # first call: the larger lattice
    got, fl = _noalloc(torch, big, precision, s0_big, 9)
    print(f"[noalloc {precision}] big: flags {fl}, max |diff| {float((got - ref_big).abs().max()):.3e}", flush=True)
    assert fl == 0
    assert torch.equal(got, ref_big)
    # second call: a smaller lattice on the same scratch
    got, fl = _noalloc(torch, small, precision, s0_small, 5)
    print(f"[noalloc {precision}] small: flags {fl}, max |diff| {float((got - ref_small).abs().max()):.3e}",
          flush=True)
    assert fl == 0
    assert torch.equal(got, ref_small)
    # and the larger one again after it
    got, fl = _noalloc(torch, big, precision, s0_big, 9)
    assert fl == 0 and torch.equal(got, ref_big)


def test_noalloc_zero_steps_and_flag(torch_cuda):
    torch = torch_cuda
    from paper_1608_03004_amd import Lattice, Tube
    tubes = [Tube(nx=64, q_xi=8, q_p=3, tau=1e-2)]
    lat = Lattice(tubes, precision="fp64", bind=False)
    good = Lattice(tubes, precision="fp64")
    good.set_initial_state(SOD_L, SOD_R)
    s = good.get_state().clone()
    before = s.clone()
    flags = torch.full((1,), 7, dtype=torch.int32, device=s.device)
    lat.step_noalloc(s, 0, flags)
    lat.stream.synchronize()
    assert torch.equal(s, before) and int(flags.item()) == 0
    # a state of negative densities raises the non-physical bit in the
    # caller's word (an ordinary run: the kernels only record it)
    bad = good.load_array(np.full((24, 64), -0.1))
    lat.step_noalloc(bad, 1, flags)
    lat.stream.synchronize()
    assert int(flags.item()) & 1
    # and a good state afterwards clears it again
    lat.step_noalloc(s, 1, flags)
    lat.stream.synchronize()
    assert int(flags.item()) == 0


def test_noalloc_rejects_lattices_beyond_the_scratch(torch_cuda):
    # a lattice whose step needs more than the static array: rejected on the
    # host before any device work (the state pointer is never touched)
    import ctypes
    torch = torch_cuda
    from paper_1608_03004_amd import Lattice, Tube
    lat = Lattice([Tube(nx=1 << 20, q_xi=64, q_p=4, tau=1e-2)], precision="fp32", bind=False)
    dummy = torch.zeros(8, dtype=torch.float32, device="cuda")
    st = lat.lib.rlb_step_noalloc(lat.h, ctypes.c_void_p(dummy.data_ptr()), 1, None,
                                  ctypes.c_void_p(lat.stream.cuda_stream))
    assert st == -1 and b"scratch" in lat.lib.rlb_last_error(lat.h)
    assert int(dummy.abs().sum().item()) == 0
