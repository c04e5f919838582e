"""The hand-written discrete adjoint on the GPU against the oracle's exact
tangent-linear model (dual numbers through the same steps).

Dot-product identity: for one step f^{n+1} = S(f^n) with Jacobian J, the GPU
adjoint returns J^T lambda; the oracle returns J v exactly (to rounding), so
<J^T lambda, v> = <lambda, J v> must hold to ~1e-12 relative in FP64, and
dL/dtau must equal <lambda, dS/dtau>.  The gradient of the profile loss with
respect to (tau, P_L, n_L) is checked against the oracle's forward-mode
gradient and against central differences of the GPU forward (h = 1e-6).
"""
import math

import numpy as np
import pytest

from tests.helpers import oracle_tube

pytestmark = pytest.mark.gpu

SOD_L = (1.0, 1.0, 0.0)
SOD_R = (0.1, 0.125, 0.0)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def _lattice(params, precision="fp64"):
    from paper_1608_03004_amd import Lattice, Tube
    return Lattice([Tube(**p) for p in params], precision=precision, adjoint=True)


CASES = [
    dict(nx=96, q_xi=8, q_p=3, tau=1e-2),
    dict(nx=70, q_xi=5, q_p=3, tau=5e-3),                     # odd q_xi
    dict(nx=64, q_xi=6, q_p=4, tau=2e-2),                     # q_p = 4 group
    dict(nx=40, q_xi=7, q_p=5, n_p=3, n_v=7, tau=3e-2),       # generic group
    dict(nx=80, q_xi=8, q_p=3, tau=1e-2, T0=0.8),
    dict(nx=300, q_xi=4, q_p=3, tau=1e-3),                    # several tiles
    # the high-order form (n_v > 7): equilibrium from the matrix-core pre-pass
    dict(nx=48, q_xi=16, q_p=3, n_v=15, tau=1e-2),
    dict(nx=36, q_xi=9, q_p=3, n_v=8, tau=2e-2),              # odd q_xi: the middle node
    dict(nx=40, q_xi=64, q_p=3, n_v=63, tau=2e-2),            # largest two-tile form
    dict(nx=24, q_xi=128, q_p=3, n_v=127, tau=2e-2),          # four row tiles
]


@pytest.mark.parametrize("params", CASES, ids=[f"case{k}" for k in range(len(CASES))])
def test_dot_product_identity_one_step(torch_cuda, params):
    torch = torch_cuda
    from oracle import oracle as O
    t = oracle_tube(params)
    left, right = (1.0, 1.0, 0.2), (0.2, 0.3, -0.1)
    F = O.run(t, left, right, 15)  # a non-trivial physical state
    rng = np.random.default_rng(7)
    v = rng.standard_normal(F.shape)
    lam = rng.standard_normal(F.shape)
    _, Jv = O.step_tangent(t, F, v, 0.0, 1)
    _, dFdtau = O.step_tangent(t, F, np.zeros_like(F), 1.0, 1)
    lat = _lattice([params])
    lat.set_initial_state(left, right)
    Fs = lat.load_array(F)
    ls = lat.load_array(lam)
    dtau = torch.zeros(1, dtype=torch.float64, device=lat.device)
    lat.adjoint_step(Fs, ls, dtau)
    torch.cuda.synchronize()
    JTl = lat.tube_view(ls, 0).cpu().numpy()
    lhs = float(np.sum(JTl * v))
    rhs = float(np.sum(lam * Jv))
    scale = np.sqrt(np.sum(JTl ** 2) * np.sum(v ** 2))
    assert abs(lhs - rhs) < 1e-12 * scale, (lhs, rhs)
    # column-wise: the adjoint of every point against the tangent of unit directions is implied;
    # the tau derivative
    g_tau = float(dtau[0])
    ref_tau = float(np.sum(lam * dFdtau))
    assert abs(g_tau - ref_tau) < 1e-11 * max(abs(ref_tau), np.sqrt(np.sum(lam ** 2) * np.sum(dFdtau ** 2))), (g_tau, ref_tau)


def test_adjoint_of_collisionless_step_is_the_transposed_stencil(torch_cuda):
    torch = torch_cuda
    from oracle import oracle as O
    params = dict(nx=50, q_xi=6, q_p=3, tau=math.inf)
    t = oracle_tube(params)
    F = O.run(t, SOD_L, SOD_R, 8)
    rng = np.random.default_rng(3)
    v, lam = rng.standard_normal(F.shape), rng.standard_normal(F.shape)
    _, Jv = O.step_tangent(t, F, v, 0.0, 1)
    lat = _lattice([params])
    lat.set_initial_state(SOD_L, SOD_R)
    ls = lat.load_array(lam)
    dtau = torch.zeros(1, dtype=torch.float64, device=lat.device)
    lat.adjoint_step(lat.load_array(F), ls, dtau)
    JTl = lat.tube_view(ls, 0).cpu().numpy()
    assert abs(np.sum(JTl * v) - np.sum(lam * Jv)) < 1e-12 * np.sqrt(np.sum(JTl ** 2) * np.sum(v ** 2))
    assert float(dtau[0]) == 0.0


@pytest.mark.parametrize("params", [dict(nx=120, q_xi=8, q_p=3, tau=1e-2),
                                    dict(nx=120, q_xi=16, q_p=3, n_v=15, tau=1e-2),
                                    dict(nx=300, q_xi=33, q_p=3, n_v=30, tau=1e-2)],
                         ids=["low_order", "high_order", "high_order_odd_two_blocks"])
def test_fields_and_initial_state_adjoints(torch_cuda, params):
    torch = torch_cuda
    from oracle import oracle as O
    t = oracle_tube(params)
    left, right = (1.0, 1.0, 0.3), (0.2, 0.4, -0.2)
    F = O.run(t, left, right, 10)
    rng = np.random.default_rng(11)
    w = rng.standard_normal((10, t.nx))
    v = rng.standard_normal(F.shape)
    _, dfields = O.fields_tangent(t, F, v)
    lat = _lattice([params])
    lat.set_initial_state(left, right)
    lam = lat.new_state().zero_()
    lat.fields_adjoint(0, lat.load_array(F), torch.tensor(w, device=lat.device), lam)
    g = lat.tube_view(lam, 0).cpu().numpy()
    lhs, rhs = np.sum(g * v), np.sum(w * dfields)
    assert abs(lhs - rhs) < 1e-12 * np.sqrt(np.sum(g ** 2) * np.sum(v ** 2))
    # initial state: <lambda0, dF0/dtheta> = grad . dtheta
    lam0 = rng.standard_normal(F.shape)
    dl, dr = (0.3, -0.2, 0.5), (0.1, 0.7, -0.4)
    _, dF0 = O.init_tangent(t, left, right, dl, dr)
    gl, gr = lat.initial_state_adjoint(0, lat.load_array(lam0))
    lhs = float(np.dot(gl, dl) + np.dot(gr, dr))
    rhs = float(np.sum(lam0 * dF0))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(rhs))


def _loss_and_grad(params, nsteps, start, target_e, every, precision="fp64"):
    import torch
    from paper_1608_03004_amd.autograd import profile_loss
    lat = _lattice([params], precision)
    dev, f64 = lat.device, torch.float64
    theta = [torch.tensor(v, dtype=f64, device=dev, requires_grad=True) for v in start]
    L = profile_loss(*theta, torch.tensor(0.1, dtype=f64, device=dev), torch.tensor(0.125, dtype=f64, device=dev),
                     lat, nsteps, target_e, every)
    L.backward()
    return float(L.detach()), np.array([float(p.grad) for p in theta]), lat


def _gpu_loss(params, nsteps, theta, target_e):
    import torch
    from paper_1608_03004_amd import Lattice, Tube
    lat = Lattice([Tube(**params)], precision="fp64")
    lat.set_initial_state((theta[1], theta[2], 0.0), SOD_R)
    lat.set_tau(theta[0])
    lat.step(nsteps)
    e = lat.moments(0)[5]
    return float(np.sum((e - target_e) ** 2) * (params.get("z_max", 0.5) - params.get("z_min", -0.5)) / params["nx"])


def test_profile_gradient_against_oracle_forward_mode_and_differences(torch_cuda):
    torch = torch_cuda
    from oracle import oracle as O
    # the adjoint configuration scaled down: Q = 32 x 3, 200 steps; dt fixed
    params = dict(nx=512, q_xi=32, q_p=3, tau=0.02, dt=0.5 / 512)
    nsteps = 200
    start = (0.02, 1.0, 1.0)
    # target profile from the forward at (tau = 0.05, P_L = 1.5)
    t_tgt = oracle_tube(dict(params, tau=0.05))
    target = O.fields(t_tgt, O.run(t_tgt, (1.5, 1.0, 0.0), SOD_R, nsteps))[5]
    target_e = torch.tensor(target, dtype=torch.float64, device="cuda")
    L, grad, _ = _loss_and_grad(params, nsteps, start, target_e, every=0)
    # oracle forward mode: one tangent run per parameter
    t = oracle_tube(params)
    dz = 1.0 / params["nx"]
    ref = []
    for k in range(3):
        dl = (1.0, 0.0, 0.0) if k == 1 else ((0.0, 1.0, 0.0) if k == 2 else (0.0, 0.0, 0.0))
        F0, dF0 = O.init_tangent(t, (start[1], start[2], 0.0), SOD_R, dl, (0.0, 0.0, 0.0))
        F, dF = O.step_tangent(t, F0, dF0, 1.0 if k == 0 else 0.0, nsteps)
        f, df = O.fields_tangent(t, F, dF)
        ref.append(float(np.sum(2 * dz * (f[5] - target) * df[5])))
    ref = np.array(ref)
    gnorm = np.abs(ref).max()
    print(f"[adjoint grad] gpu {grad} oracle {ref}", flush=True)
    assert abs(grad[0] - ref[0]) < 1e-9 * abs(ref[0])
    assert abs(grad[1] - ref[1]) < 1e-9 * abs(ref[1])
    # d e / d n_L vanishes identically: e depends on the initial P and u only
    assert abs(grad[2]) < 1e-6 * gnorm and abs(ref[2]) < 1e-6 * gnorm
    # central differences of the GPU forward, h = 1e-6 (relative)
    for k in (0, 1):
        h = 1e-6 * start[k]
        tp = list(start); tp[k] += h
        tm = list(start); tm[k] -= h
        fd = (_gpu_loss(params, nsteps, tp, target) - _gpu_loss(params, nsteps, tm, target)) / (2 * h)
        assert abs(fd - grad[k]) < 1e-6 * abs(grad[k]), (k, fd, grad[k])


def test_checkpointed_gradient_equals_store_all(torch_cuda):
    torch = torch_cuda
    params = dict(nx=256, q_xi=16, q_p=3, tau=0.03, dt=0.5 / 256)
    nsteps = 37
    target = torch.linspace(0.2, 2.5, 256, dtype=torch.float64, device="cuda")
    _, g_ck, _ = _loss_and_grad(params, nsteps, (0.03, 1.2, 0.9), target, every=0)
    _, g_all, _ = _loss_and_grad(params, nsteps, (0.03, 1.2, 0.9), target, every=1)
    _, g_5, _ = _loss_and_grad(params, nsteps, (0.03, 1.2, 0.9), target, every=5)
    assert np.array_equal(g_ck, g_all) and np.array_equal(g_5, g_all)


def test_fp32_adjoint_against_fp64_adjoint(torch_cuda):
    torch = torch_cuda
    params = dict(nx=512, q_xi=32, q_p=3, tau=0.02, dt=0.5 / 512)
    nsteps = 100
    target = torch.linspace(0.3, 2.8, 512, dtype=torch.float64, device="cuda")
    _, g64, _ = _loss_and_grad(params, nsteps, (0.02, 1.0, 1.0), target, every=0, precision="fp64")
    _, g32, _ = _loss_and_grad(params, nsteps, (0.02, 1.0, 1.0), target, every=0, precision="fp32")
    print(f"[adjoint fp32 vs fp64] {g32} {g64}", flush=True)
    scale = np.abs(g64).max()
    assert np.abs(g32 - g64).max() < 1e-3 * scale


@pytest.mark.parametrize("params", [dict(nx=300, q_xi=12, q_p=3, tau=2e-2),
                                    dict(nx=300, q_xi=32, q_p=3, n_v=31, tau=2e-2)], ids=["low_order", "high_order"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_segment_equals_step_by_step_adjoint(torch_cuda, precision, params):
    # One reverse sweep over a segment (stage states recomputed once and kept)
    # against rlb_adjoint_step applied to each recomputed state in turn; the
    # high-order form's forward recompute on a side stream writes its own
    # equilibrium buffer, not the one the reverse half reads.
    torch = torch_cuda
    lat = _lattice([params], precision)
    lat.set_initial_state((1.0, 1.0, 0.1), (0.2, 0.3, -0.1))
    lat.step(4)
    state0 = lat.get_state().clone()
    nseg = 6
    states = [state0]
    for _ in range(nseg - 1):
        lat.step(1)
        states.append(lat.get_state().clone())
    g = torch.Generator(device="cuda").manual_seed(3)
    lam0 = torch.rand(lat.state_elems, dtype=lat.dtype, device="cuda", generator=g) - 0.5
    lam_a, lam_b = lam0.clone(), lam0.clone()
    da = torch.zeros(1, dtype=torch.float64, device="cuda")
    db = torch.zeros(1, dtype=torch.float64, device="cuda")
    for F in reversed(states):
        lat.adjoint_step(F, lam_a, da)
    scratch = torch.empty(lat.adjoint_segment_size(nseg), dtype=torch.uint8, device="cuda")
    lat.adjoint_segment(state0, nseg, scratch, lam_b, db)
    torch.cuda.synchronize()
    assert torch.equal(lam_a, lam_b) and torch.equal(da, db)
    # the two halves, the forward on a side stream
    lam_c, dc = lam0.clone(), torch.zeros(1, dtype=torch.float64, device="cuda")
    scratch2 = torch.empty_like(scratch)
    side = torch.cuda.Stream()
    side.wait_stream(lat.stream)
    lat.adjoint_segment_forward(state0, nseg, scratch2, side)
    ev = torch.cuda.Event()
    ev.record(side)
    lat.stream.wait_event(ev)
    lat.adjoint_segment_reverse(nseg, scratch2, lam_c, dc)
    torch.cuda.synchronize()
    assert torch.equal(lam_a, lam_c) and torch.equal(da, dc)
    # the lattice's own state is untouched by the sweep
    assert torch.equal(lat.tube_view(lat.get_state()), lat.tube_view(states[-1]))


def test_high_order_profile_gradient_against_differences(torch_cuda):
    # the gradient of the profile loss through the high-order form (Q = 32 x 3,
    # N_v = 31, 60 steps) against central differences of the GPU forward
    torch = torch_cuda
    params = dict(nx=256, q_xi=32, q_p=3, n_v=31, tau=0.02, dt=0.5 / 256)
    nsteps = 60
    start = (0.02, 1.0, 1.0)
    target = torch.linspace(0.3, 2.8, 256, dtype=torch.float64, device="cuda")
    _, grad, _ = _loss_and_grad(params, nsteps, start, target, every=7)
    print(f"[high-order adjoint grad] {grad}", flush=True)
    for k in (0, 1):
        h = 1e-6 * start[k]
        tp = list(start); tp[k] += h
        tm = list(start); tm[k] -= h
        tgt = target.cpu().numpy()
        fd = (_gpu_loss(params, nsteps, tp, tgt) - _gpu_loss(params, nsteps, tm, tgt)) / (2 * h)
        assert abs(fd - grad[k]) < 1e-6 * abs(grad[k]), (k, fd, grad[k])
