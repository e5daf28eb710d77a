"""Pins of the oracle's adjoint reference: the reverse-mode gradient of J = w0 mean P + w1 mean T with
frozen WENO weights equals central finite differences of the forward that replays the recorded weights
(directional derivatives in the force scalings s and in the initial field); the frozen-weight
linearisation differs from the true derivative by a small, reported amount."""
import numpy as np
import pytest
import torch

from oracle import WenoControl, rotor_gradient, rotor_objective
from synth import make_case

F64 = torch.float64
W = (1.0, 0.5)
NSTEPS = 2


@pytest.fixture(scope="module")
def case():
    return make_case("adjoint", grid=(20, 20, 20))


def _frozen_fd(cfg, s0, v, h, q0=None, dq=None):
    store = WenoControl("record")
    rotor_objective(cfg, torch.tensor(s0), NSTEPS, W, store, q0=q0)
    vals = []
    for sign in (1.0, -1.0):
        ctl = WenoControl("replay", store.store)
        s = torch.tensor(s0 + sign * h * v)
        qq = None if dq is None else q0 + sign * h * dq
        J, _ = rotor_objective(cfg, s, NSTEPS, W, ctl, q0=qq)
        vals.append(float(J))
    return (vals[0] - vals[1]) / (2 * h)


def test_scaling_gradient_matches_frozen_finite_differences(case):
    rng = np.random.default_rng(0)
    n = case.rotor.n_act
    s0 = 1.0 + 0.1 * rng.standard_normal(n)
    J, g = rotor_gradient(case, s0, NSTEPS, W, frozen=True)
    v = rng.standard_normal(n)
    fd = _frozen_fd(case, s0, v, 1e-3)
    ad = float(g.numpy() @ v)
    assert abs(fd - ad) < 1e-8 * abs(ad), (fd, ad)


def test_field_gradient_matches_frozen_finite_differences(case):
    rng = np.random.default_rng(1)
    n = case.rotor.n_act
    s0 = np.ones(n)
    q0 = torch.tensor(case.q0).clone().requires_grad_(True)
    s = torch.tensor(s0)
    J, _ = rotor_objective(case, s, NSTEPS, W, WenoControl("detach"), q0=q0)
    J.backward()
    gq = q0.grad.detach()
    dq = torch.tensor(rng.standard_normal(case.q0.shape))
    dq[0] *= 0.01
    fd = _frozen_fd(case, s0, np.zeros(n), 1e-4, q0=torch.tensor(case.q0), dq=dq)
    ad = float((gq * dq).sum())
    assert abs(fd - ad) < 1e-7 * abs(ad), (fd, ad)


def test_frozen_weights_close_to_true_derivative(case):
    n = case.rotor.n_act
    _, gf = rotor_gradient(case, np.ones(n), NSTEPS, W, frozen=True)
    _, gt = rotor_gradient(case, np.ones(n), NSTEPS, W, frozen=False)
    rel = float((gf - gt).norm() / gt.norm())
    print(f"frozen-weight gradient error (relative L2): {rel:.3e}")
    assert rel < 1e-2


def _body_case(case):
    """The 20^3 rotor box with the tower and nacelle behind the rotor, its points at rest but given a
    prescribed velocity (a moving surface), so that the forcing targets a non-zero v-bar."""
    from dataclasses import replace
    from synth.cases import tower_and_nacelle
    ib = tower_and_nacelle(case.rotor.hub, 1.0, case.dx, spacing=0.5 * case.dx, z_ground=2.0 * case.dx)
    rng = np.random.default_rng(7)
    ib = replace(ib, vel=0.2 * rng.standard_normal((ib.n, 3)))
    return case.with_(ibm=ib)


def test_forcing_transpose_is_the_closed_form(case):
    # the S direct-forcing iterations are affine per cell: m_S = c m + (1 - c) rho v-bar with
    # c = (1 - V-bar/|Omega|)^S, so the reverse mode through ibm_apply must give lambda_m c and
    # lambda_rho + (1 - c) v-bar . lambda_m at the forced cells and leave the rest unchanged
    from oracle.gks_oracle import ibm_apply, ibm_setup
    cfg = _body_case(case)
    cache = ibm_setup(cfg, cfg.ibm)
    rng = np.random.default_rng(3)
    Q = torch.tensor(cfg.q0).clone().requires_grad_(True)
    lam = torch.tensor(rng.standard_normal(cfg.q0.shape))
    iters, dt = 3, 1e-3
    Qn, _ = ibm_apply(Q, dt, cfg, cache, iters)
    (g,) = torch.autograd.grad(Qn, Q, lam)
    ref = lam.clone()
    i, j, k = (cache.vbar_index[:, a] for a in range(3))
    c = (1.0 - cache.vbar / cache.vol) ** iters
    lm = lam[1:, k, j, i]
    ref[1:, k, j, i] = lm * torch.tensor(c)
    ref[0, k, j, i] = lam[0, k, j, i] + torch.tensor(1.0 - c) * (torch.tensor(cache.vbar_vel.T) * lm).sum(0)
    assert len(cache.vbar) > 50 and np.abs(cache.vbar_vel).max() > 0.01
    assert torch.allclose(g, ref, rtol=1e-13, atol=1e-15)


def test_body_at_rest_field_gradient_matches_frozen_finite_differences(case):
    # the whole window with the forced body: reverse mode against central differences of the forward
    # that replays the recorded WENO weights, along a random direction of the initial field
    cfg = _body_case(case)
    rng = np.random.default_rng(4)
    n = cfg.rotor.n_act
    s0 = 1.0 + 0.1 * rng.standard_normal(n)
    q0 = torch.tensor(cfg.q0).clone().requires_grad_(True)
    J, _ = rotor_objective(cfg, torch.tensor(s0), NSTEPS, W, WenoControl("detach"), q0=q0)
    J.backward()
    dq = torch.tensor(rng.standard_normal(cfg.q0.shape))
    dq[0] *= 0.01
    fd = _frozen_fd(cfg, s0, np.zeros(n), 1e-4, q0=torch.tensor(cfg.q0), dq=dq)
    ad = float((q0.grad * dq).sum())
    assert abs(fd - ad) < 1e-7 * abs(ad), (fd, ad)
    # and in the force scalings
    _, g = rotor_gradient(cfg, s0, NSTEPS, W, frozen=True)
    v = rng.standard_normal(n)
    fd = _frozen_fd(cfg, s0, v, 1e-3)
    assert abs(fd - float(g.numpy() @ v)) < 1e-8 * abs(fd)


def _inflow_case():
    """The rotor workload's boundaries (inflow x-, outflow x+, periodic y, slip z) on 48 x 24 x 24 with a
    fixed dt, the hub moved to 7.2 cells from the inflow side so that the inflow ghost cells reach the
    actuator points within the window."""
    from dataclasses import replace
    cfg = make_case("alm", grid=(48, 24, 24))
    return cfg.with_(cfl=0.0, dt_fixed=0.3 * cfg.dx / 11.0, rotor=replace(cfg.rotor, hub=(0.9, 1.5, 1.5)))


def test_inflow_window_field_gradient_matches_frozen_finite_differences():
    # reverse mode through the Riemann-invariant inflow ghost cells, along a perturbation of the cells
    # next to the inflow side, against central differences of the weight-replaying forward
    cfg = _inflow_case()
    assert cfg.bc[0] == "inflow" and cfg.bc[1] == "outflow" and cfg.bc[4] == "slip"
    rng = np.random.default_rng(6)
    n = cfg.rotor.n_act
    s0 = np.ones(n)
    q0 = torch.tensor(cfg.q0).clone().requires_grad_(True)
    J, _ = rotor_objective(cfg, torch.tensor(s0), NSTEPS, W, WenoControl("detach"), q0=q0)
    J.backward()
    dq = torch.zeros(cfg.q0.shape, dtype=F64)
    dq[:, :, :, :4] = torch.tensor(rng.standard_normal((4, cfg.nz, cfg.ny, 4)))
    dq[0] *= 0.01
    fd = _frozen_fd(cfg, s0, np.zeros(n), 1e-4, q0=torch.tensor(cfg.q0), dq=dq)
    ad = float((q0.grad * dq).sum())
    assert abs(ad) > 1e-6
    assert abs(fd - ad) < 1e-6 * abs(ad), (fd, ad)


def _stretched_case():
    """The locally refined grid of Section 4.3.3 (the rotor in a uniform block with dx = 0.125 and
    dy = dz = 0.1, cells growing outside it along all three axes; inflow, outflow and slip walls) with
    a fixed dt."""
    from test_gpu_stretched import _refined_block_case
    cfg = _refined_block_case()
    h = min(float(np.diff(f).min()) for f in cfg.faces)
    return cfg.with_(cfl=0.0, dt_fixed=0.3 * h / 11.0)


def test_stretched_window_field_gradient_matches_frozen_finite_differences():
    # reverse mode through the stretched-mesh scheme (chain-rule derivatives with the local widths,
    # flux difference over the cell width) against central differences of the weight-replaying forward
    cfg = _stretched_case()
    rng = np.random.default_rng(8)
    n = cfg.rotor.n_act
    s0 = np.ones(n)
    q0 = torch.tensor(cfg.q0).clone().requires_grad_(True)
    J, _ = rotor_objective(cfg, torch.tensor(s0), NSTEPS, W, WenoControl("detach"), q0=q0)
    J.backward()
    dq = torch.tensor(rng.standard_normal(cfg.q0.shape))
    dq[0] *= 0.01
    fd = _frozen_fd(cfg, s0, np.zeros(n), 1e-4, q0=torch.tensor(cfg.q0), dq=dq)
    ad = float((q0.grad * dq).sum())
    assert abs(fd - ad) < 1e-7 * abs(ad), (fd, ad)
