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
