"""GPU adjoint (gks_adjoint through the C ABI) against the oracle's reverse-mode reference and against
central finite differences of the GPU FP64 forward. The adjoint freezes the WENO nonlinear weights;
the oracle reference does the same, so those two agree to rounding; against true finite differences
the difference is the frozen-weight linearisation error (reported)."""
import math

import numpy as np
import pytest
import torch

from gpu_util import print_case
from oracle import WenoControl, rotor_gradient, rotor_objective
from synth import make_case

pytestmark = pytest.mark.gpu
W = (1.0, 0.5)


def _gpu_window(cfg, scales, nsteps, w=W, want_field=False, q0=None):
    from paper_2603_11102_amd import GksSolver
    s = GksSolver(cfg, precision="fp64", q0=q0)
    sc = torch.as_tensor(scales, dtype=torch.float64, device="cuda").contiguous()
    s.set_rotor(cfg.rotor, scale=sc)
    s.set_checkpoints(nsteps)
    s.step(nsteps)
    f = s.forces()
    J = (w[0] * f["window_power"] + w[1] * f["window_thrust"]) / f["window_steps"]
    return s, J, sc


@pytest.mark.parametrize("tip", [False, True])
def test_adjoint_matches_oracle_reference(tip):
    from dataclasses import replace
    cfg = make_case("adjoint", grid=(20, 20, 20))
    cfg = cfg.with_(rotor=replace(cfg.rotor, tip_correction=tip))
    n = cfg.rotor.n_act
    rng = np.random.default_rng(0)
    s0 = 1.0 + 0.1 * rng.standard_normal(n)
    nsteps = 2
    print_case("adjoint-vs-oracle", grid=(20, 20, 20), nsteps=nsteps)
    s, J, _ = _gpu_window(cfg, s0, nsteps)
    g, gq = s.adjoint(nsteps, W, want_field=True)
    Jo, go = rotor_gradient(cfg, s0, nsteps, W, frozen=True)
    assert abs(J - Jo) < 1e-12 * abs(Jo)
    rel = float((g.cpu() - go).abs().max() / go.abs().max())
    assert rel < 1e-10, rel
    # field sensitivity dJ/dQ^0
    q0 = torch.tensor(cfg.q0).clone().requires_grad_(True)
    Jt, _ = rotor_objective(cfg, torch.tensor(s0), nsteps, W, WenoControl("detach"), q0=q0)
    Jt.backward()
    ref = q0.grad.detach()
    gq = gq.cpu()
    for v in range(4):
        e = float((gq[v] - ref[v]).abs().max() / ref[v].abs().max())
        assert e < 1e-9, (v, e)


def test_adjoint_matches_gpu_finite_differences():
    # On this coarse grid (9.4 cells per rotor diameter) the WENO weights vary strongly; the frozen-weight
    # linearisation differs from the true derivative by about 1e-4 here (the exact frozen-weight
    # gradient is pinned against the oracle above), so the bar is 1e-3. The full-size case below holds
    # the 1e-4 bar.
    cfg = make_case("adjoint", grid=(24, 24, 24))
    n = cfg.rotor.n_act
    nsteps = 3
    print_case("adjoint-vs-fd", grid=(24, 24, 24), nsteps=nsteps)
    s, J0, _ = _gpu_window(cfg, np.ones(n), nsteps)
    g, _ = s.adjoint(nsteps, W)
    g = g.cpu().numpy()
    rng = np.random.default_rng(1)
    h = 1e-4
    for _ in range(2):
        v = rng.standard_normal(n)
        _, Jp, _ = _gpu_window(cfg, 1.0 + h * v, nsteps)
        _, Jm, _ = _gpu_window(cfg, 1.0 - h * v, nsteps)
        fd = (Jp - Jm) / (2 * h)
        ad = float(g @ v)
        print(f"directional derivative: adjoint {ad:.12e} fd {fd:.12e} rel {abs(fd - ad) / abs(fd):.3e}")
        assert abs(fd - ad) < 1e-3 * abs(fd)


def test_autograd_function_backward():
    from paper_2603_11102_amd.adjoint import rotor_window
    cfg = make_case("adjoint", grid=(20, 20, 20))
    n = cfg.rotor.n_act
    sc = torch.ones(n, dtype=torch.float64, device="cuda", requires_grad=True)
    out = rotor_window(sc, cfg, 2)
    J = W[0] * out[0] + W[1] * out[1]
    J.backward()
    s, _, _ = _gpu_window(cfg, np.ones(n), 2)
    g, _ = s.adjoint(2, W)
    assert torch.equal(sc.grad, g)


def test_adjoint_full_size_vs_finite_differences():
    cfg = make_case("adjoint")  # 128^3, 3 x 32 points, 20 steps
    n = cfg.rotor.n_act
    nsteps = cfg.steps
    print_case("adjoint-128", grid=(cfg.nx, cfg.ny, cfg.nz), nsteps=nsteps)
    s, J0, _ = _gpu_window(cfg, np.ones(n), nsteps)
    torch.cuda.synchronize()
    import time
    t0 = time.perf_counter()
    g, _ = s.adjoint(nsteps, W)
    t_adj = time.perf_counter() - t0
    g = g.cpu().numpy()
    rng = np.random.default_rng(5)
    h = 1e-4
    v = rng.standard_normal(n)
    _, Jp, _ = _gpu_window(cfg, 1.0 + h * v, nsteps)
    _, Jm, _ = _gpu_window(cfg, 1.0 - h * v, nsteps)
    fd = (Jp - Jm) / (2 * h)
    ad = float(g @ v)
    print(f"128^3 directional derivative: adjoint {ad:.12e} fd {fd:.12e} rel {abs(fd - ad) / abs(fd):.3e}; "
          f"adjoint {t_adj:.3f} s")
    assert abs(fd - ad) < 1e-4 * abs(fd)
