"""Scheme-level pins of the oracle: S2O4 amplification factor, free-stream preservation with every
boundary kind, discrete conservation in a periodic box, measured convergence order on a smooth
acoustic wave, and the initial viscous dissipation of the Taylor-Green vortex (Section 2)."""
import math

import numpy as np
import pytest
import torch

from oracle import Oracle, cfl_dt, constants, conservation_sums, s2o4_final, s2o4_stage1
from synth import make_case

F64 = torch.float64


def test_s2o4_amplification_is_fourth_order_taylor():
    # dQ/dt = k Q: L = k Q, L_t = k^2 Q. The two-stage scheme must give 1 + z + z^2/2 + z^3/6 + z^4/24.
    for k in (-1.3, 0.7, 2.0):
        for dt in (0.01, 0.1, 0.5):
            Q = torch.tensor(1.0, dtype=F64)
            Qs = s2o4_stage1(Q, k * Q, k * k * Q, dt)
            Qn = s2o4_final(Q, k * Q, k * k * Q, k * k * Qs, dt)
            z = k * dt
            assert abs(float(Qn) - (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24)) < 1e-14


def test_sound_speed_and_cfl():
    cfg = make_case("tgv", grid=(8, 8, 8))
    k = constants(cfg)
    assert abs(k["c"] - cfg.u_ref / cfg.ma) < 1e-12  # C = sqrt(1/(2 lambda)) = U_inf / Ma
    q = np.zeros((4, 8, 8, 8))
    q[0] = 1.0
    q[1] = 3.0
    q[2] = 4.0  # |U| = 5
    dt = cfl_dt(torch.tensor(q), cfg)
    assert abs(dt - 0.5 * (2 * math.pi / 8) / (5.0 + 10.0)) < 1e-15


def _uniform(cfg, rho, u):
    q = np.zeros((4, cfg.nz, cfg.ny, cfg.nx))
    q[0] = rho
    for j in range(3):
        q[1 + j] = rho * u[j]
    return q


@pytest.mark.parametrize("bc,u", [
    (("periodic",) * 6, (0.4, -0.3, 0.2)),
    (("periodic", "periodic", "noslip", "noslip", "periodic", "periodic"), (0.0, 0.0, 0.0)),
    (("periodic", "periodic", "periodic", "periodic", "slip", "slip"), (0.5, -0.4, 0.0)),
    (("inflow", "outflow", "periodic", "periodic", "slip", "slip"), (1.0, 0.0, 0.0)),
    (("slip", "slip", "noslip", "noslip", "slip", "slip"), (0.0, 0.0, 0.0)),
])
def test_free_stream_preserved(bc, u):
    cfg = make_case("tgv", grid=(10, 9, 8)).with_(bc=bc, u_in=(1.0, 0.0, 0.0), mu=0.01)
    q = _uniform(cfg, 1.05, u)
    o = Oracle(cfg, q0=q)
    for _ in range(2):
        o.step()
    assert float((o.Q - torch.tensor(q)).abs().max()) < 1e-13


def test_periodic_conservation():
    cfg = make_case("tgv", grid=(12, 12, 12))
    o = Oracle(cfg)
    s0 = conservation_sums(o.Q)
    for _ in range(3):
        o.step()
    s1 = conservation_sums(o.Q)
    n = cfg.n_cells
    for a, b in zip(s0, s1):
        assert abs(a - b) < 1e-13 * n


def _wave_case(axes, n, amp=1e-2):
    grid = [4, 4, 4]
    for a in axes:
        grid[a] = n
    cfg = make_case("tgv", grid=tuple(grid))
    h = 2 * math.pi / n
    lengths = [4 * h, 4 * h, 4 * h]
    for a in axes:
        lengths[a] = 2 * math.pi
    cfg = cfg.with_(lx=lengths[0], ly=lengths[1], lz=lengths[2], mu=0.0, cfl=0.0, dt_fixed=0.2 * h / 10.0)
    kvec = np.zeros(3)
    for a in axes:
        kvec[a] = 1.0
    khat = kvec / np.linalg.norm(kvec)
    hs = (cfg.dx, cfg.dy, cfg.dz)
    cen = [(np.arange(m) + 0.5) * hh for m, hh in zip((cfg.nx, cfg.ny, cfg.nz), hs)]
    Z, Y, X = np.meshgrid(cen[2], cen[1], cen[0], indexing="ij")
    avg = np.prod([np.sinc(kvec[i] * hs[i] / 2 / math.pi) for i in range(3)])
    s = np.sin(kvec[0] * X + kvec[1] * Y + kvec[2] * Z) * avg  # exact cell averages of sin(k.x)
    um = np.array([0.3, -0.2, 0.1])
    c = 10.0
    q = np.zeros((4,) + X.shape)
    q[0] = 1.0 + amp * s
    for j in range(3):
        q[1 + j] = um[j] * (1.0 + amp * s) + c * amp * khat[j] * s
    return cfg, q


def _restrict(Q, axes):
    sl = Q
    for a in axes:
        dim = 3 - a
        shp = list(sl.shape)
        shp[dim] //= 2
        shp.insert(dim + 1, 2)
        sl = sl.reshape(shp).mean(dim + 1)
    return sl


def _run_wave(axes, n, steps):
    cfg, q = _wave_case(axes, n)
    o = Oracle(cfg, q0=q)
    for _ in range(steps):
        o.step()
    return o.Q


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_convergence_order_1d_wave(axis):
    ns = (16, 32, 64)
    sol = {n: _run_wave((axis,), n, n // 8) for n in ns}
    e1 = float((sol[16] - _restrict(sol[32], (axis,))).abs().max())
    e2 = float((sol[32] - _restrict(sol[64], (axis,))).abs().max())
    order = math.log2(e1 / e2)
    assert order > 3.8, (e1, e2, order)


@pytest.mark.parametrize("axes", [(0, 1), (1, 2)])
def test_convergence_order_2d_wave(axes):
    ns = (8, 16, 32)
    sol = {n: _run_wave(axes, n, n // 8) for n in ns}
    e1 = float((sol[8] - _restrict(sol[16], axes)).abs().max())
    e2 = float((sol[16] - _restrict(sol[32], axes)).abs().max())
    order = math.log2(e1 / e2)
    assert order > 3.5, (e1, e2, order)


def test_taylor_green_initial_dissipation():
    # divergence-free start, uniform density: dE/dt = -nu <|grad u|^2> = -6 nu E for the k^2 = 3 mode
    n = 32
    cfg = make_case("tgv", grid=(n, n, n))
    nu = 0.01
    cfg = cfg.with_(mu=nu, cfl=0.0, dt_fixed=1e-4)
    q = cfg.q0.copy()
    L = 2 * math.pi
    x = (np.arange(n) + 0.5) * L / n
    s = np.sinc(L / n / 2 / math.pi)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    q[1] = np.sin(X) * np.cos(Y) * np.cos(Z) * s ** 3
    q[2] = -np.cos(X) * np.sin(Y) * np.cos(Z) * s ** 3
    q[3] = 0.0
    q[0] = 1.0
    o = Oracle(cfg, q0=q)

    def energy(Q):
        return float((0.5 * (Q[1:] ** 2).sum(0) / Q[0]).mean())

    e0 = energy(o.Q)
    o.step()
    rate = (energy(o.Q) - e0) / cfg.dt_fixed
    expect = -6.0 * nu * e0
    assert abs(rate / expect - 1.0) < 0.02, (rate, expect)


def test_flow_statistics_definitions():
    from oracle import flow_statistics
    rng = np.random.default_rng(0)
    base = np.zeros((4, 3, 4, 5))
    base[0] = 1.0
    # constant field: zero fluctuations
    s = flow_statistics([torch.tensor(base + 0.0) for _ in range(4)])
    assert float(s["rms"].abs().max()) == 0.0 and float(s["tke"].abs().max()) == 0.0
    # two states U = 1 +- a (rho = 2): mean 1, rms a, TKE a^2/2, zero shear stress
    a = 0.3
    q1, q2 = base.copy(), base.copy()
    q1[0] = q2[0] = 2.0
    q1[1] = 2.0 * (1 + a)
    q2[1] = 2.0 * (1 - a)
    s = flow_statistics([torch.tensor(q1), torch.tensor(q2)], u_inf=1.0)
    assert torch.allclose(s["mean"][0], torch.tensor(1.0, dtype=torch.float64))
    assert torch.allclose(s["rms"][0], torch.tensor(a, dtype=torch.float64))
    assert torch.allclose(s["tke"], torch.tensor(0.5 * a * a, dtype=torch.float64))
    # correlated U, V: <U'V'> = a b
    q1[2] = 2.0 * 0.5
    q2[2] = -2.0 * 0.5
    s = flow_statistics([torch.tensor(q1), torch.tensor(q2)])
    assert torch.allclose(s["stress"][0], torch.tensor(a * 0.5, dtype=torch.float64))
