"""Pins of the oracle's body forces: the ALM Gaussian projection (Section 3.1, Eq. (Gaussian); 1 % decay
at 2.15 eps and truncation at 3 eps from Section 4.3.1), the blade-element forces on a uniform inflow,
the rotor reductions and coefficients (Section 4.4.1), Peskin's 4-point delta identities and the
closed form of the stationary-body direct-forcing iteration (Section 3.2)."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import Oracle, alm_apply, ibm_apply, ibm_setup, phi4, rotor_points
from synth import make_case
from synth.cases import IbmSpec

F64 = torch.float64
HERE = os.path.dirname(__file__)
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))


def test_gaussian_one_percent_radius():
    r = GOLD["gaussian_one_percent_radius_over_eps"]["value"]
    # exp(-(r/eps)^2) = 0.01 at r/eps = sqrt(ln 100) = 2.146; the paper rounds to 2.15
    assert abs(math.sqrt(math.log(100.0)) - r) < 0.005
    assert abs(math.exp(-r * r) - 0.01) < 2e-4


def _uniform_alm_case(grid=(48, 24, 24)):
    cfg = make_case("alm", grid=grid)
    q = np.zeros((4, cfg.nz, cfg.ny, cfg.nx))
    q[0] = 1.0
    q[1] = 1.0
    return cfg, torch.tensor(q)


def test_alm_uniform_inflow_hand_computed():
    cfg, Q = _uniform_alm_case()
    rot = cfg.rotor
    t = 0.013
    _, out = alm_apply(Q, t, 0.0, cfg, rot)
    # uniform U = (1, 0, 0): U_x = 1, U_theta = 0 at every point
    r = np.tile(rot.r, rot.n_blades)
    c = np.tile(rot.chord, rot.n_blades)
    g = np.tile(rot.twist, rot.n_blades)
    w = np.tile(rot.width, rot.n_blades)
    om = rot.omega
    phi0 = np.arctan2(1.0, om * r)
    cd0 = rot.cd0 + rot.cd2 * (phi0 - g) ** 2
    f = 1.0 / (1.0 - cd0 * c / (4 * math.sqrt(math.pi) * rot.eps))
    phi = np.arctan2(f, om * r)
    alpha = phi - g
    urel2 = f * f + (om * r) ** 2
    cl = 2 * math.pi * np.clip(alpha, -math.radians(12), math.radians(12))
    cd = 0.01 + 0.02 * alpha ** 2
    L = 0.5 * c * w * cl * urel2
    D = 0.5 * c * w * cd * urel2
    assert np.allclose(out["alpha"].numpy(), alpha, rtol=1e-12, atol=1e-14)
    assert np.allclose(out["fx"].numpy(), L * np.cos(phi) + D * np.sin(phi), rtol=1e-12)
    assert np.allclose(out["ftheta"].numpy(), L * np.sin(phi) - D * np.cos(phi), rtol=1e-12)
    assert float(out["thrust"]) > 0 and float(out["power"]) > 0  # a turbine extracts energy


def test_alm_reductions_and_coefficients():
    cfg, Q = _uniform_alm_case()
    rot = cfg.rotor
    _, out = alm_apply(Q, 0.0, 0.0, cfg, rot)
    r = np.tile(rot.r, rot.n_blades)
    fx, ft = out["fx"].numpy(), out["ftheta"].numpy()
    T = math.fsum(fx.tolist())
    Qt = math.fsum((r * ft).tolist())
    assert abs(float(out["thrust"]) - T) < 1e-13 * abs(T)
    assert abs(float(out["torque"]) - Qt) < 1e-13 * abs(Qt)
    area = math.pi * rot.radius ** 2
    assert abs(float(out["cp"]) - 2 * rot.omega * Qt / (area * 1.0)) < 1e-12
    assert abs(float(out["ct"]) - 2 * T / (area * 1.0)) < 1e-12


def test_alm_projection_momentum_budget():
    # the truncated Gaussian deposits F (1 - deficit) with deficit ~ erfc(3) + (6/sqrt(pi)) exp(-9) = 4.4e-4
    cfg, Q = _uniform_alm_case(grid=(96, 48, 48))
    rot = cfg.rotor
    dt = 0.01
    Qn, out = alm_apply(Q, 0.0, dt, cfg, rot)
    vol = cfg.dx * cfg.dy * cfg.dz
    dmom = ((Qn[1:] - Q[1:]).sum((1, 2, 3)) * vol / dt).numpy()
    _, et = rotor_points(rot, 0.0)
    F = np.stack([out["fx"].numpy(), out["ftheta"].numpy() * et[:, 1], out["ftheta"].numpy() * et[:, 2]], 1)
    tot = -F.sum(0)
    cont = math.erfc(3.0) + 6.0 / math.sqrt(math.pi) * math.exp(-9.0)
    assert abs(cont - 4.40e-4) < 1e-6
    ratio = dmom[0] / tot[0]
    assert 1 - 5.0e-4 < ratio < 1 - 3.5e-4, ratio


def test_gaussian_lattice_sum_untruncated():
    # the lattice sum of the normalised Gaussian at eps = 2 dx is 1 to 1e-12 (Poisson summation)
    eps = 2.0
    rng = np.random.default_rng(0)
    for _ in range(3):
        off = rng.uniform(-0.5, 0.5, 3)
        ax = np.arange(-20, 21)
        Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
        r2 = (X - off[0]) ** 2 + (Y - off[1]) ** 2 + (Z - off[2]) ** 2
        s = np.sum(np.exp(-r2 / eps ** 2)) / (eps ** 3 * math.pi ** 1.5)
        assert abs(s - 1.0) < 1e-12


def test_phi4_identities():
    rng = np.random.default_rng(1)
    for r in rng.uniform(-3, 3, 50):
        j = np.arange(-6, 7)
        v = phi4(r - j)
        assert abs(v.sum() - 1.0) < 1e-14
        assert abs(((r - j) * v).sum()) < 1e-14
        assert abs((v * v).sum() - 3.0 / 8.0) < 1e-14
        even = v[(j % 2) == 0].sum()
        assert abs(even - 0.5) < 1e-14


def _ibm_case():
    cfg = make_case("tgv", grid=(16, 16, 16)).with_(bc=("periodic",) * 6)
    rng = np.random.default_rng(4)
    xyz = rng.uniform(2.5 * cfg.dx, cfg.lx - 2.5 * cfg.dx, size=(40, 3))
    dS = rng.uniform(0.02, 0.05, size=40) * cfg.dx ** 2
    return cfg.with_(ibm=IbmSpec(xyz=xyz, dS=dS))


def test_ibm_volume_partition_of_unity():
    cfg = _ibm_case()
    cache = ibm_setup(cfg, cfg.ibm)
    assert abs(cache.vbar.sum() - cfg.dx * cfg.ibm.dS.sum()) < 1e-13 * cfg.dx * cfg.ibm.dS.sum()
    assert np.allclose(cache.weights.sum(1), 1.0, atol=1e-14)


def test_ibm_closed_form_iteration():
    cfg = _ibm_case()
    cache = ibm_setup(cfg, cfg.ibm)
    Q = torch.tensor(cfg.q0)
    dt, S = 0.02, 3
    Qn, out = ibm_apply(Q, dt, cfg, cache, S)
    vol = cfg.dx * cfg.dy * cfg.dz
    i, j, k = cache.vbar_index.T
    fac = (1.0 - cache.vbar / vol) ** S
    U0 = (Q[1:, k, j, i] / Q[0, k, j, i]).numpy()
    US = (Qn[1:, k, j, i] / Qn[0, k, j, i]).numpy()
    assert np.allclose(US, U0 * fac, rtol=1e-12, atol=1e-15)
    rho = Q[0, k, j, i].numpy()
    Fsum = -(rho * vol * U0 * (1.0 - fac) / dt).sum(1)
    assert np.allclose(out["force_on_fluid"].numpy(), Fsum, rtol=1e-11)
    # untouched cells unchanged
    mask = np.ones((cfg.nz, cfg.ny, cfg.nx), bool)
    mask[k, j, i] = False
    assert torch.equal(Qn[:, torch.tensor(mask)], Q[:, torch.tensor(mask)])


def test_oracle_step_with_rotor_and_body_runs():
    cfg = make_case("alm_ibm", grid=(64, 32, 32))
    o = Oracle(cfg)
    out = o.step()
    assert math.isfinite(float(out["alm"]["power"]))
    assert float(out["ibm"]["residual"]) >= 0
    assert torch.isfinite(o.Q).all()


def test_tip_correction_factor():
    # Section 4.4, Eq. (tip-correction): printed constants, f -> 0 at the tip, f -> 1 inboard, f in [0, 1]
    from oracle import tip_factor
    cfg, Q = _uniform_alm_case()
    rot = cfg.rotor
    ax = GOLD["tip_correction_axial_c1_c2"]["value"]
    tg = GOLD["tip_correction_tangential_c1_c2"]["value"]
    assert ax == [0.1219, 21.52] and tg == [0.0984, 13.026]
    phi = torch.tensor(0.15, dtype=F64)
    rr = torch.tensor(np.linspace(0.05, 0.5, 200) * rot.radius / 0.5, dtype=F64)
    for c1, c2 in (ax, tg):
        f = tip_factor(rot, rr, phi, c1, c2)
        assert float(f[-1]) == 0.0
        assert float(f.min()) >= 0.0 and float(f.max()) <= 1.0
        assert torch.all(f[1:] <= f[:-1] + 1e-15)
        # by hand at r = 0.8 R
        N, lam = rot.n_blades, rot.omega * rot.radius / rot.u_inf
        g1 = math.exp(-c1 * (N * lam - c2)) + 0.1
        r8 = 0.8 * rot.radius
        ref = 2 / math.pi * math.acos(math.exp(-g1 * N * (rot.radius - r8) / (2 * r8 * math.sin(0.15))))
        got = float(tip_factor(rot, torch.tensor(r8, dtype=F64), phi, c1, c2))
        assert abs(got - ref) < 1e-14


def test_tip_correction_reduces_tip_loads():
    cfg, Q = _uniform_alm_case()
    rot = cfg.rotor
    from dataclasses import replace
    _, a = alm_apply(Q, 0.0, 0.0, cfg, rot)
    _, b = alm_apply(Q, 0.0, 0.0, cfg, replace(rot, tip_correction=True))
    assert float(b["thrust"]) < float(a["thrust"]) and float(b["power"]) < float(a["power"])
    n = rot.n_per_blade
    assert float(b["fx"][n - 1]) < 0.5 * float(a["fx"][n - 1])
    assert abs(float(b["fx"][0]) / float(a["fx"][0]) - 1.0) < 1e-3


def test_ibm_uniform_point_velocity_closed_form():
    # every point moves with the same V: v-bar = V at each forced cell, and per cell
    # U^S = V + (U^0 - V)(1 - V-bar/|Omega|)^S, sum_s F^s = rho |Omega| (V - U^0)(1 - (1 - V-bar/|Omega|)^S)/dt
    cfg = _ibm_case()
    V = np.array([0.3, -0.2, 0.1])
    ib = IbmSpec(xyz=cfg.ibm.xyz, dS=cfg.ibm.dS, vel=np.tile(V, (cfg.ibm.n, 1)))
    cache = ibm_setup(cfg, ib)
    assert np.allclose(cache.vbar_vel, V[None, :], rtol=0, atol=1e-15)
    Q = torch.tensor(cfg.q0)
    dt, S = 0.02, 3
    Qn, out = ibm_apply(Q, dt, cfg, cache, S)
    vol = cfg.dx * cfg.dy * cfg.dz
    i, j, k = cache.vbar_index.T
    fac = (1.0 - cache.vbar / vol) ** S
    U0 = (Q[1:, k, j, i] / Q[0, k, j, i]).numpy()
    US = (Qn[1:, k, j, i] / Qn[0, k, j, i]).numpy()
    assert np.allclose(US, V[:, None] + (U0 - V[:, None]) * fac, rtol=1e-12, atol=1e-15)
    rho = Q[0, k, j, i].numpy()
    Fsum = (rho * vol * (V[:, None] - U0) * (1.0 - fac) / dt).sum(1)
    assert np.allclose(out["force_on_fluid"].numpy(), Fsum, rtol=1e-11)


def test_ibm_body_moving_with_the_fluid_feels_no_force():
    cfg = _ibm_case()
    V = np.array([0.25, 0.1, -0.05])
    q = np.zeros_like(cfg.q0)
    q[0] = 1.1
    for d in range(3):
        q[1 + d] = 1.1 * V[d]
    ib = IbmSpec(xyz=cfg.ibm.xyz, dS=cfg.ibm.dS, vel=np.tile(V, (cfg.ibm.n, 1)))
    cache = ibm_setup(cfg, ib)
    Q = torch.tensor(q)
    Qn, out = ibm_apply(Q, 0.01, cfg, cache, 3)
    assert float((Qn - Q).abs().max()) < 1e-15
    assert float(out["force_on_fluid"].abs().max()) < 1e-12
    assert float(out["residual"]) < 1e-14  # sum_c W = 1: the interpolated U equals V


def test_ibm_point_velocity_is_volume_weighted():
    # one cell in the support of two points with different areas and velocities
    cfg = make_case("tgv", grid=(16, 16, 16)).with_(bc=("periodic",) * 6)
    h = cfg.dx
    xyz = np.array([[8.3 * h, 8.1 * h, 7.6 * h], [8.9 * h, 7.7 * h, 8.4 * h]])
    dS = np.array([0.02, 0.05]) * h * h
    vel = np.array([[1.0, 0.0, -0.5], [0.0, 2.0, 0.5]])
    cache = ibm_setup(cfg, IbmSpec(xyz=xyz, dS=dS, vel=vel))
    c = np.array([8, 8, 8])  # cell (i, j, k) = (8, 8, 8), centre (8.5 h, 8.5 h, 8.5 h)
    row = int(np.nonzero((cache.vbar_index == c).all(1))[0][0])
    w = [phi4(8.5 - xyz[p, 0] / h) * phi4(8.5 - xyz[p, 1] / h) * phi4(8.5 - xyz[p, 2] / h) for p in range(2)]
    Vp = h * dS
    expect = (w[0] * Vp[0] * vel[0] + w[1] * Vp[1] * vel[1]) / (w[0] * Vp[0] + w[1] * Vp[1])
    assert np.allclose(cache.vbar_vel[row], expect, rtol=1e-13, atol=0)
    assert abs(cache.vbar[row] - (w[0] * Vp[0] + w[1] * Vp[1])) < 1e-15 * cache.vbar[row] + 1e-30
