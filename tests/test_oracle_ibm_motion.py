"""Pins of the oracle's rigidly moving immersed bodies (reading R16: the Lagrangian points follow the
body's translation and rotation, introduction and Section 3.2): the rotation against scipy and closed
forms, rigidity, point velocities as time derivatives of the positions, the special cases of no motion
and of a body carried by a uniform stream, and the time level at which the forcing takes the points."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import Oracle, ibm_apply, ibm_motion_state, ibm_setup, rotation_matrix
from oracle.gks_oracle import IbmPoints
from synth import make_case
from synth.cases import IbmMotion, IbmSpec


def _body(n=60, seed=7):
    cfg = make_case("tgv", grid=(16, 16, 16)).with_(bc=("periodic",) * 6)
    rng = np.random.default_rng(seed)
    c0 = np.array([0.5, 0.5, 0.5]) * cfg.lx
    d = rng.normal(size=(n, 3))
    d *= (1.8 * cfg.dx) / np.linalg.norm(d, axis=1, keepdims=True)  # a sphere of radius 1.8 dx
    xyz = c0 + d
    dS = np.full(n, 4.0 * math.pi * (1.8 * cfg.dx) ** 2 / n)
    return cfg, c0, xyz, dS


def test_rotation_matrix_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(20):
        w = rng.normal(size=3) * rng.uniform(0.0, 3.0)
        R = rotation_matrix(w)
        assert np.abs(R - Rotation.from_rotvec(w).as_matrix()).max() < 1e-14
        assert np.abs(R @ R.T - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(R) - 1.0) < 1e-14
    assert np.array_equal(rotation_matrix([0.0, 0.0, 0.0]), np.eye(3))


def test_quarter_turns():
    Rz = rotation_matrix([0.0, 0.0, math.pi / 2])
    assert np.allclose(Rz @ [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], atol=1e-15)
    assert np.allclose(Rz @ [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], atol=1e-15)
    Rx = rotation_matrix([math.pi / 2, 0.0, 0.0])
    assert np.allclose(Rx @ [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], atol=1e-15)
    # a half turn about (1, 1, 0)/sqrt(2) swaps x and y and flips z
    Rd = rotation_matrix(np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0) * math.pi)
    assert np.allclose(Rd @ [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], atol=1e-15)
    assert np.allclose(Rd @ [0.0, 0.0, 1.0], [0.0, 0.0, -1.0], atol=1e-15)


def test_motion_is_rigid_and_starts_at_the_reference_positions():
    cfg, c0, xyz, dS = _body()
    ib = IbmSpec(xyz=xyz, dS=dS, motion=IbmMotion(center=c0, velocity=(0.2, -0.1, 0.05), omega=(0.3, -0.7, 1.1),
                                                   t0=0.25))
    X0, _ = ibm_motion_state(ib, 0.25)
    assert np.abs(X0 - xyz).max() < 1e-15
    X, _ = ibm_motion_state(ib, 1.9)
    D0 = np.linalg.norm(xyz[:, None] - xyz[None], axis=2)
    D1 = np.linalg.norm(X[:, None] - X[None], axis=2)
    assert np.abs(D1 - D0).max() < 1e-14
    # the centre moves with V: the mean offset from c(t) is the rotated mean offset from c0
    ct = c0 + np.array([0.2, -0.1, 0.05]) * (1.9 - 0.25)
    m0 = (xyz - c0).mean(0)
    m1 = (X - ct).mean(0)
    assert abs(np.linalg.norm(m1) - np.linalg.norm(m0)) < 1e-15


def test_point_velocity_is_the_time_derivative_of_the_position():
    cfg, c0, xyz, dS = _body()
    ib = IbmSpec(xyz=xyz, dS=dS, motion=IbmMotion(center=c0, velocity=(0.2, -0.1, 0.05), omega=(0.3, -0.7, 1.1)))
    t, h = 0.8, 1e-4
    Xp, _ = ibm_motion_state(ib, t + h)
    Xm, _ = ibm_motion_state(ib, t - h)
    _, v = ibm_motion_state(ib, t)
    # central difference error h^2/6 |X'''| <= h^2/6 |omega|^3 r
    bound = h * h / 6 * np.linalg.norm([0.3, -0.7, 1.1]) ** 3 * 1.8 * cfg.dx + 1e-11
    assert np.abs((Xp - Xm) / (2 * h) - v).max() < bound


def test_spinning_ring_speed_closed_form():
    cfg = make_case("tgv", grid=(16, 16, 16))
    c0 = np.array([3.0, 3.0, 3.0])
    ang = np.linspace(0.0, 2.0 * math.pi, 12, endpoint=False)
    r = 0.7
    xyz = c0 + r * np.stack([np.cos(ang), np.sin(ang), np.zeros_like(ang)], 1)
    W = 2.5
    ib = IbmSpec(xyz=xyz, dS=np.ones(12), motion=IbmMotion(center=c0, omega=(0.0, 0.0, W)))
    t = 0.3
    X, v = ibm_motion_state(ib, t)
    expect = c0 + r * np.stack([np.cos(ang + W * t), np.sin(ang + W * t), np.zeros_like(ang)], 1)
    assert np.abs(X - expect).max() < 1e-15 * 8
    vexp = r * W * np.stack([-np.sin(ang + W * t), np.cos(ang + W * t), np.zeros_like(ang)], 1)
    assert np.abs(v - vexp).max() < 1e-14


def test_body_at_rest_gives_the_stationary_result():
    cfg, c0, xyz, dS = _body()
    q0 = cfg.q0
    still = Oracle(cfg.with_(ibm=IbmSpec(xyz=xyz, dS=dS)), q0=q0)
    moving = Oracle(cfg.with_(ibm=IbmSpec(xyz=xyz, dS=dS, motion=IbmMotion(center=c0))), q0=q0)
    for _ in range(2):
        a = still.step()
        b = moving.step()
        assert np.abs((a["ibm"]["body_force"] - b["ibm"]["body_force"]).numpy()).max() < 1e-13
    assert float((still.Q - moving.Q).abs().max()) < 1e-13


def test_body_carried_by_a_uniform_stream_leaves_it_uniform():
    cfg, c0, xyz, dS = _body()
    V = np.array([0.3, -0.15, 0.1])
    q = np.zeros_like(cfg.q0)
    q[0] = 1.0
    for d in range(3):
        q[1 + d] = V[d]
    o = Oracle(cfg.with_(ibm=IbmSpec(xyz=xyz, dS=dS, motion=IbmMotion(center=c0, velocity=V))), q0=q)
    for _ in range(3):
        out = o.step(dt=0.01)
        assert float(out["ibm"]["body_force"].abs().max()) < 1e-11
        assert float(out["ibm"]["residual"]) < 1e-13
    assert float((o.Q - torch.tensor(q)).abs().max()) < 1e-13


def test_forcing_takes_the_points_at_the_end_of_the_step():
    # one step from t = 0 with a fixed dt equals the stationary step whose points sit at X(dt)
    cfg, c0, xyz, dS = _body()
    ib = IbmSpec(xyz=xyz, dS=dS, motion=IbmMotion(center=c0, velocity=(0.4, 0.0, 0.0), omega=(0.0, 2.0, 0.0)))
    dt = 0.05
    X1, v1 = ibm_motion_state(ib, dt)
    a = Oracle(cfg.with_(ibm=ib)).step(dt=dt)
    b = Oracle(cfg.with_(ibm=IbmSpec(xyz=X1, dS=dS, vel=v1))).step(dt=dt)
    assert np.array_equal(a["ibm"]["body_force"].numpy(), b["ibm"]["body_force"].numpy())
    # and differs from taking them at the start of the step
    X0, v0 = ibm_motion_state(ib, 0.0)
    c = Oracle(cfg.with_(ibm=IbmSpec(xyz=X0, dS=dS, vel=v0))).step(dt=dt)
    assert np.abs((a["ibm"]["body_force"] - c["ibm"]["body_force"]).numpy()).max() > 1e-6


def test_body_leaving_the_interior_is_rejected():
    cfg, c0, xyz, dS = _body()
    ib = IbmSpec(xyz=xyz, dS=dS, motion=IbmMotion(center=c0, velocity=(40.0, 0.0, 0.0)))
    X, v = ibm_motion_state(ib, 0.2)
    with pytest.raises(ValueError):
        ibm_setup(cfg, IbmPoints(X, dS, v))


def test_support_rule_at_the_edge_of_the_run():
    # reading R17: a point's 4-cell support b-1 .. b+2 (b the cell below it relative to the centres)
    # must lie in the run of cells of the body's width; z is uniform for 24 cells, then grows
    from oracle.gks_oracle import body_run, support_inside
    cfg = make_case("alm_ibm", grid=(64, 32, 32)).with_(rotor=None, ibm=None)
    h = cfg.dz
    w = np.concatenate([np.full(24, h), h * 1.1 ** np.arange(1, 9)])
    zf = np.concatenate([[0.0], np.cumsum(w)])
    cfg = cfg.with_(lz=float(zf[-1]), faces=(None, None, zf))
    runs = body_run(cfg, np.array([3.0, 2.0, 10 * h]), np.array([3.0, 2.0, 11 * h]), 2)
    assert runs[2] == (0, 23) and runs[0] == (0, 63)
    grid = ((0.0, 0.0, 0.0), (cfg.dx, cfg.dy, h))
    at_edge = np.array([[3.0, 2.0, (21 + 0.5 + 0.99) * h]])     # b = 21: support cells 20 .. 23
    past = np.array([[3.0, 2.0, (22 + 0.5 + 0.01) * h]])        # b = 22: support reaches cell 24
    low_edge = np.array([[3.0, 2.0, (1 + 0.5) * h]])            # b = 1: support cells 0 .. 3
    below = np.array([[3.0, 2.0, (0.5 + 0.99) * h]])            # b = 0: support reaches cell -1
    assert support_inside(at_edge, grid, runs) and support_inside(low_edge, grid, runs)
    assert not support_inside(past, grid, runs) and not support_inside(below, grid, runs)
