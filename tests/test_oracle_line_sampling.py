"""Pins of the oracle's line sampling of the actuator points (reading R18 of the NTNU rotor, Sections 3.1
and 4.4): it reduces to point sampling, reproduces linear velocity fields at the point, and gives the
closed-form mean of a field that trilinear interpolation reproduces exactly (a product of the two
in-plane coordinates) along the blade's direction of motion; a wrong direction, half-length or sample
count changes that mean."""
import math
from dataclasses import replace

import numpy as np
import torch

from oracle.gks_oracle import _trilinear, alm_apply, line_sample, rotor_points
from synth import make_case


def _cfg():
    cfg = make_case("alm", grid=(48, 24, 24))
    return cfg.with_(rotor=replace(cfg.rotor, theta0=0.3))


def _centres(cfg):
    n = (cfg.nx, cfg.ny, cfg.nz)
    h = (cfg.dx, cfg.dy, cfg.dz)
    o = (cfg.x0, cfg.y0, cfg.z0)
    return [o[a] + (np.arange(n[a]) + 0.5) * h[a] for a in range(3)]


def _field(cfg, ufun, seed=4):
    """Cells with random density and velocity ufun(x, y, z) at the cell centre (oracle layout)."""
    x, y, z = _centres(cfg)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    rho = 1.0 + 0.1 * np.random.default_rng(seed).uniform(-1, 1, size=X.shape)
    u = ufun(X, Y, Z)
    q = np.concatenate([rho[None], rho[None] * u], 0)
    return torch.tensor(q, dtype=torch.float64)


def test_one_sample_or_zero_length_is_point_sampling():
    cfg = _cfg()
    Q = _field(cfg, lambda X, Y, Z: np.stack([1 + 0.1 * np.sin(3 * X + Y), 0.2 * np.cos(Z), 0.1 * Y * X]))
    P, et = rotor_points(cfg.rotor, 0.37)
    ref = _trilinear(Q, cfg, P)
    assert torch.equal(line_sample(Q, cfg, P, et, 0.4, 1), ref)
    assert torch.equal(line_sample(Q, cfg, P, et, 0.0, 9), ref)
    assert not torch.allclose(line_sample(Q, cfg, P, et, 0.4, 9), ref, rtol=0, atol=1e-6)


def test_linear_field_is_reproduced_at_the_point():
    cfg = _cfg()
    a = np.array([1.0, -0.2, 0.3])
    B = np.array([[0.1, -0.3, 0.2], [0.05, 0.4, -0.1], [-0.2, 0.1, 0.3]])
    Q = _field(cfg, lambda X, Y, Z: np.stack([a[c] + B[c, 0] * X + B[c, 1] * Y + B[c, 2] * Z for c in range(3)]))
    P, et = rotor_points(cfg.rotor, 0.11)
    for npts, half in ((2, 0.3), (5, 0.5), (9, 0.5)):
        U = line_sample(Q, cfg, P, et, half, npts).numpy()
        assert np.abs(U - (a[None, :] + P @ B.T)).max() < 1e-13


def test_bilinear_field_closed_form_along_the_direction_of_motion():
    # U_x = c0 + c1 (y - y0)(z - z0) is reproduced exactly by trilinear interpolation; along
    # X_p + s e_theta, e_theta = (0, -sin th, cos th), it is A + B s - sin th cos th s^2, whose mean over
    # the midpoints s_k = l ((2k + 1)/N - 1) is A - sin th cos th l^2 (N^2 - 1) / (3 N^2)
    cfg = _cfg()
    c0, c1, y0, z0 = 0.9, 0.7, 1.1, 1.6
    Q = _field(cfg, lambda X, Y, Z: np.stack([c0 + c1 * (Y - y0) * (Z - z0), 0 * X, 0 * X]))
    t = 0.23
    P, et = rotor_points(cfg.rotor, t)
    nb, npb = cfg.rotor.n_blades, cfg.rotor.n_per_blade
    th = np.repeat(cfg.rotor.theta0 + cfg.rotor.omega * t + 2 * math.pi * np.arange(nb) / nb, npb)
    assert np.abs(np.sin(2 * th)).min() > 0.1  # generic blade angles: the quadratic term is visible
    for npts, half in ((3, 0.4), (7, 0.5), (8, 0.25)):
        U = line_sample(Q, cfg, P, et, half, npts).numpy()
        A = c0 + c1 * (P[:, 1] - y0) * (P[:, 2] - z0)
        exact = A - c1 * np.sin(th) * np.cos(th) * half * half * (npts * npts - 1) / (3.0 * npts * npts)
        assert np.abs(U[:, 0] - exact).max() < 1e-13
        # the spanwise direction e_r = (0, cos th, sin th) would flip the sign of the quadratic term
        wrong = A + c1 * np.sin(th) * np.cos(th) * half * half * (npts * npts - 1) / (3.0 * npts * npts)
        assert np.abs(U[:, 0] - wrong).max() > 1e-3


def test_uniform_stream_gives_the_point_sampled_loads():
    cfg = _cfg()
    Q = _field(cfg, lambda X, Y, Z: np.stack([1.0 + 0 * X, 0.1 + 0 * X, -0.05 + 0 * X]))
    line = replace(cfg.rotor, line_points=9, line_half_length=2 * cfg.rotor.eps)
    _, a = alm_apply(Q, 0.05, 1e-3, cfg, cfg.rotor)
    _, b = alm_apply(Q, 0.05, 1e-3, cfg, line)
    for k in ("alpha", "fx", "ftheta"):
        assert torch.allclose(a[k], b[k], rtol=1e-14, atol=1e-15), k
    Q2 = _field(cfg, lambda X, Y, Z: np.stack([1.0 + 0.2 * np.sin(4 * Y) * np.cos(3 * Z), 0 * X, 0 * X]))
    _, c = alm_apply(Q2, 0.05, 1e-3, cfg, cfg.rotor)
    _, d = alm_apply(Q2, 0.05, 1e-3, cfg, line)
    assert not torch.allclose(c["fx"], d["fx"], rtol=1e-6, atol=0)
