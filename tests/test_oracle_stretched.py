"""Pins of the oracle on stretched meshes (reading R17: reconstruction in index space, chain-rule
derivatives with the local spacings, face fluxes times the face area): a uniform mesh given as faces is
the uniform scheme, a uniform stream stays uniform on random stretching, mass is conserved with the cell
volumes, a Poiseuille profile is steady to rounding on a uniform mesh and to second order on the tanh
mesh of Section 4.1, and swapping two axes swaps the result."""
import math

import numpy as np
import pytest
import torch

from oracle import Oracle, axis_metrics, conservation_sums, operator
from synth import make_case
from synth.cases import tanh_faces


def _random_faces(n, lo, hi, seed, ratio=3.0):
    rng = np.random.default_rng(seed)
    w = rng.uniform(1.0, ratio, size=n)
    f = np.concatenate([[0.0], np.cumsum(w)])
    f = lo + (hi - lo) * f / f[-1]
    f[0], f[-1] = lo, hi
    return f


def test_uniform_faces_give_the_uniform_scheme():
    cfg = make_case("channel", grid=(12, 10, 8))
    yf = -1.0 + 2.0 * np.arange(11) / 10
    a, b = Oracle(cfg), Oracle(cfg.with_(faces=(None, yf, None)))
    for _ in range(2):
        a.step(dt=2e-3)
        b.step(dt=2e-3)
    assert float((a.Q - b.Q).abs().max()) < 1e-13


@pytest.mark.parametrize("order", [5, 2])
def test_uniform_stream_stays_uniform_on_a_stretched_mesh(order):
    cfg = make_case("channel", grid=(8, 14, 6)).with_(bc=("periodic", "periodic", "slip", "slip", "periodic",
                                                          "periodic"), body_force=(0.0, 0.0, 0.0), order=order)
    q = np.zeros((4, 6, 14, 8))
    q[0], q[1], q[3] = 1.02, 0.7, -0.2
    cfg = cfg.with_(q0=q, faces=(None, _random_faces(14, -1.0, 1.0, 3), None))
    o = Oracle(cfg)
    for _ in range(2):
        o.step()
    assert float((o.Q - torch.tensor(q)).abs().max()) < 1e-13


@pytest.mark.parametrize("order", [5, 2])
def test_mass_is_conserved_with_the_cell_volumes(order):
    cfg = make_case("channel_tanh", grid=(8, 16, 6)).with_(order=order)
    cfg = cfg.with_(faces=(None, _random_faces(16, -1.0, 1.0, 5), None))
    o = Oracle(cfg)
    m0 = conservation_sums(o.Q, cfg)[0]
    for _ in range(2):
        o.step()
    m1 = conservation_sums(o.Q, cfg)[0]
    assert abs(m1 - m0) < 1e-13 * abs(m0)
    # the unweighted sum is not conserved on this mesh (the weights matter)
    assert abs(conservation_sums(o.Q)[0] - conservation_sums(torch.tensor(cfg.q0))[0]) > 1e-10


def _poiseuille_residual(ny, stretched, order=5, mu=1e-2):
    """max |L(Q) + G| of the x momentum over cells 4 or more cells from the walls, for the exact cell
    averages of U = 1.5 (1 - y^2) driven by G = 3 mu (a steady solution of the viscous equations)."""
    yf = tanh_faces(ny) if stretched else -1.0 + 2.0 * np.arange(ny + 1) / ny
    cfg = make_case("channel_tanh", grid=(4, ny, 4))
    q = np.zeros((4, 4, ny, 4))
    q[0] = 1.0
    ya, yb = yf[:-1], yf[1:]
    q[1] = (1.5 * (1.0 - (yb ** 3 - ya ** 3) / (3.0 * (yb - ya))))[None, :, None]
    cfg = cfg.with_(q0=q, faces=(None, yf, None), mu=mu, body_force=(3.0 * mu, 0.0, 0.0), order=order)
    L0, _ = operator(torch.tensor(q), cfg, True)
    return float((L0[1] + 3.0 * mu)[:, 4:-4, :].abs().max())


@pytest.mark.parametrize("order", [5, 2])
def test_poiseuille_steady_exactly_on_uniform_and_second_order_on_tanh(order):
    assert _poiseuille_residual(32, False, order) < 1e-13
    r64, r128 = _poiseuille_residual(64, True, order), _poiseuille_residual(128, True, order)
    assert r128 < 5e-5
    assert math.log2(r64 / r128) > 1.8


def test_swapping_axes_swaps_the_result():
    # y stretched with walls in y, against x stretched with walls in x and the field transposed; the
    # field does not vary along z, so the z faces (whose two sweeps would run in swapped order) carry
    # equal fluxes on both sides of every cell
    cfg = make_case("channel", grid=(10, 12, 6)).with_(body_force=(0.0, 0.0, 0.0))
    f = _random_faces(12, -1.0, 1.0, 7)
    a_cfg = cfg.with_(nx=10, ny=12, x0=0.0, lx=cfg.lx, y0=-1.0, ly=2.0, faces=(None, f, None))
    qa = np.ascontiguousarray(np.repeat(cfg.q0[:, :1], 6, axis=1))
    qa[3] = 0.0
    qb = np.ascontiguousarray(np.stack([qa[0], qa[2], qa[1], qa[3]]).transpose(0, 1, 3, 2))
    b_cfg = cfg.with_(nx=12, ny=10, x0=-1.0, lx=2.0, y0=0.0, ly=cfg.lx,
                      bc=("noslip", "noslip", "periodic", "periodic", "periodic", "periodic"),
                      faces=(f, None, None), q0=qb)
    La0, La1 = operator(torch.tensor(qa), a_cfg, True)
    Lb0, Lb1 = operator(torch.tensor(qb), b_cfg, True)
    for A, B in ((La0, Lb0), (La1, Lb1)):
        Bt = torch.stack([B[0], B[2], B[1], B[3]]).permute(0, 1, 3, 2)
        assert float((A - Bt).abs().max()) < 1e-12 * float(A.abs().max())


def test_metrics_of_a_stretched_axis():
    cfg = make_case("channel_tanh", grid=(4, 8, 4))
    w, hf = axis_metrics(cfg, 1)
    f = tanh_faces(8)
    assert np.allclose(w, np.diff(f), rtol=0, atol=0)
    assert abs(w.sum() - 2.0) < 1e-15
    assert hf[0] == w[0] and hf[-1] == w[-1]
    # interior face spacing = distance of the adjacent cell centres
    c = 0.5 * (f[:-1] + f[1:])
    assert np.allclose(hf[1:-1], np.diff(c), rtol=1e-15, atol=0)
    with pytest.raises(ValueError):
        axis_metrics(cfg.with_(bc=("periodic",) * 6), 1)


def _top_stretched_faces(n_uniform, h, n_grow, ratio):
    """Uniform cells of size h, then n_grow cells growing by ratio (a mesh refined around the body)."""
    w = np.concatenate([np.full(n_uniform, h), h * ratio ** np.arange(1, n_grow + 1)])
    return np.concatenate([[0.0], np.cumsum(w)])


def test_rotor_in_a_uniform_block_sees_the_uniform_grid():
    from oracle import alm_apply
    cfg = make_case("alm", grid=(48, 24, 24))
    h = cfg.dz
    zf = cfg.z0 + h * np.arange(25.0)
    zf[0] = cfg.z0 - 0.3 * h  # the first cell is wider; every other cell is where it was
    st = cfg.with_(z0=float(zf[0]), lz=float(zf[-1] - zf[0]), faces=(None, None, zf))
    Q = torch.tensor(cfg.q0)
    Q[1] += 0.1 * torch.rand(Q[1].shape, generator=torch.Generator().manual_seed(3), dtype=torch.float64)
    qa, oa = alm_apply(Q, 0.05, 0.01, cfg, cfg.rotor)
    qb, ob = alm_apply(Q, 0.05, 0.01, st, st.rotor)
    for k in ("thrust", "power", "torque"):
        assert abs(float(oa[k]) - float(ob[k])) < 1e-13 * abs(float(oa[k]))
    assert float((qa - qb).abs().max()) < 1e-13 * float(qa.abs().max())


def test_body_in_a_uniform_block_sees_the_uniform_grid():
    from oracle import ibm_setup
    cfg = make_case("alm_ibm", grid=(64, 32, 32))
    zf = _top_stretched_faces(24, cfg.dz, 8, 1.1)
    st = cfg.with_(lz=float(zf[-1]), faces=(None, None, zf))
    a, b = ibm_setup(cfg, cfg.ibm), ibm_setup(st, st.ibm)
    assert np.array_equal(a.vbar_index, b.vbar_index)
    assert np.abs(a.weights - b.weights).max() < 1e-13
    assert np.abs(a.vbar - b.vbar).max() < 1e-13 * a.vbar.max()
    assert abs(a.vol - b.vol) < 1e-15 * a.vol


def test_body_across_a_width_change_is_rejected():
    from oracle import body_grid
    cfg = make_case("alm_ibm", grid=(64, 32, 32))
    zf = _top_stretched_faces(12, cfg.dz, 20, 1.05)  # widths change at z = 1.5, inside the rotor box
    st = cfg.with_(lz=float(zf[-1]), faces=(None, None, zf))
    with pytest.raises(ValueError):
        body_grid(st, (1.0, 1.0, 0.7), (1.2, 3.0, 1.7), 1)
    # and a box below the change is accepted with the block's grid
    org, h = body_grid(st, (1.0, 1.0, 0.3), (1.2, 3.0, 1.0), 1)
    assert h[2] == cfg.dz and abs(org[2]) < 1e-15


def _closed_box_three_axes(seed=7):
    """A box stretched along x, y and z (random widths, ratio up to 3), slip walls on all six sides."""
    cfg = make_case("channel", grid=(10, 9, 8)).with_(bc=("slip",) * 6, body_force=(0.0, 0.0, 0.0))
    faces = (_random_faces(10, 0.0, 2.0, seed), _random_faces(9, -1.0, 1.0, seed + 1),
             _random_faces(8, 0.0, 1.5, seed + 2))
    return cfg.with_(x0=0.0, lx=2.0, z0=0.0, lz=1.5, faces=faces)


@pytest.mark.parametrize("order", [5, 2])
def test_three_stretched_axes_free_stream_and_mass(order):
    # a fluid at rest stays at rest, and a perturbed one keeps its mass (volume-weighted), on a mesh
    # stretched along all three axes at once
    cfg = _closed_box_three_axes().with_(order=order)
    q = np.zeros((4, 8, 9, 10))
    q[0] = 1.01
    o = Oracle(cfg.with_(q0=q))
    for _ in range(2):
        o.step()
    assert float((o.Q - torch.tensor(q)).abs().max()) < 1e-13
    rng = np.random.default_rng(2)
    q[0] += 0.01 * rng.uniform(-1, 1, size=q[0].shape)
    q[1:] += 0.05 * rng.uniform(-1, 1, size=q[1:].shape)
    cfg = cfg.with_(q0=q)
    o = Oracle(cfg)
    m0 = conservation_sums(o.Q, cfg)[0]
    for _ in range(2):
        o.step()
    assert abs(conservation_sums(o.Q, cfg)[0] - m0) < 1e-13 * abs(m0)


def test_stretched_inflow_axis_keeps_a_uniform_stream():
    # inflow/outflow along a stretched x axis (the refined block of Section 4.3.3): the inflow state
    # itself stays uniform
    from synth.cases import block_faces
    cfg = make_case("alm", grid=(24, 12, 12)).with_(rotor=None)
    xf = block_faces(4, 10, 10, 0.25, 1.15, 1.0)
    cfg = cfg.with_(x0=float(xf[0]), lx=float(xf[-1] - xf[0]), faces=(xf, None, None))
    o = Oracle(cfg)
    for _ in range(2):
        o.step()
    assert float((o.Q - torch.tensor(cfg.q0)).abs().max()) < 1e-13
