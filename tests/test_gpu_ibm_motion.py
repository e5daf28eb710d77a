"""GPU parity of rigidly moving immersed bodies (gks_set_ibm_motion): every step places the Lagrangian
points at t^{n+1} and rebuilds their supports, V-bar and v-bar on the device before the forcing.
Bars as for the other parity tests: FP64 1e-12 relative against the oracle, FP32 1e-5; a body at rest
reproduces the stationary path bitwise (the device rebinning orders cells and points as the host one)."""
import numpy as np
import pytest
import torch

from gpu_util import oracle_dev, print_case, rel_errors, rel_l2, run_gpu, run_oracle
from synth import make_case
from synth.cases import IbmMotion, IbmSpec

pytestmark = pytest.mark.gpu

GRID = (64, 32, 32)


def _yawing_body(omega=8.0, vel=(0.3, 0.0, 0.0)):
    """Tower and nacelle of the rotor box turning about the tower axis and drifting downstream."""
    cfg = make_case("alm_ibm", grid=GRID).with_(rotor=None)
    tower = np.array([2.0 + 0.16, 2.0, 0.0])
    ib = IbmSpec(xyz=cfg.ibm.xyz, dS=cfg.ibm.dS, motion=IbmMotion(center=tower, velocity=vel,
                                                                   omega=(0.0, 0.0, omega), t0=0.0))
    return cfg.with_(ibm=ib)


def test_moving_body_fp64_vs_oracle():
    cfg = _yawing_body()
    steps = 6
    print_case("ibm-motion-fp64", grid=GRID, n_ibm=cfg.ibm.n, steps=steps)
    s, gouts = run_gpu(cfg, "fp64", steps)
    o, oouts = run_oracle(cfg, steps)
    err = rel_errors(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-12, err
    for g, b in zip(gouts, oouts):
        assert g["status"] == 0
        ref_f = b["ibm"]["body_force"].numpy()
        assert np.allclose(g["ibm_force"], ref_f, rtol=1e-11, atol=1e-14 * np.abs(ref_f).max())
        assert abs(g["ibm_residual"] - float(b["ibm"]["residual"])) < 1e-12 * max(1.0, float(b["ibm"]["residual"]))
    # the body did move across cells: the first and last supports differ
    from oracle import ibm_motion_state, ibm_setup
    from oracle.gks_oracle import IbmPoints
    X1, v1 = ibm_motion_state(cfg.ibm, oouts[0]["t"])
    X6, v6 = ibm_motion_state(cfg.ibm, oouts[-1]["t"])
    c1 = ibm_setup(cfg, IbmPoints(X1, cfg.ibm.dS, v1)).vbar_index
    c6 = ibm_setup(cfg, IbmPoints(X6, cfg.ibm.dS, v6)).vbar_index
    assert not np.array_equal(c1, c6)


def test_moving_body_fp32_vs_oracle():
    cfg = _yawing_body()
    steps = 4
    print_case("ibm-motion-fp32", grid=GRID, n_ibm=cfg.ibm.n, steps=steps)
    s, gouts = run_gpu(cfg, "fp32", steps)
    o, oouts = run_oracle(cfg, steps)
    err = rel_l2(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-5, err
    for g, b in zip(gouts, oouts):
        ref_f = b["ibm"]["body_force"].numpy()
        assert np.abs(np.asarray(g["ibm_force"]) - ref_f).max() < 1e-4 * np.abs(ref_f).max()


def test_body_at_rest_reproduces_the_stationary_path_bitwise():
    from paper_2603_11102_amd import GksSolver
    base = make_case("alm_ibm", grid=GRID)
    still = base.with_(ibm=IbmSpec(xyz=base.ibm.xyz, dS=base.ibm.dS))
    rest = base.with_(ibm=IbmSpec(xyz=base.ibm.xyz, dS=base.ibm.dS, motion=IbmMotion(center=(2.0, 2.0, 1.0))))
    print_case("ibm-motion-at-rest", grid=GRID, n_ibm=base.ibm.n)
    a = GksSolver(still, precision="fp32")
    b = GksSolver(rest, precision="fp32")
    for _ in range(3):
        a.step(1)
        b.step(1)
        fa, fb = a.forces(), b.forces()
        assert fa["ibm_force"] == fb["ibm_force"]
        assert fa["ibm_residual"] == fb["ibm_residual"]
    assert torch.equal(a.interior(), b.interior())


def test_several_steps_per_call_match_single_steps():
    from paper_2603_11102_amd import GksSolver
    cfg = _yawing_body()
    print_case("ibm-motion-multistep", grid=GRID, n_ibm=cfg.ibm.n)
    a = GksSolver(cfg, precision="fp32")
    b = GksSolver(cfg, precision="fp32")
    a.step(4)
    for _ in range(4):
        b.step(1)
    fa, fb = a.forces(), b.forces()
    assert fa["t"] == fb["t"] and fa["ibm_force"] == fb["ibm_force"]
    assert torch.equal(a.interior(), b.interior())


def test_body_leaving_the_interior_is_reported_and_stops_the_forcing():
    from paper_2603_11102_amd import GksSolver
    from paper_2603_11102_amd._lib import GKS_E_BODY_LEFT
    cfg = make_case("tgv", grid=(24, 24, 24)).with_(bc=("periodic",) * 6)
    h = cfg.dx
    rng = np.random.default_rng(3)
    d = rng.normal(size=(40, 3))
    d *= 1.5 * h / np.linalg.norm(d, axis=1, keepdims=True)
    c0 = np.array([cfg.lx - 6.0 * h, 0.5 * cfg.ly, 0.5 * cfg.lz])
    xyz = c0 + d
    dS = np.full(40, 0.005 * h * h)
    # 3 cells per step for a CFL step of about 0.5 h / (|U| + C): out of the interior within 2 steps
    fast = IbmSpec(xyz=xyz, dS=dS, motion=IbmMotion(center=c0, velocity=(60.0, 0.0, 0.0)))
    print_case("ibm-motion-leaves", grid=(24, 24, 24))
    s = GksSolver(cfg.with_(ibm=fast), precision="fp64")
    outs = []
    for _ in range(4):
        s.step(1)
        outs.append(s.forces(check=False))
    assert outs[0]["status"] == 0 and any(f != 0.0 for f in outs[0]["ibm_force"])
    assert [o["status"] for o in outs[2:]] == [GKS_E_BODY_LEFT] * 2
    assert bool(torch.isfinite(s.interior()).all())
    # once reported, the forcing is off for every later step: no load, no residual
    for o in outs:
        if o["status"] == GKS_E_BODY_LEFT:
            assert o["ibm_force"] == [0.0, 0.0, 0.0] and o["ibm_residual"] == 0.0
    # new points clear the report
    s.set_ibm(IbmSpec(xyz=xyz, dS=dS))
    s.step(1)
    assert s.forces()["status"] == 0


def test_moving_body_step_in_a_hip_graph_replays_like_eager_steps():
    # the per-step placement and rebinning are kernels only (no memset, no host work), so a captured
    # step replays exactly like eager steps; each replay is checked, with eager work in between
    from paper_2603_11102_amd import GksSolver
    cfg = _yawing_body()
    print_case("ibm-motion-graph", grid=GRID, n_ibm=cfg.ibm.n)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a = GksSolver(cfg, precision="fp32")
        b = GksSolver(cfg, precision="fp32")
    a.step(1)
    b.step(1)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        a.step(1)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        b.step(1)
        torch.cuda.synchronize()
        assert torch.equal(a.interior(), b.interior())
        fa, fb = a.forces(), b.forces()
        assert fa["t"] == fb["t"] and fa["ibm_force"] == fb["ibm_force"]


@pytest.mark.parametrize("order,rotor", [(2, False), (5, True)])
def test_moving_body_with_the_second_order_scheme_or_a_rotor_fp64_vs_oracle(order, rotor):
    base = make_case("alm_ibm", grid=GRID)
    cfg = _yawing_body().with_(order=order, rotor=base.rotor if rotor else None)
    print_case(f"ibm-motion-order{order}-rotor{int(rotor)}", grid=GRID, n_ibm=cfg.ibm.n)
    s, gouts = run_gpu(cfg, "fp64", 3)
    o, oouts = run_oracle(cfg, 3)
    err = rel_errors(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-12, err
    for g, b in zip(gouts, oouts):
        ref_f = b["ibm"]["body_force"].numpy()
        assert np.allclose(g["ibm_force"], ref_f, rtol=1e-11, atol=1e-14 * np.abs(ref_f).max())
        if rotor:
            assert abs(g["power"] - float(b["alm"]["power"])) < 1e-11 * abs(float(b["alm"]["power"]))


def _top_stretched(cfg, n_uniform, n_grow, ratio):
    """The same box with the cells above the first n_uniform growing by ratio (z axis)."""
    w = np.concatenate([np.full(n_uniform, cfg.dz), cfg.dz * ratio ** np.arange(1, n_grow + 1)])
    zf = np.concatenate([[0.0], np.cumsum(w)])
    return cfg.with_(lz=float(zf[-1]), faces=(None, None, zf))


def test_moving_body_on_a_stretched_mesh_fp64_vs_oracle():
    # the yawing tower and nacelle stay in the uniform cells under the growing ones
    cfg = _top_stretched(_yawing_body(), 24, 8, 1.1)
    print_case("ibm-motion-stretched-fp64", grid=GRID, n_ibm=cfg.ibm.n)
    s, gouts = run_gpu(cfg, "fp64", 4)
    o, oouts = run_oracle(cfg, 4)
    err = rel_errors(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-12, err
    for g, b in zip(gouts, oouts):
        assert g["status"] == 0
        ref_f = b["ibm"]["body_force"].numpy()
        assert np.allclose(g["ibm_force"], ref_f, rtol=1e-11, atol=1e-14 * np.abs(ref_f).max())


def test_moving_body_leaving_its_uniform_cells_is_reported():
    from paper_2603_11102_amd import GksSolver
    from paper_2603_11102_amd._lib import GKS_E_BODY_LEFT
    base = make_case("alm_ibm", grid=GRID).with_(rotor=None)
    # a small sphere below the growing cells, driven upwards into them
    h = base.dz
    rng = np.random.default_rng(5)
    d = rng.normal(size=(40, 3))
    d *= 1.5 * h / np.linalg.norm(d, axis=1, keepdims=True)
    c0 = np.array([3.0, 2.0, 24 * h - 6.0 * h])
    ib = IbmSpec(xyz=c0 + d, dS=np.full(40, 0.005 * h * h), motion=IbmMotion(center=c0, velocity=(0.0, 0.0, 60.0)))
    cfg = _top_stretched(base.with_(ibm=ib), 24, 8, 1.1)
    print_case("ibm-motion-stretched-leaves", grid=GRID)
    s = GksSolver(cfg, precision="fp64")
    outs = []
    for _ in range(4):
        s.step(1)
        outs.append(s.forces(check=False))
    assert outs[0]["status"] == 0
    assert outs[-1]["status"] == GKS_E_BODY_LEFT
    assert outs[-1]["ibm_force"] == [0.0, 0.0, 0.0]
    assert bool(torch.isfinite(s.interior()).all())


def _edge_case(velocity_cells_per_step=2.5, steps=4):
    """A small sphere below the growing cells driven upwards at a fixed dt so that its supports reach
    the last cell of the run of uniform cells at one step and leave the run at the next."""
    base = make_case("alm_ibm", grid=GRID).with_(rotor=None)
    h = base.dz
    dt = 0.04 * h
    rng = np.random.default_rng(5)
    d = rng.normal(size=(40, 3))
    d *= 1.5 * h / np.linalg.norm(d, axis=1, keepdims=True)
    c0 = np.array([3.0, 2.0, 24 * h - 6.0 * h])
    ib = IbmSpec(xyz=c0 + d, dS=np.full(40, 0.005 * h * h),
                 motion=IbmMotion(center=c0, velocity=(0.0, 0.0, velocity_cells_per_step * h / dt)))
    return _top_stretched(base.with_(ibm=ib, cfl=0.0, dt_fixed=dt), 24, 8, 1.1)


def test_moving_body_at_and_past_the_edge_of_its_run_fp64_vs_oracle():
    # the oracle applies the same rule as the device: a support may reach the last cell of the run of
    # the body's width; past it the forcing stops for good and the step reports it
    from oracle.gks_oracle import body_run, body_grid, ibm_motion_state
    from paper_2603_11102_amd._lib import GKS_E_BODY_LEFT
    cfg = _edge_case()
    steps = 4
    X0 = np.asarray(cfg.ibm.xyz)
    org, hh = body_grid(cfg, X0.min(0), X0.max(0), 2)
    run_hi = body_run(cfg, X0.min(0), X0.max(0), 2)[2][1]
    top = []
    for n in range(1, steps + 1):
        X, _ = ibm_motion_state(cfg.ibm, n * cfg.dt_fixed)
        top.append(int(np.floor((X[:, 2] - org[2]) / hh[2] - 0.5).max()) + 2)
    assert run_hi in top and top[-1] > run_hi  # the supports reach the edge cell, then pass it
    print_case("ibm-motion-edge", grid=GRID, run_hi=run_hi, support_top=top)
    from paper_2603_11102_amd import GksSolver
    s = GksSolver(cfg, precision="fp64")
    gouts = []
    for _ in range(steps):
        s.step(1)
        gouts.append(s.forces(check=False))  # the body-left status is a result here, not an error
    o, oouts = run_oracle(cfg, steps)
    err = rel_errors(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-12, err
    left = False
    for g, b, t in zip(gouts, oouts, top):
        left = left or t > run_hi
        assert b["ibm"]["left"] == left
        assert (g["status"] == GKS_E_BODY_LEFT) == left
        ref_f = b["ibm"]["body_force"].numpy()
        if left:
            assert g["ibm_force"] == [0.0, 0.0, 0.0] and not ref_f.any()
        else:
            assert any(f != 0.0 for f in g["ibm_force"])
            assert np.allclose(g["ibm_force"], ref_f, rtol=1e-11, atol=1e-14 * np.abs(ref_f).max())
