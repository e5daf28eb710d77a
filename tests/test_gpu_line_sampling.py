"""Line sampling of the actuator points (the NTNU rotor's sampling, Sections 3.1 and 4.4; reading R18)
on the GPU against the oracle: the forced field, the per-point angles and forces and the rotor loads
in FP64 (1e-12 field, 1e-11 per point) and FP32, the adjoint with line sampling against the oracle's
frozen-weight reverse mode, one sample reproducing point sampling bitwise, and the refusal of a
sampling segment that leaves the interior."""
from dataclasses import replace

import numpy as np
import pytest
import torch

from gpu_util import oracle_dev, print_case, rel_errors, rel_l2, run_gpu, run_oracle
from oracle import rotor_gradient
from synth import make_case

pytestmark = pytest.mark.gpu


def _ntnu_like(grid=(48, 24, 24), seed=3):
    cfg = make_case("alm", grid=grid)
    rng = np.random.default_rng(seed)
    q = cfg.q0.copy()
    q[1:] += 0.02 * rng.uniform(-1, 1, size=q[1:].shape)
    q[0] += 0.002 * rng.uniform(-1, 1, size=q[0].shape)
    rotor = replace(cfg.rotor, tip_correction=True, line_points=9, line_half_length=2.0 * cfg.rotor.eps,
                    theta0=0.3)
    return cfg.with_(q0=q, rotor=rotor)


def test_line_sampling_fp64_vs_oracle():
    cfg = _ntnu_like()
    print_case("line-sampling-fp64", grid=(48, 24, 24), points=cfg.rotor.line_points)
    s, gouts = run_gpu(cfg, "fp64", 2)
    o, oouts = run_oracle(cfg, 2)
    err = rel_errors(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-12, err
    for a, b in zip(gouts, oouts):
        alm = b["alm"]
        assert np.allclose(a["alpha"], alm["alpha"].numpy(), rtol=1e-12, atol=1e-14)
        assert np.abs(a["fx"] - alm["fx"].numpy()).max() <= 1e-11 * np.abs(alm["fx"].numpy()).max()
        assert np.abs(a["ftheta"] - alm["ftheta"].numpy()).max() <= 1e-11 * np.abs(alm["ftheta"].numpy()).max()
        for k in ("thrust", "torque", "power", "cp", "ct"):
            assert abs(a[k] - float(alm[k])) <= 1e-12 * abs(float(alm[k])), k
    # the sampling matters: point sampling gives different loads on this field
    p, pouts = run_gpu(cfg.with_(rotor=replace(cfg.rotor, line_points=1)), "fp64", 1)
    assert abs(pouts[0]["thrust"] - gouts[0]["thrust"]) > 1e-8 * abs(gouts[0]["thrust"])


def test_line_sampling_fp32_vs_oracle():
    cfg = _ntnu_like()
    print_case("line-sampling-fp32", grid=(48, 24, 24))
    s, gouts = run_gpu(cfg, "fp32", 2)
    o, oouts = run_oracle(cfg, 2)
    err = rel_l2(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-5, err
    assert abs(gouts[-1]["power"] - float(oouts[-1]["alm"]["power"])) < 1e-5 * abs(float(oouts[-1]["alm"]["power"]))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_one_sample_is_point_sampling(precision):
    cfg = _ntnu_like()
    print_case("line-sampling-one", precision=precision)
    a, oa = run_gpu(cfg.with_(rotor=replace(cfg.rotor, line_points=1)), precision, 2)
    b, ob = run_gpu(cfg.with_(rotor=replace(cfg.rotor, line_points=0, line_half_length=0.0)), precision, 2)
    assert torch.equal(a.interior(), b.interior())
    assert oa[-1]["thrust"] == ob[-1]["thrust"] and oa[-1]["power"] == ob[-1]["power"]


def test_line_sampling_adjoint_vs_oracle():
    from paper_2603_11102_amd import GksSolver
    cfg = make_case("adjoint", grid=(20, 20, 20))
    cfg = cfg.with_(rotor=replace(cfg.rotor, tip_correction=True, line_points=5, line_half_length=1.5 * cfg.rotor.eps))
    n = cfg.rotor.n_act
    s0 = 1.0 + 0.1 * np.random.default_rng(0).standard_normal(n)
    nsteps = 2
    w = (1.0, 0.5)
    print_case("line-sampling-adjoint", grid=(20, 20, 20), nsteps=nsteps)
    s = GksSolver(cfg, precision="fp64")
    s.set_rotor(cfg.rotor, scale=torch.as_tensor(s0, dtype=torch.float64, device="cuda").contiguous())
    s.set_checkpoints(nsteps)
    s.step(nsteps)
    f = s.forces()
    J = (w[0] * f["window_power"] + w[1] * f["window_thrust"]) / f["window_steps"]
    g, _ = s.adjoint(nsteps, w)
    Jo, go = rotor_gradient(cfg, s0, nsteps, w, frozen=True)
    assert abs(J - Jo) < 1e-12 * abs(Jo)
    rel = float((g.cpu() - go).abs().max() / go.abs().max())
    assert rel < 1e-10, rel


def test_sampling_segment_must_stay_inside():
    from paper_2603_11102_amd import GksSolver
    from paper_2603_11102_amd._lib import GksError
    cfg = _ntnu_like()
    print_case("line-sampling-refusal")
    s = GksSolver(cfg.with_(rotor=None), precision="fp64", max_act=cfg.rotor.n_act)
    with pytest.raises(GksError):
        s.set_rotor(replace(cfg.rotor, line_half_length=1.6))  # the swept segments reach 1.68 from the hub axis
    with pytest.raises(GksError):
        s.set_rotor(replace(cfg.rotor, line_points=2, line_half_length=-0.1))
    s.set_rotor(cfg.rotor)
