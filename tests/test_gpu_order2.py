"""GPU parity of the second-order GKS variant (config order = 2, reading R15) against the FP64 oracle
through the C ABI: FP64 to 1e-12 relative per variable (every boundary kind, a rotor case), FP32 to 1e-5
relative L2, free stream, periodic conservation."""
import numpy as np
import pytest
import torch

from gpu_util import oracle_dev, print_case, rel_errors, rel_l2, run_gpu, run_oracle
from synth import make_case

pytestmark = pytest.mark.gpu


def _perturbed_stream(cfg, seed=9, amp=0.05):
    rng = np.random.default_rng(seed)
    q = cfg.q0.copy()
    q[1:] += amp * rng.uniform(-1, 1, size=q[1:].shape)
    q[0] += 0.2 * amp * rng.uniform(-1, 1, size=q[0].shape)
    return q


@pytest.mark.parametrize("case,grid,steps", [
    ("tgv", (17, 33, 20), 2),          # periodic, ragged tiles in every direction
    ("channel", (21, 18, 35), 2),      # no-slip walls, body force
])
def test_order2_fp64_vs_oracle(case, grid, steps):
    cfg = make_case(case, grid=grid).with_(order=2)
    print_case(case + "-order2-fp64", grid=grid, steps=steps)
    s, gouts = run_gpu(cfg, "fp64", steps)
    o, oouts = run_oracle(cfg, steps)
    err = rel_errors(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-12, err
    for a, b in zip(gouts, oouts):
        assert abs(a["dt"] - b["dt"]) < 1e-14 * b["dt"]


def test_order2_inflow_outflow_rotor_fp64_vs_oracle():
    cfg = make_case("alm", grid=(48, 24, 24)).with_(order=2)
    cfg = cfg.with_(q0=_perturbed_stream(cfg, seed=4, amp=0.02))
    print_case("order2-alm-fp64", grid=(48, 24, 24))
    s, gouts = run_gpu(cfg, "fp64", 2)
    o, oouts = run_oracle(cfg, 2)
    err = rel_errors(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-12, err
    for a, b in zip(gouts, oouts):
        assert abs(a["power"] - float(b["alm"]["power"])) <= 1e-12 * abs(float(b["alm"]["power"]))


def test_order2_fp32_vs_oracle():
    cfg = make_case("tgv", grid=(24, 20, 18)).with_(order=2)
    print_case("order2-fp32", grid=(24, 20, 18))
    s, _ = run_gpu(cfg, "fp32", 3)
    o, _ = run_oracle(cfg, 3)
    err = rel_l2(s.interior(), oracle_dev(o.Q, cfg.rho_ref))
    assert max(err) < 1e-5, err


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-14), ("fp32", 2e-6)])
def test_order2_free_stream(precision, tol):
    cfg = make_case("alm", grid=(36, 18, 18)).with_(rotor=None, order=2)
    print_case("order2-free-stream", precision=precision)
    s, _ = run_gpu(cfg, precision, 3)
    ref = oracle_dev(torch.tensor(cfg.q0), cfg.rho_ref)
    assert float((s.interior() - ref).abs().max()) < tol


def test_order2_periodic_conservation_fp64():
    cfg = make_case("tgv", grid=(24, 24, 24)).with_(order=2)
    print_case("order2-conservation")
    from paper_2603_11102_amd import GksSolver
    s = GksSolver(cfg, precision="fp64")
    f0 = s.forces()
    s.step(5)
    f1 = s.forces()
    scale = cfg.n_cells * cfg.dx * cfg.dy * cfg.dz
    assert abs(f1["mass"] - f0["mass"]) < 1e-13 * scale
    for a, b in zip(f0["mom"], f1["mom"]):
        assert abs(a - b) < 1e-13 * scale
