"""Body-force parity at the full sizes of the rotor workloads (384 x 192 x 192 with the 192-point rotor;
512 x 256 x 256 with the rotor and the 24,139 Lagrangian points of tower and nacelle).

The force update of Section 3.3 acts after the S2O4 step. Two contexts step the same perturbed state
once with the same fixed dt, one with and one without the body forces; their flow steps are the same
kernels on the same inputs, so the force-free result is the field the forces act on. The oracle then
applies its own actuator-line model (Section 3.1) and direct forcing (Section 3.2) to that field, and
the forced context must match it in every cell, in the per-point angles and forces, and in the rotor
and body loads.

Bars: FP64 1e-11 (relative to each variable's largest magnitude; per-point and reduced loads relative);
FP32: the forces are evaluated in FP64 from the FP32 field, so per-point values and loads agree to 1e-11
as well, the forced field to 2 ulp of FP32 (2.4e-7 of the largest magnitude) and the IBM force and
residual, which see the FP32-rounded field after the actuator-line update, to 1e-6."""
import gc

import numpy as np
import pytest
import torch

from gpu_util import print_case
from oracle.gks_oracle import alm_apply, ibm_apply, ibm_setup
from synth import make_case

pytestmark = pytest.mark.gpu


def _perturbed(cfg, seed):
    rng = np.random.default_rng(seed)
    q = cfg.q0.copy()
    q[1:] += 0.05 * rng.uniform(-1, 1, size=q[1:].shape)
    q[0] += 0.005 * rng.uniform(-1, 1, size=q[0].shape)
    return cfg.with_(q0=q)


def _interior_dev(s):
    torch.cuda.synchronize()
    return s.q[:, 3:-3, 3:-3, 3:-3]


@pytest.mark.parametrize("case,precision", [
    ("alm", "fp64"), ("alm", "fp32"), ("alm_ibm", "fp64"), ("alm_ibm", "fp32"),
])
def test_full_size_body_forces_vs_oracle(case, precision):
    from paper_2603_11102_amd import GksSolver
    cfg = _perturbed(make_case(case), 17)
    dt = 0.5 * cfg.dx / (1.0 + cfg.u_ref / cfg.ma)
    cfg = cfg.with_(cfl=0.0, dt_fixed=dt)
    print_case("fullsize-forces", case=case, precision=precision, grid=(cfg.nx, cfg.ny, cfg.nz),
               n_act=cfg.rotor.n_act, n_ibm=cfg.ibm.n if cfg.ibm is not None else 0)
    plain = GksSolver(cfg.with_(rotor=None, ibm=None), precision=precision)
    plain.step(1)
    pre = _interior_dev(plain).to(torch.float64).cpu()
    plain.close()
    del plain
    gc.collect()
    torch.cuda.empty_cache()
    s = GksSolver(cfg, precision=precision)
    s.step(1)
    f = s.forces(per_point=True)
    got = _interior_dev(s).to(torch.float64)
    assert abs(f["dt"] - dt) == 0.0 and abs(f["t"] - dt) == 0.0

    # the oracle's force update on the GPU's own force-free field (oracle layout: rho, not rho - rho_ref)
    Q = pre.clone()
    Q[0] += cfg.rho_ref
    Q, alm = alm_apply(Q, dt, dt, cfg, cfg.rotor)
    ib = None
    if cfg.ibm is not None:
        Q, ib = ibm_apply(Q, dt, cfg, ibm_setup(cfg, cfg.ibm), cfg.ibm_iters)
    Q[0] -= cfg.rho_ref
    ref = Q.to(got.device)
    del Q

    # per-point values and rotor loads: FP64 arithmetic on the same sampled field in both precisions
    assert np.allclose(f["alpha"], alm["alpha"].numpy(), rtol=1e-11, atol=1e-13)
    fx, ft = alm["fx"].numpy(), alm["ftheta"].numpy()
    assert np.abs(f["fx"] - fx).max() <= 1e-11 * np.abs(fx).max()
    assert np.abs(f["ftheta"] - ft).max() <= 1e-11 * np.abs(ft).max()
    for k in ("thrust", "torque", "power", "cp", "ct"):
        assert abs(f[k] - float(alm[k])) <= 1e-11 * abs(float(alm[k])), k

    # every cell, forced or not
    tol_field = 1e-11 if precision == "fp64" else 2.4e-7
    moved = (got - pre.to(got.device)).abs().amax(dim=(1, 2, 3))
    assert float(moved[1]) > 0.0  # the actuator line did act
    for v in range(4):
        scale = float(ref[v].abs().max()) if v > 0 else cfg.rho_ref
        err = float((got[v] - ref[v]).abs().max())
        print(f"[fullsize-forces] {case} {precision} variable {v}: max error {err:.3e} (scale {scale:.3e})")
        assert err <= tol_field * scale, (v, err, scale)
    if ib is not None:
        tol_ibm = 1e-11 if precision == "fp64" else 1e-6
        bf = ib["body_force"].numpy()
        assert np.abs(np.asarray(f["ibm_force"]) - bf).max() <= tol_ibm * np.abs(bf).max()
        res = float(ib["residual"])
        assert abs(f["ibm_residual"] - res) <= tol_ibm * max(res, 1e-300)
        assert f["ibm_iters_used"] == cfg.ibm_iters
    s.close()
    del s, got, ref
    gc.collect()
    torch.cuda.empty_cache()


def test_full_size_channel_fp32_vs_fp64_hundred_steps():
    # the benchmark workload itself: 192 x 96 x 96 channel, FP32 (compensated state, density as its
    # deviation) against FP64 after 100 steps, relative L2 per variable
    from paper_2603_11102_amd import GksSolver
    from gpu_util import rel_l2
    cfg = make_case("channel")
    print_case("channel-fp32-vs-fp64-100", grid=(cfg.nx, cfg.ny, cfg.nz))
    a = GksSolver(cfg, precision="fp32")
    b = GksSolver(cfg, precision="fp64")
    a.step(100)
    b.step(100)
    err = rel_l2(a.interior(), b.interior())
    print(f"[channel-fp32-vs-fp64-100] rel L2 per variable {err}")
    assert max(err) < 1e-5, err
    fa, fb = a.forces(), b.forces()
    assert fa["step"] == fb["step"] == 100
    assert abs(fa["t"] - fb["t"]) <= 1e-6 * fb["t"]
