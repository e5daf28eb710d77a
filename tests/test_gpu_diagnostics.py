"""FP64 conservation sums, |U|max and the error and warning reports of gks_forces, against the oracle and
against exact sums of the field the library holds.

gks_forces returns mass = sum (rho - rho_ref) |Omega_ijk| and mom = sum rho U |Omega_ijk| over the
interior cells (the finite-volume telescoping of Section 2 keeps both constant in a periodic box) and
umax = max |U|; the CFL step of Section 2 uses the same maximum. The test cases carry a uniform drift
and a density offset so that none of the sums is zero by symmetry."""
import math

import numpy as np
import pytest
import torch

from gpu_util import print_case
from oracle import Oracle
from oracle.gks_oracle import axis_metrics, conservation_sums
from synth import make_case

pytestmark = pytest.mark.gpu


def _drifting(cfg, seed=21):
    """The case's field plus a uniform drift (0.3, -0.2, 0.1), a density offset and 2 % density noise."""
    rng = np.random.default_rng(seed)
    q = cfg.q0.copy()
    rho = q[0] * (1.0 + 0.002 + 0.02 * rng.uniform(-1, 1, size=q[0].shape))
    u = q[1:] / q[0]
    u = u + np.array([0.3, -0.2, 0.1])[:, None, None, None]
    return cfg.with_(q0=np.concatenate([rho[None], rho[None] * u], 0))


def _volumes(cfg):
    w = [axis_metrics(cfg, a)[0] for a in range(3)]
    return np.asarray(w[2])[:, None, None] * np.asarray(w[1])[None, :, None] * np.asarray(w[0])[None, None, :]


def _exact_sums(q, vol):
    """math.fsum of (rho - rho_ref) |Omega| and of the momenta |Omega| (q holds rho - rho_ref)."""
    a = q.numpy() * vol[None]
    return [math.fsum(a[v].reshape(-1).tolist()) for v in range(4)]


def _umax(q, rho_ref):
    rho = q[0] + rho_ref
    return float(torch.sqrt(((q[1:] / rho) ** 2).sum(0)).max())


@pytest.mark.parametrize("case,grid,steps,precision", [
    ("tgv", (32, 32, 32), 10, "fp64"),
    ("channel_tanh", (20, 24, 18), 3, "fp64"),
    ("tgv", (32, 32, 32), 10, "fp32"),
])
def test_conservation_sums_and_umax_vs_oracle(case, grid, steps, precision):
    from paper_2603_11102_amd import GksSolver
    cfg = _drifting(make_case(case, grid=grid))
    print_case("diag-sums", case=case, grid=grid, steps=steps, precision=precision)
    s = GksSolver(cfg, precision=precision)
    s.step(steps)
    f = s.forces()
    q = s.interior()
    vol = _volumes(cfg)
    o = Oracle(cfg)
    for _ in range(steps):
        o.step()
    ref = conservation_sums(o.Q, cfg)
    cell = cfg.dx * cfg.dy * cfg.dz  # the oracle's sums are per uniform cell volume
    ref_mass = (ref[0] - cfg.rho_ref * float(vol.sum()) / cell) * cell
    ref_mom = [r * cell for r in ref[1:]]
    got = [f["mass"]] + list(f["mom"])
    scale = [float((q[v].abs().numpy() * vol).sum()) for v in range(4)]
    own = _exact_sums(q, vol)
    if precision == "fp64":
        # the device's fixed-order FP64 tree sum of the field it holds, against the exact sum
        for v in range(4):
            assert abs(got[v] - own[v]) <= 1e-13 * scale[v], (v, got[v], own[v])
        tol, utol = 1e-12, 1e-12
    else:
        # FP32: the sums include the low-order part of the compensated state; the field read back is
        # its high part only, so the two differ by at most the low part (< 1 ulp of FP32 per cell)
        for v in range(4):
            assert abs(got[v] - own[v]) <= 6e-8 * scale[v], (v, got[v], own[v])
        tol, utol = 2e-6, 1e-5
    for v, r in enumerate([ref_mass] + ref_mom):
        assert abs(got[v] - r) <= tol * scale[v], (v, got[v], r)
    um_ref = _umax(o.Q - torch.tensor([cfg.rho_ref, 0, 0, 0], dtype=torch.float64).view(4, 1, 1, 1), cfg.rho_ref)
    # |U|max of the field read back (FP32: its high part, within 2e-7 relative of the state)
    assert abs(f["umax"] - _umax(q, cfg.rho_ref)) <= (1e-14 if precision == "fp64" else 2e-7) * um_ref
    assert abs(f["umax"] - um_ref) <= utol * um_ref


def test_mass_conserved_in_periodic_box_fp32_with_low_part():
    # FP32 periodic box: the mass of the compensated state (field + low part) stays at its initial value
    # to FP32 rounding of the increments
    from paper_2603_11102_amd import GksSolver
    cfg = _drifting(make_case("tgv", grid=(32, 32, 32)))
    print_case("diag-mass-fp32")
    s = GksSolver(cfg, precision="fp32")
    f0 = s.forces()
    s.step(20)
    f1 = s.forces()
    scale = float(np.abs(cfg.q0[0] - cfg.rho_ref).sum()) * cfg.dx * cfg.dy * cfg.dz
    assert abs(f1["mass"] - f0["mass"]) < 1e-6 * scale


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_non_finite_field_is_reported(precision):
    from paper_2603_11102_amd import GksSolver
    from paper_2603_11102_amd import _lib as L
    cfg = make_case("tgv", grid=(16, 16, 16))
    print_case("diag-nonfinite", precision=precision)
    s = GksSolver(cfg, precision=precision)
    assert s.forces()["status"] == L.GKS_OK
    q = cfg.q0.copy()
    q[2, 3, 5, 7] = np.nan
    s.set_interior(q)
    f = s.forces(check=False)
    assert f["status"] == L.GKS_E_NONFINITE
    assert "non-finite" in L.last_error(s.lib, s.ctx)
    q = cfg.q0.copy()
    q[0, 9, 1, 2] = np.inf
    s.set_interior(q)
    assert s.forces(check=False)["status"] == L.GKS_E_NONFINITE
    s.set_interior(cfg.q0)
    assert s.forces(check=False)["status"] == L.GKS_OK


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_velocity_at_sound_speed_is_reported(precision):
    from paper_2603_11102_amd import GksSolver
    from paper_2603_11102_amd import _lib as L
    cfg = make_case("tgv", grid=(16, 16, 16))
    c = cfg.u_ref / cfg.ma  # sqrt(1 / (2 lambda)), lambda = Ma^2 / (2 U_ref^2)
    print_case("diag-unstable", precision=precision, c=c)
    s = GksSolver(cfg, precision=precision)
    q = cfg.q0.copy()
    q[3, 4, 4, 4] = 0.99 * c * q[0, 4, 4, 4]
    q[1:, 4, 4, 4] *= np.array([0.0, 0.0, 1.0])  # |U| = 0.99 c: still below the sound speed
    s.set_interior(q)
    f = s.forces(check=False)
    assert f["status"] == L.GKS_OK
    assert abs(f["umax"] - 0.99 * c) < 1e-5 * c
    q[3, 4, 4, 4] = 1.01 * c * q[0, 4, 4, 4]
    s.set_interior(q)
    f = s.forces(check=False)
    assert f["status"] == L.GKS_E_UNSTABLE
    assert abs(f["umax"] - 1.01 * c) < 1e-5 * c
    assert "sound speed" in L.last_error(s.lib, s.ctx)


def test_warning_flags():
    from dataclasses import replace
    from paper_2603_11102_amd import GksSolver
    from paper_2603_11102_amd import _lib as L
    cfg = make_case("alm", grid=(48, 24, 24))
    print_case("diag-flags", grid=(48, 24, 24))
    s = GksSolver(cfg, precision="fp64")
    assert s.forces()["flags"] == 0  # eps = 2 dx, Ma = 0.1
    s.set_rotor(replace(cfg.rotor, eps=1.5 * cfg.dx))
    assert s.forces()["flags"] == L.GKS_WARN_EPS_SMALL  # Section 4.3.1: eps >= 2 dx
    s.set_rotor(cfg.rotor)
    assert s.forces()["flags"] == 0
    fast = GksSolver(make_case("tgv", grid=(16, 16, 16)).with_(ma=0.35), precision="fp64")
    assert fast.forces()["flags"] == L.GKS_WARN_MACH
    slow = GksSolver(make_case("tgv", grid=(16, 16, 16)).with_(ma=0.3), precision="fp64")
    assert slow.forces()["flags"] == 0
