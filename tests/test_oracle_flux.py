"""Pins of the oracle's gas-kinetic flux: Maxwellian moments (Appendix) against Gauss-Hermite
quadrature, the kinetic average against numerical half-space integrals, the microscopic coefficients
against the analytic derivative of ln g0 and the paper's printed inversion, and the flux against the
Chapman-Enskog closed form of f = g0 (1 - tau (a.u + A) + A t) (Section 2, Eq. (flux))."""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import gks_point_flux, kinetic_average, maxwellian_moment, micro_coefficients

F64 = torch.float64
HERE = os.path.dirname(__file__)
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))


def test_golden_constants_present():
    assert GOLD["gaussian_one_percent_radius_over_eps"]["value"] == 2.15
    assert "Appendix" in GOLD["moment_recurrence"]["source"]


@pytest.mark.parametrize("lam", [0.005, 0.3, 1.7])
def test_moments_vs_gauss_hermite(lam):
    # <u^a v^b w^c> of rho^-1 g0 by direct quadrature: u = U + x / sqrt(lam), weight exp(-x^2)/sqrt(pi)
    x, w = np.polynomial.hermite.hermgauss(20)
    U = [0.3, -1.2, 0.7]
    U3 = [torch.tensor(u, dtype=F64) for u in U]
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                q = 1.0
                for comp, p in zip(range(3), (a, b, c)):
                    vals = U[comp] + x / math.sqrt(lam)
                    q *= float(np.sum(w * vals ** p) / math.sqrt(math.pi))
                m = float(maxwellian_moment(U3, lam, (a, b, c)))
                assert abs(m - q) < 1e-11 * max(1.0, abs(q))


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_kinetic_average_vs_half_space_quadrature(normal):
    lam = 0.02
    rng = np.random.default_rng(normal)
    qL = np.array([1.1, *rng.standard_normal(3)])
    qR = np.array([0.9, *rng.standard_normal(3)])
    Q0 = kinetic_average(torch.tensor(qL), torch.tensor(qR), normal, lam).numpy()

    def half(q, sign):
        rho = q[0]
        U = q[1:] / rho
        g1 = lambda u, m: math.sqrt(lam / math.pi) * math.exp(-lam * (u - m) ** 2)  # noqa: E731
        lo, hi = (0.0, np.inf) if sign > 0 else (-np.inf, 0.0)
        un = U[normal]
        p0 = integrate.quad(lambda u: g1(u, un), lo, hi, epsabs=1e-14, epsrel=1e-13)[0]
        p1 = integrate.quad(lambda u: u * g1(u, un), lo, hi, epsabs=1e-14, epsrel=1e-13)[0]
        out = np.zeros(4)
        out[0] = rho * p0
        for j in range(3):
            out[1 + j] = rho * (p1 if j == normal else U[j] * p0)
        return out

    ref = half(qL, +1) + half(qR, -1)
    assert np.allclose(Q0, ref, rtol=1e-10, atol=1e-12)


def _random_state(rng, shape=(50,)):
    rho = torch.tensor(1.0 + 0.1 * rng.standard_normal(shape), dtype=F64)
    U = [torch.tensor(rng.standard_normal(shape), dtype=F64) for _ in range(3)]
    Q0 = torch.stack([rho, rho * U[0], rho * U[1], rho * U[2]], 0)
    grads = [torch.tensor(rng.standard_normal((4,) + shape), dtype=F64) for _ in range(3)]
    return Q0, grads


def test_coefficients_equal_dlng0():
    # a_k must equal d(ln g0)/dx_k = rho_k/rho - 2 lam U.dU_k + 2 lam u.dU_k (expanded in psi)
    rng = np.random.default_rng(1)
    lam = 0.37
    Q0, grads = _random_state(rng)
    a, _, _ = micro_coefficients(Q0, grads, lam)
    rho = Q0[0]
    U = Q0[1:] / rho
    for k in range(3):
        drho = grads[k][0]
        dU = (grads[k][1:] - U * drho) / rho
        a1 = drho / rho - 2 * lam * (U * dU).sum(0)
        assert torch.allclose(a[k][0], a1, rtol=1e-11, atol=1e-11)
        for j in range(3):
            assert torch.allclose(a[k][1 + j], 2 * lam * dU[j], rtol=1e-11, atol=1e-11)


def test_coefficients_equal_printed_inversion():
    # Appendix: a^{2,3,4} = 2 lam (d_{2,3,4} - (U,V,W) d1), a^1 = d1 - U a^2 - V a^3 - W a^4, d = dQ0/rho0
    rng = np.random.default_rng(2)
    lam = 0.05
    Q0, grads = _random_state(rng)
    a, _, _ = micro_coefficients(Q0, grads, lam)
    rho = Q0[0]
    U = Q0[1:] / rho
    for k in range(3):
        d = grads[k] / rho
        a2 = [2 * lam * (d[1 + j] - U[j] * d[0]) for j in range(3)]
        a1 = d[0] - U[0] * a2[0] - U[1] * a2[1] - U[2] * a2[2]
        assert torch.allclose(a[k][0], a1, rtol=1e-11, atol=1e-11)
        for j in range(3):
            assert torch.allclose(a[k][1 + j], a2[j], rtol=1e-11, atol=1e-11)


def _euler_flux(Q, n, c2):
    rho = Q[0]
    U = Q[1:] / rho
    out = [Q[1 + n]]
    for j in range(3):
        out.append(Q[1 + n] * U[j] + (c2 * rho if j == n else 0.0))
    return torch.stack(out, 0)


def _jac_times(Q, n, dQ, c2):
    rho = Q[0]
    U = Q[1:] / rho
    out = [dQ[1 + n]]
    for j in range(3):
        v = U[j] * dQ[1 + n] + U[n] * dQ[1 + j] - U[n] * U[j] * dQ[0]
        if j == n:
            v = v + c2 * dQ[0]
        out.append(v)
    return torch.stack(out, 0)


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_flux_equals_chapman_enskog_closed_form(normal):
    # F0 = E_n(Q0) - mu (dU_i/dx_n + dU_n/dx_i) (no viscous mass flux, no bulk term);
    # F1 = J_n(Q0) Qdot with Qdot = -sum_k J_k(Q0) dQ0/dx_k (the Euler time derivative)
    rng = np.random.default_rng(10 + normal)
    lam, mu = 0.005, 3e-3
    c2 = 1.0 / (2 * lam)
    Q0, grads = _random_state(rng)
    F0, F1 = gks_point_flux(Q0, grads, normal, lam, mu)
    rho = Q0[0]
    U = Q0[1:] / rho
    dU = [(grads[k][1:] - U * grads[k][0]) / rho for k in range(3)]  # dU[k][j] = dU_j/dx_k
    ref0 = _euler_flux(Q0, normal, c2)
    for j in range(3):
        ref0[1 + j] = ref0[1 + j] - mu * (dU[normal][j] + dU[j][normal])
    assert torch.allclose(F0, ref0, rtol=1e-10, atol=1e-9)
    qdot = -sum(_jac_times(Q0, k, grads[k], c2) for k in range(3))
    ref1 = _jac_times(Q0, normal, qdot, c2)
    assert torch.allclose(F1, ref1, rtol=1e-10, atol=1e-8)


def test_flux_uniform_state_is_euler():
    lam = 0.005
    Q0 = torch.tensor([[1.2], [0.6], [-0.1], [0.3]], dtype=F64)
    z = [torch.zeros(4, 1, dtype=F64)] * 3
    F0, F1 = gks_point_flux(Q0, z, 0, lam, 1e-2)
    assert torch.allclose(F0[:, 0], _euler_flux(Q0, 0, 1 / (2 * lam))[:, 0], rtol=1e-13)
    assert torch.allclose(F1, torch.zeros_like(F1), atol=1e-12)
