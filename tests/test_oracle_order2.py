"""Pins of the oracle's second-order variant (reading R15 for the comparison scheme of Section 4.3.3):
van Leer limiter properties, exactness of the limited reconstruction for linear data, free stream with
every boundary kind, periodic conservation, and a measured second-order convergence rate on a smooth
acoustic wave."""
import math

import numpy as np
import pytest
import torch

from oracle import Oracle, conservation_sums, muscl_faces, van_leer
from synth import make_case

F64 = torch.float64


def test_van_leer_limiter_properties():
    rng = np.random.default_rng(0)
    a = torch.tensor(rng.uniform(-2, 2, 2000), dtype=F64)
    b = torch.tensor(rng.uniform(-2, 2, 2000), dtype=F64)
    s = van_leer(a, b)
    assert torch.equal(s, van_leer(b, a))                       # symmetric
    same = a * b > 0
    assert torch.all(s[~same] == 0)                             # extrema and sign changes: flat
    lo = torch.minimum(a.abs(), b.abs())
    hi = torch.maximum(a.abs(), b.abs())
    assert torch.all(s[same].abs() >= lo[same] - 1e-15)         # between the smaller difference ...
    assert torch.all(s[same].abs() <= 2 * lo[same] + 1e-15)     # ... and twice it (TVD region)
    assert torch.all(s[same].abs() <= hi[same] + 1e-15)
    assert torch.all(torch.sign(s[same]) == torch.sign(a[same]))
    x = torch.tensor([0.3, -1.7, 2.5], dtype=F64)
    assert torch.allclose(van_leer(x, x), x, rtol=1e-15, atol=0)  # equal slopes pass through


def test_muscl_exact_for_linear_data():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a0, b0 = rng.uniform(-1, 1, 2)
        q = [torch.tensor(a0 + b0 * i, dtype=F64) for i in (-2, -1, 0, 1)]
        qL, qR = muscl_faces(*q)
        face = a0 + b0 * (-0.5)
        assert abs(float(qL) - face) < 1e-15 and abs(float(qR) - face) < 1e-15


def test_muscl_first_order_at_an_extremum():
    q = [torch.tensor(v, dtype=F64) for v in (0.0, 1.0, 0.0, -1.0)]  # cell -1 is a local maximum
    qL, qR = muscl_faces(*q)
    assert float(qL) == 1.0          # flat profile in the extremal cell
    assert float(qR) == 0.5          # cell 0 is monotone: slope vL(-1, -1) = -1


def _uniform(cfg, rho, u):
    q = np.zeros((4, cfg.nz, cfg.ny, cfg.nx))
    q[0] = rho
    for j in range(3):
        q[1 + j] = rho * u[j]
    return q


@pytest.mark.parametrize("bc,u", [
    (("periodic",) * 6, (0.4, -0.3, 0.2)),
    (("periodic", "periodic", "noslip", "noslip", "periodic", "periodic"), (0.0, 0.0, 0.0)),
    (("inflow", "outflow", "periodic", "periodic", "slip", "slip"), (1.0, 0.0, 0.0)),
])
def test_order2_free_stream_preserved(bc, u):
    cfg = make_case("tgv", grid=(10, 9, 8)).with_(bc=bc, u_in=(1.0, 0.0, 0.0), mu=0.01, order=2)
    q = _uniform(cfg, 1.05, u)
    o = Oracle(cfg, q0=q)
    for _ in range(2):
        o.step()
    assert float((o.Q - torch.tensor(q)).abs().max()) < 1e-13


def test_order2_periodic_conservation():
    cfg = make_case("tgv", grid=(12, 12, 12)).with_(order=2)
    o = Oracle(cfg)
    s0 = conservation_sums(o.Q)
    for _ in range(3):
        o.step()
    s1 = conservation_sums(o.Q)
    for a, b in zip(s0, s1):
        assert abs(a - b) < 1e-13 * cfg.n_cells


def _wave(n, steps):
    grid = [n, 4, 4]
    cfg = make_case("tgv", grid=tuple(grid))
    h = 2 * math.pi / n
    cfg = cfg.with_(lx=2 * math.pi, ly=4 * h, lz=4 * h, mu=0.0, cfl=0.0, dt_fixed=0.2 * h / 10.0, order=2)
    x = (np.arange(n) + 0.5) * h
    s = np.sin(x) * np.sinc(h / 2 / math.pi)  # exact cell averages of sin(x)
    q = np.zeros((4, 4, 4, n))
    amp, c, um = 1e-2, 10.0, 0.3
    q[0] = 1.0 + amp * s[None, None, :]
    q[1] = um * q[0] + c * amp * s[None, None, :]
    o = Oracle(cfg, q0=q)
    for _ in range(steps):
        o.step()
    return o.Q


def test_order2_convergence_rate():
    # self-convergence in the mean absolute difference of restricted solutions at a fixed time; the
    # limiter flattens the profile at the extrema, so the rate is measured in L1
    sol = {n: _wave(n, n // 8) for n in (32, 64, 128)}

    def restrict(Q):
        return Q.reshape(4, 4, 4, -1, 2).mean(-1)

    e1 = float((sol[32] - restrict(sol[64])).abs().mean())
    e2 = float((sol[64] - restrict(sol[128])).abs().mean())
    order = math.log2(e1 / e2)
    assert 1.7 < order < 2.6, (e1, e2, order)
