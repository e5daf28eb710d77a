"""The box recomputation behind the full-size sampled parity tests reproduces full-domain oracle steps:
for cells in the interior, at tile and chunk seams and next to every kind of non-periodic boundary
(no-slip walls, a stretched wall-normal axis, inflow, outflow and slip sides), one oracle step of the
15^3 box around the cell equals the same cell of one oracle step of the whole domain."""
import numpy as np
import pytest
import torch

from oracle import Oracle
from sampling import box_ranges, box_reference, near_boundary, take_box
from synth import make_case


def _perturb(cfg, seed):
    rng = np.random.default_rng(seed)
    q = cfg.q0.copy()
    q[1:] += 0.05 * rng.uniform(-1, 1, size=q[1:].shape)
    q[0] += 0.005 * rng.uniform(-1, 1, size=q[0].shape)
    return cfg.with_(q0=q)


@pytest.mark.parametrize("case,grid", [
    ("channel", (20, 18, 17)),                     # no-slip walls in y
    ("channel_tanh", (17, 20, 16)),                # tanh-stretched wall-normal axis
    ("alm", (36, 18, 18)),                         # inflow / outflow in x, periodic y, slip z
])
def test_box_step_equals_full_domain_step(case, grid):
    cfg = _perturb(make_case(case, grid=grid).with_(rotor=None, ibm=None), 5)
    o = Oracle(cfg)
    out = o.step()
    full = o.Q.clone()
    full[0] -= cfg.rho_ref
    pre = torch.tensor(cfg.q0, dtype=torch.float64)
    pre[0] -= cfg.rho_ref
    nb = near_boundary(cfg)
    rng = np.random.default_rng(3)
    cells = list(np.argwhere(nb)[rng.choice(int(nb.sum()), size=4, replace=False)])
    cells += [np.array([0, 0, 0]), np.array([cfg.nz - 1, cfg.ny - 1, cfg.nx - 1]), np.array([cfg.nz // 2, 1, 6])]
    for cell in cells:
        rg = box_ranges(cfg, cell)
        ref = box_reference(cfg, take_box(pre, rg), rg, cell, out["dt"])
        k, j, i = (int(c) for c in cell)
        assert torch.allclose(ref, full[:, k, j, i], rtol=0, atol=1e-13), (case, cell)
