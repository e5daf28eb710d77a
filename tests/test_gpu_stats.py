"""GPU running statistics and load history against the oracle's definitions (two-pass statistics of
the same trajectory)."""
import numpy as np
import pytest
import torch

from gpu_util import print_case
from oracle import Oracle, flow_statistics
from synth import make_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("interval", [1, 2])
def test_statistics_and_history_vs_oracle(interval):
    from paper_2603_11102_amd import GksSolver
    cfg = make_case("alm", grid=(48, 24, 24))
    rng = np.random.default_rng(8)
    q = cfg.q0.copy()
    q[1:] += 0.03 * rng.uniform(-1, 1, size=q[1:].shape)
    cfg = cfg.with_(q0=q)
    nsteps = 4
    print_case("statistics", interval=interval, nsteps=nsteps)
    s = GksSolver(cfg, precision="fp64")
    s.enable_statistics(interval)
    s.enable_history(nsteps)
    s.step(nsteps)
    st = s.statistics(u_inf=1.0)
    hist = s.history()
    o = Oracle(cfg)
    samples, outs = [], []
    for n in range(1, nsteps + 1):
        outs.append(o.step())
        if n % interval == 0:
            samples.append(o.Q.clone())
    ref = flow_statistics(samples, u_inf=1.0)
    assert st["n"] == ref["n"]
    for k in ("mean", "rms", "stress", "tke"):
        got = st[k].cpu()
        scale = max(float(ref[k].abs().max()), 1e-30)
        err = float((got - ref[k]).abs().max()) / scale
        assert err < 1e-9, (k, err)
    assert hist.shape == (nsteps, 10)
    for n in range(nsteps):
        a = outs[n]["alm"]
        assert abs(float(hist[n, 0]) - outs[n]["t"]) < 1e-14
        assert abs(float(hist[n, 5]) - float(a["cp"])) < 1e-12 * abs(float(a["cp"]))
        assert abs(float(hist[n, 6]) - float(a["ct"])) < 1e-12 * abs(float(a["ct"]))
