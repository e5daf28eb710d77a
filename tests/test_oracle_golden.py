"""The stored oracle result of the GPU parity tests (tests/golden/make_golden.py) is reproduced
exactly by the oracle as it stands: a change to its arithmetic shows up here before it silently moves
the reference the GPU is held to."""
import os

import numpy as np

from oracle import Oracle
from synth import make_case

HERE = os.path.dirname(__file__)


def test_oracle_reproduces_the_stored_taylor_green_result():
    cfg = make_case("tgv")
    o = Oracle(cfg)
    dts = [o.step()["dt"] for _ in range(cfg.steps)]
    g = np.load(os.path.join(HERE, "golden", "tgv32_oracle_10steps.npz"))
    assert np.array_equal(o.Q.numpy(), g["q"])
    assert np.array_equal(np.array(dts), g["dt"])
    assert float(o.t) == float(g["t"])
