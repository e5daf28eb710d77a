"""Write the stored oracle results used by the GPU parity tests. Calls only the CPU oracle and the
seeded case generators. Run from the repository root: python tests/golden/make_golden.py"""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
from synth import make_case  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def tgv32():
    """32^3 Taylor-Green case, FP64 oracle, 10 CFL steps."""
    cfg = make_case("tgv")
    o = Oracle(cfg)
    dts = [o.step()["dt"] for _ in range(cfg.steps)]
    np.savez_compressed(os.path.join(HERE, "tgv32_oracle_10steps.npz"), q=o.Q.numpy(), dt=np.array(dts),
                        t=np.array(o.t))


if __name__ == "__main__":
    torch.set_num_threads(min(8, os.cpu_count() or 1))
    tgv32()
