"""FP64 CPU oracle of one S2O4 step of the isothermal high-order gas-kinetic scheme with actuator-line
(ALM) and immersed-boundary (IBM) body forcing.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its Python binding) may
import, call or link anything in this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It is plain, slow, whole-array PyTorch CPU code in float64
and shares no code, table or constant with the HIP path.

Parity pins: every function here is checked in ``tests/test_oracle_*.py`` against closed forms,
invariants, brute force or special cases (free-stream preservation, periodic conservation, measured
convergence order, the Chapman-Enskog closed form of the flux, WENO polynomial exactness, S2O4
amplification factor, Gaussian-kernel sums, discrete-delta partition of unity, the closed-form IBM
iteration). Parity unpinned (oracle <-> GPU only, no outside reference): the choice of the
equilibrium average at the interface, the tangential sweep order, the WENO epsilon, the ALM force
sign and sampling time, the IBM iteration count.
"""
from .gks_oracle import *  # noqa: F401,F403
