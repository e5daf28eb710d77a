"""Seeded synthetic inputs (initial fields, rotor geometry, immersed-body surface points).

This package only produces input data. It holds none of the scheme's arithmetic, so both the
FP64 CPU oracle (test infrastructure) and the HIP library's tests and benchmark may use it.
"""
from .cases import (  # noqa: F401
    CaseConfig,
    RotorSpec,
    IbmSpec,
    make_case,
    CASE_NAMES,
)
