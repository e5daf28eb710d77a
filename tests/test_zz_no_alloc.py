"""gks_init_static (the workspace in the library's static device scratch, for callers that cannot allocate)
against gks_init with a caller workspace: the same steps give the same fields and loads, bitwise, on two
contexts in a row, the second on a smaller grid; oversize configurations and a second live static
context on the same GPU are refused."""
import numpy as np
import pytest
import torch

from gpu_util import print_case
from synth import make_case

pytestmark = pytest.mark.gpu


def _pair(cfg, precision, steps):
    from paper_2603_11102_amd import GksSolver
    ref = GksSolver(cfg, precision=precision)
    st = GksSolver(cfg, precision=precision, static_scratch=True)
    try:
        assert st.workspace is None
        ref.step(steps)
        st.step(steps)
        fr, fs = ref.forces(per_point=ref.n_act > 0), st.forces(per_point=st.n_act > 0)
        assert torch.equal(ref.interior(), st.interior())
        for k in ("t", "dt", "step", "mass", "umax", "thrust", "power"):
            assert fr[k] == fs[k], k
        assert fr["mom"] == fs["mom"]
        if ref.n_act:
            assert np.array_equal(fr["fx"], fs["fx"]) and np.array_equal(fr["alpha"], fs["alpha"])
    finally:
        st.close()
        ref.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_static_workspace_matches_caller_workspace(precision):
    # call 1: a 48 x 24 x 24 rotor box; call 2: a smaller channel with walls and a body force
    a = make_case("alm", grid=(48, 24, 24))
    print_case("no-alloc", precision=precision, grid=(48, 24, 24))
    _pair(a, precision, 3)
    b = make_case("channel", grid=(24, 20, 18))
    print_case("no-alloc", precision=precision, grid=(24, 20, 18))
    _pair(b, precision, 4)


def test_static_workspace_refusals():
    from paper_2603_11102_amd import GksSolver
    from paper_2603_11102_amd import _lib as L
    print_case("no-alloc-refusals")
    big = make_case("channel", grid=(192, 96, 96))
    with pytest.raises(L.GksError) as e:
        GksSolver(big, precision="fp32", static_scratch=True)
    assert e.value.code == L.GKS_E_INVALID_ARG and "static scratch" in str(e.value)
    cfg = make_case("tgv", grid=(16, 16, 16))
    first = GksSolver(cfg, precision="fp64", static_scratch=True)
    try:
        with pytest.raises(L.GksError) as e:
            GksSolver(cfg, precision="fp64", static_scratch=True)
        assert e.value.code == L.GKS_E_STATE
    finally:
        first.close()
    again = GksSolver(cfg, precision="fp64", static_scratch=True)  # released by the destroy above
    again.step(1)
    assert again.forces()["step"] == 1
    again.close()
