"""CPU-side checks of the C ABI: the library loads, exports every symbol include/gks.h declares, sizes
its workspace, and rejects invalid arguments before any device work (no compute calls here)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2603_11102_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gks_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)
    assert set(L.EXPORTS) == set(names)


def _cfg(**kw):
    c = L.gks_config()
    c.nx = c.ny = c.nz = 16
    c.precision = L.GKS_FP32
    c.lx = c.ly = c.lz = 1.0
    c.ma, c.u_ref, c.rho_ref, c.mu = 0.1, 1.0, 1.0, 1e-3
    c.cfl = 0.5
    for s in range(6):
        c.bc[s] = 0
    c.ibm_iters = 3
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_workspace_bytes_grows_with_capacity():
    lib = L.load()
    a = lib.gks_workspace_bytes(C.byref(_cfg()))
    b = lib.gks_workspace_bytes(C.byref(_cfg(max_act=192)))
    c = lib.gks_workspace_bytes(C.byref(_cfg(max_act=192, max_ibm=1000)))
    d = lib.gks_workspace_bytes(C.byref(_cfg(precision=L.GKS_FP64)))
    assert 0 < a < b < c
    assert d > a
    # two residual arrays of 4 variables over 16^3 cells dominate the fixed part
    assert a >= 2 * 4 * 16 ** 3 * 4


@pytest.mark.parametrize("bad", [dict(nx=2), dict(precision=7), dict(lx=0.0), dict(ma=0.0), dict(cfl=0.0),
                                 dict(max_act=2000), dict(mu=-1.0)])
def test_invalid_config_rejected(bad):
    lib = L.load()
    assert lib.gks_workspace_bytes(C.byref(_cfg(**bad))) == 0
    ctx = C.c_void_p()
    f = L.gks_field()
    rc = lib.gks_init(C.byref(_cfg(**bad)), f, f, f, None, 0, None, C.byref(ctx))
    assert rc == L.GKS_E_INVALID_ARG
    assert ctx.value is None
    assert len(lib.gks_last_error(None)) > 0


def test_unpaired_periodic_rejected():
    lib = L.load()
    c = _cfg()
    c.bc[0] = 1
    assert lib.gks_workspace_bytes(C.byref(c)) == 0


def test_init_null_pointers_rejected():
    lib = L.load()
    c = _cfg()
    f = L.gks_field()
    ctx = C.c_void_p()
    rc = lib.gks_init(C.byref(c), f, f, f, C.c_void_p(256), 1 << 30, None, C.byref(ctx))
    assert rc == L.GKS_E_INVALID_ARG
    assert b"null" in lib.gks_last_error(None)


def test_checkpoint_slot_bytes():
    lib = L.load()
    c = _cfg(precision=L.GKS_FP64)
    n = lib.gks_checkpoint_slot_bytes(C.byref(c))
    assert n >= 4 * 22 ** 3 * 8


def test_solver_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2603_11102_amd import GksSolver
    from synth import make_case
    with pytest.raises(RuntimeError):
        GksSolver(make_case("tgv", grid=(8, 8, 8)))


def test_field_changed_null_rejected():
    lib = L.load()
    assert lib.gks_field_changed(None) == L.GKS_E_INVALID_ARG


def test_oversized_axis_rejected():
    lib = L.load()
    assert lib.gks_workspace_bytes(C.byref(_cfg(nx=70000, ny=3, nz=3))) == 0


def test_fp32_workspace_holds_the_low_order_state():
    # FP32 carries Q^n, Q* and S with a low-order part of four variables per cell each
    lib = L.load()
    a = lib.gks_workspace_bytes(C.byref(_cfg()))
    assert a >= (2 + 3) * 4 * 16 ** 3 * 4


def test_ibm_motion_null_rejected():
    lib = L.load()
    m = L.gks_motion()
    assert lib.gks_set_ibm_motion(None, C.byref(m)) == L.GKS_E_INVALID_ARG


def test_ibm_workspace_holds_the_rebinning_pairs():
    # a context that may hold immersed points reserves, per point, its 64 (cell, point) pairs twice
    # over for the sort that rebuilds the supports of a moving body
    lib = L.load()
    a = lib.gks_workspace_bytes(C.byref(_cfg(max_ibm=1000)))
    b = lib.gks_workspace_bytes(C.byref(_cfg(max_ibm=0)))
    assert a - b >= 1000 * 64 * 4 * 4


def test_stretched_faces_validated():
    import numpy as np
    lib = L.load()
    ok = np.tanh(2.0 * (np.arange(17) / 8.0 - 1.0)) / np.tanh(2.0) * 0.5 + 0.5  # 17 faces on [0, 1]
    ok[0], ok[-1] = 0.0, 1.0
    P = C.POINTER(C.c_double)
    c = _cfg(bc=(C.c_int32 * 6)(0, 0, 1, 1, 0, 0))
    c.faces[1] = ok.ctypes.data_as(P)
    assert lib.gks_workspace_bytes(C.byref(c)) > 0
    bad = ok[::-1].copy()                                  # decreasing
    c.faces[1] = bad.ctypes.data_as(P)
    assert lib.gks_workspace_bytes(C.byref(c)) == 0
    short = ok * 0.9                                       # does not reach origin + length
    c.faces[1] = short.ctypes.data_as(P)
    assert lib.gks_workspace_bytes(C.byref(c)) == 0
    p = _cfg()                                             # periodic axis with its own faces
    p.faces[0] = ok.ctypes.data_as(P)
    assert lib.gks_workspace_bytes(C.byref(p)) == 0


def test_static_init_refuses_oversize_before_device_work():
    # gks_init_static checks the configuration's workspace against its static scratch before any HIP call
    lib = L.load()
    f = L.gks_field()
    ctx = C.c_void_p()
    big = _cfg(nx=192, ny=96, nz=96)
    assert lib.gks_workspace_bytes(C.byref(big)) > L.GKS_STATIC_SCRATCH_BYTES
    rc = lib.gks_init_static(C.byref(big), f, f, f, None, C.byref(ctx))
    assert rc == L.GKS_E_INVALID_ARG and ctx.value is None
    assert b"static scratch" in lib.gks_last_error(None)
    assert lib.gks_init_static(C.byref(_cfg(nx=2)), f, f, f, None, C.byref(ctx)) == L.GKS_E_INVALID_ARG
    assert lib.gks_init_static(C.byref(_cfg()), f, f, f, None, None) == L.GKS_E_INVALID_ARG
