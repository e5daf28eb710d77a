"""GksSolver: owns the device buffers (torch tensors) and drives the C ABI of libgks.so.

PyTorch supplies device memory and the HIP stream; every computation runs in the library's kernels.
There is no CPU fallback: without a GPU or without the built library the constructor raises.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional

import numpy as np
import torch

from . import _lib as L

NG = 3


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class GksSolver:
    """One simulation context.

    Fields are torch tensors of shape [4, nz+6, ny+6, nx+6] (rho - rho_ref, rho U, rho V, rho W) with
    3 ghost layers, dtype float32 or float64 on ``device``.
    """

    def __init__(self, cfg, precision: str = "fp32", device: str = "cuda:0", max_act: Optional[int] = None,
                 max_ibm: Optional[int] = None, q0: Optional[np.ndarray] = None, stream=None,
                 static_scratch: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("GksSolver needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = L.load()
        self.cfg = cfg
        self.device = torch.device(device)
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.precision = precision
        rotor = getattr(cfg, "rotor", None)
        ibm = getattr(cfg, "ibm", None)
        if max_act is None:
            max_act = rotor.n_blades * rotor.n_per_blade if rotor is not None else 0
        if max_ibm is None:
            max_ibm = ibm.n if ibm is not None else 0
        c = L.gks_config()
        c.nx, c.ny, c.nz = cfg.nx, cfg.ny, cfg.nz
        c.precision = L.GKS_FP32 if precision == "fp32" else L.GKS_FP64
        c.x0, c.y0, c.z0 = cfg.x0, cfg.y0, cfg.z0
        c.lx, c.ly, c.lz = cfg.lx, cfg.ly, cfg.lz
        c.ma, c.u_ref, c.rho_ref, c.mu = cfg.ma, cfg.u_ref, cfg.rho_ref, cfg.mu
        c.cfl, c.dt_fixed = cfg.cfl, cfg.dt_fixed
        for s in range(6):
            c.bc[s] = L.BC[cfg.bc[s]]
        for j in range(3):
            c.u_in[j] = cfg.u_in[j]
            c.body_force[j] = cfg.body_force[j]
        c.weno_eps = cfg.weno_eps
        c.ibm_iters = cfg.ibm_iters
        c.order = int(getattr(cfg, "order", 5))
        c.max_act = max_act
        c.max_ibm = max_ibm
        faces = getattr(cfg, "faces", None) or (None, None, None)
        self._faces = [None if f is None else np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in faces]
        for a in range(3):
            if self._faces[a] is not None:
                c.faces[a] = self._faces[a].ctypes.data_as(C.POINTER(C.c_double))
        self.c_cfg = c
        shape = (4, cfg.nz + 2 * NG, cfg.ny + 2 * NG, cfg.nx + 2 * NG)
        self.q = torch.zeros(shape, dtype=self.dtype, device=self.device)
        self.q_stage = torch.zeros_like(self.q)
        self.q_acc = torch.zeros_like(self.q)
        q0 = cfg.q0 if q0 is None else q0
        self.set_interior(q0)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        if static_scratch:
            # the workspace is the library's static device array (gks_init_static allocates nothing)
            self.workspace = None
            with torch.cuda.device(self.device):
                rc = self.lib.gks_init_static(C.byref(c), self._field(self.q), self._field(self.q_stage),
                                              self._field(self.q_acc), C.c_void_p(self.stream.cuda_stream),
                                              C.byref(ctx))
        else:
            nbytes = self.lib.gks_workspace_bytes(C.byref(c))
            if nbytes == 0:
                raise L.GksError(L.GKS_E_INVALID_ARG, "invalid configuration")
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = _ptr(self.workspace)
            self._ws_ptr = (base + 255) // 256 * 256
            self._ws_bytes = nbytes
            rc = self.lib.gks_init(C.byref(c), self._field(self.q), self._field(self.q_stage),
                                   self._field(self.q_acc), C.c_void_p(self._ws_ptr), C.c_size_t(nbytes),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        L.check(self.lib, None, rc)
        self.ctx = ctx
        self.n_act = 0
        self.scale = None
        self.checkpoints = None
        if rotor is not None:
            self.set_rotor(rotor)
        if ibm is not None:
            self.set_ibm(ibm)

    # ------------------------------------------------------------------ buffers
    def _field(self, t: torch.Tensor) -> L.gks_field:
        f = L.gks_field()
        f.rho, f.mx, f.my, f.mz = (_ptr(t[v]) for v in range(4))
        return f

    def set_interior(self, q0):
        """Load cell averages [4, nz, ny, nx] of (rho, rho U, rho V, rho W) into the field."""
        q = torch.as_tensor(np.asarray(q0), dtype=torch.float64).clone()
        q[0] -= self.cfg.rho_ref
        self.q[:, NG:-NG, NG:-NG, NG:-NG] = q.to(self.dtype).to(self.device)
        if getattr(self, "ctx", None):
            L.check(self.lib, self.ctx, self.lib.gks_field_changed(self.ctx))

    def interior(self) -> torch.Tensor:
        """Interior cell averages [4, nz, ny, nx]: (rho - rho_ref, rho U, rho V, rho W), float64 on the host."""
        torch.cuda.synchronize(self.device)
        return self.q[:, NG:-NG, NG:-NG, NG:-NG].to(torch.float64).cpu()

    # ------------------------------------------------------------------ body forces
    def set_rotor(self, rotor, scale: Optional[torch.Tensor] = None):
        n_act = rotor.n_blades * rotor.n_per_blade
        self._rotor_arrays = [np.ascontiguousarray(np.asarray(a, dtype=np.float64))
                              for a in (rotor.r, rotor.chord, rotor.twist, rotor.width)]
        if scale is None:
            scale = torch.as_tensor(rotor.scales(), dtype=torch.float64, device=self.device)
        self.scale = scale
        r = L.gks_rotor()
        r.n_blades, r.n_per_blade = rotor.n_blades, rotor.n_per_blade
        for j in range(3):
            r.hub[j] = rotor.hub[j]
        r.omega, r.theta0, r.radius, r.u_inf = rotor.omega, rotor.theta0, rotor.radius, rotor.u_inf
        dp = C.POINTER(C.c_double)
        r.r, r.chord, r.twist, r.width = (a.ctypes.data_as(dp) for a in self._rotor_arrays)
        r.eps, r.cl_slope, r.alpha_clip = rotor.eps, rotor.cl_slope, rotor.alpha_clip
        r.cd0, r.cd2 = rotor.cd0, rotor.cd2
        r.u_inf_correction = 1 if rotor.u_inf_correction else 0
        r.tip_correction = 1 if getattr(rotor, "tip_correction", False) else 0
        r.scale = C.c_void_p(_ptr(self.scale))
        r.line_points = int(getattr(rotor, "line_points", 1) or 1)
        r.line_half_length = float(getattr(rotor, "line_half_length", 0.0) or 0.0)
        L.check(self.lib, self.ctx, self.lib.gks_set_actuators(self.ctx, C.byref(r)))
        self.n_act = n_act

    def set_ibm(self, ibm):
        xyz = np.ascontiguousarray(np.asarray(ibm.xyz, dtype=np.float64))
        ds = np.ascontiguousarray(np.asarray(ibm.dS, dtype=np.float64))
        vel = getattr(ibm, "vel", None)
        vel = None if vel is None else np.ascontiguousarray(np.asarray(vel, dtype=np.float64).reshape(-1, 3))
        dp = C.POINTER(C.c_double)
        L.check(self.lib, self.ctx, self.lib.gks_set_ibm_points(self.ctx, xyz.shape[0], xyz.ctypes.data_as(dp),
                                                                ds.ctypes.data_as(dp),
                                                                None if vel is None else vel.ctypes.data_as(dp)))
        motion = getattr(ibm, "motion", None)
        if motion is not None:
            self.set_ibm_motion(motion)

    def set_ibm_motion(self, motion):
        """Rigid motion (centre, translation velocity, angular velocity, t0) of the body set last."""
        m = L.gks_motion()
        for d in range(3):
            m.center[d] = float(motion.center[d])
            m.velocity[d] = float(motion.velocity[d])
            m.omega[d] = float(motion.omega[d])
        m.t0 = float(motion.t0)
        L.check(self.lib, self.ctx, self.lib.gks_set_ibm_motion(self.ctx, C.byref(m)))

    # ------------------------------------------------------------------ stepping
    def step(self, n: int = 1):
        L.check(self.lib, self.ctx, self.lib.gks_step(self.ctx, int(n)))

    def forces(self, per_point: bool = False, check: bool = True) -> dict:
        out = L.gks_forces_out()
        arrs = {}
        if per_point and self.n_act:
            for k in ("alpha", "fx", "ftheta", "urel"):
                arrs[k] = np.zeros(self.n_act)
                setattr(out, k, arrs[k].ctypes.data_as(C.POINTER(C.c_double)))
        rc = self.lib.gks_forces(self.ctx, C.byref(out))
        if check:
            L.check(self.lib, self.ctx, rc)
        d = {k: getattr(out, k) for k in ("t", "dt", "step", "thrust", "torque", "power", "cp", "ct",
                                           "ibm_residual", "ibm_iters_used", "flags", "mass", "umax",
                                           "window_power", "window_thrust", "window_steps")}
        d["ibm_force"] = list(out.ibm_force)
        d["mom"] = list(out.mom)
        d["status"] = rc
        d.update(arrs)
        return d

    def set_timing(self, enable: bool = True):
        L.check(self.lib, self.ctx, self.lib.gks_set_timing(self.ctx, 1 if enable else 0))

    def read_timing(self) -> dict:
        """Accumulated milliseconds and launch-group counts per category since timing was enabled."""
        n = len(L.TIMERS)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        L.check(self.lib, self.ctx, self.lib.gks_read_timing(self.ctx, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(L.TIMERS)}

    # ------------------------------------------------------------------ statistics and histories
    def enable_statistics(self, interval: int = 1):
        nbytes = self.lib.gks_statistics_bytes(C.byref(self.c_cfg))
        self._stats = torch.empty(nbytes // 8, dtype=torch.float64, device=self.device)
        L.check(self.lib, self.ctx, self.lib.gks_set_statistics(self.ctx, C.c_void_p(self._stats.data_ptr()), int(interval)))

    def statistics(self, u_inf: float = 1.0) -> dict:
        """Mean [3, nz, ny, nx], rms [3, ...], stress (<U'V'>, <U'W'>, <V'W'>) [3, ...], tke [...] on the device."""
        shp = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        out = {k: torch.empty((3,) + shp, dtype=torch.float64, device=self.device) for k in ("mean", "rms", "stress")}
        out["tke"] = torch.empty(shp, dtype=torch.float64, device=self.device)
        n = C.c_int64()
        L.check(self.lib, self.ctx, self.lib.gks_read_statistics(
            self.ctx, float(u_inf), *(C.c_void_p(out[k].data_ptr()) for k in ("mean", "rms", "stress", "tke")),
            C.byref(n)))
        torch.cuda.synchronize(self.device)
        out["n"] = n.value
        return out

    def enable_history(self, capacity: int):
        self._hist = torch.zeros((capacity, 10), dtype=torch.float64, device=self.device)
        L.check(self.lib, self.ctx, self.lib.gks_set_history(self.ctx, C.c_void_p(self._hist.data_ptr()), int(capacity)))

    def history(self) -> torch.Tensor:
        """Records (t, dt, thrust, torque, power, C_P, C_T, IBM force x, y, z) of the steps so far."""
        n = C.c_int64()
        L.check(self.lib, self.ctx, self.lib.gks_history_count(self.ctx, C.byref(n)))
        torch.cuda.synchronize(self.device)
        return self._hist[: n.value].cpu()

    # ------------------------------------------------------------------ adjoint
    def set_checkpoints(self, capacity: int):
        """Register a device buffer of `capacity` checkpoint slots; the next steps store Q^n per step."""
        slot = self.lib.gks_checkpoint_slot_bytes(C.byref(self.c_cfg))
        self._ckpt = torch.empty(capacity * slot + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ckpt.data_ptr() + 255) // 256 * 256
        L.check(self.lib, self.ctx, self.lib.gks_set_checkpoints(self.ctx, C.c_void_p(ptr), int(capacity)))

    def adjoint(self, nsteps: int, w, want_field: bool = False, exact: bool = False):
        """Gradient of J = w0 mean P + w1 mean T over the checkpointed window with respect to the force
        scalings (device float64 [n_act]); optionally dJ/dQ^0 as [4, nz, ny, nx]. The WENO nonlinear
        weights are frozen unless ``exact``."""
        nbytes = self.lib.gks_adjoint_workspace_bytes(C.byref(self.c_cfg), self.n_act)
        if getattr(self, "_adj_ws", None) is None or self._adj_ws.numel() < nbytes + 256:
            self._adj_ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._adj_ws.data_ptr() + 255) // 256 * 256
        grad_s = torch.empty(self.n_act, dtype=torch.float64, device=self.device)
        gq = None
        if want_field:
            gq = torch.empty((4, self.cfg.nz, self.cfg.ny, self.cfg.nx), dtype=torch.float64, device=self.device)
        wv = (C.c_double * 2)(float(w[0]), float(w[1]))
        rc = self.lib.gks_adjoint(self.ctx, int(nsteps), wv, C.c_void_p(grad_s.data_ptr()),
                                  C.c_void_p(gq.data_ptr()) if gq is not None else None,
                                  C.c_void_p(ptr), C.c_size_t(nbytes), L.GKS_ADJ_EXACT_WENO if exact else 0)
        L.check(self.lib, self.ctx, rc)
        return grad_s, gq

    def reset_window(self):
        L.check(self.lib, self.ctx, self.lib.gks_reset_window(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.gks_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
