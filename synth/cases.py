"""Seeded synthetic workloads for the isothermal GKS step with actuator-line and immersed-boundary forcing.

Five workloads stand in for the paper's test cases (their data are not public here):

* ``tgv``      32^3 triply periodic box of side 2*pi, Taylor-Green velocity plus a 1 % RMS
               random-phase solenoidal perturbation over modes 1 <= |k| <= 4, Ma = 0.1, Re = 400.
* ``channel``  192 x 96 x 96 cells on 4*pi x 2 x 4*pi/3, no-slip walls at y = -1, 1, periodic x and z,
               laminar profile 1.5 (1 - y^2) plus 5 % uniform cell noise, constant pressure-gradient body
               force for Re_tau = 180 (shape class of the paper's turbulent channel, section 4.1).
* ``alm``      384 x 192 x 192 uniform cells, rotor diameter 64 cells, uniform inflow, three blades with
               64 actuator points each (shape class of the NREL 5 MW case, section 4.3).
* ``alm_ibm``  512 x 256 x 256 cells, the ``alm`` rotor plus a cylindrical tower and a capsule nacelle
               sampled by ~25k Lagrangian surface points (shape class of the NTNU case, section 4.4).
* ``adjoint``  128^3 periodic box, uniform stream with 5 % RMS random-phase turbulence, a 3 x 32 point
               rotor of diameter 40 cells, fixed time step, 20 steps.

Every initial field is an exact cell average (Fourier modes are averaged with their sinc factors, the
parabolic profile with its y^2 cell average). Everything here is input data only; none of the scheme's
arithmetic lives in this module.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence

import numpy as np

CASE_NAMES = ("tgv", "channel", "alm", "alm_ibm", "adjoint", "channel_tanh")


@dataclass
class RotorSpec:
    n_blades: int
    n_per_blade: int
    hub: tuple
    omega: float
    theta0: float
    radius: float
    r_hub: float
    u_inf: float
    r: np.ndarray
    chord: np.ndarray
    twist: np.ndarray
    width: np.ndarray
    eps: float
    cl_slope: float = 2.0 * math.pi
    alpha_clip: float = math.radians(12.0)
    cd0: float = 0.01
    cd2: float = 0.02
    u_inf_correction: bool = True
    tip_correction: bool = False        # Shen tip correction of the NTNU case (Section 4.4)
    line_points: int = 1                # line sampling of the NTNU case: samples along e_theta (1: point)
    line_half_length: float = 0.0       # half-length of the sampling segment
    scale: Optional[np.ndarray] = None  # per actuator point, n_blades * n_per_blade

    @property
    def n_act(self) -> int:
        return self.n_blades * self.n_per_blade

    def scales(self) -> np.ndarray:
        if self.scale is None:
            return np.ones(self.n_act)
        return np.asarray(self.scale, dtype=np.float64)


@dataclass
class IbmMotion:
    """Rigid motion of an immersed body: centre c0 at time t0, constant translation velocity and
    constant angular velocity (rad per unit time, about the moving centre)."""
    center: Sequence[float]
    velocity: Sequence[float] = (0.0, 0.0, 0.0)
    omega: Sequence[float] = (0.0, 0.0, 0.0)
    t0: float = 0.0


@dataclass
class IbmSpec:
    xyz: np.ndarray  # [n, 3] (positions at time motion.t0 when the body moves)
    dS: np.ndarray   # [n]
    vel: Optional[np.ndarray] = None  # [n, 3] prescribed point velocities (None: stationary)
    motion: Optional[IbmMotion] = None  # rigid motion (point velocities then follow from it)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


@dataclass
class CaseConfig:
    name: str
    nx: int
    ny: int
    nz: int
    x0: float
    y0: float
    z0: float
    lx: float
    ly: float
    lz: float
    ma: float
    u_ref: float
    rho_ref: float
    mu: float
    cfl: float
    dt_fixed: float
    bc: tuple  # (x-, x+, y-, y+, z-, z+) from {'periodic','noslip','slip','inflow','outflow'}
    u_in: tuple = (1.0, 0.0, 0.0)
    body_force: tuple = (0.0, 0.0, 0.0)
    weno_eps: float = 1e-6
    ibm_iters: int = 3
    order: int = 5  # 5: WENO-JS to 2x2 Gauss points (the high-order GKS); 2: the second-order variant
    steps: int = 10
    rotor: Optional[RotorSpec] = None
    ibm: Optional[IbmSpec] = None
    q0: Optional[np.ndarray] = field(default=None, repr=False)  # [4, nz, ny, nx]: rho, rho U, rho V, rho W
    seed: int = 0
    # cell faces per axis (n + 1 increasing coordinates from the origin to origin + length) of a
    # stretched mesh, None for a uniform axis
    faces: Optional[tuple] = field(default=None, repr=False)

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    @property
    def dz(self) -> float:
        return self.lz / self.nz

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    def with_(self, **kw) -> "CaseConfig":
        return replace(self, **kw)


# ----------------------------------------------------------------------------------------------
# exact cell averages
# ----------------------------------------------------------------------------------------------

def _centres(n: int, x0: float, length: float) -> np.ndarray:
    h = length / n
    return x0 + (np.arange(n) + 0.5) * h


def _sinc(x: np.ndarray) -> np.ndarray:
    return np.sinc(np.asarray(x) / math.pi)  # sin(x)/x


def random_solenoidal_field(shape, lengths, origin, kmax, rms, rng, kmin=1.0):
    """Cell averages of a random-phase solenoidal velocity over integer modes kmin <= |n| <= kmax.

    shape = (nz, ny, nx), lengths = (lz, ly, lx), origin = (z0, y0, x0). The field is
    Re sum_n a(n) exp(i k.x) with k = 2 pi n / L and a(n) a complex Gaussian vector projected
    normal to k (equal expected amplitude per mode, uniformly random phase). Each mode is averaged
    exactly over a cell with its sinc factors; the result is scaled so that
    sqrt(mean(|u|^2) / 3) = rms. Returns [3, nz, ny, nx] ordered (u_x, u_y, u_z).
    """
    nz, ny, nx = shape
    lz, ly, lx = lengths
    z0, y0, x0 = origin
    kk = int(math.floor(kmax))
    spec = np.zeros((3, nz, ny, nx), dtype=np.complex128)
    hx, hy, hz = lx / nx, ly / ny, lz / nz
    for a in range(-kk, kk + 1):
        for b in range(-kk, kk + 1):
            for c in range(-kk, kk + 1):
                r = math.sqrt(a * a + b * b + c * c)
                if r < kmin or r > kmax:
                    continue
                if 2 * abs(a) >= nx or 2 * abs(b) >= ny or 2 * abs(c) >= nz:
                    raise ValueError("mode not resolved by the grid")
                k = np.array([2 * math.pi * a / lx, 2 * math.pi * b / ly, 2 * math.pi * c / lz])
                amp = rng.standard_normal(3) + 1j * rng.standard_normal(3)
                kh = k / np.linalg.norm(k)
                amp = amp - np.dot(amp, kh) * kh
                # shift by the cell-centre origin and apply the cell-average sinc factors
                phase = np.exp(1j * (k[0] * (x0 + 0.5 * hx) + k[1] * (y0 + 0.5 * hy) + k[2] * (z0 + 0.5 * hz)))
                avg = _sinc(k[0] * hx / 2) * _sinc(k[1] * hy / 2) * _sinc(k[2] * hz / 2)
                spec[:, c % nz, b % ny, a % nx] += amp * phase * avg
    ntot = nx * ny * nz
    u = np.real(np.fft.ifftn(spec, axes=(1, 2, 3))) * ntot
    cur = math.sqrt(float(np.mean(np.sum(u * u, axis=0))) / 3.0)
    if cur > 0:
        u *= rms / cur
    return u


# ----------------------------------------------------------------------------------------------
# rotor and immersed-body geometry (input data)
# ----------------------------------------------------------------------------------------------

def synthetic_rotor(hub, radius, tsr, u_inf, n_blades, n_per_blade, eps, r_hub_frac=0.1,
                    design_alpha_deg=6.0, theta0=0.0, u_inf_correction=True) -> RotorSpec:
    """Rotor with textbook optimum-BEM radial profiles (no tabulated airfoil data).

    Elements of equal width between the hub radius and the tip; one actuator point per element centre.
    Flow angle phi_opt = (2/3) atan(R / (TSR r)); twist = phi_opt - design AoA; chord
    c = 8 pi r (1 - cos phi_opt) / (B C_L,design) with C_L,design = 2 pi alpha_design.
    """
    r_hub = r_hub_frac * radius
    width = (radius - r_hub) / n_per_blade
    r = r_hub + (np.arange(n_per_blade) + 0.5) * width
    phi = (2.0 / 3.0) * np.arctan(radius / (tsr * r))
    ad = math.radians(design_alpha_deg)
    cl_d = 2 * math.pi * ad
    chord = 8 * math.pi * r * (1 - np.cos(phi)) / (n_blades * cl_d)
    twist = phi - ad
    omega = tsr * u_inf / radius
    return RotorSpec(n_blades=n_blades, n_per_blade=n_per_blade, hub=tuple(float(v) for v in hub),
                     omega=omega, theta0=theta0, radius=radius, r_hub=r_hub, u_inf=u_inf,
                     r=r, chord=chord, twist=twist, width=np.full(n_per_blade, width), eps=eps,
                     u_inf_correction=u_inf_correction)


def _cylinder_z(cx, cy, z_bot, z_top, diam, h):
    """Lateral surface of a vertical cylinder, elements of equal area, points at element centres."""
    circ = math.pi * diam
    length = z_top - z_bot
    nt = max(8, int(round(circ / h)))
    nzp = max(1, int(round(length / h)))
    th = 2 * math.pi * (np.arange(nt) + 0.5) / nt
    zz = z_bot + (np.arange(nzp) + 0.5) * length / nzp
    T, Z = np.meshgrid(th, zz, indexing="ij")
    xyz = np.stack([cx + 0.5 * diam * np.cos(T), cy + 0.5 * diam * np.sin(T), Z], -1).reshape(-1, 3)
    dS = np.full(xyz.shape[0], (circ / nt) * (length / nzp))
    return xyz, dS


def _capsule_x(x_a, x_b, cy, cz, rad, h):
    """Capsule along x: cylinder between x_a and x_b plus hemispherical caps centred at x_a and x_b."""
    pts, ds = [], []
    circ = 2 * math.pi * rad
    nt = max(8, int(round(circ / h)))
    length = x_b - x_a
    nxp = max(1, int(round(length / h)))
    th = 2 * math.pi * (np.arange(nt) + 0.5) / nt
    xx = x_a + (np.arange(nxp) + 0.5) * length / nxp
    T, X = np.meshgrid(th, xx, indexing="ij")
    pts.append(np.stack([X, cy + rad * np.cos(T), cz + rad * np.sin(T)], -1).reshape(-1, 3))
    ds.append(np.full(T.size, (circ / nt) * (length / nxp)))
    nlat = max(2, int(round(0.5 * math.pi * rad / h)))
    for centre, sign in ((x_a, -1.0), (x_b, 1.0)):
        for i in range(nlat):
            t1, t2 = 0.5 * math.pi * i / nlat, 0.5 * math.pi * (i + 1) / nlat
            tm = 0.5 * (t1 + t2)
            nl = max(3, int(round(2 * math.pi * rad * math.sin(tm) / h)))
            ph = 2 * math.pi * (np.arange(nl) + 0.5) / nl
            x = centre + sign * rad * math.cos(tm)
            pts.append(np.stack([np.full(nl, x), cy + rad * math.sin(tm) * np.cos(ph),
                                 cz + rad * math.sin(tm) * np.sin(ph)], -1))
            ds.append(np.full(nl, rad * rad * (math.cos(t1) - math.cos(t2)) * 2 * math.pi / nl))
    return np.concatenate(pts, 0), np.concatenate(ds, 0)


def tower_and_nacelle(hub, D, dx, spacing, z_ground):
    """Stationary tower (diameter 0.08 D, axis 0.16 D behind the rotor plane, from the ground to hub
    height) and capsule nacelle (diameter 0.1 D, total length 0.54 D, hemispherical ends of radius
    0.05 D), as Lagrangian surface points of the given spacing (geometry after section 4.4)."""
    hx, hy, hz = hub
    tower_xyz, tower_ds = _cylinder_z(hx + 0.16 * D, hy, z_ground, hz, 0.08 * D, spacing)
    rad = 0.05 * D
    nac_xyz, nac_ds = _capsule_x(hx, hx + 0.54 * D - 2 * rad, hy, hz, rad, spacing)
    xyz = np.concatenate([nac_xyz, tower_xyz], 0)
    dS = np.concatenate([nac_ds, tower_ds], 0)
    return IbmSpec(xyz=xyz, dS=dS)


# ----------------------------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------------------------

def make_case(name: str, grid: Optional[Sequence[int]] = None, seed: Optional[int] = None,
              steps: Optional[int] = None, **overrides) -> CaseConfig:
    """Build a workload. ``grid`` = (nx, ny, nz) shrinks/enlarges it at fixed physics (the domain and
    rotor keep their size in rotor diameters; the cell count per diameter follows the grid)."""
    if name not in CASE_NAMES:
        raise ValueError(f"unknown case {name!r}")
    builder = {"tgv": _tgv, "channel": _channel, "alm": _alm, "alm_ibm": _alm_ibm, "adjoint": _adjoint,
               "channel_tanh": _channel_tanh}[name]
    cfg = builder(grid, seed)
    if steps is not None:
        cfg = cfg.with_(steps=steps)
    if overrides:
        cfg = cfg.with_(**overrides)
    return cfg


def _tgv(grid, seed):
    nx, ny, nz = grid or (32, 32, 32)
    seed = 1 if seed is None else seed
    rng = np.random.default_rng(seed)
    L = 2 * math.pi
    x, y, z = _centres(nx, 0.0, L), _centres(ny, 0.0, L), _centres(nz, 0.0, L)
    sx, sy, sz = _sinc(L / nx / 2), _sinc(L / ny / 2), _sinc(L / nz / 2)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    u0 = 1.0
    q = np.zeros((4, nz, ny, nx))
    q[0] = 1.0
    q[1] = u0 * (np.sin(X) * sx) * (np.cos(Y) * sy) * (np.cos(Z) * sz)
    q[2] = -u0 * (np.cos(X) * sx) * (np.sin(Y) * sy) * (np.cos(Z) * sz)
    kmax = min(4.0, min(nx, ny, nz) // 2 - 1)   # small test grids keep only the modes they resolve
    if kmax >= 1.0:
        q[1:] += random_solenoidal_field((nz, ny, nx), (L, L, L), (0.0, 0.0, 0.0), kmax, 0.01 * u0, rng)
    return CaseConfig(name="tgv", nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, lx=L, ly=L, lz=L,
                      ma=0.1, u_ref=1.0, rho_ref=1.0, mu=1.0 / 400.0, cfl=0.5, dt_fixed=0.0,
                      bc=("periodic",) * 6, steps=10, q0=q, seed=seed)


def _channel(grid, seed):
    nx, ny, nz = grid or (192, 96, 96)
    seed = 2 if seed is None else seed
    rng = np.random.default_rng(seed)
    lx, ly, lz = 4 * math.pi, 2.0, 4 * math.pi / 3
    hy = ly / ny
    y = _centres(ny, -1.0, ly)
    u_tau = 1.0 / 15.6          # bulk velocity 1, U_b / u_tau ~ 15.6 at Re_tau = 180
    re_tau = 180.0
    nu = u_tau * 1.0 / re_tau
    q = np.zeros((4, nz, ny, nx))
    q[0] = 1.0
    prof = 1.5 * (1.0 - (y * y + hy * hy / 12.0))   # exact cell average of 1.5 (1 - y^2)
    q[1] = prof[None, :, None]
    q[1:] += 0.05 * rng.uniform(-1.0, 1.0, size=(3, nz, ny, nx))
    return CaseConfig(name="channel", nx=nx, ny=ny, nz=nz, x0=0.0, y0=-1.0, z0=0.0, lx=lx, ly=ly, lz=lz,
                      ma=0.1, u_ref=1.0, rho_ref=1.0, mu=nu, cfl=0.5, dt_fixed=0.0,
                      bc=("periodic", "periodic", "noslip", "noslip", "periodic", "periodic"),
                      body_force=(u_tau * u_tau, 0.0, 0.0), steps=100, q0=q, seed=seed)


def tanh_faces(n: int, b: float = 2.0) -> np.ndarray:
    """Wall-clustered faces on [-1, 1]: y = tanh(b (eta / (1.5 pi) - 1)) / tanh(b) at eta = 3 pi j / n,
    j = 0..n (the channel mapping of Section 4.1)."""
    eta = 3.0 * math.pi * np.arange(n + 1) / n
    y = np.tanh(b * (eta / (1.5 * math.pi) - 1.0)) / math.tanh(b)
    y[0], y[-1] = -1.0, 1.0
    return y


def block_faces(n_lo, n_block, n_hi, h, ratio, start):
    """Faces of a locally refined axis (the refined block around the turbines of Section 4.3.3):
    n_block cells of width h beginning at `start`, with n_lo cells below and n_hi above whose widths grow
    by `ratio` per cell away from the block."""
    lo = h * ratio ** np.arange(n_lo, 0, -1)
    hi = h * ratio ** np.arange(1, n_hi + 1)
    w = np.concatenate([lo, np.full(n_block, h), hi])
    return (start - lo.sum()) + np.concatenate([[0.0], np.cumsum(w)])


def _channel_tanh(grid, seed):
    """The channel of Section 4.1 on its own mesh: [0, 2 pi] x [-1, 1] x [0, pi], 128^3 cells uniform in
    (xi, eta, zeta), tanh clustering towards the walls with b = 2; Poiseuille start with 5 % noise."""
    nx, ny, nz = grid or (128, 128, 128)
    seed = 5 if seed is None else seed
    rng = np.random.default_rng(seed)
    lx, ly, lz = 2 * math.pi, 2.0, math.pi
    yf = tanh_faces(ny)
    u_tau = 1.0 / 15.6
    nu = u_tau / 180.0
    q = np.zeros((4, nz, ny, nx))
    q[0] = 1.0
    ya, yb = yf[:-1], yf[1:]
    prof = 1.5 * (1.0 - (yb ** 3 - ya ** 3) / (3.0 * (yb - ya)))  # exact cell average of 1.5 (1 - y^2)
    q[1] = prof[None, :, None]
    q[1:] += 0.05 * rng.uniform(-1.0, 1.0, size=(3, nz, ny, nx))
    return CaseConfig(name="channel_tanh", nx=nx, ny=ny, nz=nz, x0=0.0, y0=-1.0, z0=0.0, lx=lx, ly=ly, lz=lz,
                      ma=0.1, u_ref=1.0, rho_ref=1.0, mu=nu, cfl=0.5, dt_fixed=0.0,
                      bc=("periodic", "periodic", "noslip", "noslip", "periodic", "periodic"),
                      body_force=(u_tau * u_tau, 0.0, 0.0), steps=100, q0=q, seed=seed,
                      faces=(None, yf, None))


def _uniform_stream(nx, ny, nz, u=1.0):
    q = np.zeros((4, nz, ny, nx))
    q[0] = 1.0
    q[1] = u
    return q


def _alm(grid, seed):
    nx, ny, nz = grid or (384, 192, 192)
    seed = 3 if seed is None else seed
    D = 1.0
    lx, ly, lz = 6 * D, 3 * D, 3 * D
    dx = lx / nx
    if not (abs(ly / ny - dx) < 1e-12 * dx and abs(lz / nz - dx) < 1e-12 * dx):
        raise ValueError("alm case needs cubic cells: grid must be proportional to 6:3:3")
    rotor = synthetic_rotor(hub=(1.5 * D, 1.5 * D, 1.5 * D), radius=0.5 * D, tsr=7.0, u_inf=1.0,
                            n_blades=3, n_per_blade=64, eps=2 * dx)
    re_r = 3.38e7
    return CaseConfig(name="alm", nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, lx=lx, ly=ly, lz=lz,
                      ma=0.1, u_ref=1.0, rho_ref=1.0, mu=1.0 * 0.5 * D / re_r, cfl=0.5, dt_fixed=0.0,
                      bc=("inflow", "outflow", "periodic", "periodic", "slip", "slip"),
                      u_in=(1.0, 0.0, 0.0), steps=5, rotor=rotor, q0=_uniform_stream(nx, ny, nz), seed=seed)


def _alm_ibm(grid, seed):
    nx, ny, nz = grid or (512, 256, 256)
    seed = 4 if seed is None else seed
    D = 1.0
    lx, ly, lz = 8 * D, 4 * D, 4 * D
    dx = lx / nx
    if not (abs(ly / ny - dx) < 1e-12 * dx and abs(lz / nz - dx) < 1e-12 * dx):
        raise ValueError("alm_ibm case needs cubic cells: grid must be proportional to 8:4:4")
    hub = (2.0 * D, 2.0 * D, 1.2 * D)
    rotor = synthetic_rotor(hub=hub, radius=0.5 * D, tsr=7.0, u_inf=1.0, n_blades=3, n_per_blade=64,
                            eps=2 * dx)
    ibm = tower_and_nacelle(hub, D, dx, spacing=0.28 * dx, z_ground=2.0 * dx)
    re_r = 3.38e7
    return CaseConfig(name="alm_ibm", nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, lx=lx, ly=ly, lz=lz,
                      ma=0.1, u_ref=1.0, rho_ref=1.0, mu=1.0 * 0.5 * D / re_r, cfl=0.5, dt_fixed=0.0,
                      bc=("inflow", "outflow", "periodic", "periodic", "slip", "slip"),
                      u_in=(1.0, 0.0, 0.0), steps=5, rotor=rotor, ibm=ibm,
                      q0=_uniform_stream(nx, ny, nz), seed=seed, ibm_iters=3)


def _adjoint(grid, seed):
    nx, ny, nz = grid or (128, 128, 128)
    seed = 5 if seed is None else seed
    rng = np.random.default_rng(seed)
    D = 1.0
    dx = D / 40.0 * (128.0 / nx)   # 40 cells per diameter at 128^3; the domain stays 3.2 D
    L = nx * dx
    if not (ny == nx and nz == nx):
        raise ValueError("adjoint case is a cube")
    q = _uniform_stream(nx, ny, nz)
    kmax = min(8.0, (nx // 2) - 1)
    q[1:] += random_solenoidal_field((nz, ny, nx), (L, L, L), (0.0, 0.0, 0.0), kmax, 0.05, rng)
    rotor = synthetic_rotor(hub=(0.5 * L, 0.5 * L, 0.5 * L), radius=0.5 * D, tsr=7.0, u_inf=1.0,
                            n_blades=3, n_per_blade=32, eps=2 * dx)
    re_r = 3.38e7
    return CaseConfig(name="adjoint", nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, lx=L, ly=L, lz=L,
                      ma=0.1, u_ref=1.0, rho_ref=1.0, mu=1.0 * 0.5 * D / re_r, cfl=0.0,
                      dt_fixed=1.0e-3 * (128.0 / nx), bc=("periodic",) * 6, steps=20, rotor=rotor,
                      q0=q, seed=seed)
