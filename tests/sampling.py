"""Sampled parity at full size: which cells to sample and how the oracle recomputes one of them.

The update of a cell in one S2O4 step (Section 2) depends on Q^n within 6 cells (3 per stage along each
axis: the normal reconstruction reaches 3 cells, the tangential sweeps 2). A sampled cell is recomputed
by the oracle on a 15^3 box of the pre-step field around it: centred (and periodic) away from the
domain boundary; cut at the boundary, with the domain's own boundary condition there, for a cell within
7 cells of a non-periodic side (the box's far side is then at least 8 cells away). Either way every
cell that the sample's update reads is exact (tests/test_sampling_boxes.py checks this against
full-domain oracle steps)."""
import numpy as np
import torch

from oracle import Oracle

R = 7  # box half-width


def excluded(cfg):
    """Boolean mask [nz, ny, nx] of cells a sample must avoid (those the body forces reach)."""
    ex = np.zeros((cfg.nz, cfg.ny, cfg.nx), bool)
    n = (cfg.nx, cfg.ny, cfg.nz)
    h = (cfg.dx, cfg.dy, cfg.dz)
    org = (cfg.x0, cfg.y0, cfg.z0)
    cen = [org[a] + (np.arange(n[a]) + 0.5) * h[a] for a in range(3)]
    if cfg.rotor is not None:
        r = cfg.rotor
        reach = r.r.max() + 3 * r.eps + (R + 2) * max(h)
        near = [np.abs(cen[0] - r.hub[0]) < 3 * r.eps + (R + 2) * h[0],
                np.abs(cen[1] - r.hub[1]) < reach, np.abs(cen[2] - r.hub[2]) < reach]
        ex |= near[2][:, None, None] & near[1][None, :, None] & near[0][None, None, :]
    if cfg.ibm is not None:
        lo = cfg.ibm.xyz.min(0) - (R + 4) * max(h)
        hi = cfg.ibm.xyz.max(0) + (R + 4) * max(h)
        inb = [(cen[a] > lo[a]) & (cen[a] < hi[a]) for a in range(3)]
        ex |= inb[2][:, None, None] & inb[1][None, :, None] & inb[0][None, None, :]
    return ex


def near_boundary(cfg):
    """Boolean mask of cells within R cells of a non-periodic side."""
    nb = np.zeros((cfg.nz, cfg.ny, cfg.nx), bool)
    n = (cfg.nx, cfg.ny, cfg.nz)
    for axis in range(3):
        for side in range(2):
            if cfg.bc[2 * axis + side] != "periodic":
                sl = [slice(None)] * 3
                sl[2 - axis] = slice(0, R) if side == 0 else slice(n[axis] - R, n[axis])
                nb[tuple(sl)] = True
    return nb


def face_chunk(n_n, tiles, slots=256):
    """March chunk of a face-kernel launch: the chunk that minimises rounds x (chunk + 2) for `slots`
    resident workgroups (one face workgroup per compute unit at these register and LDS sizes)."""
    best, best_chunk = None, n_n
    for nc in range(1, n_n + 1):
        chunk = -(-n_n // nc)
        wgs = tiles * (-(-n_n // chunk))
        cost = (-(-wgs // slots)) * (chunk + 2)
        if best is None or cost < best:
            best, best_chunk = cost, chunk
    return best_chunk


def face_plan(n_n, tiles, chunk, slots=256):
    """Work split of an order-5 face launch: (seg_len, n_wg). seg_len 0 is one aligned chunk per
    workgroup; seg_len > 0 gives workgroup w the cells [w seg_len, (w + 1) seg_len) of the tile-major
    (tile, cell) order, when its worst workgroup (cells + 2 per tile it meets, times the rounds of
    `slots`) beats the chunks'."""
    best = (-(-tiles * (-(-n_n // chunk)) // slots)) * (chunk + 2)
    plan = (0, tiles * (-(-n_n // chunk)))
    total = tiles * n_n
    for rounds in range(1, 9):
        ln = -(-total // (rounds * slots))
        wgs = -(-total // ln)
        w = np.arange(wgs)
        c0, c1 = w * ln, np.minimum(w * ln + ln, total)
        worst = int(((c1 - c0) + 2 * ((c1 - 1) // n_n - c0 // n_n + 1)).max())
        cost = (-(-wgs // slots)) * worst
        if cost < best:
            best, plan = cost, (ln, wgs)
        if ln == 1:
            break
    return plan


def seams(cfg, precision):
    """Per axis, a (nz, ny, nx) mask of the cells on either side of a seam of the face kernels along that
    axis: the first and last cell of each march of the pass normal to it (aligned chunks, or the runs of
    the tile-major split, which start and end at different cells in different tiles), and the tile edges
    across the faces of the other passes (16 x 16 faces in FP32, 16 x 8 in FP64)."""
    n = (cfg.nx, cfg.ny, cfg.nz)
    t2 = 16 if precision == "fp32" else 8
    axes = ((0, 1, 2), (1, 0, 2), (2, 0, 1))  # (normal, t1, t2) of the x, y and z faces
    seam = [np.zeros((cfg.nz, cfg.ny, cfg.nx), bool) for _ in range(3)]

    def along(a, mask1d):  # broadcast a 1-D mask over axis a of the (z, y, x) array
        shape = [1, 1, 1]
        shape[2 - a] = n[a]
        return mask1d.reshape(shape)

    for an, a1, a2 in axes:
        nt1, nt2 = -(-n[a1] // 16), -(-n[a2] // t2)
        tiles = nt1 * nt2
        chunk = face_chunk(n[an], tiles)
        seg_len, n_wg = face_plan(n[an], tiles, chunk)
        # march ends per tile: ends[t] marks the normal cells that start or end a march in tile t
        ends = np.zeros((tiles, n[an]), bool)
        if seg_len == 0:
            i = np.arange(n[an])
            ends[:] = (i % chunk == 0) | (i % chunk == chunk - 1) | (i == n[an] - 1)
        else:
            for w in range(n_wg):
                lin, end = w * seg_len, min(w * seg_len + seg_len, tiles * n[an])
                while lin < end:
                    t, f0 = divmod(lin, n[an])
                    f1 = min(n[an], f0 + end - lin)
                    ends[t, f0] = ends[t, f1 - 1] = True
                    lin += f1 - f0
        # spread over the cells: tile t covers t1 cells [16 (t % nt1), ...) and t2 cells [t2 (t // nt1), ...)
        i1 = np.arange(n[a1]) // 16
        i2 = np.arange(n[a2]) // t2
        tile_of = i2[:, None] * nt1 + i1[None, :]            # [t2 cell, t1 cell]
        m = ends[tile_of]                                     # [t2 cell, t1 cell, normal cell]
        # to (z, y, x): axes (a2, a1, an) -> (2, 1, 0) order
        order = {a2: 0, a1: 1, an: 2}
        seam[an] |= np.transpose(m, (order[2], order[1], order[0]))
        seam[a1] |= along(a1, (np.arange(n[a1]) % 16 == 0) | (np.arange(n[a1]) % 16 == 15))
        seam[a2] |= along(a2, (np.arange(n[a2]) % t2 == 0) | (np.arange(n[a2]) % t2 == t2 - 1))
    return seam


def box_range(c, n, periodic):
    """Index range of the 15 cells of the box along one axis and whether it is cut at the low or the
    high boundary (0: centred, -1: starts at cell 0, +1: ends at cell n - 1)."""
    if periodic or (R <= c < n - R):
        return np.arange(c - R, c + R + 1) % n, 0
    if c < R:
        return np.arange(0, 2 * R + 1), -1
    return np.arange(n - 2 * R - 1, n), 1


def box_ranges(cfg, cell):
    """Per axis (x, y, z) the box's index range and cut flag around interior cell (k, j, i)."""
    k, j, i = (int(c) for c in cell)
    n = (cfg.nx, cfg.ny, cfg.nz)
    return [box_range(c, n[a], cfg.bc[2 * a] == "periodic") for a, c in zip((0, 1, 2), (i, j, k))]


def take_box(field, ranges, pad=0):
    """The box of a [4, nz, ny, nx] field (pad: ghost layers of the array) as float64 on the host."""
    ii = [np.asarray(ranges[a][0]) + pad for a in (2, 1, 0)]
    t = field[:, ii[0]][:, :, ii[1]][:, :, :, ii[2]]
    return t.to(torch.float64).cpu()


def box_reference(cfg, box, ranges, cell, dt):
    """One oracle step (fixed dt, no body forces) of the box `box` ([4, W, W, W], rho - rho_ref) cut out
    of cfg's domain at `ranges`; returns the new state (rho - rho_ref, momenta) of interior cell
    (k, j, i)."""
    k, j, i = (int(c) for c in cell)
    W = 2 * R + 1
    h = (cfg.dx, cfg.dy, cfg.dz)
    x0 = (cfg.x0, cfg.y0, cfg.z0)
    faces = cfg.faces or (None, None, None)
    bc = list(cfg.bc)
    org = list(x0)
    lens = [W * h[a] for a in range(3)]
    bfaces = [None, None, None]
    centre = []
    for a in range(3):
        idx, cut = ranges[a]
        c = (i, j, k)[a]
        periodic = cfg.bc[2 * a] == "periodic"
        if cut == 0 and not periodic:
            # centred box away from the boundary: its ends are 7 cells from the sample, any boundary
            # condition there leaves the sample exact
            bc[2 * a] = bc[2 * a + 1] = "outflow"
        elif cut == -1:
            bc[2 * a + 1] = "outflow"
        elif cut == 1:
            bc[2 * a] = "outflow"
        lo = int(idx[0])
        if faces[a] is not None:
            fb = np.asarray(faces[a][lo:lo + W + 1], dtype=np.float64)
            bfaces[a] = fb
            org[a], lens[a] = float(fb[0]), float(fb[-1] - fb[0])
        elif not periodic:
            org[a] = x0[a] + lo * h[a]
        centre.append(R if cut == 0 else int(c - lo))
    bcfg = cfg.with_(nx=W, ny=W, nz=W, x0=org[0], y0=org[1], z0=org[2], lx=lens[0], ly=lens[1], lz=lens[2],
                     bc=tuple(bc), cfl=0.0, dt_fixed=dt, rotor=None, ibm=None,
                     faces=tuple(bfaces) if any(x is not None for x in bfaces) else None)
    q0 = box.clone()
    q0[0] += cfg.rho_ref
    o = Oracle(bcfg, q0=q0)
    o.step()
    ref = o.Q[:, centre[2], centre[1], centre[0]].clone()
    ref[0] -= cfg.rho_ref
    return ref
