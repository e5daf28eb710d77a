"""Helpers shared by the GPU tests: run the HIP library and the oracle on the same seeded case."""
import numpy as np
import torch

from oracle import Oracle


def run_gpu(cfg, precision, steps, **kw):
    from paper_2603_11102_amd import GksSolver
    s = GksSolver(cfg, precision=precision, **kw)
    outs = []
    for _ in range(steps):
        s.step(1)
        outs.append(s.forces(per_point=s.n_act > 0))
    return s, outs


def run_oracle(cfg, steps):
    o = Oracle(cfg)
    outs = [o.step() for _ in range(steps)]
    return o, outs


def oracle_dev(Q, rho_ref):
    """Oracle field (rho, m) -> (rho - rho_ref, m)."""
    q = Q.detach().clone()
    q[0] = q[0] - rho_ref
    return q


def rel_errors(gpu, ref, rho_ref=1.0):
    """Per variable: max |gpu - ref| / max |ref|. Arrays hold (rho - rho_ref, rho U, rho V, rho W); the
    density error is taken relative to the density rho = rho_ref + (rho - rho_ref), because the FP64
    oracle carries rho itself (its rho - rho_ref is only known to ~1e-16 rho absolute)."""
    out = []
    for v in range(4):
        d = float((gpu[v] - ref[v]).abs().max())
        s = float((ref[v] + rho_ref).abs().max()) if v == 0 else float(ref[v].abs().max())
        out.append(d / s if s > 0 else d)
    return out


def rel_errors_dev(gpu, ref):
    """Density deviation error relative to max |rho - rho_ref| (informational)."""
    d = float((gpu[0] - ref[0]).abs().max())
    s = float(ref[0].abs().max())
    return d / s if s > 0 else d


def rel_l2(gpu, ref):
    out = []
    for v in range(4):
        d = float(torch.linalg.vector_norm(gpu[v] - ref[v]))
        s = float(torch.linalg.vector_norm(ref[v]))
        out.append(d / s if s > 0 else d)
    return out


def print_case(tag, **kw):
    print(f"[gpu-case] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
