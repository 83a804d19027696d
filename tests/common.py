"""Helpers shared by the tests: oracle parameters for a seeded workload, error
norms, and GPU availability."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def oracle_params(w, collision: int = 0) -> O.Params:
    return O.Params(D=w.D, n=tuple(w.n) + (1,) * (3 - len(w.n)), bc=tuple(w.bc) + (0,) * (3 - len(w.bc)),
                    collision=collision, a=w.eos["eos_a"], b=w.eos["eos_b"], R=w.eos["eos_R"],
                    acentric=w.eos["acentric"], Tr=w.T_over_Tc, kappa=w.kappa_tilde,
                    nu_l=w.nu_liquid, nu_v=w.nu_vapour, rho_l=w.rho_l, rho_v=w.rho_v)


def rel_max(a, b) -> float:
    """max |a - b| / max |b| (the parity norm on macroscopic fields)."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2"""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def velocity_map(c_lib: np.ndarray, D: int) -> np.ndarray:
    """index of each library velocity in the oracle's numbering"""
    c_ora = O.velocities(D)
    out = []
    for v in c_lib[:, :D]:
        out.append(int(np.where((c_ora == v).all(axis=1))[0][0]))
    return np.array(out)
