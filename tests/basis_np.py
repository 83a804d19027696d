"""Independent numpy construction of the modified central Hermite basis
(Appendix A), used by the tests to pin the oracle.  Nothing here is imported by
the oracle or by the HIP library.

A moment is identified by its exponents (p, q[, r]) on (c - u); the modified
second-order diagonal block is labelled 'xx-yy', 'xx-zz' and 'trace'.
"""
from __future__ import annotations

import itertools

import numpy as np

CS2 = 1.0 / 3.0


def velocities(D: int) -> np.ndarray:
    Q = 3 ** D
    i = np.arange(Q)
    cols = [i % 3 - 1, (i // 3) % 3 - 1]
    if D == 3:
        cols.append(i // 9 - 1)
    return np.stack(cols, axis=1)


def H1(m: int, xi):
    """Central Hermite polynomial of order m in one variable."""
    if m == 0:
        return np.ones_like(xi, dtype=float)
    if m == 1:
        return xi
    return xi * xi - CS2


def labels(D: int):
    """Moment labels of the modified basis (Appendix A ordering is not needed)."""
    out = []
    for m in itertools.product(range(3), repeat=D):
        m = tuple(m)
        if sum(m) == 2 and max(m) == 2:
            continue                    # diagonal tensor moments are replaced
        out.append(m)
    out += ["xx-yy", "trace"] if D == 2 else ["xx-yy", "xx-zz", "trace"]
    return out


def moment_row(D: int, lab, u) -> np.ndarray:
    c = velocities(D).astype(float)
    xi = c - np.asarray(u, dtype=float)[None, :D]
    if isinstance(lab, tuple):
        row = np.ones(len(c))
        for a in range(D):
            row = row * H1(lab[a], xi[:, a])
        return row
    sq = [H1(2, xi[:, a]) for a in range(D)]
    if lab == "xx-yy":
        return sq[0] - sq[1]
    if lab == "xx-zz":
        return sq[0] - sq[2]
    if lab == "trace":
        return sum(sq)
    raise KeyError(lab)


def matrix(D: int, u):
    labs = labels(D)
    return labs, np.stack([moment_row(D, l, u) for l in labs])


def category(lab, trace_in_s: bool = False) -> str:
    """conserved / stress / h (the trace goes to h, or to s with trace_in_s;
    higher orders go to h)."""
    if isinstance(lab, tuple):
        o = sum(lab)
        if o <= 1:
            return "conserved"
        if o == 2:
            return "stress"            # off-diagonal second order
        return "h"
    if lab == "trace":
        return "stress" if trace_in_s else "h"
    return "stress"


def project(D: int, u, f, cat: str, trace_in_s: bool = False) -> np.ndarray:
    """Projection of f on the moments of one category, by explicit inversion."""
    labs, M = matrix(D, u)
    a = M @ f
    mask = np.array([category(l, trace_in_s) == cat for l in labs], dtype=float)
    return np.linalg.solve(M, mask * a)


def appendix_astar(D: int, rho, F, Phi):
    """Closed-form central Hermite moments of f* printed in Appendix A
    (retyped per moment identity; dt = 1)."""
    Fx, Fy = F[0], F[1]
    X = Fx * Fx + rho * Phi[0]
    Y = Fy * Fy + rho * Phi[1]
    if D == 2:
        return {
            (0, 0): rho, (1, 0): Fx, (0, 1): Fy,
            (1, 1): Fx * Fy / rho,
            "xx-yy": (Fx ** 2 - Fy ** 2 + rho * (Phi[0] - Phi[1])) / rho,
            "trace": (Fx ** 2 + Fy ** 2 + rho * (Phi[0] + Phi[1])) / rho,
            (2, 1): Fy * X / rho ** 2,
            (1, 2): Fx * Y / rho ** 2,
            (2, 2): X * Y / rho ** 3,
        }
    Fz = F[2]
    Z = Fz * Fz + rho * Phi[2]
    return {
        (0, 0, 0): rho, (1, 0, 0): Fx, (0, 1, 0): Fy, (0, 0, 1): Fz,
        (1, 1, 0): Fx * Fy / rho, (1, 0, 1): Fx * Fz / rho, (0, 1, 1): Fy * Fz / rho,
        "xx-yy": (Fx ** 2 - Fy ** 2 + rho * (Phi[0] - Phi[1])) / rho,
        "xx-zz": (Fx ** 2 - Fz ** 2 + rho * (Phi[0] - Phi[2])) / rho,
        "trace": (Fx ** 2 + Fy ** 2 + Fz ** 2 + rho * (Phi[0] + Phi[1] + Phi[2])) / rho,
        (2, 1, 0): Fy * X / rho ** 2, (2, 0, 1): Fz * X / rho ** 2,
        (1, 2, 0): Fx * Y / rho ** 2, (0, 2, 1): Fz * Y / rho ** 2,
        (1, 0, 2): Fx * Z / rho ** 2, (0, 1, 2): Fy * Z / rho ** 2,
        (1, 1, 1): Fx * Fy * Fz / rho ** 2,
        (2, 2, 0): X * Y / rho ** 3, (2, 0, 2): X * Z / rho ** 3, (0, 2, 2): Y * Z / rho ** 3,
        (2, 1, 1): Fy * Fz * X / rho ** 3, (1, 2, 1): Fx * Fz * Y / rho ** 3,
        (1, 1, 2): Fx * Fy * Z / rho ** 3,
        (2, 2, 1): Fz * X * Y / rho ** 4, (2, 1, 2): Fy * X * Z / rho ** 4,
        (1, 2, 2): Fx * Y * Z / rho ** 4,
        (2, 2, 2): X * Y * Z / rho ** 5,
    }
