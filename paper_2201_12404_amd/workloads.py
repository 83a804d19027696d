"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds initial fields (tanh density profiles of drops and
films, seeded velocity noise) and parameter sets; it holds none of the
method's arithmetic.  Both the oracle and the HIP library are started from
these fields.

The coexistence densities below are the Maxwell equal-area values of the
Peng-Robinson EOS (acentric factor 0.344) at the stated reduced temperature;
they are parameters of the initial profile and of the viscosity
interpolation.  Both Maxwell solvers (the oracle's and the library's) are
checked against them in the tests.

Initial interface width: W = 5 for the static drop; W = 7 for the impacts.
At the impact viscosity (nu_l = 0.005) liquid layers of <= 20 cells started
from a W = 5 profile diverge in the first 50 steps (oracle and GPU alike),
while W = 7, close to the model's own converged width at this kappa~ (6.4),
is stable; the drop-to-film gap is 2W.

Shared definitions (lattice units, node coordinates 0..n-1):
  tanh profile      : tanh(2 x / W), so that max |grad rho| = (rho_l - rho_v)/W
  drop indicator    : phi_d = (1 - tanh(2 (|r - c| - R)/W)) / 2
  film indicator    : phi_f = (1 - tanh(2 (z - h)/W)) / 2, z = wall-normal
                      coordinate, first fluid node at 0, wall plane at -1/2
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

# Peng-Robinson parameter sets
EOS_A = dict(eos_a=2.0 / 49.0, eos_b=2.0 / 21.0, eos_R=1.0, acentric=0.344)   # static-drop set
EOS_B = dict(eos_a=0.003, eos_b=0.095, eos_R=1.0, acentric=0.344)             # paper's coexistence set

# Maxwell coexistence (rho_v, rho_l) at the temperatures used
COEX = {
    ("A", 0.8): (0.1971219064812592, 7.203851671377542),
    ("B", 0.592454): (0.008788568917849803, 8.78865484765582),    # density ratio 1000
}
TR_RATIO_1000 = 0.592454
KAPPA_W5_RATIO_1000 = 0.01219     # square-gradient kappa~ for W = 5 at ratio 1000, EOS set B


@dataclass(frozen=True)
class Workload:
    name: str
    lattice: int            # 0 D2Q9, 1 D3Q27
    n: tuple
    bc: tuple
    precision: int          # 0 FP32, 1 FP64
    eos: dict
    T_over_Tc: float
    kappa_tilde: float
    nu_liquid: float
    nu_vapour: float
    rho_v: float
    rho_l: float
    kind: str               # "drop" or "impact"
    radius: float
    width: float = 5.0
    film: float = 0.0       # film thickness h (impact)
    centre: tuple = ()
    u_impact: float = 0.0
    noise: float = 0.0      # uniform velocity noise amplitude
    seed: int = 0
    steps: int = 1000

    @property
    def D(self) -> int:
        return 2 if self.lattice == 0 else 3

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    def scaled(self, n, radius, film, centre, steps=None, name=None) -> "Workload":
        return replace(self, n=tuple(n), radius=radius, film=film, centre=tuple(centre),
                       steps=self.steps if steps is None else steps, name=name or self.name + "-scaled")


def _coords(n):
    axes = [np.arange(k, dtype=np.float64) for k in n]
    mesh = np.meshgrid(*axes, indexing="ij")
    # cell order x fastest
    return [m.transpose(tuple(range(len(n)))[::-1]).reshape(-1) for m in mesh]


def initial_fields(w: Workload):
    """rho0 (N,), u0 (D, N) in float64, cell = x + nx*(y + ny*z)."""
    X = _coords(w.n)
    D = w.D
    c = w.centre if w.centre else tuple((k - 1) / 2 for k in w.n)
    r = np.sqrt(sum((X[a] - c[a]) ** 2 for a in range(D)))
    phi_d = 0.5 * (1.0 - np.tanh(2.0 * (r - w.radius) / w.width))
    if w.kind == "drop":
        rho0 = w.rho_v + (w.rho_l - w.rho_v) * phi_d
        u0 = np.zeros((D, w.N))
    elif w.kind == "impact":
        zn = X[D - 1]                                   # wall-normal coordinate
        phi_f = 0.5 * (1.0 - np.tanh(2.0 * (zn - w.film) / w.width))
        rho0 = w.rho_v + (w.rho_l - w.rho_v) * np.maximum(phi_f, phi_d)
        u0 = np.zeros((D, w.N))
        u0[D - 1] = -w.u_impact * phi_d
    else:
        raise ValueError(w.kind)
    if w.noise > 0:
        rng = np.random.default_rng(w.seed)
        u0 = u0 + rng.uniform(-w.noise, w.noise, (D, w.N))
    return rho0, u0


def _nu_vapour(nu_l, rv, rl, mu_ratio=55.0):
    """Vapour kinematic viscosity for a liquid/vapour dynamic viscosity ratio."""
    return nu_l * (rl / rv) / mu_ratio


_rv_b, _rl_b = COEX[("B", TR_RATIO_1000)]

# 128^2 periodic static drop, FP64 (T/Tc = 0.8, EOS set A)
STATIC_DROP_FP64 = Workload(
    name="static-drop-d2q9-128-fp64", lattice=0, n=(128, 128), bc=(0, 0), precision=1,
    eos=EOS_A, T_over_Tc=0.8, kappa_tilde=0.03, nu_liquid=0.02, nu_vapour=0.02,
    rho_v=COEX[("A", 0.8)][0], rho_l=COEX[("A", 0.8)][1], kind="drop", radius=25.0,
    centre=(64.0, 64.0), noise=1e-4, seed=0, steps=1000)

# 1024 x 512 drop impact on a film, x periodic, walls in y, FP32, ratio 1000
IMPACT_2D = Workload(
    name="impact-d2q9-1024x512-fp32", lattice=0, n=(1024, 512), bc=(0, 1), precision=0,
    eos=EOS_B, T_over_Tc=TR_RATIO_1000, kappa_tilde=KAPPA_W5_RATIO_1000, nu_liquid=0.005,
    nu_vapour=_nu_vapour(0.005, _rv_b, _rl_b), rho_v=_rv_b, rho_l=_rl_b, kind="impact",
    radius=80.0, width=7.0, film=16.0, centre=(512.0, 16.0 + 80.0 + 14.0), u_impact=0.05, steps=20000)

# 256^3 drop impact on a film, x/y periodic, walls in z, FP32, ratio 1000
IMPACT_3D = Workload(
    name="impact-d3q27-256-fp32", lattice=1, n=(256, 256, 256), bc=(0, 0, 1), precision=0,
    eos=EOS_B, T_over_Tc=TR_RATIO_1000, kappa_tilde=KAPPA_W5_RATIO_1000, nu_liquid=0.005,
    nu_vapour=_nu_vapour(0.005, _rv_b, _rl_b), rho_v=_rv_b, rho_l=_rl_b, kind="impact",
    radius=40.0, width=7.0, film=8.0, centre=(128.0, 128.0, 8.0 + 40.0 + 14.0), u_impact=0.04, steps=10000)
