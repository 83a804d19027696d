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
  slab indicator    : phi_s = (tanh(2 (x - x1)/W) - tanh(2 (x - x2)/W)) / 2,
                      liquid between x1 and x2
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

# Maxwell coexistence (rho_v, rho_l) of EOS set B by reduced temperature:
# T/Tc = 0.60 .. 0.90 in steps of 0.01, and the temperatures of the density
# ratios 1000, 100, 10 (written by tests/golden/make_coexistence_table.py).
COEX_B_TABLE = {
    0.6: (0.010256254041444899, 8.746713113967818),
    0.61: (0.012499227237872022, 8.689831850259097),
    0.62: (0.015120352686928098, 8.631415610172784),
    0.63: (0.01816437335895818, 8.571403009734869),
    0.64: (0.021679157297824013, 8.509728867127127),
    0.65: (0.02571584579789224, 8.446323881152825),
    0.66: (0.030329039696676947, 8.381114270987307),
    0.67: (0.03557703115829154, 8.314021371206149),
    0.68: (0.04152208902592476, 8.244961174947885),
    0.69: (0.04823080681247406, 8.17384381666729),
    0.7: (0.055774523760970016, 8.100572984196372),
    0.71: (0.06422983124239237, 8.025045247658579),
    0.72: (0.07367917919673458, 7.94714929004974),
    0.73: (0.08421160053251234, 7.866765020838681),
    0.74: (0.0959235756065201, 7.783762549520429),
    0.75: (0.10892006441815894, 7.698000990363289),
    0.76: (0.12331574139881563, 7.609327062193561),
    0.77: (0.1392364772558622, 7.517573437353024),
    0.78: (0.15682112509460644, 7.42255678108655),
    0.79: (0.17622368521466736, 7.324075405339272),
    0.8: (0.1976159463471271, 7.2219064374712225),
    0.81: (0.2211907333132178, 7.115802372079132),
    0.82: (0.24716593613455512, 7.005486828954025),
    0.83: (0.27578955963457163, 6.890649276069038),
    0.84: (0.3073461251417693, 6.770938383778612),
    0.85: (0.3421648924312004, 6.645953539718899),
    0.86: (0.38063057583931903, 6.515233847907654),
    0.87: (0.4231975463981391, 6.3782436174044275),
    0.88: (0.4704090166979872, 6.234352840763261),
    0.89: (0.5229235325754982, 6.082810334811679),
    0.9: (0.5815525016166778, 5.922705810032623),
    0.592454: (0.008788568917849803, 8.78865484765582),
    0.725237: (0.07905400211939459, 7.905370373963834),
    0.901356: (0.5900262283184834, 5.900277847492134),
}
TR_OF_RATIO = {1000: 0.592454, 100: 0.725237, 10: 0.901356}


def kappa_w5(tr: float) -> float:
    """kappa~ giving an equilibrium interface width of ~5 for EOS set B at
    T/Tc = tr: the square-gradient values 0.01219, 0.007348, 0.005019 and
    0.002270 (T/Tc = 0.5925, 0.7252, 0.8, 0.9014) follow
    0.01219 ((1 - tr) / 0.407546)^1.25 within 8%."""
    return KAPPA_W5_RATIO_1000 * ((1.0 - tr) / (1.0 - TR_RATIO_1000)) ** 1.25


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
    kind: str               # "drop", "impact" or "slab"
    radius: float
    width: float = 5.0
    film: float = 0.0       # film thickness h (impact)
    centre: tuple = ()
    u_impact: float = 0.0
    noise: float = 0.0      # uniform velocity noise amplitude
    noise_liquid: float = 0.0   # impacts: Gaussian velocity noise in the liquid, std / u_impact
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
    elif w.kind == "slab":
        # liquid column of half-width 'radius' centred at centre[0] along x
        x = X[0]
        phi_s = 0.5 * (np.tanh(2.0 * (x - (w.centre[0] - w.radius)) / w.width)
                       - np.tanh(2.0 * (x - (w.centre[0] + w.radius)) / w.width))
        rho0 = w.rho_v + (w.rho_l - w.rho_v) * phi_s
        u0 = np.zeros((D, w.N))
    elif w.kind == "impact":
        zn = X[D - 1]                                   # wall-normal coordinate
        phi_f = 0.5 * (1.0 - np.tanh(2.0 * (zn - w.film) / w.width))
        rho0 = w.rho_v + (w.rho_l - w.rho_v) * np.maximum(phi_f, phi_d)
        u0 = np.zeros((D, w.N))
        u0[D - 1] = -w.u_impact * phi_d
        if w.noise_liquid > 0:
            # white noise on the liquid's velocity, std noise_liquid * U0
            # (Sec. 3.3, largest We), weighted by the liquid indicator
            liquid = np.maximum(phi_f, phi_d)
            rng = np.random.default_rng(w.seed)
            for a in range(D):
                u0[a] += rng.normal(0.0, w.noise_liquid * w.u_impact, w.N) * liquid
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


# ------------------------------------------------------------- job sets


def batch_static_drops(count: int = 64, seed: int = 0, steps: int = 2000, lo: int = 64, hi: int = 512):
    """Independent D2Q9 static drops of uneven size (FP32): edge N uniform in
    {lo..hi}, radius 0.2 N, T/Tc uniform on the 0.60 .. 0.90 grid of the
    coexistence table, EOS set B, kappa~ for W ~ 5, nu = 0.02 in both phases,
    velocity noise 1e-4 (seed k for job k), periodic."""
    rng = np.random.default_rng(seed)
    grid = [round(0.60 + 0.01 * k, 2) for k in range(31)]
    jobs = []
    for k in range(count):
        N = int(rng.integers(lo, hi + 1))
        tr = grid[int(rng.integers(0, len(grid)))]
        rv, rl = COEX_B_TABLE[tr]
        jobs.append(Workload(
            name=f"drop-{k}-d2q9-{N}-fp32", lattice=0, n=(N, N), bc=(0, 0), precision=0, eos=EOS_B,
            T_over_Tc=tr, kappa_tilde=kappa_w5(tr), nu_liquid=0.02, nu_vapour=0.02, rho_v=rv, rho_l=rl,
            kind="drop", radius=0.2 * N, centre=((N - 1) / 2, (N - 1) / 2), noise=1e-4, seed=k, steps=steps))
    return jobs


def impact_job(D: int, N: int, ratio: int, u0: float, steps: int, k: int = 0) -> Workload:
    """A drop impact of the served mix: D2Q9 on N x N (x periodic, walls in
    y) or D3Q27 on N^3 (x, y periodic, walls in z); drop diameter 0.3125 N,
    film max(0.1 D, 2W), gap 2W, W = 7, nu_l = 0.005, nu_v = nu_l max(1,
    ratio / 55), FP32."""
    tr = TR_OF_RATIO[ratio]
    rv, rl = COEX_B_TABLE[tr]
    W = 7.0
    R = 0.3125 * N / 2
    h = max(0.1 * 2 * R, 2 * W)
    zc = h + R + 2 * W
    nu_l = 0.005
    nu_v = nu_l * max(1.0, ratio / 55.0)
    if D == 2:
        n, bc, c = (N, N), (0, 1), ((N - 1) / 2, zc)
    else:
        n, bc, c = (N, N, N), (0, 0, 1), ((N - 1) / 2, (N - 1) / 2, zc)
    return Workload(
        name=f"impact-{k}-d{D}q{9 if D == 2 else 27}-{N}-r{ratio}-fp32", lattice=0 if D == 2 else 1, n=n, bc=bc,
        precision=0, eos=EOS_B, T_over_Tc=tr, kappa_tilde=kappa_w5(tr), nu_liquid=nu_l, nu_vapour=nu_v,
        rho_v=rv, rho_l=rl, kind="impact", radius=R, width=W, film=h, centre=c, u_impact=u0, seed=k, steps=steps)


def served_stream(count: int = 200, rate: float = 20.0, seed: int = 0):
    """Seeded Poisson stream of impact jobs: (arrival time [s], Workload).
    Half D2Q9 with N uniform in {128..1024}, half D3Q27 with N in {64..192};
    density ratio from {10, 100, 1000}; impact speed uniform in [0.02, 0.06];
    2000 .. 10000 steps."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        D = 2 if rng.random() < 0.5 else 3
        N = int(rng.integers(128, 1025)) if D == 2 else int(rng.integers(64, 193))
        ratio = int(rng.choice([10, 100, 1000]))
        u0 = float(rng.uniform(0.02, 0.06))
        steps = int(rng.integers(2000, 10001))
        out.append((t, impact_job(D, N, ratio, u0, steps, k)))
    return out
