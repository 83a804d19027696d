"""The paper's comparisons of the single-relaxation-time (BGK) and entropic
collisions, run through the library (every simulation step is a HIP kernel;
many runs advance together in one batch):

* spurious currents of 2-D resting drops against temperature and viscosity,
  with the (1 - T/Tc)^m fit (Sec. 3.1.2);
* the stability domain of 2-D drop impacts over viscosity and impact speed
  (Sec. 3.2).

Spurious currents are the maximum of the fluid velocity u + F/(2 rho) (the
bare velocity of a resting two-phase state is -F/(2 rho), not a current).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, replace

import numpy as np

from . import elmrt as E
from . import workloads as W


def drop(tr: float, nu: float, N: int = 128, R: float = 25.0, width: float = 5.0, precision: int = 0,
         noise: float = 0.0, seed: int = 0) -> W.Workload:
    """Resting D2Q9 drop of EOS set B at T/Tc = tr (a key of the coexistence
    table), radius R in an N x N periodic box, uniform viscosity nu."""
    rv, rl = W.COEX_B_TABLE[tr]
    return W.Workload(name=f"drop-{tr}-{nu}", lattice=0, n=(N, N), bc=(0, 0), precision=precision, eos=W.EOS_B,
                      T_over_Tc=tr, kappa_tilde=W.kappa_w5(tr), nu_liquid=nu, nu_vapour=nu, rho_v=rv, rho_l=rl,
                      kind="drop", radius=R, width=width, centre=((N - 1) / 2, (N - 1) / 2), noise=noise, seed=seed)


def impact2d(nu: float, u0: float, R0: float = 50.0, width: float = 5.0, film: float = 25.0,
             ratio: int = 1000, n=(500, 200), precision: int = 0) -> W.Workload:
    """2-D drop impact of the stability study: radius R0, interface width W,
    film thickness 'film' on the lower wall, gap 2W, x periodic, walls in y,
    uniform viscosity nu (both phases), density ratio 'ratio'."""
    tr = W.TR_OF_RATIO[ratio]
    rv, rl = W.COEX_B_TABLE[tr]
    zc = film + R0 + 2 * width
    return W.Workload(name=f"impact-{nu}-{u0}", lattice=0, n=tuple(n), bc=(0, 1), precision=precision,
                      eos=W.EOS_B, T_over_Tc=tr, kappa_tilde=W.kappa_w5(tr), nu_liquid=nu, nu_vapour=nu,
                      rho_v=rv, rho_l=rl, kind="impact", radius=R0, width=width, film=film,
                      centre=((n[0] - 1) / 2, zc), u_impact=u0)


@dataclass
class Run:
    workload: W.Workload
    collision: int
    stable: bool = True
    umax: float = float("nan")       # max |fluid velocity| at the end
    history: tuple = ()              # (step, umax) at the checkpoints


def _run_batch(runs, steps: int, checkpoints=()):
    """Advance all runs together (one batch), reading the fluid velocity of
    every run at the checkpoints and at the end; returns lattice updates / s."""
    sims = []
    for r in runs:
        sim = E.Simulation(E.params_for(r.workload, r.collision))
        sim.init_fields(*W.initial_fields(r.workload))
        sims.append(sim)
    b = E.Batch(sims)
    marks = sorted(set([c for c in checkpoints if 0 < c < steps] + [steps]))
    done, t_gpu = 0, 0.0
    hist = [[] for _ in runs]
    import torch
    for c in marks:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(c - done)
        torch.cuda.synchronize()
        t_gpu += time.perf_counter() - t0
        done = c
        for k, sim in enumerate(sims):
            if not runs[k].stable:
                continue
            try:
                u = sim.read_fluid_velocity()
            except E.ElmrtUnstable:
                runs[k].stable = False
                continue
            m = float(np.sqrt((u ** 2).sum(axis=0)).max())
            if not np.isfinite(m):
                runs[k].stable = False
                continue
            hist[k].append((c, m))
            runs[k].umax = m
    b.close()
    for k, sim in enumerate(sims):
        runs[k].history = tuple(hist[k])
        sim.close()
    lu = sum(r.workload.N for r in runs) * steps
    return lu / t_gpu if t_gpu > 0 else float("nan")


def spurious_currents(temps, nus, collisions=(E.ELMRT_BGK, E.ELMRT_ENTROPIC), steps: int = 4000, N: int = 128,
                      R: float = 25.0, checkpoints=(), precision: int = 0):
    """Max spurious current after 'steps' for every (T/Tc, nu, collision);
    returns (runs, lattice updates per second of the batched run)."""
    runs = [Run(drop(tr, nu, N, R, precision=precision), c) for c in collisions for tr in temps for nu in nus]
    rate = _run_batch(runs, steps, checkpoints)
    return runs, rate


def stability_map(nus, u0s, collisions=(E.ELMRT_BGK, E.ELMRT_ENTROPIC), steps: int = 2000, **kw):
    """Stable / unstable after 'steps' for every (nu, U0, collision) of the
    2-D impact; returns (runs, lattice updates per second)."""
    runs = [Run(impact2d(nu, u0, **kw), c) for c in collisions for nu in nus for u0 in u0s]
    rate = _run_batch(runs, steps)
    return runs, rate


def fit_power(temps, umax):
    """Least-squares fit umax = C (1 - T/Tc)^m in log space; returns (m, C)."""
    x = np.log(1.0 - np.asarray(temps, dtype=np.float64))
    y = np.log(np.asarray(umax, dtype=np.float64))
    m, logc = np.polyfit(x, y, 1)
    return float(m), float(np.exp(logc))
