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


# ------------------------------------------ thermodynamic consistency (f2)


def _eos(a: float) -> dict:
    return dict(eos_a=a, eos_b=0.095, eos_R=1.0, acentric=0.344)


def _coex(tr: float, a: float):
    p = E.Params(lattice=0, n=(8, 8, 1), T_over_Tc=tr, **_eos(a))
    rv, rl, _ = E.elmrt_coexistence(p)
    return rv, rl


def kappa_for(tr: float, a: float) -> float:
    """kappa~ for an interface width of ~5: the EOS-set-B value scaled by
    a / 0.003 (at fixed T/Tc and b the pressure scales with a)."""
    return W.kappa_w5(tr) * a / 0.003


def slab(tr: float, a: float = 0.003, n=(800, 10), half: float = 200.0, width: float = 5.0, nu: float = 0.1,
         precision: int = 0) -> W.Workload:
    """Flat-interface case of Sec. 3.1.1: a liquid column 2*half wide at the
    centre of a periodic n[0] x n[1] box of vapour (Maxwell densities)."""
    rv, rl = _coex(tr, a)
    return W.Workload(name=f"slab-{tr}-{a}", lattice=0, n=tuple(n), bc=(0, 0), precision=precision, eos=_eos(a),
                      T_over_Tc=tr, kappa_tilde=kappa_for(tr, a), nu_liquid=nu, nu_vapour=nu, rho_v=rv, rho_l=rl,
                      kind="slab", radius=half, width=width, centre=((n[0] - 1) / 2, (n[1] - 1) / 2))


def laplace_drop(tr: float, R: float, a: float = 0.003, width: float = 5.0, nu: float = 0.1,
                 precision: int = 0) -> W.Workload:
    """Resting drop of radius R in a periodic square box of side 4R + 20W."""
    rv, rl = _coex(tr, a)
    N = int(4 * R + 20 * width)
    return W.Workload(name=f"laplace-{tr}-{R}-{a}", lattice=0, n=(N, N), bc=(0, 0), precision=precision, eos=_eos(a),
                      T_over_Tc=tr, kappa_tilde=kappa_for(tr, a), nu_liquid=nu, nu_vapour=nu, rho_v=rv, rho_l=rl,
                      kind="drop", radius=R, width=width, centre=((N - 1) / 2, (N - 1) / 2))


def _converge(workloads, steps_max: int, chunk: int, tol: float):
    """Advance the workloads together until every density field changes by
    less than tol * max(rho) (max norm) over a chunk, or steps_max; returns
    the final density fields, the steps taken and whether each converged."""
    sims = []
    for w in workloads:
        sim = E.Simulation(E.params_for(w))
        sim.init_fields(*W.initial_fields(w))
        sims.append(sim)
    b = E.Batch(sims)
    prev = [None] * len(sims)
    conv = [False] * len(sims)
    done = 0
    while done < steps_max and not all(conv):
        b.step(chunk)
        done += chunk
        for k, sim in enumerate(sims):
            rho, _, _ = sim.read_macros()
            if prev[k] is not None and np.abs(rho - prev[k]).max() < tol * np.abs(rho).max():
                conv[k] = True
            prev[k] = rho
    b.close()
    for sim in sims:
        sim.close()
    return prev, done, conv


def coexistence_sweep(temps, a: float = 0.003, steps_max: int = 40000, chunk: int = 2000, tol: float = 1e-9,
                      **kw):
    """Converged flat interfaces at each T/Tc: simulated vapour and liquid
    densities (means over the bulk of each phase), the Maxwell values and the
    interface thickness W = (rho_l - rho_v) / max |d rho / dx| (Sec. 3.1.1)."""
    ws = [slab(tr, a, **kw) for tr in temps]
    fields, steps, conv = _converge(ws, steps_max, chunk, tol)
    out = []
    for w, rho, ok in zip(ws, fields, conv):
        nx, ny = w.n
        prof = rho.reshape(ny, nx).mean(axis=0)
        x = np.arange(nx)
        x1, x2 = w.centre[0] - w.radius, w.centre[0] + w.radius
        liquid = np.abs(x - w.centre[0]) < w.radius - 10 * w.width
        vapour = (x < x1 - 10 * w.width) | (x > x2 + 10 * w.width)
        rl, rv = float(prof[liquid].mean()), float(prof[vapour].mean())
        grad = np.abs(np.roll(prof, -1) - np.roll(prof, 1)) / 2.0
        out.append(dict(T_over_Tc=w.T_over_Tc, a=a, rho_l=rl, rho_v=rv, rho_l_maxwell=w.rho_l,
                        rho_v_maxwell=w.rho_v, W=float((rl - rv) / grad.max()), steps=steps, converged=ok))
    return out


def laplace_sweep(temps, radii, a: float = 0.003, steps_max: int = 40000, chunk: int = 2000, tol: float = 1e-9,
                  **kw):
    """Converged resting drops: pressure jump dP = P(rho_in) - P(rho_out)
    between the drop centre and the box corner, the equimolar radius R_e
    (pi R_e^2 (rho_in - rho_out) = sum (rho - rho_out), D = 2) and the
    surface tension sigma = dP R_e of the Laplace law (Sec. 3.1.2)."""
    ws = [laplace_drop(tr, R, a, **kw) for tr in temps for R in radii]
    fields, steps, conv = _converge(ws, steps_max, chunk, tol)
    out = []
    for w, rho, ok in zip(ws, fields, conv):
        N = w.n[0]
        f2 = rho.reshape(N, N)
        c = N // 2
        r_in, r_out = float(f2[c - 2:c + 3, c - 2:c + 3].mean()), float(f2[:3, :3].mean())
        P = E.elmrt_pressure(E.params_for(w), np.array([r_in, r_out]))
        dP = float(P[0] - P[1])
        Re = float(np.sqrt((rho - r_out).sum() / (np.pi * (r_in - r_out))))
        out.append(dict(T_over_Tc=w.T_over_Tc, a=a, R0=w.radius, rho_in=r_in, rho_out=r_out, dP=dP, R_e=Re,
                        sigma=dP * Re, steps=steps, converged=ok))
    return out
