"""FP32 parity at the configurations' real shape after 1000 steps, through
the C ABI, against the FP64 oracle:

  * the 2-D impact at its full 1024 x 512 size and a 96^3 3-D impact (the
    3-D recipe: walls in z, two x-tiles of the default tiling, 24 y-tiles,
    several marching blocks), each run alone;
  * eight members of the 64-drop batch (its eight smallest grids) advanced in
    the batch itself;
  * eight jobs of the served stream (its six smallest D2Q9 and two smallest
    D3Q27 jobs, density ratios 10 to 1000) taken out of the request loop while
    other jobs share its rounds.

The oracle's fields come from tests/golden/parity_<case>.npz (written by
tests/golden/make_parity_goldens.py, which calls only the oracle) for the
impacts, and from the oracle run in the test for the batch members.

Bars.  Each norm -- e_rho, e_j (max norm on j = rho u), l2_j, and e_u, l2_u
on the bare velocity u = j / rho -- is held to max(1e-5, 3 x the
conditioning spread of that case at that instant).  The batch members
(static drops) and the 3-D impact at step 500 are held to 1e-5 on every
norm, the 2-D impact at step 600 on its moments.  The spread is what
FP32-sized perturbations do to the exact method: the FP64 build (equal to the
oracle within 1e-12) run once plainly and once with every population
multiplied by (1 + 2^-24 eta), eta uniform in [-1, 1], before every step; it
is measured by this module (test_conditioning_spread) and recorded in SPREAD
below.  Where a drop meets a film or another drop, the draining vapour layer
makes it exceed 1e-5 on u, and on the max norms of rho and j through a
rupture.
"""
import os
import sys
from dataclasses import replace

import numpy as np
import pytest

import parity_cases as PC
from common import oracle_params, rel_l2, rel_max
from oracle import oracle as O
from paper_2201_12404_amd import elmrt as E
from paper_2201_12404_amd import workloads as W

pytestmark = pytest.mark.gpu

NORMS = ("e_rho", "e_j", "l2_j", "e_u", "l2_u")

# Conditioning spread per case and norm at step 1000: the largest departure,
# over four noise seeds, of the FP64 build with FP32-sized noise injected
# before every step from the plain FP64 build (measured on the MI355X by
# conditioning_spread below; test_conditioning_spread re-measures it).
SPREAD = {
    'c2-full': {'e_rho': 9.51e-06, 'e_j': 0.000191, 'l2_j': 1.73e-05, 'e_u': 0.000133, 'l2_u': 2.56e-05},
    'c3-96': {'e_rho': 5.42e-07, 'e_j': 1.26e-05, 'l2_j': 1.53e-06, 'e_u': 4.18e-05, 'l2_u': 2.51e-06},
    'c5-33': {'e_rho': 2.14e-05, 'e_j': 0.000272, 'l2_j': 2.08e-05, 'e_u': 0.000314, 'l2_u': 3.05e-05},
    'c5-56': {'e_rho': 9.64e-07, 'e_j': 2.22e-06, 'l2_j': 1.26e-06, 'e_u': 2.79e-06, 'l2_u': 1.16e-06},
    'c5-3': {'e_rho': 1.58e-05, 'e_j': 0.000828, 'l2_j': 0.000109, 'e_u': 0.00153, 'l2_u': 0.000204},
    'c5-35': {'e_rho': 8.99e-05, 'e_j': 0.000904, 'l2_j': 0.000117, 'e_u': 0.00146, 'l2_u': 0.000214},
    'c5-59': {'e_rho': 1.6e-05, 'e_j': 2.43e-05, 'l2_j': 9.57e-06, 'e_u': 8.13e-05, 'l2_u': 3.45e-05},
    'c5-78': {'e_rho': 1.42e-06, 'e_j': 2.16e-06, 'l2_j': 1.18e-06, 'e_u': 5.5e-06, 'l2_u': 7.47e-06},
    'c5-89': {'e_rho': 1.45e-07, 'e_j': 3.33e-06, 'l2_j': 1.33e-06, 'e_u': 2.65e-06, 'l2_u': 1.14e-06},
    'c5-118': {'e_rho': 3.84e-07, 'e_j': 1.73e-05, 'l2_j': 3.28e-06, 'e_u': 1.02e-05, 'l2_u': 2.36e-06},
}


# The same spread at the earlier stored instants, where measured.  On the 2-D
# impact the velocity spread stays near 1e-5 or above from the approach of the
# drop (the draining vapour layer) to step 1000: 6.3e-4 at step 200, 1.6e-5
# at 600, 1.2e-5 at 700 (e_u), while the moments' spread at 600 is ~2e-6.
SPREAD_AT = {
    ('c2-full', 600): {'e_rho': 2.17e-06, 'e_j': 2.95e-06, 'l2_j': 1.55e-06, 'e_u': 1.58e-05, 'l2_u': 1.03e-05},
}


def bar(name, k):
    return max(1e-5, 3.0 * SPREAD.get(name, {}).get(k, 0.0))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    O.set_threads(min(16, os.cpu_count() or 1))
    yield


def norms(rho_g, j_g, rho_o, j_o):
    u_g, u_o = j_g / rho_g, j_o / rho_o
    return dict(e_rho=rel_max(rho_g, rho_o), e_j=rel_max(j_g, j_o), l2_j=rel_l2(j_g, j_o),
                e_u=rel_max(u_g, u_o), l2_u=rel_l2(u_g, u_o))


def fmt(d):
    return " ".join(f"{k}={v:.3e}" for k, v in d.items())


def check(name, n, strict=False, spread=None):
    """Every norm <= 1e-5 (strict), else <= max(1e-5, 3 x the case's spread);
    with 'spread' given: the moments' norms <= 1e-5 and those of u <=
    max(1e-5, 3 x spread)."""
    say(f"{name}: {fmt(n)}")
    for k in NORMS:
        if spread is not None:
            lim = max(1e-5, 3.0 * spread[k]) if k in ("e_u", "l2_u") else 1e-5
        else:
            lim = 1e-5 if strict else bar(name, k)
        assert n[k] <= lim, (name, k, n[k], lim)


def golden(name, step=None):
    path = PC.golden_path(name, step)
    if not os.path.exists(path):
        pytest.fail(f"missing golden {path}: run tests/golden/make_parity_goldens.py {name}")
    return PC.load_golden(name, step)


def compare_with_golden(name, w, rho, u, sums, step=PC.STEPS, strict=False, spread=None):
    g = golden(name, step)
    assert g["steps"] == step
    j = rho[None, :] * u
    if g["planes"] is not None:
        cells = PC.plane_cells(w, g["planes"])
        rho, j = rho[cells], j[:, cells]
    n = norms(rho, j, g["rho"], g["j"])
    # global sums of the whole grid (FP64 sums on both sides)
    n["mass"] = abs(sums[0] / g["sums"][0] - 1)
    check(name, n, strict, spread)
    assert n["mass"] <= 1e-6


def run_alone(w, steps):
    rho0, u0 = W.initial_fields(w)
    sim = E.Simulation(E.params_for(w))
    sim.init_fields(rho0, u0)
    sim.step(steps)
    rho, u, sums = sim.read_macros()
    sim.close()
    return rho, u, sums


@pytest.mark.parametrize("name", ["c2-full", "c3-96"])
def test_impact_real_shape_1000_steps(name):
    """The 2-D impact at 1024 x 512 and a 96^3 3-D impact, alone, default
    tiling, 1000 steps (past the contact), against the oracle's golden fields
    (whole field in 2-D, the sampled planes in 3-D) and global mass."""
    w = PC.cases()[name]
    say(f"[gpu] {name} {w.name} n={w.n} {PC.STEPS} steps")
    rho, u, sums = run_alone(w, PC.STEPS)
    compare_with_golden(name, w, rho, u, sums)


@pytest.mark.parametrize("name", ["c2-full", "c3-96"])
def test_impact_real_shape_checkpoint(name):
    """The same runs at an earlier stored instant: the 3-D impact at step
    500, every norm within 1e-5 of the oracle; the 2-D impact at step 600,
    where the moments' conditioning spread is ~2e-6: e_rho, e_j and l2_j
    within 1e-5, the velocity norms within 3 x their spread there (1.6e-5 and
    1.0e-5, SPREAD_AT)."""
    w = PC.cases()[name]
    (step,) = PC.CHECKPOINTS[name]
    say(f"[gpu] {name} {w.name} n={w.n} {step} steps")
    rho, u, sums = run_alone(w, step)
    compare_with_golden(name, w, rho, u, sums, step=step, strict=True, spread=SPREAD_AT.get((name, step)))


def test_batch_members_1000_steps():
    """The 64 uneven static drops as one batch (autotuned tiling, graph
    replay) for 1000 steps, the autotuning trials included; the eight smallest
    members against the oracle run here: every norm <= 1e-5."""
    jobs = [replace(j, steps=PC.STEPS) for j in W.batch_static_drops(count=64, seed=0)]
    sims = []
    for j in jobs:
        s = E.Simulation(E.params_for(j))
        s.init_fields(*W.initial_fields(j))
        sims.append(s)
    say(f"[gpu] batch of {len(sims)} drops, {PC.STEPS} steps")
    b = E.Batch(sims)
    taken = b.autotune(2)
    b.step(PC.STEPS - taken)
    small = sorted(range(len(jobs)), key=lambda k: jobs[k].N)[:8]
    for k in small:
        rho, u, _ = sims[k].read_macros()
        w = jobs[k]
        p = oracle_params(w)
        f = O.init_fluid(p, *W.initial_fields(w))
        O.step(p, f, PC.STEPS)
        rho_o, u_o, _ = O.macros(p, f)
        n = norms(rho, rho[None] * u, rho_o, rho_o[None] * u_o)
        check(f"c4-{k}-{w.n[0]}", n, strict=True)
    b.close()
    for s in sims:
        s.close()


def test_served_jobs_1000_steps():
    """Eight jobs of the served stream (six D2Q9, two D3Q27; ratios 10, 100,
    1000) submitted to the request loop with 1000 steps each, between six
    other jobs of the stream that share its rounds; each result against the
    oracle's golden fields."""
    cases = PC.cases()
    names = [k for k in cases if k.startswith("c5-")]
    stream = W.served_stream(count=200, rate=20.0, seed=0)
    others = [stream[k][1] for k in (0, 7, 13, 23, 33 + 1, 9)]
    srv = E.Server(pool_bytes=8 << 30, chunk_steps=200)
    ids = {}
    order = names[:4] + ["o0", "o1", "o2"] + names[4:] + ["o3", "o4", "o5"]
    for key in order:
        if key.startswith("o"):
            w = others[int(key[1])]
            srv.submit(E.params_for(w), *W.initial_fields(w), 300)
        else:
            w = cases[key]
            ids[key] = srv.submit(E.params_for(w), *W.initial_fields(w), PC.STEPS)
    say(f"[gpu] served: {len(order)} jobs")
    while True:
        q, r = srv.run(4)
        if q == 0 and r == 0:
            break
    for key in names:
        st, _, done = srv.job(ids[key])
        assert st == E.Server.DONE and done == PC.STEPS, (key, st, done)
        rho, u, sums = srv.result(ids[key])
        compare_with_golden(key, cases[key], rho, u, sums)
    srv.close()


def _fp64_run(w, steps, eps=0.0, seed=0):
    """rho, j of the FP64 build after 'steps' steps; with eps > 0 every
    population is multiplied by (1 + eps eta), eta uniform in [-1, 1] (seeded),
    before every step."""
    import torch
    w64 = replace(w, precision=1)
    sim = E.Simulation(E.params_for(w64))
    sim.init_fields(*W.initial_fields(w64))
    if eps > 0:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        for _ in range(steps):
            snap = sim.save_state()
            f = snap[512:].view(torch.float64)
            f.mul_(1 + eps * (torch.rand(f.shape, generator=gen, dtype=torch.float64, device=f.device) * 2 - 1))
            sim.load_state(snap)
            sim.step(1)
    else:
        sim.step(steps)
    rho, u, _ = sim.read_macros()
    sim.close()
    return rho, rho[None] * u


def conditioning_spread(w, steps=PC.STEPS, eps=2.0 ** -24, seeds=(1, 2, 3, 4)):
    """Largest norms, over the seeds, between the FP64 build with FP32-sized
    noise and the plain FP64 build (the FP64 build equals the oracle within
    1e-12: test_gpu_parity)."""
    r0, j0 = _fp64_run(w, steps)
    out = {k: 0.0 for k in NORMS}
    for s in seeds:
        r1, j1 = _fp64_run(w, steps, eps, s)
        n = norms(r1, j1, r0, j0)
        for k in NORMS:
            out[k] = max(out[k], n[k])
    return out


@pytest.mark.parametrize("name", ["c2-full", "c3-96"] + [f"c5-{k}" for k in PC.C5_D2Q9 + PC.C5_D3Q27])
def test_conditioning_spread(name):
    """The conditioning spread of each impact reproduces the recorded one
    (SPREAD) within a factor 2, so the bars rest on a measurement of the
    problem, not of the FP32 kernels."""
    w = PC.cases()[name]
    n = conditioning_spread(w)
    say(f"spread {name}: {fmt(n)}")
    assert name in SPREAD
    for k in NORMS:
        assert SPREAD[name][k] / 2 <= n[k] <= 2 * SPREAD[name][k], (name, k, n[k])
