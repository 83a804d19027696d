"""Batched launches (many simulations per launch, HIP-graph replay, the
autotuners), through the C ABI.  The bar is bitwise: every member of a batch
must evolve exactly as the same simulation stepped alone (same kernels, same
arithmetic, tile shapes do not change results), and one member is also
checked against the FP64 oracle."""
import os
import sys

import numpy as np
import pytest

from common import oracle_params, rel_l2, rel_max
from oracle import oracle as O
from paper_2201_12404_amd import elmrt as E
from paper_2201_12404_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def make(w, tiling=None):
    sim = E.Simulation(E.params_for(w))
    if tiling:
        sim.set_tiling(*tiling)
    rho0, u0 = W.initial_fields(w)
    sim.init_fields(rho0, u0)
    return sim


def drops(count=5, hi=160):
    return W.batch_static_drops(count=count, seed=3, lo=64, hi=hi)


def test_batch_equals_individual_d2q9_graph_and_direct():
    jobs = drops()
    say("[gpu] batch d2q9", [j.n for j in jobs])
    tilings = [None, (128, 1, 8), None, (256, 1, 4), (64, 1, 32)]
    ref = [make(j, t) for j, t in zip(jobs, tilings)]
    for s in ref:
        s.step(7)
    f_ref = [s.read_populations() for s in ref]
    for use_graph in (True, False):
        sims = [make(j, t) for j, t in zip(jobs, tilings)]
        b = E.Batch(sims)
        b.set_graph(use_graph)
        b.step(7)
        for k, s in enumerate(sims):
            assert np.array_equal(s.read_populations(), f_ref[k]), (use_graph, k)
        b.close()
        for s in sims:
            s.close()
    for s in ref:
        s.close()


def test_graph_replays_with_eager_work_between():
    """Replays of the captured graph, with reads (eager kernels and
    synchronisations) between them, each against sims stepped alone."""
    jobs = drops(4, 128)
    ref = [make(j) for j in jobs]
    sims = [make(j) for j in jobs]
    b = E.Batch(sims)
    for rnd in range(3):
        b.step(4)
        for s in ref:
            s.step(4)
        for k in range(len(jobs)):
            r_b, u_b, _ = sims[k].read_macros()
            r_r, u_r, _ = ref[k].read_macros()
            assert np.array_equal(r_b, r_r) and np.array_equal(u_b, u_r), (rnd, k)
    b.close()


def test_member_stepped_alone_between_batch_steps():
    """Stepping one member through its own handle flips its buffer parity;
    the batch notices and rebuilds its table (odd step counts included)."""
    jobs = drops(3, 96)
    ref = [make(j) for j in jobs]
    sims = [make(j) for j in jobs]
    b = E.Batch(sims)
    b.step(3)
    sims[0].step(1)
    b.step(5)
    for k, s in enumerate(ref):
        s.step(3 + 5 + (1 if k == 0 else 0))
    for k in range(3):
        assert np.array_equal(sims[k].read_populations(), ref[k].read_populations()), k
    b.close()


def test_batch_equals_individual_d3q27():
    ws = [W.IMPACT_3D.scaled(n=(72, 40, 40), radius=10.0, film=8.0, centre=(36.0, 20.0, 28.0), name="a"),
          W.impact_job(3, 48, 100, 0.04, 10, 1)]
    say("[gpu] batch d3q27", [w.n for w in ws])
    ref = [make(w) for w in ws]
    for s in ref:
        s.step(6)
    sims = [make(w, t) for w, t in zip(ws, [(32, 8, 5), None])]
    b = E.Batch(sims)
    b.step(6)
    for k in range(2):
        assert np.array_equal(sims[k].read_populations(), ref[k].read_populations()), k
    b.close()


def test_autotuners_keep_results():
    jobs = drops(3, 128)
    sims = [make(j) for j in jobs]
    b = E.Batch(sims)
    taken = b.autotune(2)
    say("[gpu] batch autotune steps", taken)
    assert taken > 0
    b.step(3)
    ref = [make(j) for j in jobs]
    for k, s in enumerate(ref):
        s.step(taken + 3)
        assert np.array_equal(sims[k].read_populations(), s.read_populations()), k
    b.close()
    one = make(jobs[0])
    t1 = one.autotune(1)
    alone = make(jobs[0])
    alone.step(t1)
    assert np.array_equal(one.read_populations(), alone.read_populations())


def test_batch_member_against_oracle():
    """A 64^2 FP32 static drop stepped in a batch with a larger one, 300
    steps, against the FP64 oracle."""
    jobs = W.batch_static_drops(count=2, seed=11, lo=64, hi=64) + W.batch_static_drops(count=1, seed=5, lo=200, hi=200)
    sims = [make(j) for j in jobs]
    b = E.Batch(sims)
    b.step(300)
    rho_g, u_g, _ = sims[0].read_macros()
    w = jobs[0]
    rho0, u0 = W.initial_fields(w)
    p = oracle_params(w)
    f = O.init_fluid(p, rho0, u0)
    O.step(p, f, 300)
    rho_o, u_o, _ = O.macros(p, f)
    e_rho, l2_j = rel_max(rho_g, rho_o), rel_l2(rho_g * u_g, rho_o * u_o)
    say(f"batch member vs oracle: e_rho={e_rho:.3e} l2_j={l2_j:.3e}")
    assert e_rho < 1e-5 and l2_j < 1e-5
    b.close()


def test_batch_rejects_mixed_members():
    a = make(drops(1, 64)[0])
    c = make(W.impact_job(3, 48, 100, 0.04, 10, 2))
    with pytest.raises(E.ElmrtError, match="lattice"):
        E.Batch([a, c])
    with pytest.raises(E.ElmrtError, match="twice"):
        E.Batch([a, a])


def test_set_stream_keeps_results_and_batch_rejects_a_moved_member():
    """A simulation moved to another stream mid-run (after synchronising the
    old one) ends bitwise where the same simulation stepped on one stream
    ends; a batch refuses to step once a member has moved away from its
    stream."""
    import torch
    w = drops(count=1, hi=96)[0]
    a, b = make(w), make(w)
    other = torch.cuda.Stream()
    a.step(5)
    torch.cuda.current_stream().synchronize()
    a.set_stream(other)
    a.step(7)
    other.synchronize()
    b.step(12)
    ra, ua, sa = a.read_macros()
    rb, ub, sb = b.read_macros()
    assert np.array_equal(ra, rb) and np.array_equal(ua, ub) and np.array_equal(sa, sb)
    c, d = make(w), make(w)
    batch = E.Batch([c, d])
    batch.step(2)
    torch.cuda.current_stream().synchronize()
    c.set_stream(other)
    with pytest.raises(E.ElmrtError, match="another stream"):
        batch.step(2)
    batch.close()
    for s in (a, b, c, d):
        s.close()
