"""The request loop (elmrt_server_*): jobs of both lattices arriving while
others run, admitted by footprint, advanced in shared batches; every result
must be bitwise the one of the same job run alone."""
import sys

import numpy as np
import pytest

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
    yield


def alone(w, steps):
    sim = E.Simulation(E.params_for(w))
    rho0, u0 = W.initial_fields(w)
    sim.init_fields(rho0, u0)
    sim.step(steps)
    out = sim.read_macros()
    sim.close()
    return out


def mix():
    return [
        (W.impact_job(2, 128, 1000, 0.05, 37, 0), 37),
        (W.impact_job(3, 48, 100, 0.04, 21, 1), 21),
        (W.impact_job(2, 160, 10, 0.03, 50, 2), 50),
        (W.batch_static_drops(count=1, seed=4, lo=96, hi=96, steps=44)[0], 44),
        (W.impact_job(3, 40, 1000, 0.06, 33, 4), 33),
        (W.impact_job(2, 96, 100, 0.02, 9, 5), 9),
    ]


def test_results_same_alone_and_in_the_mix():
    jobs = mix()
    srv = E.Server(pool_bytes=1 << 30, chunk_steps=8)
    ids = []
    for k, (w, steps) in enumerate(jobs):
        rho0, u0 = W.initial_fields(w)
        ids.append(srv.submit(E.params_for(w), rho0, u0, steps))
        if k % 2 == 1:
            srv.run(2)          # later jobs arrive while earlier ones run
    while True:
        q, r = srv.run(4)
        if q == 0 and r == 0:
            break
    for (w, steps), jid in zip(jobs, ids):
        st, t, done = srv.job(jid)
        assert st == E.Server.DONE and done == steps
        assert t[0] <= t[1] <= t[2]
        rho_s, u_s, s_s = srv.result(jid)
        rho_a, u_a, s_a = alone(w, steps)
        say(f"[gpu] {w.name}: max|drho| {np.abs(rho_s - rho_a).max():.1e}")
        assert np.array_equal(rho_s, rho_a) and np.array_equal(u_s, u_a), w.name
        assert np.array_equal(s_s, s_a)
    lu, free = srv.stats()
    assert lu == sum(w.N * steps for w, steps in jobs)
    assert free == 1 << 30
    srv.close()


def test_admission_waits_for_memory():
    """A pool that holds one 128^2 impact job at a time: the second waits
    queued until the first is retired, and both finish correctly."""
    w1, w2 = W.impact_job(2, 128, 1000, 0.05, 20, 0), W.impact_job(2, 128, 100, 0.03, 12, 1)
    need = E.elmrt_workspace_bytes(E.params_for(w1))
    srv = E.Server(pool_bytes=need + need // 2, chunk_steps=5)
    a = srv.submit(E.params_for(w1), *W.initial_fields(w1), 20)
    b = srv.submit(E.params_for(w2), *W.initial_fields(w2), 12)
    q, r = srv.run(1)
    assert (q, r) == (1, 1)
    assert srv.job(b)[0] == E.Server.QUEUED
    while srv.run(1) != (0, 0):
        pass
    for jid, w, steps in ((a, w1, 20), (b, w2, 12)):
        rho_s, u_s, _ = srv.result(jid)
        rho_a, u_a, _ = alone(w, steps)
        assert np.array_equal(rho_s, rho_a) and np.array_equal(u_s, u_a)
    assert srv.job(b)[1][1] >= srv.job(a)[1][2]    # admitted after the first finished
    srv.close()


def test_server_rejects_invalid_job():
    srv = E.Server(pool_bytes=1 << 24, chunk_steps=4)
    p = E.Params(lattice=0, n=(3, 16, 1))
    with pytest.raises(E.ElmrtError, match="rejected"):
        srv.submit(p, np.zeros(48), np.zeros(96), 10)
    srv.close()


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_fill_budget_takes_turns(policy):
    """With a fill budget of one cell only one resident job advances in a
    round: the oldest (policies 0 and 2) or the one with the least remaining
    work, cells x steps (policy 1); the other starts when it is done, and both
    results are those of the jobs run alone."""
    w1, w2 = W.impact_job(2, 128, 1000, 0.05, 12, 0), W.impact_job(2, 96, 10, 0.03, 8, 1)
    srv = E.Server(pool_bytes=1 << 28, chunk_steps=4)
    srv.set_fill(1)
    srv.set_policy(policy)
    a = srv.submit(E.params_for(w1), *W.initial_fields(w1), 12)
    b = srv.submit(E.params_for(w2), *W.initial_fields(w2), 8)
    srv.run(1)          # the first pass admits both and advances one
    first, second = (a, b) if policy in (0, 2) else (b, a)
    assert srv.job(first)[2] == 4 and srv.job(second)[2] == 0
    while srv.run(1) != (0, 0):
        pass
    for jid, w, steps in ((a, w1, 12), (b, w2, 8)):
        rho_s, u_s, _ = srv.result(jid)
        rho_a, u_a, _ = alone(w, steps)
        assert np.array_equal(rho_s, rho_a) and np.array_equal(u_s, u_a)
    srv.close()


def test_round_takes_only_jobs_that_fit():
    """A round takes its first job, then only the later jobs that fit the
    rest of the fill budget: with a budget of two 64^2 grids, arrival order
    64^2, 128^2, 64^2, the first round advances the two small jobs (as one
    batch) and not the large one; every result is that of the job alone."""
    ws = [W.impact_job(2, 64, 10, 0.03, 8, 0), W.impact_job(2, 128, 1000, 0.05, 8, 1),
          W.impact_job(2, 64, 100, 0.04, 8, 2)]
    srv = E.Server(pool_bytes=1 << 28, chunk_steps=4)
    srv.set_fill(2 * 64 * 64)
    ids = [srv.submit(E.params_for(w), *W.initial_fields(w), 8) for w in ws]
    srv.run(1)          # the first pass admits all three and runs one round
    assert [srv.job(j)[2] for j in ids] == [4, 0, 4]
    while srv.run(1) != (0, 0):
        pass
    for jid, w in zip(ids, ws):
        rho_s, u_s, _ = srv.result(jid)
        rho_a, u_a, _ = alone(w, 8)
        assert np.array_equal(rho_s, rho_a) and np.array_equal(u_s, u_a)
    srv.close()


def test_unstable_job_is_evicted():
    """A job that goes unstable (BGK at nu = 0.0005 on a density-ratio-1000
    drop) is evicted once its polled flag is seen: it stops short of its step
    count, reports ELMRT_E_UNSTABLE with its fields, and frees its memory,
    while the job beside it finishes bitwise as if run alone."""
    from paper_2201_12404_amd import studies as S
    bad_w = S.drop(W.TR_OF_RATIO[1000], 0.0005, N=96, R=20.0)
    bad_steps = 4000
    sim = E.Simulation(E.params_for(bad_w, E.ELMRT_BGK))
    sim.init_fields(*W.initial_fields(bad_w))
    sim.step(bad_steps)
    with pytest.raises(E.ElmrtUnstable):
        sim.read_macros()
    sim.close()
    good_w, good_steps = W.impact_job(2, 128, 100, 0.03, 60, 1), 600
    srv = E.Server(pool_bytes=1 << 28, chunk_steps=20)
    bad = srv.submit(E.params_for(bad_w, E.ELMRT_BGK), *W.initial_fields(bad_w), bad_steps)
    good = srv.submit(E.params_for(good_w), *W.initial_fields(good_w), good_steps)
    while srv.run(1) != (0, 0):
        pass
    st, _, done = srv.job(bad)
    say(f"unstable job evicted after {done} of {bad_steps} steps")
    assert st == E.Server.DONE and done < bad_steps
    with pytest.raises(E.ElmrtUnstable) as ei:
        srv.result(bad)
    assert ei.value.rho.shape == (bad_w.N,)
    rho_s, u_s, _ = srv.result(good)
    rho_a, u_a, _ = alone(good_w, good_steps)
    assert np.array_equal(rho_s, rho_a) and np.array_equal(u_s, u_a)
    assert srv.stats()[1] == 1 << 28
    srv.close()
