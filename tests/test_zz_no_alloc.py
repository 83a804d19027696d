"""The entry point that allocates nothing, elmrt_read_sums_noalloc, against
elmrt_read_macros: the same compensated sums (bitwise) and the same
instability flag, on two calls in a row, the second on a smaller grid, in
both precisions and lattices, through the C ABI."""
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


def _sums_noalloc(sim):
    import torch
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    flag = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    E.elmrt_read_sums_noalloc(sim.handle, out.data_ptr(), flag.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(flag.cpu().item())


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_sums_equal_read_macros(prec):
    """Two sims, the second smaller, each stepped and read through both entry
    points: the device sums equal the host ones bitwise, the flag is 0."""
    from dataclasses import replace
    cases = [replace(W.IMPACT_3D.scaled(n=(72, 40, 40), radius=10.0, film=8.0, centre=(36.0, 20.0, 28.0),
                                        name="noalloc-3d"), precision=prec),
             replace(W.IMPACT_2D.scaled(n=(70, 44), radius=9.0, film=8.0, centre=(33.0, 27.0), name="noalloc-2d"),
                     precision=prec)]
    assert cases[1].N < cases[0].N
    for w in cases:
        say(f"[gpu] noalloc {w.name} n={w.n} prec={prec}")
        sim = E.Simulation(E.params_for(w))
        sim.init_fields(*W.initial_fields(w))
        sim.step(17)
        dev, flag = _sums_noalloc(sim)
        _, _, host = sim.read_macros()
        say(f"  device {dev} host {np.asarray(host)} flag {flag}")
        assert flag == 0
        assert np.array_equal(dev, np.asarray(host))
        sim.close()


def test_noalloc_flag_of_an_unstable_state():
    """A uniform state beyond 1/b (the pole of the pressure): one step raises
    the sticky flag, which both entry points report; a uniform state below
    1/b leaves it clear."""
    w = W.STATIC_DROP_FP64.scaled(n=(40, 36), radius=9.0, film=0.0, centre=(20.0, 18.0), name="beyond-1/b")
    b = w.eos["eos_b"]
    for rho0, unstable in ((0.95 / b, False), (1.05 / b, True)):
        sim = E.Simulation(E.params_for(w))
        sim.init_fields(np.full(w.N, rho0), np.zeros((2, w.N)))
        sim.step(1)
        dev, flag = _sums_noalloc(sim)
        if unstable:
            assert flag != 0
            with pytest.raises(E.ElmrtUnstable):
                sim.read_macros()
        else:
            assert flag == 0
            _, _, host = sim.read_macros()
            assert np.array_equal(dev, np.asarray(host))
        assert abs(dev[0] / (rho0 * w.N) - 1) < 1e-14
        sim.close()
