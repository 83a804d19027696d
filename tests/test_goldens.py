"""The stored oracle fields of the FP32 parity cases (tests/golden/parity_*.npz)
are what the current oracle computes: the smallest case is recomputed here
and must match bitwise after the same FP32 rounding.  CPU only."""
import numpy as np
import pytest

import parity_cases as PC
from common import oracle_params
from oracle import oracle as O
from paper_2201_12404_amd import workloads as W


@pytest.mark.slow
def test_smallest_golden_reproduces():
    name = "c5-33"
    w = PC.cases()[name]
    g = PC.load_golden(name)
    p = oracle_params(w)
    f = O.init_fluid(p, *W.initial_fields(w))
    O.step(p, f, g["steps"])
    rho, u, sums = O.macros(p, f)
    assert np.array_equal(rho.astype(np.float32).astype(np.float64), g["rho"])
    assert np.array_equal((rho[None] * u).astype(np.float32).astype(np.float64), g["j"])
    np.testing.assert_allclose(sums, g["sums"], rtol=1e-15, atol=0)



def test_goldens_cover_every_case():
    """Every case and checkpoint has its golden file, of the stated step."""
    import os
    for name in PC.cases():
        for step in (PC.STEPS,) + tuple(PC.CHECKPOINTS.get(name, ())):
            path = PC.golden_path(name, step)
            assert os.path.exists(path), path
            assert PC.load_golden(name, step)["steps"] == step
