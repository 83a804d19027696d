"""Writes the oracle's fields after 1000 steps for the FP32 parity cases at
the configurations' real shape (tests/parity_cases.py): one
tests/golden/parity_<case>.npz per case.  Calls only the oracle (and the
seeded input generator): f = f^eq at the initial fluid velocity (reading R16),
1000 oracle steps, then rho and j = rho u of every cell, or of the sampled
planes for the 3-D cases, rounded to FP32, and the global compensated sums.

    python tests/golden/make_parity_goldens.py [--threads 8] [case ...]

Takes about 6 minutes for the 2-D cases and 20-70 minutes for each 3-D case
on 8 cores.
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import parity_cases as PC  # noqa: E402
from common import oracle_params  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2201_12404_amd import workloads as W  # noqa: E402


def save(name, w, p, f, t, st):
    rho, u, sums = O.macros(p, f)
    if st.nonfinite or not np.isfinite(rho).all():
        raise RuntimeError(f"{name}: oracle state not finite after {t} steps")
    j = rho[None, :] * u
    out = dict(steps=np.int64(t), sums=np.asarray(sums, dtype=np.float64),
               oracle_sha=np.str_(PC.oracle_source_sha()), name=np.str_(w.name),
               gamma_fallbacks_last_step=np.int64(st.cells_gamma_fallback))
    if w.D == 3:
        planes = PC.sample_planes(w)
        cells = PC.plane_cells(w, planes)
        out["planes"] = np.asarray(planes, dtype=np.int64)
        rho, j = rho[cells], j[:, cells]
    out["rho"] = rho.astype(np.float32)
    out["j"] = j.astype(np.float32)
    path = PC.golden_path(name, t)
    np.savez_compressed(path, **out)
    return path


def write(name, w):
    p = oracle_params(w)
    rho0, u0 = W.initial_fields(w)
    f = O.init_fluid(p, rho0, u0)
    t0 = time.time()
    done = 0
    for t in sorted(set(PC.CHECKPOINTS.get(name, ())) | {w.steps}):
        st = O.step(p, f, t - done)
        done = t
        path = save(name, w, p, f, t, st)
        print(f"{name}: {w.name} n={w.n} {t} steps in {time.time() - t0:.0f} s, "
              f"{os.path.getsize(path) / 1e6:.2f} MB", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("cases", nargs="*")
    args = ap.parse_args()
    O.set_threads(args.threads)
    cases = PC.cases()
    for name in (args.cases or list(cases)):
        write(name, cases[name])


if __name__ == "__main__":
    main()
