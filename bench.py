"""Throughput of the fused stream + collide step on one MI355X.

Workload: D3Q27, FP32, 256^3 drop impact on a thin film (x, y periodic, walls
in z, density ratio 1000), seeded synthetic initial state resident in HBM
before the timed region.  A step is one moment kernel plus one fused
stencil/collision kernel over all cells.

Prints one JSON line: MLUPS, ms per step, the roofline of the dominant
(collision) kernel timed with HIP events on the library's stream, and a CPU
baseline (the FP64 oracle on the host cores, on a bounded sample).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


class _Ranges:
    """roctx ranges around the benchmark's phases (visible with rocprofv3
    --marker-trace); no-ops where the roctx library is absent."""

    def __init__(self):
        import ctypes
        self._lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
            try:
                self._lib = ctypes.CDLL(name)
                self._lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                break
            except (OSError, AttributeError):
                self._lib = None

    def push(self, name: str):
        if self._lib:
            self._lib.roctxRangePushA(name.encode())

    def pop(self):
        if self._lib:
            self._lib.roctxRangePop()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for fn in ("elmrt_kernels.hip", "elmrt_internal.h"):
        with open(os.path.join(ROOT, "paper_2201_12404_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(D: int, es: int):
    """Per lattice update: (moment kernel, collision kernel) bytes.
    moment   : Q populations read, rho and D flux components written
    collision: Q populations read and written, rho and D fluxes read"""
    Q = 9 if D == 2 else 27
    return (Q * es + (1 + D) * es, 2 * Q * es + (1 + D) * es)


def measured_traffic(tag: str, tiling):
    """HBM bytes per launch of the collision and of the moment kernel from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source with this tiling; else (None, None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha") != kernel_source_hash() or d.get("tiling") != list(tiling):
        return None, None
    return d.get("bytes_per_launch"), d.get("k_macro", {}).get("bytes_per_launch")


def cpu_baseline(w, budget_s: float = 20.0):
    """The FP64 oracle as it stands, timed on a bounded sample of the same
    workload: a 128 x 128 x 96 block cut from the 256^3 initial state around the
    drop and the film (own periodic x/y, walls in z), stepped on all host
    threads."""
    import numpy as np

    from oracle import oracle as O
    from paper_2201_12404_amd import workloads as W

    threads = O.set_threads(0)
    rho0, u0 = W.initial_fields(w)
    nx, ny, nz = w.n
    sx, sy, sz = 128, 128, 96
    x0, y0 = (nx - sx) // 2, (ny - sy) // 2
    r = rho0.reshape(nz, ny, nx)[:sz, y0:y0 + sy, x0:x0 + sx].reshape(-1).copy()
    u = u0.reshape(3, nz, ny, nx)[:, :sz, y0:y0 + sy, x0:x0 + sx].reshape(3, -1).copy()
    p = O.Params(D=3, n=(sx, sy, sz), bc=(0, 0, 1), collision=0, a=w.eos["eos_a"], b=w.eos["eos_b"],
                 R=w.eos["eos_R"], acentric=w.eos["acentric"], Tr=w.T_over_Tc, kappa=w.kappa_tilde,
                 nu_l=w.nu_liquid, nu_v=w.nu_vapour, rho_l=w.rho_l, rho_v=w.rho_v)
    f = O.init_fluid(p, r, u)
    steps, elapsed = 0, 0.0
    while elapsed < budget_s and steps < 50:
        t0 = time.perf_counter()
        O.step(p, f, 1)
        elapsed += time.perf_counter() - t0
        steps += 1
        if elapsed > 0.6 * budget_s:
            break
    mlups = sx * sy * sz * steps / elapsed / 1e6
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": round(mlups, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle", "cpu": cpu,
            "affinity": len(os.sched_getaffinity(0)),
            "sample": f"{steps} step(s) of a {sx}x{sy}x{sz} block of the 256^3 impact state "
                      f"(FP64 oracle, OpenMP over cells), {elapsed:.1f} s"}


def impact_2d(steps: int = 2000, warmup: int = 100):
    """The 2-D impact configuration (D2Q9 FP32 1024 x 512, ratio 1000) from
    its initial state: time per step over 'steps' steps after 'warmup', the
    library's automatic tiling."""
    import torch

    from paper_2201_12404_amd import elmrt as E
    from paper_2201_12404_amd import workloads as W

    w = W.IMPACT_2D
    sim = E.Simulation(E.params_for(w))
    sim.init_fields(*W.initial_fields(w))
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    return {"workload": w.name, "steps": steps, "mlups": round(w.N * steps / wall / 1e6, 1),
            "us_per_step": round(wall / steps * 1e6, 2)}


def batched_vs_plain(steps: int = 2000, trial_steps: int = 4):
    """64 uneven D2Q9 static drops (FP32), each for 'steps' steps: one after
    the other through the single-simulation path, then all together as one
    batch (autotuned tiling, graph replay).  Aggregate MLUPS of both; the
    autotuning trials are steps of the run and are timed with it."""
    import torch

    from paper_2201_12404_amd import elmrt as E
    from paper_2201_12404_amd import workloads as W

    jobs = W.batch_static_drops(count=64, seed=0, steps=steps)
    cells = sum(j.N for j in jobs)

    def fresh():
        sims = []
        for j in jobs:
            sim = E.Simulation(E.params_for(j))
            sim.init_fields(*W.initial_fields(j))
            sims.append(sim)
        torch.cuda.synchronize()
        return sims

    sims = fresh()
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for sim in sims:
        sim.close()
    sims = fresh()
    b = E.Batch(sims)
    t0 = time.perf_counter()
    taken = b.autotune(trial_steps)
    b.step(steps - taken)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    for sim in sims:
        sim.close()
    return {"workload": f"64 D2Q9 static drops, edges 64..512, {cells} cells, {steps} steps, FP32",
            "plain_mlups": round(cells * steps / t_plain / 1e6, 1), "plain_s": round(t_plain, 3),
            "batched_mlups": round(cells * steps / t_batch / 1e6, 1), "batched_s": round(t_batch, 3),
            "autotune_steps": taken, "speedup": round(t_plain / t_batch, 2),
            "accuracy": "bitwise equal to the plain path (same kernels)"}


def served_jobs(count: int, step_scale: float):
    """The first 'count' jobs of the served impact stream (seeded Poisson
    arrivals, 20 jobs/s, D2Q9 and D3Q27 drop impacts of mixed size, density
    ratio and speed) with step counts scaled by 'step_scale', and their
    initial fields."""
    from paper_2201_12404_amd import workloads as W

    stream = W.served_stream(count=count, rate=20.0, seed=0)
    jobs = [(t, w, max(1, int(round(w.steps * step_scale)))) for t, w in stream]
    return jobs, [W.initial_fields(w) for _, w, _ in jobs]


def plain_fifo(jobs, inputs):
    """Each job alone through the single-simulation path (upload, steps,
    read-out), one after another; FIFO completion times follow from the
    measured service times and the arrival times."""
    import numpy as np
    import torch

    from paper_2201_12404_amd import elmrt as E

    service, unstable = [], []
    for k, ((_, w, n), (rho0, u0)) in enumerate(zip(jobs, inputs)):
        sim = E.Simulation(E.params_for(w))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.init_fields(rho0, u0)
        sim.step(n)
        try:
            sim.read_macros()
        except E.ElmrtUnstable:
            unstable.append(k)   # run to its step count, like the others
        service.append(time.perf_counter() - t0)
        sim.close()
        if k % 20 == 19:
            print(f"[bench] plain: {k + 1} of {len(jobs)} jobs", file=sys.stderr, flush=True)
    finish, lat = 0.0, []
    for (t, _, _), sv in zip(jobs, service):
        finish = max(finish, t) + sv
        lat.append(finish - t)
    lu = sum(w.N * n for _, w, n in jobs)
    return {"p50_s": round(float(np.percentile(lat, 50)), 3), "p99_s": round(float(np.percentile(lat, 99)), 3),
            "mlups": round(lu / finish / 1e6, 1), "makespan_s": round(finish, 3),
            "busy_s": round(sum(service), 3), "unstable_jobs": unstable}


def served_replay(jobs, inputs, policy: int, fill: int, chunk: int, pool_gib: float = 16.0):
    """Arrivals replayed in real time into the request loop (admission by
    footprint into a 'pool_gib' GiB pool, rounds of resident jobs up to 'fill'
    cells in the scheduling 'policy' order, 'chunk' steps for the costliest
    batch of a round).  Latency = arrival to completion; aggregate MLUPS =
    lattice updates / makespan (first arrival to last completion)."""
    import numpy as np

    from paper_2201_12404_amd import elmrt as E

    srv = E.Server(pool_bytes=int(pool_gib * (1 << 30)), chunk_steps=chunk)
    srv.set_fill(fill)
    srv.set_policy(policy)
    ids = [None] * len(jobs)
    t_start = time.monotonic()
    k = 0
    last = t_start
    while True:
        now = time.monotonic() - t_start
        while k < len(jobs) and jobs[k][0] <= now:
            _, w, n = jobs[k]
            ids[k] = srv.submit(E.params_for(w), inputs[k][0], inputs[k][1], n)
            k += 1
        q, r = srv.run(1)
        if time.monotonic() - last > 10.0:
            last = time.monotonic()
            print(f"[bench] served: {k} submitted, {q} queued, {r} resident", file=sys.stderr, flush=True)
        if k == len(jobs) and q == 0 and r == 0:
            break
        if q == 0 and r == 0 and k < len(jobs):
            time.sleep(max(0.0, min(0.01, jobs[k][0] - (time.monotonic() - t_start))))
    t_end = time.monotonic() - t_start
    lat, evicted = [], []
    for k, ((t, _, n), jid) in enumerate(zip(jobs, ids)):
        st, times, done = srv.job(jid)
        lat.append(times[2] - (t_start + t))
        if done < n:
            evicted.append(k)   # went unstable: read out early
    srv.close()
    lu = sum(w.N * n for _, w, n in jobs)
    return {"policy": ["arrival", "least remaining work", "least remaining work, oldest first"][policy],
            "fill_cells": fill, "chunk": chunk,
            "p50_s": round(float(np.percentile(lat, 50)), 3), "p99_s": round(float(np.percentile(lat, 99)), 3),
            "mlups": round(lu / t_end / 1e6, 1), "makespan_s": round(t_end, 3), "evicted_jobs": evicted}


def served_vs_plain(count: int, step_scale: float, fill: int = 2 << 20, chunk: int = 200):
    """Plain FIFO against the request loop in arrival order (the server's
    default) and with least remaining work first, on the same jobs."""
    jobs, inputs = served_jobs(count, step_scale)
    lu = sum(w.N * n for _, w, n in jobs)
    plain = plain_fifo(jobs, inputs)
    served = served_replay(jobs, inputs, 0, fill, chunk)
    print("[bench] served, least remaining work first", file=sys.stderr, flush=True)
    served_lrw = served_replay(jobs, inputs, 1, fill, chunk)
    return {"workload": f"first {count} jobs of the served stream (seed 0, 20 jobs/s), steps x {step_scale}, "
                        f"{lu:.3e} lattice updates, FP32",
            "served": served, "served_least_work_first": served_lrw, "plain": plain,
            "accuracy": "bitwise equal to the job run alone (tested)"}


def copy_probe(nbytes: int = 1 << 30):
    """A plain device copy kernel of known size (read nbytes, write nbytes),
    for calibrating the rocprofv3 FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB copy kernel (counter calibration)")
    # The library's autotuner picks 64 x 4 tiles marching 40..46 planes on this
    # grid (within 0.3% of each other); the bench fixes 46 so that its run and
    # the committed rocprofv3 counters describe the same launches.
    ap.add_argument("--tile", type=str, default="64,4,46", help="tx,ty,tm of the collision kernel")
    ap.add_argument("--autotune", action="store_true", help="let the library's autotuner pick the tiling")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched and served comparisons")
    ap.add_argument("--serve-jobs", type=int, default=200, help="jobs of the served stream to replay")
    ap.add_argument("--serve-step-scale", type=float, default=0.25, help="scale of the served jobs' step counts")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the slab decomposition over xGMI is design-only).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2201_12404_amd import elmrt as E
    from paper_2201_12404_amd import workloads as W

    torch.cuda.set_device(0)
    w = W.IMPACT_3D
    params = E.params_for(w)
    rho0, u0 = W.initial_fields(w)
    sim = E.Simulation(params)
    if not args.autotune:
        sim.set_tiling(*(int(v) for v in args.tile.split(",")))
    sim.init_fields(rho0, u0)
    mass0 = float(rho0.sum())
    del rho0, u0
    tuned = 0
    if args.autotune:
        # the library's autotuner picks the tiling; its trial steps are steps
        # of the run, taken before the warm-up and not timed
        print(f"[bench] {w.name}: autotuning the tiling", file=sys.stderr, flush=True)
        tuned = sim.autotune(4)
    tx, ty, tm = sim.get_tiling()
    print(f"[bench] tiling {tx}x{ty}x{tm}; warmup {args.warmup} steps", file=sys.stderr, flush=True)
    ranges = _Ranges()
    ranges.push("warmup")
    sim.step(args.warmup)
    torch.cuda.synchronize()

    ranges.pop()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    ranges.push("timed steps")
    t0 = time.perf_counter()
    ms_macro, ms_collide = sim.step_timed(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ranges.pop()
    _, u_end, sums = sim.read_macros()
    fallbacks = sim.gamma_fallbacks()
    umax = float(np.sqrt((u_end ** 2).sum(axis=0)).max())
    del u_end
    sim.close()

    N = w.N
    ms_per_step = wall / args.steps * 1e3
    mlups = N * args.steps / wall / 1e6
    es = 4
    b_macro, b_collide = algorithmic_bytes(3, es)
    avg_collide_s = ms_collide / args.steps / 1e3
    avg_macro_s = ms_macro / args.steps / 1e3
    achieved = N * b_collide / avg_collide_s / 1e9
    tag = "collide_d3q27_fp32_256"
    traffic, traffic_macro = measured_traffic(tag, (tx, ty, tm))
    out = {
        "metric": "MLUPS (D3Q27 FP32 256^3 drop-impact step)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": "D3Q27", "grid": list(w.n), "bc": "periodic x,y; walls z",
                   "collision": "entropic", "density_ratio": 1000, "tiling": [tx, ty, tm],
                   "autotune_steps": tuned},
        "hbm_gbs_algorithmic_step": round(N * (b_macro + b_collide) / wall * args.steps / 1e9, 1),
        # the step's HBM bytes counted by rocprofv3 (both kernels, committed
        # counters on this source) over the measured time per step
        "hbm_gbs_counted_step": (round((traffic + traffic_macro) / (ms_per_step / 1e3) / 1e9, 1)
                                 if traffic and traffic_macro else None),
        "kernels_ms": {"moments": round(avg_macro_s * 1e3, 4), "collide": round(avg_collide_s * 1e3, 4)},
        "roofline": {
            "kernel": f"k_collide<3,float,{tx},{ty}>",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            # counted HBM bytes per launch over the live launch time: the
            # rate at the memory interface, re-reads included
            "traffic_gbs": round(traffic / avg_collide_s / 1e9, 1) if traffic else None,
            "bytes_per_cell": b_collide,
        },
        "diagnostics": {"mass_drift": sums[0] / mass0 - 1.0, "gamma_fallbacks": fallbacks,
                        "max_speed": round(umax, 6), "steps_run": args.warmup + args.steps + tuned},
    }
    if args.copy_probe:
        copy_probe()
    if not args.no_batched:
        print("[bench] 2-D impact 1024x512", file=sys.stderr, flush=True)
        out["impact_2d"] = impact_2d()
        print("[bench] batched vs plain (64 static drops)", file=sys.stderr, flush=True)
        ranges.push("batched vs plain")
        out["batched"] = batched_vs_plain()
        ranges.pop()
        print("[bench] served vs plain", file=sys.stderr, flush=True)
        ranges.push("served vs plain")
        out["served"] = served_vs_plain(args.serve_jobs, args.serve_step_scale)
        ranges.pop()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
