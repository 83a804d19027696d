"""Thin ctypes binding of the C ABI declared in ``include/elmrt.h``.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libelmrt.so``.  PyTorch provides the device workspace and the stream.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libelmrt.so")

ELMRT_OK, ELMRT_E_INVALID, ELMRT_E_NOMEM, ELMRT_E_DEVICE, ELMRT_E_UNSTABLE, ELMRT_E_STATE = range(6)
ELMRT_D2Q9, ELMRT_D3Q27 = 0, 1
ELMRT_FP32, ELMRT_FP64 = 0, 1
ELMRT_ENTROPIC, ELMRT_BGK = 0, 1
ELMRT_PERIODIC, ELMRT_WALL = 0, 1
ELMRT_READING_TRACE_IN_S, ELMRT_READING_PHI_FLUID_VELOCITY = 1, 2


class ElmrtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"elmrt status {status}: {msg}")
        self.status = status


class ElmrtUnstable(ElmrtError):
    """Raised by read_macros when the sticky instability flag is set; the
    outputs read anyway are attached as ``.rho``, ``.u`` and ``.sums``."""


class elmrt_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("lattice", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("bc", ctypes.c_int32 * 3),
        ("readings", ctypes.c_int32),
        ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double), ("eos_R", ctypes.c_double),
        ("acentric", ctypes.c_double), ("T_over_Tc", ctypes.c_double),
        ("kappa_tilde", ctypes.c_double),
        ("nu_liquid", ctypes.c_double), ("nu_vapour", ctypes.c_double),
        ("rho_liquid", ctypes.c_double), ("rho_vapour", ctypes.c_double),
        ("body_accel", ctypes.c_double * 3),
        ("target_W", ctypes.c_double),
    ]


# Every function declared in include/elmrt.h: name -> (restype, argtypes).
_dp = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "elmrt_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(elmrt_params), ctypes.POINTER(ctypes.c_size_t)]),
    "elmrt_create": (ctypes.c_int, [ctypes.POINTER(elmrt_params), ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "elmrt_init_fields": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "elmrt_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "elmrt_step_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dp]),
    "elmrt_read_macros": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp]),
    "elmrt_read_populations": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "elmrt_read_sums_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "elmrt_read_fluid_velocity": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "elmrt_velocities": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "elmrt_coexistence": (ctypes.c_int, [ctypes.POINTER(elmrt_params), _dp, _dp, _dp]),
    "elmrt_pressure": (ctypes.c_int, [ctypes.POINTER(elmrt_params), _dp, _dp, ctypes.c_int64]),
    "elmrt_kappa_for_width": (ctypes.c_int, [ctypes.POINTER(elmrt_params), ctypes.c_double, _dp]),
    "elmrt_set_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "elmrt_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "elmrt_get_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "elmrt_gamma_fallbacks": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "elmrt_state_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "elmrt_poll_unstable": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "elmrt_save_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "elmrt_load_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "elmrt_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "elmrt_batch_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "elmrt_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "elmrt_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "elmrt_batch_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "elmrt_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "elmrt_batch_destroy": (None, [ctypes.c_void_p]),
    "elmrt_destroy": (None, [ctypes.c_void_p]),
    "elmrt_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "elmrt_server_set_fill": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "elmrt_server_set_policy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "elmrt_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(elmrt_params), _dp, _dp, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64)]),
    "elmrt_server_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "elmrt_server_job": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), _dp,
                                        ctypes.POINTER(ctypes.c_int64)]),
    "elmrt_server_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dp, _dp, _dp]),
    "elmrt_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "elmrt_server_destroy": (None, [ctypes.c_void_p]),
    "elmrt_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libelmrt.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != ELMRT_OK:
        raise ElmrtError(st, lib().elmrt_last_error().decode())


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


@dataclass
class Params:
    """Problem statement mirrored from elmrt_params (see include/elmrt.h)."""
    lattice: int
    n: tuple
    precision: int = ELMRT_FP32
    collision: int = ELMRT_ENTROPIC
    bc: tuple = (0, 0, 0)
    eos_a: float = 2.0 / 49.0
    eos_b: float = 2.0 / 21.0
    eos_R: float = 1.0
    acentric: float = 0.344
    T_over_Tc: float = 0.8
    kappa_tilde: float = 0.03
    nu_liquid: float = 0.02
    nu_vapour: float = 0.02
    rho_liquid: float = 0.0
    rho_vapour: float = 0.0
    body_accel: tuple = (0.0, 0.0, 0.0)
    target_W: float = 0.0
    trace_in_h: bool = True      # reading R6 (False: ELMRT_READING_TRACE_IN_S)
    phi_velocity: int = 0        # reading R4 (1: ELMRT_READING_PHI_FLUID_VELOCITY)

    @property
    def D(self) -> int:
        return 2 if self.lattice == ELMRT_D2Q9 else 3

    @property
    def Q(self) -> int:
        return 9 if self.D == 2 else 27

    @property
    def N(self) -> int:
        n = list(self.n) + [1] * (3 - len(self.n))
        return int(n[0]) * int(n[1]) * int(n[2])

    def c(self) -> elmrt_params:
        p = elmrt_params()
        p.struct_size = ctypes.sizeof(elmrt_params)
        p.lattice, p.precision, p.collision = self.lattice, self.precision, self.collision
        n = list(self.n) + [1] * (3 - len(self.n))
        bc = list(self.bc) + [0] * (3 - len(self.bc))
        for k in range(3):
            p.n[k] = int(n[k])
            p.bc[k] = int(bc[k])
        p.readings = (0 if self.trace_in_h else ELMRT_READING_TRACE_IN_S) | \
            (ELMRT_READING_PHI_FLUID_VELOCITY if self.phi_velocity else 0)
        p.eos_a, p.eos_b, p.eos_R = self.eos_a, self.eos_b, self.eos_R
        p.acentric, p.T_over_Tc = self.acentric, self.T_over_Tc
        p.kappa_tilde = self.kappa_tilde
        p.nu_liquid, p.nu_vapour = self.nu_liquid, self.nu_vapour
        p.rho_liquid, p.rho_vapour = self.rho_liquid, self.rho_vapour
        g = list(self.body_accel) + [0.0] * (3 - len(self.body_accel))
        for k in range(3):
            p.body_accel[k] = float(g[k])
        p.target_W = float(self.target_W)
        return p


def params_for(w, collision: int = ELMRT_ENTROPIC) -> Params:
    """Parameters of a seeded workload (paper_2201_12404_amd.workloads.Workload)."""
    return Params(lattice=w.lattice, n=tuple(w.n) + (1,) * (3 - len(w.n)), precision=w.precision,
                  collision=collision, bc=tuple(w.bc) + (0,) * (3 - len(w.bc)),
                  T_over_Tc=w.T_over_Tc, kappa_tilde=w.kappa_tilde, nu_liquid=w.nu_liquid,
                  nu_vapour=w.nu_vapour, rho_liquid=w.rho_l, rho_vapour=w.rho_v, **w.eos)


# ------------------------------------------------ functions of the C ABI


def elmrt_workspace_bytes(p: Params) -> int:
    cp = p.c()
    out = ctypes.c_size_t()
    _check(lib().elmrt_workspace_bytes(ctypes.byref(cp), ctypes.byref(out)))
    return out.value


def elmrt_create(p: Params, workspace_ptr: int, workspace_bytes: int, stream_ptr: int) -> int:
    cp = p.c()
    h = ctypes.c_void_p()
    _check(lib().elmrt_create(ctypes.byref(cp), ctypes.c_void_p(workspace_ptr), workspace_bytes,
                              ctypes.c_void_p(stream_ptr), ctypes.byref(h)))
    return h.value


def elmrt_init_fields(sim: int, rho0: np.ndarray, u0: np.ndarray) -> None:
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)
    _check(lib().elmrt_init_fields(ctypes.c_void_p(sim), _dptr(rho0), _dptr(u0)))


def elmrt_step(sim: int, nsteps: int) -> None:
    _check(lib().elmrt_step(ctypes.c_void_p(sim), int(nsteps)))


def elmrt_step_timed(sim: int, nsteps: int):
    ms = np.zeros(2)
    _check(lib().elmrt_step_timed(ctypes.c_void_p(sim), int(nsteps), _dptr(ms)))
    return float(ms[0]), float(ms[1])


def elmrt_read_macros(sim: int, N: int, D: int):
    """Returns (rho[N], u[D, N], sums[4]); raises ElmrtUnstable (outputs attached)."""
    rho = np.zeros(N)
    u = np.zeros((D, N))
    sums = np.zeros(4)
    st = lib().elmrt_read_macros(ctypes.c_void_p(sim), _dptr(rho), _dptr(u), _dptr(sums))
    if st == ELMRT_E_UNSTABLE:
        err = ElmrtUnstable(st, lib().elmrt_last_error().decode())
        err.rho, err.u, err.sums = rho, u, sums
        raise err
    _check(st)
    return rho, u, sums


def elmrt_read_density(sim: int, N: int) -> np.ndarray:
    """rho[N] alone (elmrt_read_macros with u and sums NULL: only the
    density crosses to the host)."""
    rho = np.zeros(N)
    st = lib().elmrt_read_macros(ctypes.c_void_p(sim), _dptr(rho), None, None)
    if st == ELMRT_E_UNSTABLE:
        err = ElmrtUnstable(st, lib().elmrt_last_error().decode())
        err.rho = rho
        raise err
    _check(st)
    return rho


def elmrt_read_fluid_velocity(sim: int, N: int, D: int) -> np.ndarray:
    u = np.zeros((D, N))
    st = lib().elmrt_read_fluid_velocity(ctypes.c_void_p(sim), _dptr(u))
    if st == ELMRT_E_UNSTABLE:
        err = ElmrtUnstable(st, lib().elmrt_last_error().decode())
        err.u = u
        raise err
    _check(st)
    return u


def elmrt_read_sums_noalloc(sim: int, dev_sums_ptr: int, dev_flag_ptr: int = 0) -> None:
    """Enqueue the compensated sums (4 FP64 at dev_sums_ptr) and the flag word
    (uint32 at dev_flag_ptr, or 0 for none) into device memory; no wait."""
    _check(lib().elmrt_read_sums_noalloc(sim, dev_sums_ptr, dev_flag_ptr or None))


def elmrt_read_populations(sim: int, Q: int, N: int) -> np.ndarray:
    f = np.zeros((Q, N))
    _check(lib().elmrt_read_populations(ctypes.c_void_p(sim), _dptr(f)))
    return f


def elmrt_velocities(lattice: int) -> np.ndarray:
    c = (ctypes.c_int32 * 81)()
    Q = lib().elmrt_velocities(int(lattice), c)
    if Q < 0:
        raise ElmrtError(ELMRT_E_INVALID, "unknown lattice")
    return np.array(c[: 3 * Q], dtype=np.int64).reshape(Q, 3)


def elmrt_coexistence(p: Params):
    cp = p.c()
    rv, rl, ps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().elmrt_coexistence(ctypes.byref(cp), ctypes.byref(rv), ctypes.byref(rl), ctypes.byref(ps)))
    return rv.value, rl.value, ps.value


def elmrt_kappa_for_width(p: Params, W: float) -> float:
    cp = p.c()
    out = ctypes.c_double()
    _check(lib().elmrt_kappa_for_width(ctypes.byref(cp), float(W), ctypes.byref(out)))
    return out.value


def elmrt_pressure(p: Params, rho: np.ndarray) -> np.ndarray:
    cp = p.c()
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    P = np.zeros_like(rho)
    _check(lib().elmrt_pressure(ctypes.byref(cp), _dptr(rho), _dptr(P), rho.size))
    return P


def elmrt_poll_unstable(sim: int, word: "ctypes.c_uint32") -> None:
    """Enqueue a copy of the sim's instability flag into ``word`` (a
    ctypes.c_uint32; valid once the sim's stream has reached the copy)."""
    _check(lib().elmrt_poll_unstable(ctypes.c_void_p(sim), ctypes.byref(word)))


def elmrt_state_bytes(sim: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().elmrt_state_bytes(ctypes.c_void_p(sim), ctypes.byref(out)))
    return out.value


def elmrt_save_state(sim: int, dev_ptr: int, nbytes: int) -> None:
    _check(lib().elmrt_save_state(ctypes.c_void_p(sim), ctypes.c_void_p(dev_ptr), nbytes))


def elmrt_load_state(sim: int, dev_ptr: int, nbytes: int) -> None:
    _check(lib().elmrt_load_state(ctypes.c_void_p(sim), ctypes.c_void_p(dev_ptr), nbytes))


def elmrt_gamma_fallbacks(sim: int) -> int:
    out = ctypes.c_int64()
    _check(lib().elmrt_gamma_fallbacks(ctypes.c_void_p(sim), ctypes.byref(out)))
    return out.value


def elmrt_get_tiling(sim: int):
    tx, ty, tm = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().elmrt_get_tiling(ctypes.c_void_p(sim), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(tm)))
    return tx.value, ty.value, tm.value


def elmrt_set_stream(sim: int, stream_ptr: int) -> None:
    _check(lib().elmrt_set_stream(ctypes.c_void_p(sim), ctypes.c_void_p(stream_ptr)))


def elmrt_set_tiling(sim: int, tx: int, ty: int, tm: int) -> None:
    _check(lib().elmrt_set_tiling(ctypes.c_void_p(sim), int(tx), int(ty), int(tm)))


def elmrt_autotune(sim: int, trial_steps: int) -> int:
    taken = ctypes.c_int64()
    _check(lib().elmrt_autotune(ctypes.c_void_p(sim), int(trial_steps), ctypes.byref(taken)))
    return taken.value


def elmrt_batch_workspace_bytes(count: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().elmrt_batch_workspace_bytes(int(count), ctypes.byref(out)))
    return out.value


def elmrt_batch_create(sims, workspace_ptr: int, workspace_bytes: int) -> int:
    arr = (ctypes.c_void_p * len(sims))(*[ctypes.c_void_p(h) for h in sims])
    h = ctypes.c_void_p()
    _check(lib().elmrt_batch_create(arr, len(sims), ctypes.c_void_p(workspace_ptr), workspace_bytes,
                                    ctypes.byref(h)))
    return h.value


def elmrt_batch_step(batch: int, nsteps: int) -> None:
    _check(lib().elmrt_batch_step(ctypes.c_void_p(batch), int(nsteps)))


def elmrt_batch_set_graph(batch: int, use_graph: bool) -> None:
    _check(lib().elmrt_batch_set_graph(ctypes.c_void_p(batch), int(bool(use_graph))))


def elmrt_batch_autotune(batch: int, trial_steps: int) -> int:
    taken = ctypes.c_int64()
    _check(lib().elmrt_batch_autotune(ctypes.c_void_p(batch), int(trial_steps), ctypes.byref(taken)))
    return taken.value


def elmrt_batch_destroy(batch: int) -> None:
    lib().elmrt_batch_destroy(ctypes.c_void_p(batch))


def elmrt_destroy(sim: int) -> None:
    lib().elmrt_destroy(ctypes.c_void_p(sim))


def elmrt_server_create(pool_ptr: int, pool_bytes: int, stream_ptr: int, chunk_steps: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().elmrt_server_create(ctypes.c_void_p(pool_ptr), pool_bytes, ctypes.c_void_p(stream_ptr),
                                     int(chunk_steps), ctypes.byref(h)))
    return h.value


def elmrt_server_set_fill(server: int, cells: int) -> None:
    _check(lib().elmrt_server_set_fill(ctypes.c_void_p(server), int(cells)))


def elmrt_server_set_policy(server: int, policy: int) -> None:
    _check(lib().elmrt_server_set_policy(ctypes.c_void_p(server), int(policy)))


def elmrt_server_submit(server: int, p: Params, rho0: np.ndarray, u0: np.ndarray, steps: int) -> int:
    cp = p.c()
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)
    jid = ctypes.c_int64()
    _check(lib().elmrt_server_submit(ctypes.c_void_p(server), ctypes.byref(cp), _dptr(rho0), _dptr(u0), int(steps),
                                     ctypes.byref(jid)))
    return jid.value


def elmrt_server_run(server: int, rounds: int):
    q, r = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().elmrt_server_run(ctypes.c_void_p(server), int(rounds), ctypes.byref(q), ctypes.byref(r)))
    return q.value, r.value


def elmrt_server_job(server: int, job_id: int):
    st, done = ctypes.c_int32(), ctypes.c_int64()
    t = np.zeros(3)
    _check(lib().elmrt_server_job(ctypes.c_void_p(server), int(job_id), ctypes.byref(st), _dptr(t), ctypes.byref(done)))
    return st.value, t, done.value


def elmrt_server_result(server: int, job_id: int, N: int, D: int):
    rho, u, sums = np.zeros(N), np.zeros((D, N)), np.zeros(4)
    st = lib().elmrt_server_result(ctypes.c_void_p(server), int(job_id), _dptr(rho), _dptr(u), _dptr(sums))
    if st == ELMRT_E_UNSTABLE:
        err = ElmrtUnstable(st, lib().elmrt_last_error().decode())
        err.rho, err.u, err.sums = rho, u, sums
        raise err
    _check(st)
    return rho, u, sums


def elmrt_server_stats(server: int):
    lu, free = ctypes.c_int64(), ctypes.c_size_t()
    _check(lib().elmrt_server_stats(ctypes.c_void_p(server), ctypes.byref(lu), ctypes.byref(free)))
    return lu.value, free.value


def elmrt_server_destroy(server: int) -> None:
    lib().elmrt_server_destroy(ctypes.c_void_p(server))


def elmrt_last_error() -> str:
    return lib().elmrt_last_error().decode()


# --------------------------------------------------- torch-backed handle


@dataclass
class Simulation:
    """A handle bound to a torch-allocated device workspace and torch's current
    stream on ``device``.  The workspace lives as long as this object."""
    params: Params
    device: str = "cuda:0"
    handle: int = field(default=0, init=False)

    def __post_init__(self):
        import torch

        lib()
        self._torch = torch
        dev = torch.device(self.device)
        nbytes = elmrt_workspace_bytes(self.params)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off: off + nbytes]
        self.stream = torch.cuda.current_stream(dev)
        self.handle = elmrt_create(self.params, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)

    def init_fields(self, rho0, u0):
        elmrt_init_fields(self.handle, rho0, u0)

    def step(self, nsteps: int):
        elmrt_step(self.handle, nsteps)

    def step_timed(self, nsteps: int):
        return elmrt_step_timed(self.handle, nsteps)

    def read_macros(self):
        return elmrt_read_macros(self.handle, self.params.N, self.params.D)

    def save_state(self):
        """Snapshot of the current state in a new torch uint8 device tensor."""
        n = elmrt_state_bytes(self.handle)
        raw = self._torch.empty(n + 256, dtype=self._torch.uint8, device=self.workspace.device)
        off = (-raw.data_ptr()) % 256
        snap = raw[off: off + n]
        elmrt_save_state(self.handle, snap.data_ptr(), n)
        return snap

    def load_state(self, snap):
        elmrt_load_state(self.handle, snap.data_ptr(), snap.numel())

    def gamma_fallbacks(self) -> int:
        return elmrt_gamma_fallbacks(self.handle)

    def read_density(self):
        return elmrt_read_density(self.handle, self.params.N)

    def read_populations(self):
        return elmrt_read_populations(self.handle, self.params.Q, self.params.N)

    def read_fluid_velocity(self):
        return elmrt_read_fluid_velocity(self.handle, self.params.N, self.params.D)

    def set_tiling(self, tx, ty, tm):
        elmrt_set_tiling(self.handle, tx, ty, tm)

    def get_tiling(self):
        return elmrt_get_tiling(self.handle)

    def set_stream(self, stream):
        """Enqueue later calls on ``stream`` (a torch.cuda.Stream); work
        already enqueued on the old stream must be ordered by the caller."""
        elmrt_set_stream(self.handle, stream.cuda_stream)
        self.stream = stream

    def autotune(self, trial_steps: int = 4) -> int:
        return elmrt_autotune(self.handle, trial_steps)

    def close(self):
        if self.handle:
            elmrt_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Simulations of one lattice, precision and stream advanced together
    (one launch per pass and step, pairs of steps replayed from a HIP graph).
    The members stay usable through their own handles; the job table lives in
    a torch-allocated device buffer owned by this object."""

    def __init__(self, sims, device: str = "cuda:0"):
        import torch

        self.sims = list(sims)
        nbytes = elmrt_batch_workspace_bytes(len(self.sims))
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=torch.device(device))
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off: off + nbytes]
        self.handle = elmrt_batch_create([s.handle for s in self.sims], self.workspace.data_ptr(), nbytes)

    def step(self, nsteps: int):
        elmrt_batch_step(self.handle, nsteps)

    def set_graph(self, use_graph: bool):
        elmrt_batch_set_graph(self.handle, use_graph)

    def autotune(self, trial_steps: int = 4) -> int:
        return elmrt_batch_autotune(self.handle, trial_steps)

    def close(self):
        if self.handle:
            elmrt_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop over a torch-allocated device pool on torch's current
    stream (see elmrt_server_* in include/elmrt.h)."""

    QUEUED, RESIDENT, DONE, FAILED = 0, 1, 2, 3

    def __init__(self, pool_bytes: int, chunk_steps: int = 100, device: str = "cuda:0"):
        import torch

        lib()
        raw = torch.empty(pool_bytes + 256, dtype=torch.uint8, device=torch.device(device))
        off = (-raw.data_ptr()) % 256
        self.pool = raw[off: off + pool_bytes]
        self.stream = torch.cuda.current_stream(torch.device(device))
        self.handle = elmrt_server_create(self.pool.data_ptr(), pool_bytes, self.stream.cuda_stream, chunk_steps)
        self.shapes = {}

    def set_fill(self, cells: int):
        elmrt_server_set_fill(self.handle, cells)

    def set_policy(self, policy: int):
        elmrt_server_set_policy(self.handle, policy)

    def submit(self, p: Params, rho0, u0, steps: int) -> int:
        jid = elmrt_server_submit(self.handle, p, rho0, u0, steps)
        self.shapes[jid] = (p.N, p.D)
        return jid

    def run(self, rounds: int = 1):
        return elmrt_server_run(self.handle, rounds)

    def job(self, jid: int):
        return elmrt_server_job(self.handle, jid)

    def result(self, jid: int):
        N, D = self.shapes[jid]
        return elmrt_server_result(self.handle, jid, N, D)

    def stats(self):
        return elmrt_server_stats(self.handle)

    def close(self):
        if self.handle:
            elmrt_server_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
