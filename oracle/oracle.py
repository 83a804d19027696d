"""Python access to the FP64 CPU oracle (``elmrt_oracle.c``).

TEST INFRASTRUCTURE ONLY: import it from the tests, from the smoke check or
from the CPU-baseline leg of the benchmark, never from the product path.  It
shares no code with the HIP library; both read their inputs from the seeded
generators in ``paper_2201_12404_amd.workloads``.

Array conventions (numpy, float64):
  * populations ``f``: shape (N, Q), cell-major, cell = x + nx*(y + ny*z);
    velocity i has c = (i%3-1, (i//3)%3-1, i//9-1) (no z for D2Q9);
  * vector fields ``u``: shape (D, N).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "elmrt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over cells)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
             "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 3),
        ("collision", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
        ("acentric", ctypes.c_double), ("Tr", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("nu_l", ctypes.c_double), ("nu_v", ctypes.c_double),
        ("rho_l", ctypes.c_double), ("rho_v", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("trace_in_s", ctypes.c_int32),
        ("phi_half_force", ctypes.c_int32),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("cells_p_above_p0", ctypes.c_int64),
        ("cells_gamma_fallback", ctypes.c_int64),
        ("min_2_over_omega_gamma", ctypes.c_double),
        ("max_2_over_omega_gamma", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
    ]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.ora_Q.argtypes = [ctypes.c_int]
        L.ora_Q.restype = ctypes.c_int
        L.ora_weights.argtypes = [ctypes.c_int, _dp]
        L.ora_product_form.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.ora_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.ora_extended_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.ora_moment_class.argtypes = [ctypes.c_int, ctypes.c_int]
        L.ora_moment_class.restype = ctypes.c_int
        L.ora_moments.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.ora_split.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.ora_collide.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp,
                                  _dp, ctypes.POINTER(ctypes.c_int)]
        L.ora_Tc.argtypes = [ctypes.c_double] * 3
        L.ora_Tc.restype = ctypes.c_double
        L.ora_alpha.argtypes = [ctypes.c_double] * 2
        L.ora_alpha.restype = ctypes.c_double
        L.ora_pressure.argtypes = [ctypes.POINTER(_Params), ctypes.c_double]
        L.ora_pressure.restype = ctypes.c_double
        L.ora_maxwell.argtypes = [ctypes.c_double] * 5 + [_dp, _dp, _dp]
        L.ora_maxwell.restype = ctypes.c_int
        L.ora_kappa_for_width.argtypes = [ctypes.c_double] * 6 + [_dp]
        L.ora_kappa_for_width.restype = ctypes.c_int
        L.ora_omega.argtypes = [ctypes.POINTER(_Params), ctypes.c_double]
        L.ora_omega.restype = ctypes.c_double
        L.ora_force_field.argtypes = [ctypes.POINTER(_Params), _dp, _dp]
        L.ora_force_field.restype = ctypes.c_int
        L.ora_init_equilibrium.argtypes = [ctypes.POINTER(_Params), _dp, _dp, _dp]
        L.ora_init_equilibrium.restype = ctypes.c_int
        L.ora_init_fluid.argtypes = [ctypes.POINTER(_Params), _dp, _dp, _dp]
        L.ora_init_fluid.restype = ctypes.c_int
        L.ora_step.argtypes = [ctypes.POINTER(_Params), _dp, ctypes.c_int64,
                               ctypes.POINTER(_Stats), _dp]
        L.ora_step.restype = ctypes.c_int
        L.ora_macros.argtypes = [ctypes.POINTER(_Params), _dp, _dp, _dp, _dp]
        L.ora_macros.restype = ctypes.c_int
        L.ora_update_cells.argtypes = [ctypes.POINTER(_Params), _dp, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64), _dp]
        L.ora_update_cells.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _vec(x, D):
    v = np.zeros(3, dtype=np.float64)
    v[:D] = np.asarray(x, dtype=np.float64)[:D]
    return v


# --------------------------------------------------------------- lattice


def Q_of(D: int) -> int:
    return 9 if D == 2 else 27


def velocities(D: int) -> np.ndarray:
    Q = Q_of(D)
    i = np.arange(Q)
    c = np.stack([i % 3 - 1, (i // 3) % 3 - 1, (i // 9) - 1 if D == 3 else 0 * i], axis=1)
    return c[:, :D].astype(np.int64)


def weights(D: int) -> np.ndarray:
    w = np.zeros(Q_of(D))
    lib().ora_weights(D, _ptr(w))
    return w


def product_form(D, rho, xi, zeta):
    out = np.zeros(Q_of(D))
    lib().ora_product_form(D, float(rho), _ptr(_vec(xi, D)), _ptr(_vec(zeta, D)), _ptr(out))
    return out


def equilibrium(D, rho, u):
    out = np.zeros(Q_of(D))
    lib().ora_equilibrium(D, float(rho), _ptr(_vec(u, D)), _ptr(out))
    return out


def extended_equilibrium(D, rho, u, F, Phi):
    out = np.zeros(Q_of(D))
    lib().ora_extended_equilibrium(D, float(rho), _ptr(_vec(u, D)), _ptr(_vec(F, D)),
                                   _ptr(_vec(Phi, D)), _ptr(out))
    return out


def moment_classes(D):
    return np.array([lib().ora_moment_class(D, k) for k in range(Q_of(D))])


def moments(D, u, f):
    a = np.zeros(Q_of(D))
    lib().ora_moments(D, _ptr(_vec(u, D)), _ptr(np.ascontiguousarray(f, dtype=np.float64)), _ptr(a))
    return a


def split(D, u, f, trace_in_s: int = 0):
    Q = Q_of(D)
    k, s, h = np.zeros(Q), np.zeros(Q), np.zeros(Q)
    lib().ora_split(D, int(trace_in_s), _ptr(_vec(u, D)), _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                    _ptr(k), _ptr(s), _ptr(h))
    return k, s, h


def collide(D, collision, omega, f, F, Phi, trace_in_s: int = 0):
    """One cell's collision; returns (post-collision populations, gamma, fell_back)."""
    out = np.zeros(Q_of(D))
    g = ctypes.c_double()
    fb = ctypes.c_int()
    lib().ora_collide(D, int(collision), int(trace_in_s), float(omega),
                      _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                      _ptr(_vec(F, D)), _ptr(_vec(Phi, D)), _ptr(out), ctypes.byref(g), ctypes.byref(fb))
    return out, g.value, bool(fb.value)


# -------------------------------------------------------- thermodynamics


def Tc(a, b, R=1.0):
    return lib().ora_Tc(a, b, R)


def alpha(acentric, Tr):
    return lib().ora_alpha(acentric, Tr)


def maxwell(a, b, R, acentric, Tr):
    """Brute-force equal-area coexistence: returns (rho_v, rho_l, p_sat)."""
    rv, rl, ps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib().ora_maxwell(a, b, R, acentric, Tr, ctypes.byref(rv), ctypes.byref(rl), ctypes.byref(ps))
    if rc != 0:
        raise ValueError(f"ora_maxwell failed ({rc}) for Tr={Tr}")
    return rv.value, rl.value, ps.value


def kappa_for_width(a, b, R, acentric, Tr, W):
    """Square-gradient kappa~ of an interface of width W (brute force)."""
    k = ctypes.c_double()
    rc = lib().ora_kappa_for_width(a, b, R, acentric, Tr, W, ctypes.byref(k))
    if rc != 0:
        raise ValueError(f"ora_kappa_for_width failed ({rc})")
    return k.value


# ------------------------------------------------------------------ grid


@dataclass
class Params:
    D: int
    n: tuple
    bc: tuple = (0, 0, 0)
    collision: int = 0          # 0 entropic, 1 BGK
    a: float = 2.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    acentric: float = 0.344
    Tr: float = 0.8
    kappa: float = 0.03
    nu_l: float = 0.02
    nu_v: float = 0.02
    rho_l: float = 0.0
    rho_v: float = 0.0
    g: tuple = (0.0, 0.0, 0.0)      # uniform body acceleration
    trace_in_h: bool = True         # reading R6; False puts the trace in s
    phi_velocity: int = 0           # reading R4: 0 bare u, 1 fluid velocity u + F/(2 rho)

    def c(self) -> _Params:
        p = _Params()
        p.D = self.D
        n = list(self.n) + [1] * (3 - len(self.n))
        bc = list(self.bc) + [0] * (3 - len(self.bc))
        for k in range(3):
            p.n[k] = int(n[k])
            p.bc[k] = int(bc[k])
        p.collision = int(self.collision)
        p.a, p.b, p.R, p.acentric, p.Tr = self.a, self.b, self.R, self.acentric, self.Tr
        p.kappa = self.kappa
        p.nu_l, p.nu_v, p.rho_l, p.rho_v = self.nu_l, self.nu_v, self.rho_l, self.rho_v
        g = list(self.g) + [0.0] * (3 - len(self.g))
        for k in range(3):
            p.g[k] = float(g[k])
        p.trace_in_s = 0 if self.trace_in_h else 1
        p.phi_half_force = int(self.phi_velocity)
        return p

    @property
    def N(self) -> int:
        n = list(self.n) + [1] * (3 - len(self.n))
        return int(n[0] * n[1] * n[2])

    @property
    def Q(self) -> int:
        return Q_of(self.D)


def pressure(p: Params, rho):
    cp = p.c()
    rho = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    return np.array([lib().ora_pressure(ctypes.byref(cp), float(r)) for r in rho])


def omega(p: Params, rho: float) -> float:
    cp = p.c()
    return lib().ora_omega(ctypes.byref(cp), float(rho))


def force_field(p: Params, rho: np.ndarray) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    assert rho.size == p.N
    F = np.zeros((p.N, 3))
    cp = p.c()
    rc = lib().ora_force_field(ctypes.byref(cp), _ptr(rho), _ptr(F))
    assert rc == 0
    return F[:, : p.D].T.copy()


def init_equilibrium(p: Params, rho0: np.ndarray, u0: np.ndarray) -> np.ndarray:
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(p.D, -1)
    f = np.zeros((p.N, p.Q))
    cp = p.c()
    rc = lib().ora_init_equilibrium(ctypes.byref(cp), _ptr(rho0), _ptr(u0), _ptr(f))
    if rc != 0:
        raise ValueError("invalid oracle parameters")
    return f


def init_fluid(p: Params, rho0: np.ndarray, u0: np.ndarray) -> np.ndarray:
    """f = f^eq at the bare velocity u0 - F(rho0)/(2 rho0): u0 is the fluid velocity."""
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(p.D, -1)
    f = np.zeros((p.N, p.Q))
    cp = p.c()
    rc = lib().ora_init_fluid(ctypes.byref(cp), _ptr(rho0), _ptr(u0), _ptr(f))
    if rc != 0:
        raise ValueError("invalid oracle parameters")
    return f


@dataclass
class Stats:
    cells_p_above_p0: int = 0
    cells_gamma_fallback: int = 0
    min_2_over_omega_gamma: float = 0.0
    max_2_over_omega_gamma: float = 0.0
    nonfinite: int = 0
    gamma: np.ndarray | None = field(default=None, repr=False)


def step(p: Params, f: np.ndarray, nsteps: int, want_gamma: bool = False) -> Stats:
    """Advance f (N, Q) in place by nsteps; returns the last step's statistics."""
    assert f.shape == (p.N, p.Q) and f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
    st = _Stats()
    g = np.zeros(p.N) if want_gamma else None
    cp = p.c()
    rc = lib().ora_step(ctypes.byref(cp), _ptr(f), int(nsteps), ctypes.byref(st),
                        _ptr(g) if g is not None else None)
    if rc != 0:
        raise RuntimeError(f"ora_step failed ({rc})")
    return Stats(st.cells_p_above_p0, st.cells_gamma_fallback, st.min_2_over_omega_gamma,
                 st.max_2_over_omega_gamma, st.nonfinite, g)


def macros(p: Params, f: np.ndarray):
    """Returns (rho (N,), u (D, N), sums[4]) with compensated sums."""
    rho = np.zeros(p.N)
    u = np.zeros((p.D, p.N))
    sums = np.zeros(4)
    cp = p.c()
    rc = lib().ora_macros(ctypes.byref(cp), _ptr(np.ascontiguousarray(f)), _ptr(rho), _ptr(u), _ptr(sums))
    assert rc == 0
    return rho, u, sums


def update_cells(p: Params, f: np.ndarray, cells) -> np.ndarray:
    """f(r, t+1) at the given cells (flat indices) from the whole field f(t)."""
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((cells.size, p.Q))
    cp = p.c()
    rc = lib().ora_update_cells(ctypes.byref(cp), _ptr(np.ascontiguousarray(f)), cells.size,
                                cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(out))
    assert rc == 0
    return out


def set_threads(n: int = 0) -> int:
    return lib().ora_set_threads(int(n))
