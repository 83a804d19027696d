"""CPU checks of the C ABI library: it loads, exports every symbol the header
declares, and its host-only calls (workspace size, validation, coexistence,
velocity table) behave as documented.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2201_12404_amd import elmrt as E
from paper_2201_12404_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "elmrt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(elmrt_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    names = _declared_functions()
    assert "elmrt_create" in names and "elmrt_step" in names and "elmrt_read_macros" in names
    lib = ctypes.CDLL(E.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps every declared function under the same name
    for n in names:
        assert n in E._SIGS, n
        assert hasattr(E, n), n


def test_params_struct_size_matches_header():
    # layout from the header: u32, 3 x i32, 3 x i64, 3 x i32, i32, 10 x f64,
    # 3 x f64 (body acceleration), f64 (target width); the library itself
    # rejects a struct_size other than its sizeof
    assert ctypes.sizeof(E.elmrt_params) == 4 + 12 + 24 + 12 + 4 + 10 * 8 + 3 * 8 + 8
    E.elmrt_workspace_bytes(E.Params(lattice=0, n=(8, 8, 1)))


@pytest.mark.parametrize("w", [W.STATIC_DROP_FP64, W.IMPACT_2D, W.IMPACT_3D])
def test_workspace_bytes(w):
    p = E.params_for(w)
    nb = E.elmrt_workspace_bytes(p)
    es = 8 if w.precision == 1 else 4
    Q = 9 if w.D == 2 else 27
    assert nb >= (2 * Q + 1 + w.D) * w.N * es
    assert nb <= (2 * Q + 1 + w.D) * w.N * es + 128 * 1024


@pytest.mark.parametrize("change,msg", [
    (dict(lattice=7), "lattice"),
    (dict(precision=3), "precision"),
    (dict(collision=2), "collision"),
    (dict(n=(3, 16, 1)), "extent"),
    (dict(n=(16, 16, 2)), "n[2]"),
    (dict(T_over_Tc=1.0), "T/Tc"),
    (dict(eos_b=0.0), "EOS"),
    (dict(kappa_tilde=-1.0), "kappa"),
    (dict(nu_liquid=0.0), "viscosities"),
    (dict(nu_liquid=0.01, nu_vapour=0.1, rho_liquid=0.1, rho_vapour=1.0), "rho_liquid"),
    (dict(bc=(2, 0, 0)), "bc"),
    (dict(body_accel=(0.0, 0.0, 1e-5)), "body_accel"),
    (dict(body_accel=(float("nan"), 0.0, 0.0)), "body_accel"),
    (dict(target_W=-1.0), "target_W"),
    (dict(target_W=5.0, kappa_tilde=0.01), "not both"),
])
def test_invalid_params_rejected(change, msg):
    base = dict(lattice=E.ELMRT_D2Q9, n=(16, 16, 1))
    base.update(change)
    p = E.Params(**base)
    with pytest.raises(E.ElmrtError) as ei:
        E.elmrt_workspace_bytes(p)
    assert ei.value.status == E.ELMRT_E_INVALID
    assert msg in E.elmrt_last_error()


def test_cells_limit():
    p = E.Params(lattice=E.ELMRT_D3Q27, n=(2048, 1024, 1024))
    with pytest.raises(E.ElmrtError):
        E.elmrt_workspace_bytes(p)


@pytest.mark.parametrize("key", list(W.COEX.keys()))
def test_coexistence_matches_oracle_and_workload_table(key):
    """The library's Maxwell solver (closed-form antiderivative) agrees with
    the oracle's brute-force equal-area construction and with the densities
    the workloads use."""
    eos = W.EOS_A if key[0] == "A" else W.EOS_B
    p = E.Params(lattice=0, n=(16, 16, 1), T_over_Tc=key[1], **eos)
    rv, rl, ps = E.elmrt_coexistence(p)
    orv, orl, ops = O.maxwell(eos["eos_a"], eos["eos_b"], eos["eos_R"], eos["acentric"], key[1])
    assert abs(rv / orv - 1) < 1e-9 and abs(rl / orl - 1) < 1e-11 and abs(ps / ops - 1) < 1e-8
    wrv, wrl = W.COEX[key]
    assert abs(rv / wrv - 1) < 1e-9 and abs(rl / wrl - 1) < 1e-11


def test_velocity_tables():
    for lat, D in ((E.ELMRT_D2Q9, 2), (E.ELMRT_D3Q27, 3)):
        c = E.elmrt_velocities(lat)
        assert c.shape == (3 ** D, 3)
        assert len({tuple(v) for v in c}) == 3 ** D
        assert np.all(np.abs(c) <= 1)
        if D == 2:
            assert np.all(c[:, 2] == 0)
        # opposite of i is Q-1-i
        np.testing.assert_array_equal(c[::-1], -c)
    with pytest.raises(E.ElmrtError):
        E.elmrt_velocities(5)


def test_no_cpu_fallback_in_product_package():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2201_12404_amd")
    for dp, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dp, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, fn
                assert "elmrt_oracle" not in txt, fn


def test_batch_workspace_bytes():
    assert E.elmrt_batch_workspace_bytes(1) >= 128
    assert E.elmrt_batch_workspace_bytes(64) >= 64 * 128
    assert E.elmrt_batch_workspace_bytes(64) % 256 == 0
    with pytest.raises(E.ElmrtError):
        E.elmrt_batch_workspace_bytes(0)


def test_batch_create_rejects_bad_arguments_without_a_device():
    # every argument check precedes any device call
    with pytest.raises(E.ElmrtError, match="no sims"):
        E.elmrt_batch_create([], 256, 1 << 20)
    with pytest.raises(E.ElmrtError, match="aligned"):
        E.elmrt_batch_create([1], 8, 1 << 20)


def test_plane_block_limit():
    # Q x cells per plane x value size must stay below 2^31 bytes
    p = E.Params(lattice=1, n=(5000, 5000, 4), precision=1, bc=(0, 0, 1))
    with pytest.raises(E.ElmrtError, match="plane block"):
        E.elmrt_workspace_bytes(p)


def test_server_create_rejects_bad_arguments_without_a_device():
    with pytest.raises(E.ElmrtError, match="aligned"):
        E.elmrt_server_create(0, 1 << 20, 0, 10)
    with pytest.raises(E.ElmrtError, match="chunk"):
        E.elmrt_server_create(256, 1 << 20, 0, 0)


def test_null_handles_rejected_without_a_device():
    """Every entry point that takes a handle refuses NULL with
    ELMRT_E_INVALID before touching the device."""
    L = E.lib()
    null = ctypes.c_void_p(0)
    i64, i32, sz, u32 = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_uint32()
    d = np.zeros(4)
    calls = {
        "elmrt_step": lambda: L.elmrt_step(null, 1),
        "elmrt_set_tiling": lambda: L.elmrt_set_tiling(null, 64, 1, 0),
        "elmrt_get_tiling": lambda: L.elmrt_get_tiling(null, None, None, None),
        "elmrt_set_stream": lambda: L.elmrt_set_stream(null, null),
        "elmrt_autotune": lambda: L.elmrt_autotune(null, 2, ctypes.byref(i64)),
        "elmrt_gamma_fallbacks": lambda: L.elmrt_gamma_fallbacks(null, ctypes.byref(i64)),
        "elmrt_poll_unstable": lambda: L.elmrt_poll_unstable(null, ctypes.byref(u32)),
        "elmrt_state_bytes": lambda: L.elmrt_state_bytes(null, ctypes.byref(sz)),
        "elmrt_save_state": lambda: L.elmrt_save_state(null, null, 0),
        "elmrt_load_state": lambda: L.elmrt_load_state(null, null, 0),
        "elmrt_read_macros": lambda: L.elmrt_read_macros(null, None, None, None),
        "elmrt_batch_step": lambda: L.elmrt_batch_step(null, 1),
        "elmrt_batch_autotune": lambda: L.elmrt_batch_autotune(null, 2, ctypes.byref(i64)),
        "elmrt_server_run": lambda: L.elmrt_server_run(null, 1, ctypes.byref(i32), ctypes.byref(i32)),
        "elmrt_server_stats": lambda: L.elmrt_server_stats(null, ctypes.byref(i64), ctypes.byref(sz)),
    }
    for name, call in calls.items():
        assert call() == E.ELMRT_E_INVALID, name


def test_unknown_readings_rejected():
    p = E.Params(lattice=0, n=(16, 16, 1)).c()
    p.readings = 4
    out = ctypes.c_size_t()
    assert E.lib().elmrt_workspace_bytes(ctypes.byref(p), ctypes.byref(out)) == E.ELMRT_E_INVALID
    assert "readings" in E.elmrt_last_error()


@pytest.mark.parametrize("tr", [0.592454, 0.7, 0.8, 0.9])
@pytest.mark.parametrize("eos", [W.EOS_A, W.EOS_B])
def test_kappa_for_width_matches_oracle(tr, eos):
    """The library's kappa~(W) (closed-form antiderivative of P/rho^2, golden
    section on the potential's peak) against the oracle's (Simpson
    quadrature, scan), host FP64."""
    p = E.Params(lattice=0, n=(16, 16, 1), T_over_Tc=tr, **eos)
    for Wd in (5.0, 12.0):
        k_lib = E.elmrt_kappa_for_width(p, Wd)
        k_ora = O.kappa_for_width(eos["eos_a"], eos["eos_b"], eos["eos_R"], eos["acentric"], tr, Wd)
        assert abs(k_lib / k_ora - 1) < 1e-7, (k_lib, k_ora)
    with pytest.raises(E.ElmrtError):
        E.elmrt_kappa_for_width(p, 0.0)
