"""C-ABI checks that need no GPU: the library loads, exports every function
include/fdtd.h declares, validates its arguments before touching a device,
and derives the same FP32 coefficients as the oracle (FP64, rounded once)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "fdtd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdtd_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = _declared()
    assert len(names) >= 15
    L = fdtd.lib()
    for n in names:
        assert hasattr(L, n), n


def test_workspace_bytes():
    assert fdtd.workspace_bytes(1, 4, 4) == 0
    assert fdtd.workspace_bytes(4, 4, 4, 7) == 0
    b32 = fdtd.workspace_bytes(256, 256, 256, W.FP32)
    b16 = fdtd.workspace_bytes(256, 256, 256, W.FP16)
    assert b32 > 2 * 6 * 4 * 257 ** 3 and b16 < b32
    assert b32 % 256 == 0


def _create(nx=8, ny=8, nz=8, d=1e-3, dt=None, eps=(1.0,), sig=(0.0,), mu=None, mat=None, storage=0):
    arr, n = fdtd._materials(eps, sig, mu)
    dt = W.courant_dt(d, d, d) if dt is None else dt
    h = C.c_void_p()
    mptr = None if mat is None else np.ascontiguousarray(mat, np.uint8).ctypes.data
    rc = fdtd.lib().fdtd_create(C.byref(h), nx, ny, nz, d, d, d, dt, arr, n, mptr, storage, None, 0, None)
    return rc


def test_create_rejects_before_touching_the_device():
    d = 1e-3
    limit = 1.0 / (W.C0 * np.sqrt(3.0 / d ** 2))
    assert _create(dt=limit * 1.0001) == fdtd.ECFL
    assert "Courant" in fdtd.lib().fdtd_last_error().decode()
    assert _create(nx=1) == fdtd.EINVAL
    assert _create(mu=(2.0,)) == fdtd.EINVAL
    assert _create(eps=(0.0,)) == fdtd.EINVAL
    assert _create(sig=(-1.0,)) == fdtd.EINVAL
    assert _create(storage=3) == fdtd.EINVAL
    bad = np.zeros((8, 8, 8), np.uint8)
    bad[3, 2, 1] = 1                      # only one material in the table
    assert _create(mat=bad) == fdtd.EINVAL
    assert "material index" in fdtd.lib().fdtd_last_error().decode()


def test_coefficients_match_oracle_rounded_once():
    rng = np.random.default_rng(0)
    eps = np.concatenate([[1.0], rng.uniform(1, 12, 255)])
    sig = np.concatenate([[0.0], rng.uniform(0, 0.05, 255)])
    for d in [(1e-3, 1e-3, 1e-3), (1e-3, 1.3e-3, 0.7e-3)]:
        dt = W.courant_dt(*d)
        ours, ch = fdtd.coefficients(eps, sig, *d, dt)
        ref, ref_ch = oracle.coefficients(eps, sig, dt, *d)
        assert np.array_equal(ours, ref.astype(np.float32))
        assert np.array_equal(ch, ref_ch.astype(np.float32))


def test_graded_coefficients_match_oracle_rounded_once():
    rng = np.random.default_rng(1)
    eps = np.concatenate([[1.0], rng.uniform(1, 12, 15)])
    sig = np.concatenate([[0.0], rng.uniform(0, 0.05, 15)])
    sx, sy, sz = (rng.uniform(0.4e-3, 2e-3, n) for n in (9, 5, 7))
    dt = W.courant_dt_graded(sx, sy, sz)
    cag, gc = fdtd.graded_coefficients(eps, sig, sx, sy, sz, dt)
    ref_cag, ref_hc, ref_ec = oracle.graded_coefficients(eps, sig, dt, sx, sy, sz)
    assert np.array_equal(cag, ref_cag.astype(np.float32))
    assert np.array_equal(gc[:, 0], ref_hc.astype(np.float32))
    assert np.array_equal(gc[:, 1], ref_ec.astype(np.float32))


def test_graded_coefficients_reject_bad_sizes():
    sx = np.full(4, 1e-3)
    bad = sx.copy()
    bad[2] = 0.0
    with pytest.raises(fdtd.FdtdError) as e:
        fdtd.graded_coefficients([1.0], [0.0], bad, sx, sx, 1e-12)
    assert e.value.code == fdtd.EINVAL


def test_cpml_coefficients_match_oracle_rounded_once():
    rng = np.random.default_rng(2)
    eps = np.concatenate([[1.0], rng.uniform(1, 12, 7)])
    sig = np.concatenate([[0.0], rng.uniform(0, 0.05, 7)])
    sx, sy, sz = (rng.uniform(0.5e-3, 1.5e-3, n) for n in (21, 17, 25))
    dt = W.courant_dt_graded(sx, sy, sz)
    for layer in [dict(thickness=5, order=3, sigma_factor=1.0, kappa_max=5.0, alpha_max=0.05),
                  dict(thickness=8, order=4, sigma_factor=0.7, kappa_max=1.0, alpha_max=0.0)]:
        cag, gc, cp = fdtd.cpml_coefficients(eps, sig, sx, sy, sz, dt, **layer)
        r_cag, r_hc, r_ec, r_cp = oracle.cpml_coefficients(eps, sig, dt, sx, sy, sz, **layer)
        assert np.array_equal(cag, r_cag.astype(np.float32))
        assert np.array_equal(gc[:, 0], r_hc.astype(np.float32))
        assert np.array_equal(gc[:, 1], r_ec.astype(np.float32))
        assert np.array_equal(cp, r_cp.astype(np.float32))


def test_cpml_coefficients_reject_bad_layers():
    s = np.full(10, 1e-3)
    for bad in [dict(thickness=5), dict(thickness=2, order=0), dict(thickness=2, kappa_max=0.5),
                dict(thickness=2, alpha_max=-1.0), dict(thickness=0)]:
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.cpml_coefficients([1.0], [0.0], s, s, s, 1e-12, **bad)
        assert e.value.code == fdtd.EINVAL


def test_perfect_conductor_entries_are_zero_and_match_oracle():
    inf = float("inf")
    eps, sig = np.array([1.0, 4.0, 2.0]), np.array([0.0, inf, 0.01])
    ours, ch = fdtd.coefficients(eps, sig, 1e-3, 1.1e-3, 0.9e-3, 1.5e-12)
    ref, _ = oracle.coefficients(eps, sig, 1.5e-12, 1e-3, 1.1e-3, 0.9e-3)
    assert np.array_equal(ours, ref.astype(np.float32)) and np.all(ours[1] == 0.0)
    s = np.full(6, 1e-3)
    cag, _ = fdtd.graded_coefficients(eps, sig, s, s, s, 1.5e-12)
    r_cag, _, _ = oracle.graded_coefficients(eps, sig, 1.5e-12, s, s, s)
    assert np.array_equal(cag, r_cag.astype(np.float32)) and np.all(cag[1] == 0.0)
    with pytest.raises(fdtd.FdtdError):
        fdtd.coefficients([inf], [0.0], 1e-3, 1e-3, 1e-3, 1.5e-12)      # eps_r must be finite


def test_tile_stats_rejects_null():
    import ctypes as C
    a, b = C.c_longlong(), C.c_longlong()
    assert fdtd.lib().fdtd_tile_stats(None, C.byref(a), C.byref(b)) == fdtd.EINVAL


def test_time_block_rejects_null():
    t = C.c_int()
    assert fdtd.lib().fdtd_time_block(None, C.byref(t)) == fdtd.EINVAL


def test_tune_time_block_rejects_null():
    t = C.c_int()
    assert fdtd.lib().fdtd_tune_time_block(None, 10, C.byref(t), None) == fdtd.EINVAL
