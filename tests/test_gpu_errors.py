"""Error paths of the C ABI that need a created solver.  Every condition is
forced from the host; no kernel is made to fault."""
import ctypes as C

import numpy as np
import pytest

from paper_1301_4539_amd import fdtd, workload as W

pytestmark = pytest.mark.gpu


def _solver(storage=W.FP32, n=(12, 10, 9)):
    wl = W.spheres(*n, 2, 10, seed=3, n_sources=0, n_probes=0, rmin=1, rmax=3, storage=storage)
    return wl, fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=2)


def _code(fn, *a):
    with pytest.raises(fdtd.FdtdError) as e:
        fn(*a)
    return e.value.code


def test_source_and_probe_validation():
    wl, s = _solver()
    try:
        w = np.ones(5, np.float32)
        assert _code(s.add_source, 2, 0, 3, 3, w) == fdtd.EINVAL      # Ez on the x=0 wall (PEC)
        assert _code(s.add_source, 0, 3, 0, 3, w) == fdtd.EINVAL      # Ex on the y=0 wall
        assert _code(s.add_source, 3, 3, 3, 3, w) == fdtd.EINVAL      # H component
        assert _code(s.add_probe, 0, wl.nx, 3, 3) == fdtd.EINVAL      # Ex has i < nx
        assert _code(s.add_probe, 7, 1, 1, 1) == fdtd.EINVAL          # no component 7
        assert s.add_source(2, 3, 3, 3, w) == 0
        assert s.add_probe(5, 3, 3, 3) == 0
        s.step(3)
        assert _code(s.add_probe, 1, 2, 2, 2) == fdtd.ESTATE          # probes before stepping only
        assert _code(s.read_probes, 0, 4) == fdtd.EINVAL              # step 3 not run yet
        assert s.read_probes(0, 3).shape == (3, 1)
        assert _code(s.set_tiling, 4, 0) == fdtd.EINVAL
        assert _code(s.set_kernel, fdtd.KERNEL_FUSED, 7) == fdtd.EINVAL      # T = 1..6
    finally:
        s.close()


def test_plain_kernel_needs_fp32():
    _, s = _solver(W.FP16)
    try:
        assert _code(s.set_kernel, fdtd.KERNEL_PLAIN, 1) == fdtd.EINVAL
    finally:
        s.close()


def test_workspace_too_small_or_misaligned():
    import torch
    wl, _s = _solver()
    _s.close()
    need = fdtd.workspace_bytes(wl.nx, wl.ny, wl.nz, W.FP32)
    buf = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    arr, n = fdtd._materials(wl.eps_r, wl.sigma)
    for ptr, size in ((buf.data_ptr(), need - 256), (buf.data_ptr() + 4, need)):
        h = C.c_void_p()
        rc = fdtd.lib().fdtd_create(C.byref(h), wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.dt, arr, n, None,
                                    W.FP32, C.c_void_p(ptr), size, None)
        assert rc == fdtd.ENOMEM


def test_caller_workspace_equals_library_allocation():
    wl = W.spheres(30, 20, 25, 4, 16, seed=8, n_sources=1, n_probes=3, rmin=2, rmax=5)
    outs = []
    for torch_ws in (True, False):
        s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=4, torch_workspace=torch_ws)
        try:
            s.step(16)
            outs.append(s.read_fields())
        finally:
            s.close()
    assert np.array_equal(outs[0], outs[1])


def _overflowing_state(wl):
    """Hx of order 1 next to an Ez whose largest value is 1e-6: Ez's scale
    leaves it no room for the curl of Hx within one block."""
    f = np.zeros((6, wl.nz + 1, wl.ny + 1, wl.nx + 1), np.float32)
    f[3, 3:5, 3:5, 3:6] = 1.0            # Hx
    f[2, 2, 2, 2] = 1e-6                 # Ez maximum 1e-6 -> large scale
    return f


def test_fp16_overflow_block_rerun_bitexact_with_oracle():
    """A component scaled for a tiny maximum and then driven hard within one
    block would overflow binary16: the block runs again from its input with
    that component's scale taken from the block's own maximum (the oracle's
    overflow retry), bit for bit, and nothing is reported."""
    import oracle
    from tests import gpu_helpers as G
    wl, s = _solver(W.FP16)
    f = _overflowing_state(wl)
    try:
        s.set_fields(f)
        s.step(2)
        s.step(3)
        s.synchronize()                    # no FDTD_ERANGE
        got = s.read_fields()
        scales, sat = s.storage_state()
    finally:
        s.close()
    prob = oracle.Problem.from_workload(wl)
    ref = G.pec_clean(wl, f)
    st = prob.quantize_upload(ref, W.FP16)
    rule = oracle.choose_scales(st["m_stored"], prob.a_max)
    prob.run_q(ref, 0, 2, W.FP16, 2, st)
    assert st["scales"][2] < rule[2] - 6          # the first block was re-run with a new Ez scale
    prob.run_q(ref, 2, 3, W.FP16, 2, st)
    assert not sat and not st["flag"][0]
    assert scales == list(st["scales"])
    assert G.first_mismatch(got, ref) is None, G.first_mismatch(got, ref)


def test_fp16_overflow_rerun_in_a_batch():
    """The same in a batched launch beside a solve that does not overflow:
    only the overflowing solve's block runs again; both equal the oracle."""
    import oracle
    from tests import gpu_helpers as G
    wl, a = _solver(W.FP16)
    wl2 = W.spheres(20, 14, 11, 3, 12, seed=9, n_sources=1, n_probes=2, rmin=1, rmax=3, storage=W.FP16)
    b = fdtd.Solver.from_workload(wl2, kernel=fdtd.KERNEL_FUSED, time_block=2)
    f = _overflowing_state(wl)
    try:
        a.set_fields(f)
        fdtd.step_batch([a, b], [4, 4])
        a.synchronize()
        b.synchronize()
        got_a, got_b = a.read_fields(), b.read_fields()
    finally:
        a.close()
        b.close()
    prob = oracle.Problem.from_workload(wl)
    ref = G.pec_clean(wl, f)
    st = prob.quantize_upload(ref, W.FP16)
    prob.run_q(ref, 0, 4, W.FP16, 2, st)
    ref_b, _, st_b = G.oracle_q(wl2, 4, W.FP16, 2)
    assert not st["flag"][0] and not st_b["flag"][0]
    assert G.first_mismatch(got_a, ref) is None, G.first_mismatch(got_a, ref)
    assert G.first_mismatch(got_b, ref_b) is None, G.first_mismatch(got_b, ref_b)


def test_value_beyond_the_format_reported_as_erange():
    """A value that binary16 cannot hold at any scale (1e25 > 65504 x 2^64)
    is stored saturated and reported: fdtd_synchronize gives FDTD_ERANGE."""
    wl, s = _solver(W.FP16)
    try:
        f = _overflowing_state(wl)
        f[3, 3, 3, 3] = 1e25
        s.set_fields(f)
        s.step(2)
        assert _code(s.synchronize) == fdtd.ERANGE
        scales, sat = s.storage_state()
        assert sat
    finally:
        s.close()
