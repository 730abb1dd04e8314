"""Checkpoint and resume: a run saved after n1 steps and restored into a
fresh solver of the same configuration continues bit for bit as the
straight run -- fields and the probe records after the checkpoint -- for
FP32 and FP16 storage (the scales are part of the state), with CPML layers
(the psi state is part of it), across a block boundary that is not a
multiple of T; a state does not load into a solver of another shape."""
import numpy as np
import pytest

from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def _wl(storage=W.FP32, cpml=None, seed=4280):
    wl = W.spheres(90, 70, 60, 8, 50, seed=seed, n_sources=3, n_probes=12, rmin=3, rmax=9, name="ckpt",
                   storage=storage)
    wl.waveforms = np.random.default_rng(seed).standard_normal(wl.waveforms.shape)
    wl.cpml = cpml
    return wl


def _assert_same(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


@pytest.mark.parametrize("storage,kernel,T,layers", [(W.FP32, fdtd.KERNEL_FUSED, 4, None),
                                                     (W.FP16, fdtd.KERNEL_FUSED, 3, None),
                                                     (W.FP32, fdtd.KERNEL_AUTO, 0,
                                                      dict(thickness=5, order=3, sigma_factor=1.0, kappa_max=4.0,
                                                           alpha_max=0.05))])
def test_resume_equals_straight_run(storage, kernel, T, layers):
    wl = _wl(storage, layers)
    print(f"checkpoint storage={storage} kernel={kernel} T={T} layers={bool(layers)}", flush=True)
    straight = fdtd.Solver.from_workload(wl, kernel=kernel, time_block=T)
    try:
        # the same step calls as the checkpointed run: 16-bit storage re-encodes
        # at the end of every call
        straight.step(23)
        straight.step(27)
        f_ref, p_ref = straight.read_fields(), straight.read_probes(0, 50)
    finally:
        straight.close()
    first = fdtd.Solver.from_workload(wl, kernel=kernel, time_block=T)
    try:
        first.step(23)                       # not a multiple of T: the state sits mid-block
        state = first.save_state()
        first.step(5)                        # work after the checkpoint is not in it
    finally:
        first.close()
    second = fdtd.Solver.from_workload(wl, kernel=kernel, time_block=T)
    try:
        second.load_state(state)
        assert second.steps_done() == 23
        second.step(27)
        f, p = second.read_fields(), second.read_probes(23, 27)
        assert np.all(second.read_probes(0, 23) == 0.0)
    finally:
        second.close()
    _assert_same(f, f_ref, "fields")
    _assert_same(p, p_ref[23:], "probes")


def test_state_does_not_load_into_another_configuration():
    a = fdtd.Solver.from_workload(_wl())
    b = fdtd.Solver.from_workload(W.spheres(91, 70, 60, 8, 50, seed=1, n_sources=1, n_probes=2, rmin=3, rmax=9))
    c = fdtd.Solver.from_workload(_wl(W.FP16))
    try:
        state = a.save_state()
        for other in (b, c):
            with pytest.raises(fdtd.FdtdError) as e:
                other.load_state(state)
            assert e.value.code == fdtd.EINVAL
        with pytest.raises(fdtd.FdtdError):
            a.load_state(state[:100])
    finally:
        a.close()
        b.close()
        c.close()


def test_rewind_clears_probe_rows_written_by_a_later_history():
    """Save at step 10 of a run from zero fields, perturb the whole state and
    step on (every probe row from 10 on gets a nonzero value), then restore
    the step-10 state and step again with the zero-tile skip on: probes in
    tiles the field has not reached are never written by the replayed run,
    so their rows must read 0 again -- the oracle's record of the same run."""
    from tests.test_gpu_zero_skip import spreading
    wl = spreading(n_steps=40)
    print("checkpoint rewind over written probe rows, 200x120x150, skip on", flush=True)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=4)
    try:
        s.set_zero_skip(True)
        s.step(10)
        state = s.save_state()
        rng = np.random.default_rng(77)
        s.set_fields(rng.standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1)).astype(np.float32))
        s.step(30)
        s.synchronize()
        assert np.count_nonzero(s.read_probes(10, 30)) == 30 * len(wl.probes)
        s.load_state(state)
        s.step(30)
        f, p = s.read_fields(), s.read_probes(0, 40)
    finally:
        s.close()
    fo, po = G.oracle_f32(wl, 40)
    assert np.count_nonzero(po[39] == 0.0) > 0          # some probes are still out of the field's reach
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
