"""Batched (multi-grid, persistent) launches: every solve in a mix gives
bit-for-bit the result it gives alone, and the oracle's (FP32 operation
order for FP32 storage, the 16-bit emulation on the same call schedule for
FP16 storage)."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def _mix():
    specs = [((40, 33, 29), W.FP32, 30), ((70, 48, 35), W.FP32, 23), ((31, 64, 20), W.FP16, 30),
             ((55, 21, 47), W.FP32, 17), ((64, 64, 64), W.FP16, 26), ((24, 24, 90), W.FP32, 30)]
    out = []
    for q, (n, st, steps) in enumerate(specs):
        wl = W.spheres(*n, 5, steps, seed=900 + q, n_sources=1, n_probes=6, rmin=2, rmax=6,
                       name=f"mix{q}", storage=st)
        wl.waveforms = np.random.default_rng(q).standard_normal(wl.waveforms.shape)
        out.append(wl)
    return out


def _solve_alone(wl, T, chunks):
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T)
    try:
        for c in chunks:
            s.step(c)
        return s.read_fields(), s.read_probes(0, wl.n_steps)
    finally:
        s.close()


@pytest.mark.parametrize("T", [2, 4])
def test_batch_equals_alone_and_oracle(T):
    wls = _mix()
    solvers = [fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T) for wl in wls]
    try:
        # continuous batching: solves join and leave between calls, with
        # chunks that are not multiples of T
        left = [wl.n_steps for wl in wls]
        calls = [[] for _ in wls]
        active = [0, 1, 2]
        rounds = 0
        while any(left):
            chunk = [min(left[i], 7 + (rounds % 3)) for i in active]
            fdtd.step_batch([solvers[i] for i in active], chunk)
            for i, c in zip(active, chunk):
                left[i] -= c
                calls[i].append(c)
            rounds += 1
            if rounds == 2:
                active += [3, 4, 5]
            active = [i for i in active if left[i] > 0]
        got = [(s.read_fields(), s.read_probes(0, wl.n_steps)) for s, wl in zip(solvers, wls)]
    finally:
        for s in solvers:
            s.close()
    for q, (wl, (f, p)) in enumerate(zip(wls, got)):
        # the same call schedule alone (reduced storage re-encodes at the end
        # of every call, so the schedule is part of the result)
        fa, pa = _solve_alone(wl, T, calls[q])
        assert G.first_mismatch(f, fa) is None, f"{wl.name} fields, batch vs alone: {G.first_mismatch(f, fa)}"
        assert G.first_mismatch(p, pa) is None, f"{wl.name} probes, batch vs alone: {G.first_mismatch(p, pa)}"
        if wl.storage == W.FP32:
            fo, po = G.oracle_f32(wl, wl.n_steps)
        else:
            # the emulation, called with the batch's schedule: blocks end at
            # absolute multiples of T and at the end of every call
            prob = oracle.Problem.from_workload(wl)
            fo = G.pec_clean(wl, G.init32(wl))
            st = prob.quantize_upload(fo, wl.storage)
            s0, rows = 0, []
            for c in calls[q]:
                rows.append(prob.run_q(fo, s0, c, wl.storage, T, st))
                s0 += c
            po = np.concatenate(rows, axis=0)
            assert not st["flag"][0]
        assert G.first_mismatch(f, fo) is None, f"{wl.name} fields vs oracle: {G.first_mismatch(f, fo)}"
        assert G.first_mismatch(p, po) is None, f"{wl.name} probes vs oracle: {G.first_mismatch(p, po)}"


def test_aligned_batches_equal_one_call_alone():
    """With chunks that are multiples of T (what the serving engine issues),
    reduced storage gives the same result as one fdtd_step call alone."""
    T = 4
    wls = [wl for wl in _mix() if wl.storage == W.FP16]
    solvers = [fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T) for wl in wls]
    try:
        left = [wl.n_steps for wl in wls]
        while any(left):
            act = [i for i in range(len(wls)) if left[i] > 0]
            ch = [min(left[i], 8) for i in act]
            fdtd.step_batch([solvers[i] for i in act], ch)
            for i, c in zip(act, ch):
                left[i] -= c
        got = [s.read_fields() for s in solvers]
    finally:
        for s in solvers:
            s.close()
    for wl, f in zip(wls, got):
        fa, _ = _solve_alone(wl, T, [wl.n_steps])
        assert G.first_mismatch(f, fa) is None, wl.name


def test_batch_rejects_bad_input():
    wl = _mix()[0]
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=2)
    try:
        with pytest.raises(fdtd.FdtdError):
            fdtd.step_batch([s, s], [1, 1])
        with pytest.raises(fdtd.FdtdError):
            fdtd.step_batch([s], [-1])
        s.set_kernel(fdtd.KERNEL_PLAIN, 1)
        with pytest.raises(fdtd.FdtdError):
            fdtd.step_batch([s], [2])
    finally:
        s.close()
