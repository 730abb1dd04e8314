"""fdtd_tune_time_block: T = 3, 4, 5 measured on the solver itself, the
fastest kept.  FP32 results do not depend on T, so the tuned run -- the
tuning steps included -- stays bit-exact with the oracle; the rules of the
entry point."""
import pytest

from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G
from tests.test_gpu_parity import ragged

pytestmark = pytest.mark.gpu


def test_tuned_run_is_bitexact_and_keeps_the_fastest_T():
    wl = ragged(n_steps=40)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=0)
    try:
        print("tune T on 131x75x50 over 9 steps each, then 6 more steps", flush=True)
        T, ns = s.tune_time_block(9)
        # an untimed block and the largest multiple of T up to 9 for each T
        assert s.steps_done() == (3 + 9) + (4 + 8) + (5 + 5)
        assert T in (3, 4, 5) and s.time_block == T
        assert all(v > 0 for v in ns.values()) and ns[T] == min(ns.values())
        s.step(6)
        f, p = s.read_fields(), s.read_probes(0, 40)
    finally:
        s.close()
    fo, po = G.oracle_f32(wl, 40)
    assert G.first_mismatch(f, fo) is None
    assert G.first_mismatch(p, po) is None


def test_tune_time_block_rules():
    wl = W.spheres(30, 24, 20, 2, 10, seed=5, n_sources=1, n_probes=2, rmin=2, rmax=4, name="e")
    cases = []
    s16 = fdtd.Solver.from_workload(wl, storage=W.FP16)
    cases.append((s16, lambda s: s.tune_time_block(4)))                 # T changes 16-bit results
    sp = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_PLAIN)
    cases.append((sp, lambda s: s.tune_time_block(4)))
    sl = fdtd.Solver.from_workload(wl)
    sl.set_cpml(3)
    cases.append((sl, lambda s: s.tune_time_block(4)))
    se = fdtd.Solver.from_workload(wl)
    se.set_energy_trace(2)
    cases.append((se, lambda s: s.tune_time_block(4)))
    s0 = fdtd.Solver.from_workload(wl)
    cases.append((s0, lambda s: s.tune_time_block(0)))
    try:
        for s, call in cases:
            with pytest.raises(fdtd.FdtdError) as e:
                call(s)
            assert e.value.code == fdtd.EINVAL
            assert s.steps_done() == 0
    finally:
        for s, _ in cases:
            s.close()
