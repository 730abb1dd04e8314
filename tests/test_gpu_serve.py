"""Serving on the GPU: requests that arrive while others run are admitted and
batched; each result equals the same solve run alone, bit for bit (FP32 and
FP16 storage; the engine's chunks are multiples of T)."""
import numpy as np
import pytest

from paper_1301_4539_amd import fdtd, serve, workload as W

pytestmark = pytest.mark.gpu


def test_serving_mix_equals_alone():
    reqs = W.serving_requests(n=10, rate=200.0, seed=77, dim_lo=24, dim_hi=72, steps_lo=40, steps_hi=160)
    wls = {r.rid: r.workload() for r in reqs}
    eng = serve.Engine(serve.GpuBackend(wls), budget_bytes=1 << 30, max_slots=6, chunk=24)
    rep = eng.run(reqs)
    assert not rep.rejected
    s = rep.summary()
    assert s["requests"] == len(reqs) and s["p99_s"] >= s["p50_s"] > 0
    assert any(r.storage == W.FP16 for r in reqs) and any(r.storage == W.FP32 for r in reqs)
    for r in rep.records:
        wl = wls[r.rid]
        solo = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=serve.DEFAULT_T[wl.storage])
        try:
            solo.step(wl.n_steps)
            ref = solo.read_probes(0, wl.n_steps)
        finally:
            solo.close()
        assert r.probes.shape == ref.shape
        assert np.array_equal(r.probes, ref), f"request {r.rid} differs from its solo run"
        assert np.max(np.abs(ref)) > 0
