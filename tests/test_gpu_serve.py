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


def test_serving_graded_cpml_and_conductor_requests():
    """Requests the batched launches do not take (graded sizes, CPML layers)
    are stepped alone inside the same ticks; a perfect-conductor request is
    batched like the rest.  Each result equals its solo run bit for bit."""
    reqs = W.serving_requests(n=8, rate=200.0, seed=78, dim_lo=24, dim_hi=64, steps_lo=40, steps_hi=120)
    wls = {r.rid: r.workload() for r in reqs}
    fp32 = [r.rid for r in reqs if r.storage == W.FP32]
    assert len(fp32) >= 1
    rng = np.random.default_rng(78)
    g = wls[reqs[0].rid if reqs[0].rid != fp32[-1] else reqs[1].rid]
    g.spacing = tuple(rng.uniform(0.6e-3, 1.4e-3, n) for n in (g.nx, g.ny, g.nz))
    g.dt = W.courant_dt_graded(*g.spacing)
    c = wls[fp32[-1]]
    c.cpml = dict(thickness=4, order=3, sigma_factor=1.0, kappa_max=3.0, alpha_max=0.05)
    p = next(wls[r.rid] for r in reqs if wls[r.rid] is not g and wls[r.rid] is not c)
    p.eps_r, p.mu_r, p.sigma = np.append(p.eps_r, 1.0), np.append(p.mu_r, 1.0), np.append(p.sigma, np.inf)
    p.mat[:, :, -6:] = len(p.sigma) - 1
    backend = serve.GpuBackend(wls)
    eng = serve.Engine(backend, budget_bytes=1 << 30, max_slots=5, chunk=24)
    rep = eng.run(reqs)
    assert not rep.rejected
    for r in rep.records:
        wl = wls[r.rid]
        kernel, tb, _ = backend.solver_options(wl)
        print(f"request {r.rid}: graded={wl.spacing is not None} cpml={bool(wl.cpml)}", flush=True)
        solo = fdtd.Solver.from_workload(wl, kernel=kernel, time_block=tb)
        try:
            solo.step(wl.n_steps)
            ref = solo.read_probes(0, wl.n_steps)
        finally:
            solo.close()
        assert np.array_equal(r.probes, ref), f"request {r.rid} differs from its solo run"
    assert not backend.alone
