"""GPU parity of dead-tile skipping: tiles whose owned nodes all stay +0 for
good (inside a perfect conductor, away from sources, with H +0) are left out
of the fused launches.  Every result is bit for bit the oracle's, with the
skip on and off: from zero fields and a source inside a conductor shell, at
T = 1..4 and 6, with FP16/BF16 storage against the emulation, from uploaded
fields that are nonzero deep inside the conductor, with a source added on a
conductor edge after some steps, and across a checkpoint."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def shell(n_steps=40, seed=4270, storage=W.FP32, nx=150, ny=110, nz=90):
    """A perfect conductor outside an ellipsoid filling the box (the shape of
    the paper's case S, ragged and anisotropic), a few dielectric spheres and
    two sources inside, probes inside and some deep in the conductor."""
    wl = W.spheres(nx, ny, nz, 4, n_steps, seed=seed, n_sources=0, n_probes=0, rmin=3, rmax=8,
                   name="shell", storage=storage)
    wl.eps_r = np.append(wl.eps_r, 1.0)
    wl.mu_r = np.append(wl.mu_r, 1.0)
    wl.sigma = np.append(wl.sigma, np.inf)
    pec = len(wl.sigma) - 1
    k, j, i = np.meshgrid(*(np.arange(v) for v in (nz, ny, nx)), indexing="ij")
    u = ((i + 0.5 - nx / 2) / (0.45 * nx)) ** 2 + ((j + 0.5 - ny / 2) / (0.45 * ny)) ** 2 + \
        ((k + 0.5 - nz / 2) / (0.45 * nz)) ** 2
    wl.mat[u > 1.0] = pec
    rng = np.random.default_rng(seed)
    wl.sources = [(W.EZ, nx // 2 + 3, ny // 2 - 2, nz // 2 + 1), (W.EX, nx // 2 - 9, ny // 2 + 5, nz // 2 - 4)]
    wl.waveforms = rng.standard_normal((2, n_steps))
    wl.probes = [(W.EZ, nx // 2, ny // 2, nz // 2), (W.HX, nx // 2 + 10, ny // 2, nz // 2 - 3),
                 (W.EY, 2, 3, 4), (W.HZ, nx - 3, ny - 4, nz - 5), (W.EX, nx - 6, 5, nz // 2)]
    return wl


def _assert_same(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


def _run(wl, steps, T, skip, storage=W.FP32, chunks=None, init=None):
    s = fdtd.Solver.from_workload(wl, storage=storage, kernel=fdtd.KERNEL_FUSED, time_block=T)
    try:
        s.set_zero_skip(skip)
        if init is not None:
            s.set_fields(init)
        for n in chunks or [steps]:
            s.step(n)
        return s.read_fields(), s.read_probes(0, steps)
    finally:
        s.close()


def test_shell_conductor_fraction():
    wl = shell()
    assert 0.4 < np.isinf(wl.sigma)[wl.mat].mean() < 0.7


@pytest.mark.parametrize("T", [1, 2, 3, 4, 6])
def test_dead_tiles_bitexact_from_zero(T):
    wl = shell()
    fo, po = G.oracle_f32(wl, 40)
    assert np.abs(po[:, :2]).max() > 0 and np.all(po[:, 2:] == 0)
    for skip in (True, False):
        print(f"shell T={T} skip={skip}, 40 steps in 11+29", flush=True)
        f, p = _run(wl, 40, T, skip, chunks=[11, 29])
        _assert_same(f, fo, f"fields skip={skip}")
        _assert_same(p, po, f"probes skip={skip}")


@pytest.mark.parametrize("fmt", [W.FP16, W.BF16])
def test_dead_tiles_reduced_storage_bitexact_with_emulation(fmt):
    wl = shell(n_steps=36, storage=fmt)
    print(f"shell fmt={fmt} T=3, 36 steps", flush=True)
    f, p = _run(wl, 36, 3, True, storage=fmt)
    fo, po, _ = G.oracle_q(wl, 36, fmt, 3)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_dead_tiles_upload_with_values_inside_conductor():
    """Uploaded fields: random inside the shell, zero in the conductor except
    one H value deep inside it (constant for good, so its tile must run) and
    random E on conductor edges (stored as zero, so those stay dead)."""
    wl = shell(n_steps=30, seed=4271)
    init = np.zeros((6, wl.nz + 1, wl.ny + 1, wl.nx + 1), np.float32)
    rng = np.random.default_rng(5)
    c = slice(wl.nz // 4, 3 * wl.nz // 4), slice(wl.ny // 4, 3 * wl.ny // 4), slice(wl.nx // 4, 3 * wl.nx // 4)
    init[(slice(None),) + c] = rng.standard_normal(init[(slice(None),) + c].shape)
    init[4, 3, 4, 5] = 0.75                       # Hy deep in the conductor corner
    init[0:3, :6, :6, :6] = rng.standard_normal((3, 6, 6, 6))
    print("shell upload, T=4, 30 steps", flush=True)
    f, p = _run(wl, 30, 4, True, init=init)
    prob = oracle.Problem.from_workload(wl)
    fo = G.pec_clean(wl, init.copy())
    owned = np.zeros((wl.nz + 1, wl.ny + 1, wl.nx + 1), bool)
    owned[:wl.nz, :wl.ny, :wl.nx] = np.isinf(wl.sigma)[wl.mat]
    fo[0:3][:, owned] = 0.0
    po = prob.run_f32(fo, 0, 30)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    assert f[4, 3, 4, 5] == np.float32(0.75)


def test_dead_tiles_source_added_on_conductor_edge():
    """A source placed on an edge deep inside the conductor after 10 steps
    (added after that edge's update, cleared by the next) wakes its tile."""
    wl = shell(n_steps=30, seed=4272)
    extra = (W.EZ, 3, 4, 5)
    wave = np.random.default_rng(9).standard_normal(30).astype(np.float32)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=4)
    try:
        s.step(10)
        s.add_source(*extra, wave)
        s.step(20)
        f, p = s.read_fields(), s.read_probes(0, 30)
    finally:
        s.close()
    ref = shell(n_steps=30, seed=4272)
    ref.sources = list(ref.sources) + [extra]
    w = wave.astype(np.float64).copy()
    w[:10] = 0.0
    ref.waveforms = np.vstack([ref.waveforms, w[None, :]])
    fo, po = G.oracle_f32(ref, 30)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    assert np.abs(fo[3:6, :12, :12, :12]).max() > 0      # the conductor-edge source drove H nearby


def test_dead_tiles_across_checkpoint():
    wl = shell(n_steps=32, seed=4273)
    fo, po = G.oracle_f32(wl, 32)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=4)
    try:
        s.step(12)
        state = s.save_state()
    finally:
        s.close()
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=4)
    try:
        s.step(3)                                  # some other history, then the restore
        s.load_state(state)
        s.step(20)
        f, p = s.read_fields(), s.read_probes(12, 20)
    finally:
        s.close()
    _assert_same(f, fo, "fields")
    _assert_same(p, po[12:], "probes")


def test_tile_stats_show_the_skip():
    """fdtd_tile_stats: with the skip on, a conductor shell run from zero
    fields dispatches fewer workgroups than its full tilings hold; with the
    skip off, exactly as many."""
    wl = shell(n_steps=40)
    out = {}
    for skip in (True, False):
        s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=4)
        try:
            s.set_zero_skip(skip)
            assert s.tile_stats() == (0, 0)
            s.step(40)
            out[skip] = s.tile_stats()
        finally:
            s.close()
    run, full = out[True]
    assert 0 < run < 0.8 * full
    assert out[False][0] == out[False][1] > 0


def test_dead_tiles_in_batched_launches():
    """fdtd_step_batch skips the dead tiles of each solve too: two conductor
    shells and an open dielectric grid in one batch equal each solve alone
    and the oracle, and the shells dispatch fewer workgroups than their full
    tilings hold."""
    wls = [shell(n_steps=24, seed=4271, nx=90, ny=70, nz=60), shell(n_steps=24, seed=4272, nx=70, ny=90, nz=50),
           W.spheres(60, 50, 40, 3, 24, seed=4273, n_sources=1, n_probes=4, rmin=3, rmax=6, name="open")]
    print("batched dead tiles: two shells and a dielectric grid, 24 steps at T=4 in chunks 9+15", flush=True)
    ss = [fdtd.Solver.from_workload(w, kernel=fdtd.KERNEL_FUSED, time_block=4) for w in wls]
    try:
        for n in (9, 15):
            fdtd.step_batch(ss, [n] * len(ss))
        got = [(s.read_fields(), s.read_probes(0, 24) if w.probes else None) for s, w in zip(ss, wls)]
        stats = [s.tile_stats() for s in ss]
    finally:
        for s in ss:
            s.close()
    for (f, p), w, st in zip(got, wls, stats):
        fo, po = G.oracle_f32(w, 24)
        _assert_same(f, fo, f"{w.name} fields")
        if p is not None:
            _assert_same(p, po, f"{w.name} probes")
    assert stats[0][0] < stats[0][1] and stats[1][0] < stats[1][1]
