"""Parity at the benchmark's full sizes, in the launch configurations bench.py
times (fused kernel, automatic T and tile shape; on 512^3 also T = 5, which
the bench's tuning keeps there).

Short runs from a seeded random state are compared element by element with
the oracle (the oracle takes a few seconds per step at these sizes on the
host cores).  Full-length runs are checked through properties that hold at
any size: every kernel variant gives the same bits, and probes equal the
field values they sample."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def _random_init(wl, seed):
    rng = np.random.default_rng(seed)
    f = rng.random((6, wl.nz + 1, wl.ny + 1, wl.nx + 1), dtype=np.float32)
    f -= np.float32(0.5)
    return G.pec_clean(wl, f)


def _check(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


@pytest.mark.parametrize("name,T,fixed", [("spheres256", 4, False), ("spheres512", 4, False), ("spheres512", 5, True),
                                          ("cavity402", 4, False)])
def test_fullsize_fp32_short_run_bitexact(name, T, fixed):
    """A full block and a partial one at the automatic T (or a fixed one)."""
    wl = {"spheres256": W.spheres256, "spheres512": W.spheres512, "cavity402": W.cavity402}[name]()
    steps = T + 2
    init = _random_init(wl, 11)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T if fixed else 0)
    try:
        assert s.time_block == T
        print(f"fullsize {name} FP32 T={T} ({'fixed' if fixed else 'automatic'}), {steps} steps", flush=True)
        s.set_fields(init)
        s.step(steps)
        probes = s.read_probes(0, steps)
        prob = oracle.Problem.from_workload(wl)
        ref = init.copy()
        ref_probes = prob.run_f32(ref, 0, steps)
        for c in range(6):
            _check(s.read_field(c), ref[c], f"{name} component {c}")
        _check(probes, ref_probes, f"{name} probes")
    finally:
        s.close()


@pytest.mark.parametrize("T", [3, 4])
@pytest.mark.parametrize("fmt", [W.FP16, W.BF16])
@pytest.mark.parametrize("grid", ["512", "1024x512x256"])
def test_fullsize_reduced_storage_bitexact_with_emulation(fmt, grid, T):
    """T=3 is the 16-bit default (what the bench times), T=4 the FP32 one;
    two blocks at T=3 so that the second block runs on the first one's scales."""
    steps = 2 * T if T == 3 else T
    wl = W.precision512(fmt, n_steps=steps) if grid == "512" else W.precision1024(fmt, n_steps=steps)
    init = _random_init(wl, 12)
    print(f"fullsize {grid} fmt={fmt} T={T} steps={steps}", flush=True)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T)
    try:
        s.set_fields(init)
        s.step(steps)
        prob = oracle.Problem.from_workload(wl)
        ref = init.copy()
        st = prob.quantize_upload(ref, fmt)
        prob.run_q(ref, 0, steps, fmt, T, st)
        scales, sat = s.storage_state()
        assert scales == list(st["scales"]) and not sat
        for c in range(6):
            _check(s.read_field(c), ref[c], f"{grid} fmt {fmt} component {c}")
    finally:
        s.close()


def test_fullsize_1000_steps_fused_equals_plain():
    """The benchmarked run (256^3, 1000 steps, T=4) against the plain
    two-pass kernel: identical fields and probe traces."""
    wl = W.spheres256()
    outs = []
    for kernel, T in ((fdtd.KERNEL_FUSED, 4), (fdtd.KERNEL_PLAIN, 1)):
        s = fdtd.Solver.from_workload(wl, kernel=kernel, time_block=T)
        try:
            s.step(wl.n_steps)
            outs.append((s.read_fields(), s.read_probes(0, wl.n_steps)))
        finally:
            s.close()
    (f1, p1), (f2, p2) = outs
    _check(f1, f2, "fields")
    _check(p1, p2, "probes")
    assert np.max(np.abs(f1[0:3])) > 1e-3
    # the last probe row equals the final fields at the probe positions
    for q, (c, i, j, k) in enumerate(wl.probes):
        assert p1[-1, q] == float(f1[c, k, j, i])


def test_planes_too_large_for_the_fused_kernel_run_plain():
    """4800 x 4800 x 2 cells in FP32: six components of one z-plane times T+1
    planes exceed the fused kernel's 2 GiB chunk addressing even at T = 1.
    Under AUTO the solver steps with the plain kernel, bit-exact with the
    oracle.  In 16-bit storage (fused kernel only) planes that large are
    rejected at create: 6800 x 6800."""
    big = W.spheres(6800, 6800, 2, 0, 3, seed=22, n_sources=1, n_probes=0, rmin=1, rmax=2, name="wider")
    with pytest.raises(fdtd.FdtdError) as e:
        fdtd.Solver.from_workload(big, storage=W.FP16)
    assert e.value.code == fdtd.EINVAL
    del big
    wl = W.spheres(4800, 4800, 2, 0, 3, seed=21, n_sources=1, n_probes=4, rmin=1, rmax=2, name="wide")
    init = _random_init(wl, 13)
    s = fdtd.Solver.from_workload(wl)
    try:
        s.set_fields(init)
        s.step(3)
        got = s.read_fields()
        probes = s.read_probes(0, 3)
    finally:
        s.close()
    prob = oracle.Problem.from_workload(wl)
    ref = init.copy()
    ref_probes = prob.run_f32(ref, 0, 3)
    _check(got, ref, "wide grid")
    _check(probes, ref_probes, "wide grid probes")
