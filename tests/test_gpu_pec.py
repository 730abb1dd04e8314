"""GPU parity of perfect-conductor material entries (sigma = +inf): bit for
bit with the oracle on a ragged grid holding PEC spheres (fused T = 1..4,
plain, graded, FP16 storage), with fdtd_set_fields zeroing the edges PEC
cells own; and the paper's case S (a 400-cell PEC sphere in a 402^3 box) at
full size."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def pec_ragged(n_steps=40, seed=4260, storage=W.FP32):
    """The ragged dielectric grid plus a perfect-conductor entry (index 16):
    three seeded PEC spheres and a PEC slab over the last 11 cells in x;
    random waveforms."""
    wl = W.spheres(131, 75, 50, 14, n_steps, seed=seed, n_sources=3, n_probes=16, rmin=3, rmax=12,
                   name="pec_ragged", storage=storage)
    wl.eps_r = np.append(wl.eps_r, 1.0)
    wl.mu_r = np.append(wl.mu_r, 1.0)
    wl.sigma = np.append(wl.sigma, np.inf)
    rng = np.random.default_rng(seed)
    k, j, i = np.meshgrid(*(np.arange(v) for v in (wl.nz, wl.ny, wl.nx)), indexing="ij")
    for _ in range(3):
        c = rng.uniform([10, 10, 10], [110, 65, 40])
        r = rng.uniform(5, 10)
        wl.mat[(i + 0.5 - c[0]) ** 2 + (j + 0.5 - c[1]) ** 2 + (k + 0.5 - c[2]) ** 2 <= r * r] = 16
    wl.mat[i >= 120] = 16
    wl.waveforms = rng.standard_normal(wl.waveforms.shape)
    return wl


def pec_clean(wl, f):
    """What fdtd_set_fields stores: walls, unused slots and PEC-owned E zeroed."""
    g = G.pec_clean(wl, f)
    owned = np.zeros((wl.nz + 1, wl.ny + 1, wl.nx + 1), bool)
    owned[:wl.nz, :wl.ny, :wl.nx] = np.isinf(wl.sigma)[wl.mat]
    g[0:3][:, owned] = 0.0
    return g


def _assert_same(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


def test_pec_grid_has_conductor_cells():
    wl = pec_ragged()
    frac = np.isinf(wl.sigma)[wl.mat].mean()
    assert 0.01 < frac < 0.6, frac


@pytest.mark.parametrize("kernel,T", [(fdtd.KERNEL_PLAIN, 1), (fdtd.KERNEL_FUSED, 1), (fdtd.KERNEL_FUSED, 2),
                                      (fdtd.KERNEL_FUSED, 3), (fdtd.KERNEL_FUSED, 4)])
def test_pec_bitexact_from_random_fields(kernel, T):
    wl = pec_ragged()
    init = np.random.default_rng(11).standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1)).astype(np.float32)
    print(f"pec ragged kernel={kernel} T={T}, 40 steps", flush=True)
    f, p = G.gpu_run(wl, 40, kernel=kernel, T=T, init=init, chunks=[9, 31])
    prob = oracle.Problem.from_workload(wl)
    fo = pec_clean(wl, init)
    po = prob.run_f32(fo, 0, 40)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    owned = np.isinf(wl.sigma)[wl.mat]
    assert np.all(f[0:3, :wl.nz, :wl.ny, :wl.nx][:, owned] == 0.0)


def test_pec_graded_bitexact():
    wl = pec_ragged(n_steps=30, seed=4261)
    rng = np.random.default_rng(4261)
    wl.spacing = tuple(rng.uniform(0.5e-3, 1.5e-3, n) for n in (wl.nx, wl.ny, wl.nz))
    wl.dt = W.courant_dt_graded(*wl.spacing)
    print("pec graded, automatic kernel, 30 steps", flush=True)
    f, p = G.gpu_run(wl, 30, kernel=fdtd.KERNEL_AUTO, T=0)
    fo, po = G.oracle_f32(wl, 30)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("fmt", [W.FP16, W.BF16])
def test_pec_reduced_storage_bitexact_with_emulation(fmt):
    wl = pec_ragged(n_steps=24, seed=4262, storage=fmt)
    print(f"pec reduced storage fmt={fmt} T=3, 24 steps", flush=True)
    f, p = G.gpu_run(wl, 24, kernel=fdtd.KERNEL_FUSED, T=3, storage=fmt)
    fo, po, _ = G.oracle_q(wl, 24, fmt, 3)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_sphere402_full_size_bitexact():
    """The paper's case S at full size from random fields (the conductor's
    edges zeroed on upload), automatic kernel and T, 20 steps."""
    wl = W.sphere402(n_steps=20)
    init = np.random.default_rng(402).standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1), dtype=np.float32)
    print("sphere402 full size, 20 steps", flush=True)
    f, p = G.gpu_run(wl, 20, kernel=fdtd.KERNEL_AUTO, T=0, init=init)
    prob = oracle.Problem.from_workload(wl)
    fo = pec_clean(wl, init)
    po = prob.run_f32(fo, 0, 20)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
