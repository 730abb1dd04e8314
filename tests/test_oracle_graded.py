"""Graded (per-index) spacing in the oracle, pinned by what geometry and the
mathematics fix: Stokes' theorem on primal and dual faces, the uniform case,
exact energy conservation and divergence constancy, and the stated FP32
operation order (every fmaf correctly rounded)."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import workload as W
from tests import closed_forms as cf

C0 = 299792458.0


def _sizes(rng, n, d0=1e-3, spread=2.0):
    return d0 * rng.uniform(1.0, spread, size=n)


def _graded_dt(sx, sy, sz, frac=0.9):
    return frac / (C0 * np.sqrt(1 / sx.min() ** 2 + 1 / sy.min() ** 2 + 1 / sz.min() ** 2))


def _problem(n, sizes, eps, sig, mat, dt):
    return oracle.Problem(*n, 1e-3, 1e-3, 1e-3, dt, eps, sig, mat, spacing=sizes)


def test_uniform_per_axis_spacing_equals_the_uniform_oracle():
    """dx != dy != dz but constant along each axis: the graded update is the
    uniform one (to rounding), so an axis or primal/dual swap would show."""
    n, d = (7, 5, 6), (1.0e-3, 1.3e-3, 0.8e-3)
    rng = np.random.default_rng(1)
    dt = W.courant_dt(*d)
    eps, sig = np.array([1.0, 4.0, 9.0]), np.array([0.0, 0.02, 0.04])
    mat = rng.integers(0, 3, size=n[::-1]).astype(np.uint8)
    uni = oracle.Problem(*n, *d, dt, eps, sig, mat)
    gra = oracle.Problem(*n, *d, dt, eps, sig, mat, spacing=[np.full(m, dd) for m, dd in zip(n, d)])
    f = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1))
    a, b = f.copy(), f.copy()
    uni.run_f64(a, 0, 20)
    gra.run_f64(b, 0, 20)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def _stokes_h(n, sx, sy, sz, dt, f):
    """H after one Faraday half-step from circulations of E around primal
    faces (edge lengths) over face areas."""
    nx, ny, nz = n
    g = f.copy()
    ex, ey, ez = f[0], f[1], f[2]
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                if j < ny and k < nz:     # Hx: face at x_i spanning y_j..y_j+1, z_k..z_k+1
                    circ = (ey[k, j, i] * sy[j] + ez[k, j + 1, i] * sz[k]
                            - ey[k + 1, j, i] * sy[j] - ez[k, j, i] * sz[k])
                    g[3, k, j, i] -= C0 * dt * circ / (sy[j] * sz[k])
                if i < nx and k < nz:     # Hy: face at y_j spanning z_k.., x_i..
                    circ = (ez[k, j, i] * sz[k] + ex[k + 1, j, i] * sx[i]
                            - ez[k, j, i + 1] * sz[k] - ex[k, j, i] * sx[i])
                    g[4, k, j, i] -= C0 * dt * circ / (sz[k] * sx[i])
                if i < nx and j < ny:     # Hz: face at z_k spanning x_i.., y_j..
                    circ = (ex[k, j, i] * sx[i] + ey[k, j, i + 1] * sy[j]
                            - ex[k, j + 1, i] * sx[i] - ey[k, j, i] * sy[j])
                    g[5, k, j, i] -= C0 * dt * circ / (sx[i] * sy[j])
    return g


def _dual(s):
    n = len(s)
    return np.array([s[0] / 2 if q == 0 else s[n - 1] / 2 if q == n else (s[q - 1] + s[q]) / 2
                     for q in range(n + 1)])


def _stokes_e(n, sx, sy, sz, dt, f):
    """E after one Ampere half-step (vacuum, no loss) from circulations of H
    around the dual faces of interior edges (dual edge lengths) over the dual
    face areas; tangential E on the walls stays."""
    nx, ny, nz = n
    dx, dy, dz = _dual(sx), _dual(sy), _dual(sz)
    g = f.copy()
    hx, hy, hz = f[3], f[4], f[5]
    for k in range(1, nz):
        for j in range(1, ny):
            for i in range(nx):           # Ex at (i+1/2, j, k): dual face dy_j x dz_k
                circ = (hz[k, j, i] * dz[k] - hz[k, j - 1, i] * dz[k]
                        - hy[k, j, i] * dy[j] + hy[k - 1, j, i] * dy[j])
                g[0, k, j, i] += C0 * dt * circ / (dy[j] * dz[k])
    for k in range(1, nz):
        for j in range(ny):
            for i in range(1, nx):        # Ey at (i, j+1/2, k): dual face dz_k x dx_i
                circ = (hx[k, j, i] * dx[i] - hx[k - 1, j, i] * dx[i]
                        - hz[k, j, i] * dz[k] + hz[k, j, i - 1] * dz[k])
                g[1, k, j, i] += C0 * dt * circ / (dz[k] * dx[i])
    for k in range(nz):
        for j in range(1, ny):
            for i in range(1, nx):        # Ez at (i, j, k+1/2): dual face dx_i x dy_j
                circ = (hy[k, j, i] * dy[j] - hy[k, j, i - 1] * dy[j]
                        - hx[k, j, i] * dx[i] + hx[k, j - 1, i] * dx[i])
                g[2, k, j, i] += C0 * dt * circ / (dx[i] * dy[j])
    return g


@pytest.mark.parametrize("seed", [2, 3])
def test_graded_half_steps_match_stokes_assembly(seed):
    n = (4, 3, 5)
    rng = np.random.default_rng(seed)
    sx, sy, sz = (_sizes(rng, m) for m in n)
    dt = _graded_dt(sx, sy, sz)
    prob = _problem(n, (sx, sy, sz), [1.0], [0.0], np.zeros(n[::-1], np.uint8), dt)
    f = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1))
    f[0:3][~W.interior_e_mask(*n)] = 0.0
    g = f.copy()
    prob.h_half_f64(g)
    ref = _stokes_h(n, sx, sy, sz, dt, f)
    assert np.max(np.abs(g[3:] - ref[3:])) < 1e-12 * np.max(np.abs(ref[3:]))
    h = g.copy()
    prob.e_half_f64(h)
    ref = _stokes_e(n, sx, sy, sz, dt, g)
    assert np.max(np.abs(h[0:3] - ref[0:3])) < 1e-12 * np.max(np.abs(ref[0:3]))


def test_graded_energy_conserved_lossless():
    """With volume weights (edge length x dual area for E, face area x dual
    length for H) a lossless PEC box keeps the discrete energy to rounding."""
    n = (9, 7, 8)
    rng = np.random.default_rng(4)
    sx, sy, sz = (_sizes(rng, m, spread=3.0) for m in n)
    dt = _graded_dt(sx, sy, sz)
    eps = np.array([1.0, 2.5, 7.0])
    mat = rng.integers(0, 3, size=n[::-1]).astype(np.uint8)
    prob = _problem(n, (sx, sy, sz), eps, np.zeros(3), mat, dt)
    f = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1))
    f[0:3][~W.interior_e_mask(*n)] = 0.0
    w0 = prob.energy(f)
    for _ in range(4):
        prob.run_f64(f, 0, 50)
        assert abs(prob.energy(f) - w0) < 1e-12 * w0


def test_graded_energy_detects_a_wrong_dual_size():
    """Plant a mistake in the oracle's coefficients (the uniform primal size
    where the dual size belongs): energy then drifts, so the conservation pin
    above does check the dual sizes."""
    n = (9, 7, 8)
    rng = np.random.default_rng(4)
    sx, sy, sz = (_sizes(rng, m, spread=3.0) for m in n)
    dt = _graded_dt(sx, sy, sz)
    prob = _problem(n, (sx, sy, sz), [1.0], [0.0], np.zeros(n[::-1], np.uint8), dt)
    prob.ec64[1:n[0]] = C0 * dt / sx[1:]          # primal instead of dual x sizes
    f = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1))
    f[0:3][~W.interior_e_mask(*n)] = 0.0
    w0 = prob.energy(f)
    prob.run_f64(f, 0, 200)
    assert abs(prob.energy(f) - w0) > 1e-6 * w0


def test_graded_divergence_constant_without_sources():
    n = (8, 6, 7)
    rng = np.random.default_rng(6)
    sx, sy, sz = (_sizes(rng, m, spread=2.5) for m in n)
    dt = _graded_dt(sx, sy, sz)
    eps, sig = np.array([1.0, 5.0]), np.array([0.0, 0.03])
    mat = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    prob = _problem(n, (sx, sy, sz), eps, sig, mat, dt)
    f = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1))
    f[0:3][~W.interior_e_mask(*n)] = 0.0
    de0, dh0 = prob.divergence(f)
    prob.run_f64(f, 0, 60)
    de, dh = prob.divergence(f)
    assert np.max(np.abs(dh - dh0)) < 1e-9 * np.max(np.abs(dh0))
    # with loss, div(eps E) decays towards 0 where sigma > 0; in vacuum cells it is constant
    assert np.max(np.abs(de)) <= np.max(np.abs(de0)) * (1 + 1e-9)
    lossless = oracle.Problem(*n, 1e-3, 1e-3, 1e-3, dt, eps, np.zeros(2), mat, spacing=(sx, sy, sz))
    g = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1))
    g[0:3][~W.interior_e_mask(*n)] = 0.0
    de0, _ = lossless.divergence(g)
    lossless.run_f64(g, 0, 60)
    de, _ = lossless.divergence(g)
    assert np.max(np.abs(de - de0)) < 1e-9 * np.max(np.abs(de0))


def test_graded_fp32_is_the_stated_operation_order():
    n = (3, 3, 3)
    nx, ny, nz = n
    rng = np.random.default_rng(12)
    sx, sy, sz = (_sizes(rng, m) for m in n)
    dt = _graded_dt(sx, sy, sz)
    eps, sig = np.array([1.0, 3.7]), np.array([0.0, 0.03])
    mat = rng.integers(0, 2, size=(nz, ny, nx)).astype(np.uint8)
    prob = _problem(n, (sx, sy, sz), eps, sig, mat, dt)
    hcx, hcy, hcz = np.split(prob.hc32, [nx + 1, nx + ny + 2])
    ecx, ecy, ecz = np.split(prob.ec32, [nx + 1, nx + ny + 2])
    f = rng.standard_normal((6, nz + 1, ny + 1, nx + 1)).astype(np.float32)
    g = f.copy()
    prob.h_half_f32(g)
    fma = cf.exact_fma32
    for k in range(nz):
        for j in range(ny):
            for i in range(nx + 1):
                dey = np.float32(f[1, k + 1, j, i] - f[1, k, j, i])
                dez = np.float32(f[2, k, j + 1, i] - f[2, k, j, i])
                assert g[3, k, j, i] == fma(-hcy[j], dez, fma(hcz[k], dey, f[3, k, j, i]))
    h = g.copy()
    prob.e_half_f32(h)
    for k in range(1, nz):
        for j in range(1, ny):
            for i in range(nx):
                ca, gm = prob.cag32[mat[k, j, i]]
                cby, cbz = np.float32(gm * ecy[j]), np.float32(gm * ecz[k])
                dhz = np.float32(g[5, k, j, i] - g[5, k, j - 1, i])
                dhy = np.float32(g[4, k, j, i] - g[4, k - 1, j, i])
                t = np.float32(ca * g[0, k, j, i])
                assert h[0, k, j, i] == fma(-cbz, dhy, fma(cby, dhz, t))


def test_graded_fp32_energy_close_to_fp64_energy():
    """The FP32-half-step form of the graded energy (what the GPU reports)
    agrees with the FP64 form on the same fields to FP32 rounding."""
    n = (9, 7, 8)
    rng = np.random.default_rng(14)
    sx, sy, sz = (_sizes(rng, m, spread=2.0) for m in n)
    dt = _graded_dt(sx, sy, sz)
    eps = np.array([1.0, 3.0])
    mat = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    prob = _problem(n, (sx, sy, sz), eps, np.zeros(2), mat, dt)
    f = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1)).astype(np.float32)
    f[0:3][~W.interior_e_mask(*n)] = 0.0
    w64 = prob.energy(f.astype(np.float64))
    w32 = prob.energy(f)
    assert abs(w32 - w64) < 1e-6 * w64


@pytest.mark.parametrize("fmt", [1, 2])
def test_graded_reduced_storage_composes_step_and_quantisation(fmt):
    """The graded emulation mode is the graded FP32 step with the state
    re-encoded at block ends: one block of all the steps equals the FP32
    run followed by one re-encoding, and blocks of T equal T-step FP32 runs
    each followed by one."""
    n = (10, 9, 11)
    rng = np.random.default_rng(31)
    sx, sy, sz = (_sizes(rng, m) for m in n)
    dt = _graded_dt(sx, sy, sz)
    eps, sig = np.array([1.0, 3.0]), np.array([0.0, 0.02])
    mat = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    prob = _problem(n, (sx, sy, sz), eps, sig, mat, dt)
    f0 = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1)).astype(np.float32)
    f0[0:3][~W.interior_e_mask(*n)] = 0.0
    fq = f0.copy()
    st = prob.quantize_upload(fq, fmt)
    for T, steps in ((12, 12), (4, 12)):
        a = fq.copy()
        sa = {k: v.copy() for k, v in st.items()}
        prob.run_q(a, 0, steps, fmt, T, sa)
        b = fq.copy()
        sb = {k: v.copy() for k, v in st.items()}
        for s0 in range(0, steps, T):
            prob.run_f32(b, s0, T)
            lib = oracle.lib()
            lib.orc_quantize_state(prob.nx, prob.ny, prob.nz, fmt, 0, prob.a_max, b, sb["scales"], sb["m_stored"],
                                   sb["flag"])
        assert np.array_equal(a, b) and np.array_equal(sa["scales"], sb["scales"])
        assert not np.array_equal(a, fq)
