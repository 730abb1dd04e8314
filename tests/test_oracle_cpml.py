"""CPML absorbing layers in the oracle, pinned by what physics and the
mathematics fix rather than by the oracle itself:

* a point source in a small box with CPML layers records, at probes close to
  the layers, the same signals as in a box large enough that no reflection
  returns within the window (the unbounded-space answer); a PEC box of the
  small size reflects at full strength, and a planted sign error in the psi
  recursion is caught;
* with sigma = 0, kappa = 1 and alpha = 0 the layers vanish: the update is
  the graded one exactly;
* the energy of a pulse leaves the box, and stays gone (late-time stability);
* FP32 follows the stated order (psi first, then one fmaf per layer term)."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import workload as W
from tests import closed_forms as cf

D = 1e-3
LAYER = dict(thickness=8, order=3, sigma_factor=1.0, kappa_max=5.0, alpha_max=0.05)


def _point_source_run(n, steps, cpml=None, plant=None):
    """Ez point source at the centre of an n^3 vacuum box; probes 9 cells off
    the source, the farthest 3 cells from an 8-cell layer of a 40^3 box."""
    dt = W.courant_dt(D, D, D)
    c = n // 2
    src = [(2, c, c, c)]
    w = W.gaussian_sine(steps, dt, D)[None, :]
    probes = [(2, c, c, c + 9), (2, c + 9, c, c), (0, c + 5, c + 7, c + 6), (2, c + 9, c + 9, c + 9)]
    prob = oracle.Problem(n, n, n, D, D, D, dt, [1.0], [0.0], np.zeros((n, n, n), np.uint8), src, w, probes,
                          cpml=cpml)
    if plant:
        plant(prob)
    f = oracle.zero_fields(n, n, n)
    return prob.run_f64(f, 0, steps)


@pytest.fixture(scope="module")
def unbounded():
    # 220 steps travel < 126 cells; from the centre of a 160^3 box a wall
    # reflection needs > 150 cells to come back to any probe
    return _point_source_run(160, 220)


def _rel_err(p, ref):
    return np.abs(p - ref).max(axis=0) / np.abs(ref).max(axis=0)


def test_cpml_matches_the_unbounded_reference(unbounded):
    err = _rel_err(_point_source_run(40, 220, cpml=LAYER), unbounded)
    assert err.max() < 1e-3, err
    err_pec = _rel_err(_point_source_run(40, 220), unbounded)
    assert err_pec.min() > 0.3, err_pec


def test_cpml_planted_sign_error_is_caught(unbounded):
    def flip(prob):
        prob.cp64[:, 1] *= -1.0
        prob.cp64[:, 4] *= -1.0
    err = _rel_err(_point_source_run(40, 220, cpml=LAYER, plant=flip), unbounded)
    assert err.max() > 1e-2, err


def test_cpml_without_loss_or_stretch_is_the_graded_update():
    n = (14, 12, 16)
    rng = np.random.default_rng(3)
    sizes = tuple(rng.uniform(0.5e-3, 1.5e-3, m) for m in n)
    dt = W.courant_dt_graded(*sizes)
    eps, sig = np.array([1.0, 4.0]), np.array([0.0, 0.02])
    mat = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    zero = dict(thickness=4, order=3, sigma_factor=0.0, kappa_max=1.0, alpha_max=0.0)
    g = oracle.Problem(*n, D, D, D, dt, eps, sig, mat, spacing=sizes)
    c = oracle.Problem(*n, D, D, D, dt, eps, sig, mat, spacing=sizes, cpml=zero)
    f = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1))
    f[0:3][~W.interior_e_mask(*n)] = 0.0
    a, b = f.copy(), f.copy()
    g.run_f64(a, 0, 30)
    c.run_f64(b, 0, 30)
    assert np.array_equal(a, b)
    a32, b32 = f.astype(np.float32), f.astype(np.float32)
    g.run_f32(a32, 0, 30)
    c.run_f32(b32, 0, 30)
    assert np.array_equal(a32, b32)


def test_cpml_energy_leaves_and_stays_gone():
    n = 32
    dt = W.courant_dt(D, D, D)
    c = n // 2
    # a current whose samples sum to zero leaves no static charge behind
    g = W.gaussian_sine(400, dt, D)
    w = np.diff(np.concatenate([[0.0], g]))[None, :]
    cp = dict(thickness=6, order=3, sigma_factor=1.0, kappa_max=5.0, alpha_max=0.05)
    prob = oracle.Problem(n, n, n, D, D, D, dt, [1.0], [0.0], np.zeros((n, n, n), np.uint8),
                          [(2, c, c, c)], w, [], cpml=cp)
    f = oracle.zero_fields(n, n, n)
    energy = []
    for s in range(0, 1500, 50):
        prob.run_f64(f, s, 50)
        energy.append(prob.energy(f))
    peak = max(energy)
    assert energy[-1] < 1e-6 * peak, energy
    assert energy[-1] <= energy[-5] * 1.0001          # no late-time growth
    assert np.all(np.isfinite(f))


def test_cpml_fp32_close_to_fp64():
    n = (24, 20, 22)
    rng = np.random.default_rng(9)
    sizes = tuple(rng.uniform(0.6e-3, 1.4e-3, m) for m in n)
    dt = W.courant_dt_graded(*sizes)
    eps, sig = np.array([1.0, 6.0]), np.array([0.0, 0.03])
    mat = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    cp = dict(thickness=5, order=3, sigma_factor=1.0, kappa_max=4.0, alpha_max=0.05)
    prob = oracle.Problem(*n, D, D, D, dt, eps, sig, mat, spacing=sizes, cpml=cp)
    f = rng.standard_normal((6, n[2] + 1, n[1] + 1, n[0] + 1))
    f[0:3][~W.interior_e_mask(*n)] = 0.0
    f32 = f.astype(np.float32)
    prob.run_f64(f, 0, 100)
    prob.run_f32(f32, 0, 100)
    assert W.rel_l2(f32, f) < 1e-5


def test_cpml_fp32_is_the_stated_operation_order():
    """One step on a 9x8x10 grid with 3-cell layers: Hx and Ex in a corner of
    two layers, recomputed with correctly rounded fmaf from the graded update
    and the psi recursion."""
    n = (9, 8, 10)
    nx, ny, nz = n
    rng = np.random.default_rng(21)
    sizes = tuple(rng.uniform(0.7e-3, 1.3e-3, m) for m in n)
    dt = W.courant_dt_graded(*sizes)
    eps, sig = np.array([1.0, 2.5]), np.array([0.0, 0.04])
    mat = rng.integers(0, 2, size=(nz, ny, nx)).astype(np.uint8)
    cp = dict(thickness=3, order=3, sigma_factor=1.0, kappa_max=3.0, alpha_max=0.05)
    prob = oracle.Problem(*n, D, D, D, dt, eps, sig, mat, spacing=sizes, cpml=cp)
    prob.psi32[:] = rng.standard_normal(prob.psi32.shape).astype(np.float32)
    psi0 = prob.psi32.copy()
    f = rng.standard_normal((6, nz + 1, ny + 1, nx + 1)).astype(np.float32)
    f[0:3][~W.interior_e_mask(*n)] = 0.0
    g = f.copy()
    prob.run_f32(g, 0, 1)
    fma = cf.exact_fma32
    hcx, hcy, hcz = np.split(prob.hc32, [nx + 1, nx + ny + 2])
    ecx, ecy, ecz = np.split(prob.ec32, [nx + 1, nx + ny + 2])
    cpx, cpy, cpz = np.split(prob.cp32, [nx + 1, nx + ny + 2])
    # Hx at (i, j+1/2, k+1/2) with j, k in the low layers: graded, then z term, then y term
    i, j, k = 4, 1, 2
    dey_z = np.float32(f[1, k + 1, j, i] - f[1, k, j, i])
    dez_y = np.float32(f[2, k, j + 1, i] - f[2, k, j, i])
    hx = fma(-hcy[j], dez_y, fma(hcz[k], dey_z, f[3, k, j, i]))
    pz = fma(cpz[k, 0], psi0[1, k, j, i], np.float32(cpz[k, 1] * dey_z))
    hx = fma(cpz[k, 2], pz, hx)
    py = fma(cpy[j, 0], psi0[0, k, j, i], np.float32(cpy[j, 1] * dez_y))
    hx = fma(-cpy[j, 2], py, hx)
    assert g[3, k, j, i] == hx
    assert prob.psi32[1, k, j, i] == pz and prob.psi32[0, k, j, i] == py
    # Ex at (i+1/2, j, k) with j, k in the high layers, from the new H
    i, j, k = 3, ny - 1, nz - 2
    ca, gm = prob.cag32[mat[k, j, i]]
    dhz_y = np.float32(g[5, k, j, i] - g[5, k, j - 1, i])
    dhy_z = np.float32(g[4, k, j, i] - g[4, k - 1, j, i])
    t = fma(np.float32(gm * ecy[j]), dhz_y, np.float32(ca * f[0, k, j, i]))
    ex = fma(-np.float32(gm * ecz[k]), dhy_z, t)
    qy = fma(cpy[j, 3], psi0[6, k, j, i], np.float32(cpy[j, 4] * dhz_y))
    ex = fma(np.float32(gm * cpy[j, 5]), qy, ex)
    qz = fma(cpz[k, 3], psi0[7, k, j, i], np.float32(cpz[k, 4] * dhy_z))
    ex = fma(-np.float32(gm * cpz[k, 5]), qz, ex)
    assert g[0, k, j, i] == ex
