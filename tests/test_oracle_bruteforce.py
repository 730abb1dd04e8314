"""Brute force on tiny grids: the oracle's loops against the curl operator
assembled face by face from Stokes' theorem (Yee's integral form, Sec. 2.1),
its transpose (the discrete antisymmetry that Sec. 2.1 credits for
stability) and the closed-form spectrum of the PEC box."""
import math

import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import workload as W
from tests import closed_forms as cf

C0 = cf.C0


def _vec_to_fields(n, dofs, v, offset):
    nx, ny, nz = n
    f = np.zeros((6, nz + 1, ny + 1, nx + 1))
    for r, (c, i, j, k) in enumerate(dofs):
        f[offset + c, k, j, i] = v[r]
    return f


def _fields_to_vec(f, dofs, offset):
    return np.array([f[offset + c, k, j, i] for (c, i, j, k) in dofs])


GRIDS = [((4, 3, 5), (1e-3, 1.1e-3, 0.9e-3)), ((4, 4, 4), (1e-3, 1e-3, 1e-3))]


@pytest.mark.parametrize("n,d", GRIDS)
def test_faraday_matches_stokes_assembly(n, d):
    C, edofs, hdofs = cf.stokes_curl(n, d)
    dt = W.courant_dt(*d)
    prob = oracle.Problem(*n, *d, dt, [1.0], [0.0], np.zeros(n[::-1], np.uint8))
    M = np.zeros_like(C)
    for col in range(len(edofs)):
        e = np.zeros(len(edofs)); e[col] = 1.0
        f = _vec_to_fields(n, edofs, e, 0)
        prob.h_half_f64(f)
        M[:, col] = _fields_to_vec(f, hdofs, 3)
    assert np.max(np.abs(M - (-C0 * dt) * C)) < 1e-13 * np.max(np.abs(M))


@pytest.mark.parametrize("n,d", GRIDS)
def test_ampere_is_the_transpose_on_interior_edges(n, d):
    C, edofs, hdofs = cf.stokes_curl(n, d)
    dt = W.courant_dt(*d)
    prob = oracle.Problem(*n, *d, dt, [1.0], [0.0], np.zeros(n[::-1], np.uint8))
    M = np.zeros((len(edofs), len(hdofs)))
    for col in range(len(hdofs)):
        h = np.zeros(len(hdofs)); h[col] = 1.0
        f = _vec_to_fields(n, hdofs, h, 3)
        prob.e_half_f64(f)
        M[:, col] = _fields_to_vec(f, edofs, 0)
    P = np.diag([1.0 if cf.interior_edge(n, t) else 0.0 for t in edofs])
    ref = C0 * dt * (P @ C.T)
    assert np.max(np.abs(M - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,d", GRIDS)
def test_spectrum_of_curl_curl(n, d):
    C, edofs, _ = cf.stokes_curl(n, d)
    keep = [r for r, t in enumerate(edofs) if cf.interior_edge(n, t)]
    A = C[:, keep]
    K = A.T @ A
    ev = np.sort(np.linalg.eigvalsh(K))
    scale = max(4.0 / x ** 2 for x in d)
    nx, ny, nz = n
    interior_nodes = (nx - 1) * (ny - 1) * (nz - 1)
    expect = []
    for mx in range(nx):
        for my in range(ny):
            for mz in range(nz):
                zeros = (mx == 0) + (my == 0) + (mz == 0)
                mult = 2 if zeros == 0 else (1 if zeros == 1 else 0)
                lam = sum((2.0 / d[a] * math.sin(math.pi * (mx, my, mz)[a] / (2 * n[a]))) ** 2 for a in range(3))
                expect += [lam] * mult
    expect = np.sort(np.array(expect + [0.0] * interior_nodes))
    assert len(expect) == len(ev)
    assert np.max(np.abs(ev - expect)) < 1e-12 * scale
    assert int(np.sum(ev < 1e-9 * scale)) == interior_nodes
    if n == (4, 4, 4):
        assert int(np.sum(ev > 1e-9 * scale)) == 81 and interior_nodes == 27


def _lam_max(n, d):
    return sum((2.0 / d[a] * math.sin(math.pi * (n[a] - 1) / (2 * n[a]))) ** 2 for a in range(3))


@pytest.mark.parametrize("factor,stable", [(0.99, True), (1.01, False)])
def test_stability_limit(factor, stable):
    """Leapfrog stability: c dt sqrt(lambda_max) <= 2 (lambda_max from the spectrum)."""
    n, d = (4, 3, 5), (1e-3, 1.1e-3, 0.9e-3)
    dt = factor * 2.0 / (C0 * math.sqrt(_lam_max(n, d)))
    rng = np.random.default_rng(5)
    prob = oracle.Problem(*n, *d, dt, [1.0], [0.0], np.zeros(n[::-1], np.uint8))
    f = np.zeros((6, n[2] + 1, n[1] + 1, n[0] + 1))
    mask = W.interior_e_mask(*n)
    f[0:3][mask] = rng.standard_normal(int(mask.sum()))
    a0 = float(np.max(np.abs(f)))
    prob.run_f64(f, 0, 3000)
    grow = float(np.max(np.abs(f))) / a0
    if stable:
        assert grow < 50.0
    else:
        assert not np.isfinite(grow) or grow > 1e6


def test_fp32_op_order_by_exact_fma():
    """The f32 mode equals a rational-arithmetic evaluation of the stated
    operation order (every fmaf correctly rounded), element by element."""
    n, d = (3, 3, 3), (1e-3, 1.2e-3, 0.9e-3)
    nx, ny, nz = n
    dt = W.courant_dt(*d)
    rng = np.random.default_rng(11)
    eps = np.array([1.0, 3.7]); sig = np.array([0.0, 0.03])
    mat = rng.integers(0, 2, size=(nz, ny, nx)).astype(np.uint8)
    prob = oracle.Problem(*n, *d, dt, eps, sig, mat)
    f = rng.standard_normal((6, nz + 1, ny + 1, nx + 1)).astype(np.float32)
    g = f.copy()
    prob.h_half_f32(g)
    ch = prob.ch32
    fma = cf.exact_fma32
    for k in range(nz):
        for j in range(ny):
            for i in range(nx + 1):
                dey = np.float32(f[1, k + 1, j, i] - f[1, k, j, i])
                dez = np.float32(f[2, k, j + 1, i] - f[2, k, j, i])
                assert g[3, k, j, i] == fma(-ch[1], dez, fma(ch[2], dey, f[3, k, j, i]))
    h = g.copy()
    prob.e_half_f32(h)
    for k in range(1, nz):
        for j in range(1, ny):
            for i in range(nx):
                cfm = prob.coef32[mat[k, j, i]]
                dhz = np.float32(g[5, k, j, i] - g[5, k, j - 1, i])
                dhy = np.float32(g[4, k, j, i] - g[4, k - 1, j, i])
                t = np.float32(cfm[0] * g[0, k, j, i])
                assert h[0, k, j, i] == fma(-cfm[3], dhy, fma(cfm[2], dhz, t))


def test_fp32_op_order_by_exact_fma_all_components():
    """Every component follows the stated order: H = fmaf(-ch_b, d_b, fmaf(ch_a,
    d_a, H)) and E = fmaf(-Cb_b, d_b, fmaf(Cb_a, d_a, Ca E)), with (a, b) =
    (z, y) for x, (x, z) for y and (y, x) for z (the printed hx loop's term
    order, permuted cyclically; Sec. 2.1-2.2).  The swapped order differs
    from the oracle somewhere, so the check can tell the two apart."""
    n, d = (4, 3, 5), (1e-3, 1.2e-3, 0.9e-3)
    nx, ny, nz = n
    dt = W.courant_dt(*d)
    rng = np.random.default_rng(12)
    eps = np.array([1.0, 3.7, 9.1]); sig = np.array([0.0, 0.03, 0.011])
    mat = rng.integers(0, 3, size=(nz, ny, nx)).astype(np.uint8)
    prob = oracle.Problem(*n, *d, dt, eps, sig, mat)
    f = rng.standard_normal((6, nz + 1, ny + 1, nx + 1)).astype(np.float32)
    g = f.copy()
    prob.h_half_f32(g)
    chx, chy, chz = prob.ch32
    fma = cf.exact_fma32
    swapped = 0
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                if i < nx and k < nz:          # Hy: z term (Ex), then x term (Ez)
                    dez_x = np.float32(f[2, k, j, i + 1] - f[2, k, j, i])
                    dex_z = np.float32(f[0, k + 1, j, i] - f[0, k, j, i])
                    assert g[4, k, j, i] == fma(-chz, dex_z, fma(chx, dez_x, f[4, k, j, i]))
                    swapped += g[4, k, j, i] != fma(chx, dez_x, fma(-chz, dex_z, f[4, k, j, i]))
                if i < nx and j < ny:          # Hz: y term (Ex), then x term (Ey)
                    dex_y = np.float32(f[0, k, j + 1, i] - f[0, k, j, i])
                    dey_x = np.float32(f[1, k, j, i + 1] - f[1, k, j, i])
                    assert g[5, k, j, i] == fma(-chx, dey_x, fma(chy, dex_y, f[5, k, j, i]))
                    swapped += g[5, k, j, i] != fma(chy, dex_y, fma(-chx, dey_x, f[5, k, j, i]))
    h = g.copy()
    prob.e_half_f32(h)
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                if 0 < i < nx and j < ny and 0 < k < nz:     # interior Ey
                    ca, cbx, cby, cbz = prob.coef32[mat[k, j, i]]
                    dhx_z = np.float32(g[3, k, j, i] - g[3, k - 1, j, i])
                    dhz_x = np.float32(g[5, k, j, i] - g[5, k, j, i - 1])
                    t = np.float32(ca * g[1, k, j, i])
                    assert h[1, k, j, i] == fma(-cbx, dhz_x, fma(cbz, dhx_z, t))
                    swapped += h[1, k, j, i] != fma(cbz, dhx_z, fma(-cbx, dhz_x, t))
                if 0 < i < nx and 0 < j < ny and k < nz:     # interior Ez
                    ca, cbx, cby, cbz = prob.coef32[mat[k, j, i]]
                    dhy_x = np.float32(g[4, k, j, i] - g[4, k, j, i - 1])
                    dhx_y = np.float32(g[3, k, j, i] - g[3, k, j - 1, i])
                    t = np.float32(ca * g[2, k, j, i])
                    assert h[2, k, j, i] == fma(-cby, dhx_y, fma(cbx, dhy_x, t))
                    swapped += h[2, k, j, i] != fma(cbx, dhy_x, fma(-cby, dhx_y, t))
    assert swapped > 0
