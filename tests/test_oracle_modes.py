"""Pin the oracle against the exact discrete dynamics of PEC cavity modes.

A Yee eigenmode of the PEC box evolves as E^n = cos(n theta) E^0 with
sin(theta/2) = c dt sqrt(sum_d sin^2(m_d pi/(2 n_d))/d_d^2) (the leapfrog of
Sec. 2.1 applied to an eigenvector of curl-curl).  A wrong sign, index,
stagger or wall treatment breaks this relation at O(1).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import workload as W
from tests import closed_forms as cf


def _problem(n, d, dt, eps=1.0, sigma=0.0):
    nx, ny, nz = n
    return oracle.Problem(nx, ny, nz, d[0], d[1], d[2], dt, [eps], [sigma],
                          np.zeros((nz, ny, nx), np.uint8))


def _check_mode(n, d, m, amp, steps, tol=1e-11, eps=1.0):
    dt = W.courant_dt(*d)
    f = cf.mode_state(m, amp, n, d, dt)
    e0 = f[0:3].copy()
    prob = _problem(n, d, dt, eps)
    th = cf.discrete_theta(m, n, d, dt, eps)
    worst = 0.0
    for s in range(1, steps + 1):
        prob.run_f64(f, s - 1, 1)
        worst = max(worst, float(np.max(np.abs(f[0:3] - math.cos(s * th) * e0))))
    return worst / float(np.max(np.abs(e0))), th


def test_tm110_config0_geometry():
    n, d = (32, 32, 32), (1e-3, 1e-3, 1e-3)
    err, th = _check_mode(n, d, (1, 1, 0), (0.0, 0.0, 1.0), 100)
    assert err < 1e-11
    # the numbers the config-0 geometry implies (S = 0.99/sqrt(3))
    assert abs(th - 0.0793467182043760) < 1e-14
    assert abs(math.cos(100 * th) - (-0.0806027)) < 1e-6
    # the test distinguishes discrete from continuous dispersion
    dt = W.courant_dt(*d)
    thc = cf.continuous_theta((1, 1, 0), n, d, dt)
    assert abs(math.cos(100 * th) - math.cos(100 * thc)) > 1e5 * 1e-11


@pytest.mark.parametrize("m,amp", [((0, 1, 1), (1.0, 0.0, 0.0)),
                                   ((1, 0, 1), (0.0, 1.0, 0.0)),
                                   ((1, 1, 0), (0.0, 0.0, 1.0))])
def test_axis_rotations(m, amp):
    err, _ = _check_mode((12, 10, 8), (1e-3, 1e-3, 1e-3), m, amp, 60)
    assert err < 1e-11


@pytest.mark.parametrize("m", [(1, 1, 1), (2, 1, 3), (3, 2, 1)])
def test_general_mode_anisotropic(m):
    n, d = (12, 10, 8), (1.0e-3, 1.3e-3, 0.8e-3)
    amp = cf.polarisation(m, n, d)
    f0 = cf.mode_e(m, amp, n)
    assert all(np.max(np.abs(f0[c])) > 0.02 for c in range(3))   # exercises all E (and so all H)
    err, _ = _check_mode(n, d, m, amp, 80)
    assert err < 1e-11


def test_uniform_permittivity_mode():
    """eps_r = 4: the frequency drops by sqrt(eps_r) in the discrete relation."""
    n, d = (10, 10, 6), (1e-3, 1e-3, 1e-3)
    err, th = _check_mode(n, d, (1, 1, 0), (0.0, 0.0, 1.0), 60, eps=4.0)
    assert err < 1e-11
    assert abs(th - cf.discrete_theta((1, 1, 0), n, d, W.courant_dt(*d), 1.0)) > 1e-3


def test_workload_tm110_is_the_oracle_mode():
    """The config-0 generator's H^{-1/2} equals the closed form used above,
    and is minus half of the oracle's own first H increment."""
    n, d = (32, 32, 32), (1e-3, 1e-3, 1e-3)
    dt = W.courant_dt(*d)
    f = W.tm110_state(*n, *d, dt)
    ref = cf.mode_state((1, 1, 0), (0.0, 0.0, 1.0), n, d, dt)
    assert np.max(np.abs(f - ref)) < 1e-15
    prob = _problem(n, d, dt)
    g = f.copy()
    g[3:6] = 0.0
    prob.h_half_f64(g)         # g[3:6] = -c dt curl E^0
    assert np.max(np.abs(f[3:6] + 0.5 * g[3:6])) < 1e-15


def test_fp32_mode_within_1e5_of_fp64_on_config0():
    """FP32 operation-order mode vs FP64 on the full config-0 workload."""
    wl = W.cavity32()
    prob = oracle.Problem.from_workload(wl)
    f64 = wl.init_fields.copy()
    f32 = wl.init_fields.astype(np.float32)
    p64 = prob.run_f64(f64, 0, wl.n_steps)
    p32 = prob.run_f32(f32, 0, wl.n_steps)
    err = W.rel_l2(f32, f64)
    assert err < 1e-5
    assert err > 1e-9            # it really is single precision
    assert np.max(np.abs(p32 - p64)) < 1e-5
