"""Closed forms of the Yee scheme used to pin the oracle (test helpers).

* PEC cavity eigenmodes on the staggered grid and their exact discrete
  dispersion relation.
* The discrete curl assembled face by face from Stokes' theorem (the
  integral form of Faraday's law on mesh faces, Sec. 2.1), independent of
  the update loops.
"""
import math

import numpy as np

C0 = 299792458.0


def kappa(m, n, d):
    """(2/d) sin(pi m / (2 n)) per axis."""
    return np.array([2.0 / d[a] * math.sin(math.pi * m[a] / (2.0 * n[a])) for a in range(3)])


def discrete_theta(m, n, d, dt, eps_r=1.0):
    """theta = omega~ dt with sin(theta/2) = (c dt/sqrt(eps_r)) sqrt(sum sin^2(m pi/2n)/d^2)."""
    s = C0 * dt / math.sqrt(eps_r) * math.sqrt(sum((math.sin(math.pi * m[a] / (2 * n[a])) / d[a]) ** 2
                                                   for a in range(3)))
    return 2.0 * math.asin(s)


def continuous_theta(m, n, d, dt, eps_r=1.0):
    k2 = sum((math.pi * m[a] / (n[a] * d[a])) ** 2 for a in range(3))
    return C0 / math.sqrt(eps_r) * math.sqrt(k2) * dt


def mode_e(m, amp, n):
    """E of the PEC mode m with polarisation amp (6-component array, H zero).

    Ex(i+1/2,j,k) = ax cos(pi mx (i+1/2)/nx) sin(pi my j/ny) sin(pi mz k/nz), cyclic.
    """
    nx, ny, nz = n
    f = np.zeros((6, nz + 1, ny + 1, nx + 1))
    i = np.arange(nx + 1)[None, None, :]
    j = np.arange(ny + 1)[None, :, None]
    k = np.arange(nz + 1)[:, None, None]
    sx, sy, sz = (np.sin(math.pi * m[0] * i / nx), np.sin(math.pi * m[1] * j / ny),
                  np.sin(math.pi * m[2] * k / nz))
    cx, cy, cz = (np.cos(math.pi * m[0] * (i + 0.5) / nx), np.cos(math.pi * m[1] * (j + 0.5) / ny),
                  np.cos(math.pi * m[2] * (k + 0.5) / nz))
    ex = amp[0] * cx * sy * sz
    ey = amp[1] * sx * cy * sz
    ez = amp[2] * sx * sy * cz
    f[0, :, :, :nx] = ex[:, :, :nx]
    f[1, :, :ny, :] = ey[:, :ny, :]
    f[2, :nz, :, :] = ez[:nz, :, :]
    return f


def curl_e(f, d):
    """Discrete curl of E at the H faces (by differences), shape like f[3:6]."""
    dx, dy, dz = d
    ex, ey, ez = f[0], f[1], f[2]
    out = np.zeros_like(f[3:6])
    # Hx(i, j+1/2, k+1/2): dEz/dy - dEy/dz
    out[0, :-1, :-1, :] = (ez[:-1, 1:, :] - ez[:-1, :-1, :])[:, :, :] / dy - (ey[1:, :-1, :] - ey[:-1, :-1, :]) / dz
    # Hy(i+1/2, j, k+1/2): dEx/dz - dEz/dx
    out[1, :-1, :, :-1] = (ex[1:, :, :-1] - ex[:-1, :, :-1]) / dz - (ez[:-1, :, 1:] - ez[:-1, :, :-1]) / dx
    # Hz(i+1/2, j+1/2, k): dEy/dx - dEx/dy
    out[2, :, :-1, :-1] = (ey[:, :-1, 1:] - ey[:, :-1, :-1]) / dx - (ex[:, 1:, :-1] - ex[:, :-1, :-1]) / dy
    return out


def mode_state(m, amp, n, d, dt):
    """(E^0, H^{-1/2}) for which the leapfrog gives E^n = cos(n theta) E^0."""
    f = mode_e(m, amp, n)
    f[3:6] = 0.5 * C0 * dt * curl_e(f, d)
    return f


def polarisation(m, n, d, v=(1.0, 2.0, 3.0)):
    """A polarisation orthogonal to kappa (discretely divergence-free)."""
    k = kappa(m, n, d)
    a = np.cross(k, np.asarray(v, dtype=float))
    return a / np.max(np.abs(a))


# --------------------------------------------------------------------------
# Stokes assembly of the curl: C[face, edge] = +-len(edge)/area(face)
# --------------------------------------------------------------------------
def dof_lists(n):
    """Valid E and H storage positions, as lists of (comp, i, j, k)."""
    nx, ny, nz = n
    e, h = [], []
    lim_e = [(nx, ny + 1, nz + 1), (nx + 1, ny, nz + 1), (nx + 1, ny + 1, nz)]
    lim_h = [(nx + 1, ny, nz), (nx, ny + 1, nz), (nx, ny, nz + 1)]
    for c in range(3):
        for k in range(lim_e[c][2]):
            for j in range(lim_e[c][1]):
                for i in range(lim_e[c][0]):
                    e.append((c, i, j, k))
    for c in range(3):
        for k in range(lim_h[c][2]):
            for j in range(lim_h[c][1]):
                for i in range(lim_h[c][0]):
                    h.append((c, i, j, k))
    return e, h


def stokes_curl(n, d):
    """Matrix C (n_H x n_E): (curl E) at each face = circulation / area.

    A face normal to axis a at lower corner p spans tangent axes b = a+1 and
    c = a+2 (cyclic).  Walking its boundary in the right-hand sense around
    +a: the b-edge at p (+), the c-edge at p+e_b (+), the b-edge at p+e_c
    (-), the c-edge at p (-).
    """
    e, h = dof_lists(n)
    eidx = {t: r for r, t in enumerate(e)}
    C = np.zeros((len(h), len(e)))
    for row, (a, i, j, k) in enumerate(h):
        b, c = (a + 1) % 3, (a + 2) % 3
        area = d[b] * d[c]
        p = [i, j, k]
        pb = list(p); pb[b] += 1
        pc = list(p); pc[c] += 1
        for comp, q, sgn in ((b, p, +1), (c, pb, +1), (b, pc, -1), (c, p, -1)):
            key = (comp, q[0], q[1], q[2])
            if key in eidx:
                C[row, eidx[key]] += sgn * d[comp] / area
    return C, e, h


def interior_edge(n, t):
    nx, ny, nz = n
    c, i, j, k = t
    if c == 0:
        return 0 < j < ny and 0 < k < nz
    if c == 1:
        return 0 < i < nx and 0 < k < nz
    return 0 < i < nx and 0 < j < ny


def exact_fma32(a, b, c):
    """Correctly rounded float32 fused multiply-add, via exact rationals."""
    from fractions import Fraction
    a, b, c = np.float32(a), np.float32(b), np.float32(c)
    r = Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))
    g = np.float32(float(r))
    best = None
    for cand in (np.nextafter(g, np.float32(-np.inf)), g, np.nextafter(g, np.float32(np.inf))):
        err = abs(Fraction(float(cand)) - r)
        if best is None or err < best[0] or (err == best[0] and (int(cand.view(np.uint32)) & 1) == 0):
            best = (err, cand)
    return np.float32(best[1])
