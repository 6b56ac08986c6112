"""Positively split Ewald decomposition of the periodic FT-RPY mobility (oracle).

The paper evaluates the far-field mobility with the PSE method (Section 2.2.3
and Eq. `UBff`: real-space plus wave-space parts); the details of the split
are those of Hasimoto's damping applied to the exact RPY multipliers:

    H(k)   = (1 + k^2 / (4 xi^2)) exp(-k^2 / (4 xi^2)),
    wave:  tt sinc^2(ka) H (I - kk)/(eta k^2),  rr jv^2(ka) H (I - kk)/(4 eta),
           rt (i/2) sinc(ka) jv(ka) H [k]x / (eta k^2),
    real:  the free-space RPY block minus the inverse transform S of the wave
           multipliers (a smooth, rapidly decaying function of r).

Both halves are symmetric positive semi-definite, which is what makes the
split usable for Brownian sampling.  This module evaluates S by adaptive
quadrature of the radial integrals and the wave part by a direct k-sum, so
the GPU's two halves can be checked one at a time.  It is slow by design.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from scipy.integrate import quad
from scipy.special import spherical_jn

from . import rpy


def _H(k, xi):
    q = k * k / (4 * xi * xi)
    return (1 + q) * math.exp(-q)


def _sinc_jv(y):
    if y == 0.0:
        return 1.0, 1.0
    return float(spherical_jn(0, y)), 3.0 * float(spherical_jn(1, y)) / y


@functools.lru_cache(maxsize=200000)
def smooth_part(r, a, eta, xi):
    """(tI, tR, rI, rR, c) of S(r), the inverse transform of the PSE wave multipliers."""
    kmax = 2 * xi * math.sqrt(46.0) * 1.2

    def rad(f):
        return quad(f, 0.0, kmax, limit=1000, epsabs=1e-17, epsrel=1e-13)[0]

    def phi_tt(k):
        s, _ = _sinc_jv(k * a)
        return s * s * _H(k, xi)

    def phi_rr(k):
        _, j = _sinc_jv(k * a)
        return 0.25 * k * k * j * j * _H(k, xi)

    def phi_rt(k):
        s, j = _sinc_jv(k * a)
        return s * j * _H(k, xi)

    def fI(x):
        if x < 1e-8:
            return 2.0 / 3.0
        return spherical_jn(0, x) - spherical_jn(1, x) / x

    p = 1.0 / (2 * math.pi ** 2 * eta)
    tI = p * rad(lambda k: phi_tt(k) * fI(k * r))
    tR = p * rad(lambda k: phi_tt(k) * spherical_jn(2, k * r))
    rI = p * rad(lambda k: phi_rr(k) * fI(k * r))
    rR = p * rad(lambda k: phi_rr(k) * spherical_jn(2, k * r))
    c = -1.0 / (4 * math.pi ** 2 * eta) * rad(lambda k: k * phi_rt(k) * spherical_jn(1, k * r))
    return tI, tR, rI, rR, c


def real_functions(r, a, eta, xi):
    """PSE real-space scalar functions (tI, tR, rI, rR, c) at distances r > 0."""
    r = np.atleast_1d(np.asarray(r, dtype=float))
    free = rpy.rpy_scalars(r, a, eta)
    out = np.zeros((len(r), 5))
    for m, rv in enumerate(r):
        S = smooth_part(float(rv), a, eta, xi)
        out[m] = [free[k][m] - S[k] for k in range(5)]
    return out


def self_terms(a, eta, xi):
    S = smooth_part(0.0, a, eta, xi)
    return rpy.mu_t(a, eta) - S[0], rpy.mu_r(a, eta) - S[2]


def real_mobility(x, L, a, eta, xi, r_cut, strain=0.0):
    """Dense real-space part: sum over images with |x_i - x_j + A n| < r_cut, plus self
    (A n = (n_x + strain n_y, n_y, n_z) L, the sheared lattice; the cube at strain 0)."""
    x = np.asarray(x, dtype=float)
    n = len(x)
    M = np.zeros((n, n, 6, 6))
    nmax = int(math.ceil(r_cut / L)) + 1
    d0 = x[:, None, :] - x[None, :, :]
    rng = range(-nmax, nmax + 1)
    mx = nmax + int(math.ceil(abs(strain) * nmax))
    for nx in range(-mx, mx + 1):
        for ny in rng:
            for nz in rng:
                d = d0 + L * np.array([nx + strain * ny, ny, nz], dtype=float)
                r = np.linalg.norm(d, axis=-1)
                mask = (r < r_cut) & (r > 0)
                if not mask.any():
                    continue
                idx = np.nonzero(mask)
                f = real_functions(r[idx], a, eta, xi)
                M[idx] += rpy.blocks_from_scalars(d[idx], *f.T)
    st, sr = self_terms(a, eta, xi)
    for i in range(n):
        M[i, i, :3, :3] += st * np.eye(3)
        M[i, i, 3:, 3:] += sr * np.eye(3)
    return M.transpose(0, 2, 1, 3).reshape(6 * n, 6 * n)


def wave_mobility(x, L, a, eta, xi, kc=None, strain=0.0):
    """Dense wave-space part by a direct sum over |k| < kc (default: Gaussian below 1e-20),
    over the reciprocal lattice of the (sheared) lattice."""
    if kc is None:
        kc = 2 * xi * math.sqrt(46.0)
    kv, k2 = rpy.wave_vectors(L, kc, strain)
    kn = np.sqrt(k2)
    y = kn * a
    s = np.sin(y) / y
    j = 3 * (np.sin(y) - y * np.cos(y)) / y ** 3
    small = y < 1e-2
    j[small] = 1 - y[small] ** 2 / 10
    q = k2 / (4 * xi * xi)
    H = (1 + q) * np.exp(-q)
    n = len(x)
    Mt, Mr, Mrt = rpy.wave_sum(x, L, kv, s * s * H / k2, 0.25 * j * j * H, s * j * H / kn, eta)
    return rpy.add_wave(np.zeros((6 * n, 6 * n)), Mt, Mr, Mrt)
