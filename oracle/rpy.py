"""Force-torque Rotne-Prager-Yamakawa mobility, free space and periodic.

Each bead carries a force f and a torque t; the mobility maps them to its
translational and angular velocity (u, w).  The far-field mobility of the
paper (Section 2.2, the M-infinity block of Eq. `SP1`; Section 2.3,
Eq. `spm_agg`) is taken at force-torque level: per bead pair a 6x6 block
[[tt, tr], [rt, rr]].

Spectral definition (periodic cube of side L, V = L^3, k in (2 pi / L) Z^3 minus 0,
sinc(x) = sin x / x, jv(x) = 3 (sin x - x cos x) / x^3, r = x_i - x_j):

    tt(r) = 1/(eta V) sum_k sinc^2(ka)             (I - kk/k^2) / k^2 cos(k.r)
    rt(r) = 1/(eta V) sum_k (i/2) sinc(ka) jv(ka)  [k]x / k^2       e^{i k.r}
    rr(r) = 1/(eta V) sum_k (1/4) jv^2(ka)         (I - kk/k^2)     cos(k.r)

with [v]x w = v x w.  tr equals rt.  Sums of this kind converge far too slowly
to be summed directly, so the periodic mobility is evaluated by Ewald
splitting: a multiplier m(k) is written m H + m (1 - H) with a damping H(k)
that decays like a Gaussian; the first part is summed over wave vectors, the
second is transformed to real space and summed over periodic images.

The oracle deliberately uses Beenakker's damping
    H_B(k) = (1 + u + 2 u^2) e^{-u},  u = k^2 / (4 xi^2)
applied to the far-field (point-particle RPY) multipliers
    tt: (1 - a^2 k^2 / 3),  rt: 1,  rr: 1/4 k^2 (in the (I-kk)/k^2 form),
plus the exact local correction for overlapping beads (r < 2a) and the self
term.  The GPU path uses a different split (Hasimoto damping on the exact
sinc/jv multipliers), so agreement between the two is not an artefact of a
shared formula.  The result does not depend on xi (a pinned property).

Real-space functions come from radial inverse transforms of
phi(k) = sum_p c_p k^(2p) exp(-k^2 / (4 xi^2)): for the tensor form
(1/eta) phi(k) (I - kk/k^2) / k^2 its inverse transform is

    (1/eta) [ (A + B'/r) I - (A + 3 B'/r) rr/r^2 ],
    A(r)  = IFT[phi / k^2](r),
    B'(r) = -(1/r^2) int_0^r s^2 A(s) ds,

and IFT[(i/2) phi [k]x / k^2] = (1/2) A'(r) [r_hat]x.  With
g(r) = IFT[exp(-k^2/4 xi^2)] = (xi/sqrt(pi))^3 exp(-xi^2 r^2) and
IFT[k^2 f] = -Laplacian IFT[f], every term is an erf or a polynomial times a
Gaussian, and the polynomials are manipulated exactly.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as P
from scipy.special import erf, erfc, gamma

SQPI = math.sqrt(math.pi)


def mu_t(a, eta):
    """Stokes translational self-mobility 1/(6 pi eta a) (drag of Section 2.3)."""
    return 1.0 / (6.0 * math.pi * eta * a)


def mu_r(a, eta):
    """Rotational self-mobility 1/(8 pi eta a^3)."""
    return 1.0 / (8.0 * math.pi * eta * a ** 3)


def _outer(rhat):
    return rhat[..., :, None] * rhat[..., None, :]


def _cross_matrix(v):
    """[v]x such that [v]x w = v x w, for arrays (..., 3)."""
    z = np.zeros(v.shape[:-1])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], -1),
        np.stack([v[..., 2], z, -v[..., 0]], -1),
        np.stack([-v[..., 1], v[..., 0], z], -1),
    ], -2)


# --------------------------------------------------------------------------
# free space
# --------------------------------------------------------------------------

def rpy_scalars(r, a, eta):
    """Free-space FT-RPY as scalar functions of the distance r (array).

    Returns (tI, tR, rI, rR, c) with
        tt = tI I + tR rr^,   rr = rI I + rR rr^,   rt = tr = c [r^]x.
    Non-overlapping (r >= 2a) and overlapping (r < 2a) branches; at r = 0
    tt = mu_t I, rr = mu_r I, rt = 0.
    """
    r = np.asarray(r, dtype=float)
    mt, mr = mu_t(a, eta), mu_r(a, eta)
    far = r >= 2.0 * a
    rs = np.where(far, r, 1.0)
    tI = np.where(far, (1.0 + 2.0 * a * a / (3.0 * rs * rs)) / (8.0 * math.pi * eta * rs),
                  mt * (1.0 - 9.0 * r / (32.0 * a)))
    tR = np.where(far, (1.0 - 2.0 * a * a / (rs * rs)) / (8.0 * math.pi * eta * rs),
                  mt * 3.0 * r / (32.0 * a))
    rI = np.where(far, -1.0 / (16.0 * math.pi * eta * rs ** 3),
                  mr * (1.0 - 27.0 * r / (32.0 * a) + 5.0 * r ** 3 / (64.0 * a ** 3)))
    rR = np.where(far, 3.0 / (16.0 * math.pi * eta * rs ** 3),
                  mr * (9.0 * r / (32.0 * a) - 3.0 * r ** 3 / (64.0 * a ** 3)))
    c = np.where(far, -1.0 / (8.0 * math.pi * eta * rs * rs),
                 -(r / a) * (1.0 - 3.0 * r / (8.0 * a)) / (16.0 * math.pi * eta * a * a))
    return tI, tR, rI, rR, c


def rpy_far_scalars(r, a, eta):
    """Point-particle (non-overlapping) branch used for every r > 0."""
    rs = np.asarray(r, dtype=float)
    tI = (1.0 + 2.0 * a * a / (3.0 * rs * rs)) / (8.0 * math.pi * eta * rs)
    tR = (1.0 - 2.0 * a * a / (rs * rs)) / (8.0 * math.pi * eta * rs)
    rI = -1.0 / (16.0 * math.pi * eta * rs ** 3)
    rR = 3.0 / (16.0 * math.pi * eta * rs ** 3)
    c = -1.0 / (8.0 * math.pi * eta * rs * rs)
    return tI, tR, rI, rR, c


def blocks_from_scalars(rvec, tI, tR, rI, rR, c):
    """6x6 pair blocks [[tt, tr], [rt, rr]] for displacements rvec (..., 3)."""
    r = np.linalg.norm(rvec, axis=-1)
    rhat = rvec / np.where(r > 0, r, 1.0)[..., None]
    eye = np.eye(3)
    rr_ = _outer(rhat)
    tt = tI[..., None, None] * eye + tR[..., None, None] * rr_
    rot = rI[..., None, None] * eye + rR[..., None, None] * rr_
    rt = c[..., None, None] * _cross_matrix(rhat)
    out = np.zeros(r.shape + (6, 6))
    out[..., :3, :3] = tt
    out[..., 3:, :3] = rt
    out[..., :3, 3:] = rt
    out[..., 3:, 3:] = rot
    return out


def rpy_free_block(rvec, a, eta):
    r = np.linalg.norm(rvec, axis=-1)
    return blocks_from_scalars(rvec, *rpy_scalars(r, a, eta))


def rpy_free_matrix(x, a, eta):
    """Dense 6N x 6N free-space FT-RPY mobility of bead positions x (N, 3)."""
    n = len(x)
    d = x[:, None, :] - x[None, :, :]
    B = rpy_free_block(d, a, eta)
    return B.transpose(0, 2, 1, 3).reshape(6 * n, 6 * n)


# --------------------------------------------------------------------------
# Gaussian-polynomial inverse transforms
# --------------------------------------------------------------------------

class DampedMultiplier:
    """phi(k) = sum_p c[p] k^(2p) exp(-k^2 / (4 xi^2)) and its radial transforms.

    Polynomials in t = r^2 represent functions Q(t) exp(-xi^2 t).
      Laplacian[Q e] = [6 (Q' - xi^2 Q) + 4 t (Q'' - 2 xi^2 Q' + xi^4 Q)] e
      d/dr [Q e]     = r * 2 (Q' - xi^2 Q) e
    """

    def __init__(self, c, xi):
        self.c = np.asarray(c, dtype=float)
        self.xi = float(xi)
        x2 = self.xi ** 2
        g0 = np.array([(self.xi / SQPI) ** 3])
        self.G = [g0]                               # G[q] e = (-Lap)^q g
        for _ in range(len(self.c)):
            Q = self.G[-1]
            dQ, d2Q = P.polyder(Q), P.polyder(Q, 2)
            lap = P.polyadd(6.0 * P.polysub(dQ, x2 * Q),
                            P.polymulx(4.0 * P.polyadd(P.polysub(d2Q, 2 * x2 * dQ), x2 * x2 * Q)))
            self.G.append(-lap)
        # D[q]: d/dr (G[q] e) = r D[q](t) e
        self.D = [2.0 * P.polysub(P.polyder(Q), x2 * Q) if len(Q) > 1 else -2.0 * x2 * Q
                  for Q in self.G]

    @staticmethod
    def _val(Q, t):
        return P.polyval(t, Q)

    def A(self, r):
        """IFT[phi / k^2](r), r > 0."""
        xi, t = self.xi, r * r
        e = np.exp(-xi * xi * t)
        out = self.c[0] * erf(xi * r) / (4 * math.pi * r)
        for p in range(1, len(self.c)):
            out = out + self.c[p] * self._val(self.G[p - 1], t) * e
        return out

    def dA(self, r):
        """d/dr IFT[phi / k^2](r), r > 0."""
        xi, t = self.xi, r * r
        e = np.exp(-xi * xi * t)
        out = self.c[0] * (2 * xi / SQPI * e / r - erf(xi * r) / (r * r)) / (4 * math.pi)
        for p in range(1, len(self.c)):
            out = out + self.c[p] * r * self._val(self.D[p - 1], t) * e
        return out

    def S2(self, r):
        """int_0^r s^2 A(s) ds."""
        xi, t = self.xi, r * r
        e = np.exp(-xi * xi * t)
        er = erf(xi * r)
        out = self.c[0] * ((t / 2 - 1 / (4 * xi * xi)) * er + r * e / (2 * xi * SQPI)) / (4 * math.pi)
        if len(self.c) > 1:
            out = out + self.c[1] * (er / (4 * math.pi) - xi * r * e / (2 * math.pi ** 1.5))
        for p in range(2, len(self.c)):
            out = out - self.c[p] * t * r * self._val(self.D[p - 2], t) * e
        return out

    def A0(self):
        """IFT[phi / k^2](0) = (1 / 2 pi^2) int_0^inf phi dk."""
        s = 2 * self.xi
        mom = [gamma(p + 0.5) * s ** (2 * p + 1) / 2 for p in range(len(self.c))]
        return float(np.dot(self.c, mom)) / (2 * math.pi ** 2)

    def tensor_scalars(self, r):
        """(I-coefficient, rr-coefficient) of IFT[phi (I - kk/k^2) / k^2], eta = 1."""
        A = self.A(r)
        Bp = -self.S2(r) / (r * r)
        return A + Bp / r, -(A + 3 * Bp / r)


def _poly_k2(coeffs_u, xi):
    """Convert a polynomial in u = k^2/(4 xi^2) to one in k^2."""
    return np.array([cu / (4 * xi * xi) ** p for p, cu in enumerate(coeffs_u)])


def beenakker_multipliers(a, xi):
    """Damped far-field multipliers phi_tt, phi_rr, phi_rt (coefficients in k^2)."""
    hb = _poly_k2([1.0, 1.0, 2.0], xi)                      # (1 + u + 2u^2)
    tt = P.polymul([1.0, -a * a / 3.0], hb)
    rr = P.polymulx(0.25 * hb)
    rt = hb
    return (DampedMultiplier(tt, xi), DampedMultiplier(rr, xi), DampedMultiplier(rt, xi))


# --------------------------------------------------------------------------
# periodic mobility, Beenakker split
# --------------------------------------------------------------------------

def _real_scalars(r, a, eta, mults):
    """Real-space Ewald functions at r > 0 (tI, tR, rI, rR, c)."""
    mtt, mrr, mrt = mults
    tI, tR, rI, rR, c = rpy_scalars(r, a, eta)
    sI, sR = mtt.tensor_scalars(r)
    qI, qR = mrr.tensor_scalars(r)
    sc = 0.5 * mrt.dA(r)
    return (tI - sI / eta, tR - sR / eta, rI - qI / eta, rR - qR / eta, c - sc / eta)


def self_blocks(a, eta, xi):
    """Real-space self term (n = 0, i = j) of the Beenakker split (diagonal)."""
    mtt, mrr, _ = beenakker_multipliers(a, xi)
    st = mu_t(a, eta) - (2.0 / 3.0) * mtt.A0() / eta
    sr = mu_r(a, eta) - (2.0 / 3.0) * mrr.A0() / eta
    return st, sr


def default_xi(L, n_bead, r_cut_factor=6.5):
    """Pick the oracle's own xi by balancing real-space and wave-space work.

    Cost model (seconds, measured on numpy/BLAS): every image shift touches all
    n^2 pairs (~15 ns each), every pair inside the cutoff costs ~0.5 us, and the
    wave sum costs ~216 n^2 K flops at ~1e11 flop/s.
    """
    best = None
    for xi in np.geomspace(0.03, 3.0, 200):
        rc = r_cut_factor / xi
        nshift = (2 * (math.ceil(rc / L) + 1) + 1) ** 3
        inside = n_bead * n_bead * (4 * math.pi / 3) * rc ** 3 / L ** 3
        kc = 2 * r_cut_factor * xi
        nk = (4 * math.pi / 3) * (kc * L / (2 * math.pi)) ** 3 / 2
        cost = nshift * n_bead ** 2 * 15e-9 + inside * 0.5e-6 + 216 * n_bead ** 2 * nk / 1e11
        if best is None or cost < best[0]:
            best = (cost, xi)
    return float(best[1])


def periodic_mobility(x, L, a=1.0, eta=1.0, xi=None, r_cut_factor=6.5, k_chunk=2048, strain=0.0):
    """Dense 6N x 6N periodic FT-RPY mobility (row/col order: bead, then f/t).

    Real space: all images n with |x_i - x_j + A n| < r_cut_factor / xi.
    Wave space: all k != 0 with |k| < 2 r_cut_factor xi.  r_cut_factor = 6.5
    leaves truncation errors near 1e-14 relative (exp(-42) times the
    polynomial prefactors of the split).

    The lattice is A n = (n_x L + n_y gamma L, n_y L, n_z L) for strain gamma (a cube at
    gamma = 0); its reciprocal vectors are k = 2 pi A^-T m = (2 pi / L)(m_x, m_y - gamma m_x,
    m_z) and the cell volume stays L^3.
    """
    x = np.asarray(x, dtype=float)
    n = len(x)
    if xi is None:
        xi = default_xi(L, n, r_cut_factor)
    mults = beenakker_multipliers(a, xi)
    M = np.zeros((n, n, 6, 6))

    # ---- real space -------------------------------------------------------
    rc = r_cut_factor / xi
    nmax = int(math.ceil(rc / L)) + 1
    d0 = x[:, None, :] - x[None, :, :]
    rng = range(-nmax, nmax + 1)
    mx = nmax + int(math.ceil(abs(strain) * nmax))
    for nx in range(-mx, mx + 1):
        for ny in rng:
            for nz in rng:
                d = d0 + L * np.array([nx + strain * ny, ny, nz], dtype=float)
                r = np.linalg.norm(d, axis=-1)
                mask = (r < rc) & (r > 0)
                if not mask.any():
                    continue
                idx = np.nonzero(mask)
                sc = _real_scalars(r[idx], a, eta, mults)
                M[idx] += blocks_from_scalars(d[idx], *sc)
    st, sr = self_blocks(a, eta, xi)
    for i in range(n):
        M[i, i, :3, :3] += st * np.eye(3)
        M[i, i, 3:, 3:] += sr * np.eye(3)
    M = M.transpose(0, 2, 1, 3).reshape(6 * n, 6 * n)

    # ---- wave space (half space of k; k and -k combined) --------------------
    kv, k2 = wave_vectors(L, 2 * r_cut_factor * xi, strain)
    u = k2 / (4 * xi * xi)
    hb = (1 + u + 2 * u * u) * np.exp(-u)
    Mt, Mr, Mrt = wave_sum(x, L, kv, (1 - a * a * k2 / 3) * hb / k2, 0.25 * hb, hb / np.sqrt(k2),
                           eta, k_chunk)
    return add_wave(M, Mt, Mr, Mrt)



def wave_vectors(L, kc, strain=0.0):
    """Half space of the reciprocal lattice k = (2 pi / L)(m_x, m_y - gamma m_x, m_z),
    0 < |k| < kc (one of each +-k pair)."""
    m = int(math.ceil(kc * L / (2 * math.pi)))
    g = np.arange(-m, m + 1)
    my = m + int(math.ceil(abs(strain) * m))
    gy = np.arange(-my, my + 1)
    ks = np.stack(np.meshgrid(g, gy, g, indexing="ij"), -1).reshape(-1, 3)
    pos = (ks[:, 0] > 0) | ((ks[:, 0] == 0) & ((ks[:, 1] > 0) | ((ks[:, 1] == 0) & (ks[:, 2] > 0))))
    ms = ks[pos].astype(float)
    ms[:, 1] -= strain * ms[:, 0]
    kv = (2 * math.pi / L) * ms
    k2 = np.einsum("ij,ij->i", kv, kv)
    keep = k2 < kc * kc
    return kv[keep], k2[keep]


def wave_sum(x, L, kv, m_tt, m_rr, m_rt, eta=1.0, k_chunk=2048):
    """Dense wave-space blocks for multipliers given per k (half space):

        tt: m_tt (I - kk) cos(k.r),  rr: m_rr (I - kk) cos(k.r),
        rt: (i/2) m_rt [k^]x e^{ik.r} summed with its -k partner,

    each times 2 / (eta V) (the -k partner of tt/rr), i.e. the full lattice sum.
    Returns (Mt, Mr, Mrt) as 3N x 3N arrays; Mrt maps force to angular velocity.
    """
    x = np.asarray(x, dtype=float)
    n = len(x)
    V = L ** 3
    w_tt = 2.0 / (eta * V) * m_tt
    w_rr = 2.0 / (eta * V) * m_rr
    w_rt = 1.0 / (eta * V) * m_rt
    kn = np.linalg.norm(kv, axis=1)
    khat = kv / kn[:, None]
    # two unit vectors orthogonal to k, (e1, e2, k^) right-handed
    ref = np.where(np.abs(khat[:, 2:3]) < 0.9, [[0.0, 0.0, 1.0]], [[1.0, 0.0, 0.0]])
    e1 = np.cross(ref, khat)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(khat, e1)
    Mt = np.zeros((3 * n, 3 * n))
    Mr = np.zeros((3 * n, 3 * n))
    Mrt = np.zeros((3 * n, 3 * n))
    for s in range(0, len(kv), k_chunk):
        sl = slice(s, s + k_chunk)
        ph = x @ kv[sl].T                           # (n, K)
        cs, sn = np.cos(ph), np.sin(ph)
        E1, E2 = e1[sl], e2[sl]

        def cols(a_, E):
            return (a_[:, None, :] * E.T[None, :, :]).reshape(3 * n, -1)
        C1, C2, S1, S2 = cols(cs, E1), cols(cs, E2), cols(sn, E1), cols(sn, E2)
        Z = np.concatenate([C1, C2, S1, S2], axis=1)
        Mt += (Z * np.tile(w_tt[sl], 4)) @ Z.T
        Mr += (Z * np.tile(w_rr[sl], 4)) @ Z.T
        # rt pair sum: -w sin(k.(xi - xj)) (e2 e1^T - e1 e2^T),
        # sin(k.(xi-xj)) = s_i c_j - c_i s_j
        wr = np.tile(w_rt[sl], 4)
        Zl = np.concatenate([S2, -S1, -C2, C1], axis=1)
        Mrt -= (Zl * wr) @ Z.T
    return Mt, Mr, Mrt


def add_wave(M, Mt, Mr, Mrt):
    """Add 3N x 3N wave blocks into a 6N x 6N mobility (tr = rt transposed)."""
    n = M.shape[0] // 6
    M6 = M.reshape(n, 6, n, 6)
    M6[:, :3, :, :3] += Mt.reshape(n, 3, n, 3)
    M6[:, 3:, :, 3:] += Mr.reshape(n, 3, n, 3)
    M6[:, 3:, :, :3] += Mrt.reshape(n, 3, n, 3)
    M6[:, :3, :, 3:] += Mrt.reshape(n, 3, n, 3).transpose(2, 3, 0, 1)
    return M6.reshape(6 * n, 6 * n)


HASIMOTO = 2.837297479480619   # simple-cubic lattice constant of periodic Stokes flow


def hasimoto_self(L, a=1.0, eta=1.0):
    """Periodic single-bead mobilities (translational, rotational).

    U/F = mu_t (1 - 2.8373 a/L + (4 pi / 3)(a/L)^3) and
    W/T = mu_r (1 - (4 pi / 3)(a/L)^3) for the RPY bead in a cubic lattice;
    the paper uses the leading correction 1 + 2.84 R_h / L (Section 3.1.3).
    """
    v = 4 * math.pi / 3 * (a / L) ** 3
    return mu_t(a, eta) * (1 - HASIMOTO * a / L + v), mu_r(a, eta) * (1 - v)
