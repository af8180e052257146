"""Oracle O2 -- the fast summation's steps in plain FP64 numpy.  TEST INFRASTRUCTURE ONLY.

The paper evaluates its eq. (2) with NFFTs: the point data are spread onto a
regular grid X with a smooth, localized window; the Green function is first
smoothed near the origin and corrected afterwards in the smoothing zone; a
grid of size about p^2 N (2D) with p the smoothness degree is used; an FFT is
taken and divided by the window's Fourier coefficients.  The paper stops at
the spectrum; the remaining steps are the standard regularized-kernel fast
summation (multiply by the Fourier coefficients of the smoothed kernel,
transform back, interpolate at the targets with the same window, add the
near-field correction).  This module takes those steps one by one:

  S0  torus map     c = bounding-box midpoint, D = 2 max |p - c| over all points,
                    s = (1/2 - eps_B)/D; every pairwise distance <= 1/2 - eps_B.
  S0' plan          K(r) = -(1/2pi) ln r.  K_R(r) = T_I(r) for r < eps_I (even
                    polynomial of degree 2p-2 matching K and its first p-1
                    derivatives at eps_I); K(r) for eps_I <= r <= 1/2-eps_B;
                    T_B(r) on (1/2-eps_B, 1/2] (degree 2p-2, matching K and p-1
                    derivatives at 1/2-eps_B, first p-1 derivatives zero at 1/2);
                    T_B(1/2) beyond.  b_l = (1/n^2) sum_{j in I_n} K_R(|j|/n)
                    e^{-2 pi i j.l/n}.  Kaiser-Bessel window psi(t) =
                    sinh(b sqrt(m^2-t^2)) / (pi sqrt(m^2-t^2)) on |t| < m cells,
                    b = pi (2 - 1/sigma), sigma = G/n (2 unless the bandwidth
                    n is set; the paper leaves the NFFT's oversampling to the
                    NFFT package), with its Fourier
                    transform I0(m sqrt(b^2 - (2 pi xi)^2)); both divided by
                    I0(m b) (a constant that cancels).
  S2  spread        g_k = sum_j s_j psi(G x_j1 - k1) psi(G x_j2 - k2), 2m taps/dim.
  S3  FFT           g^_l = sum_k g_k e^{-2 pi i l.k/G}.
  S4  multiply      f^_l = omega_l b_l g^_l / (psi^(l1/G) psi^(l2/G))^2 on
                    |l1|,|l2| <= n/2 (omega = 1/2 per Nyquist index n/2 so the
                    trigonometric interpolant of K_R is real), times -2 pi i l_d
                    for the gradient components.
  S5  inverse FFT   g'_k = sum_l f^_l e^{2 pi i l.k/G}.
  S6  gather        f(y_i) = sum_k g'_k psi(G y_i1 - k1) psi(G y_i2 - k2).
  S7  near field    for |y_i - x_j| < eps_I add s_j (K - T_I)(r); H adds
                    -s_j grad(K - T_I).  Then
                    phi = far + near + (ln s / 2pi) sum_j s_j,  H = s (far + near).
                    A pair at r = 0 is not part of the exact sum: it removes its far
                    value T_I(0) and its share ln(s)/2pi of the offset, i.e. adds
                    -s_j (T_I(0) + ln(s)/2pi).
  S8  adjoint       the exact transpose of S2..S7 with respect to the charges.

Every library call is a plain primitive (numpy FFT, scipy sparse matvec for the
window sums, a KD-tree for the near pairs).  direct_ndft() gives the windowless
far field for tiny inputs, which pins the window, the deconvolution constant
and the DFT sign.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np
from scipy import fft as sfft
from scipy import sparse, special
from scipy.spatial import cKDTree

TWO_PI = 2.0 * np.pi

# The 2D FFTs are scipy's (the same pocketfft transform as numpy's) with worker threads:
# a G = 8192 transform then takes a fraction of a second instead of seconds.
_WORKERS = max(1, int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1))


def fft2(a):
    return sfft.fft2(a, workers=_WORKERS)


def ifft2(a):
    return sfft.ifft2(a, workers=_WORKERS)


def fftn_w(a):
    return sfft.fftn(a, workers=_WORKERS)


def ifftn_w(a):
    return sfft.ifftn(a, workers=_WORKERS)


@dataclass
class Params:
    G: int            # FFT grid per dimension (oversampled)
    m: int            # window half-width in grid cells (2m taps per dimension)
    p: int            # regularization (smoothness) degree
    eps_I: float      # near-field radius, torus units
    eps_B: float = 1.0 / 16.0  # boundary regularization width, torus units
    band: int = 0     # bandwidth n (even, G/2 <= n < G); 0 means n = G/2 (oversampling 2)

    @property
    def n(self):
        return self.band if self.band else self.G // 2

    @property
    def kb_b(self):
        sigma = self.G / self.n
        return np.pi * (2.0 - 1.0 / sigma)


# ----------------------------------------------------------------------------
# S0' the regularized kernel
# ----------------------------------------------------------------------------

def K(r):
    return -np.log(r) / TWO_PI


def K_scaled_deriv(q, r):
    """r^q K^{(q)}(r)."""
    if q == 0:
        return float(K(r))
    return -((-1.0) ** (q - 1)) * math.factorial(q - 1) / TWO_PI


def _ff(a, q):
    """Falling factorial a (a-1) ... (a-q+1); zero if q > a."""
    if q > a:
        return 0.0
    out = 1.0
    for i in range(q):
        out *= (a - i)
    return out


def inner_coeffs(p, eps_I):
    """a_k with T_I(r) = sum_{k<p} a_k (r/eps_I)^{2k}, T_I^{(q)}(eps_I) = K^{(q)}(eps_I), q < p."""
    A = np.array([[_ff(2 * k, q) for k in range(p)] for q in range(p)])
    rhs = np.array([K_scaled_deriv(q, eps_I) for q in range(p)])
    return np.linalg.solve(A, rhs)


def boundary_coeffs(p, eps_B):
    """c_k with T_B(r) = sum_{k<=2p-2} c_k t^k, t = (r - r_B)/eps_B, r_B = 1/2 - eps_B.

    T_B^{(q)}(r_B) = K^{(q)}(r_B) for q < p and T_B^{(q)}(1/2) = 0 for 1 <= q < p.
    """
    rB = 0.5 - eps_B
    c = np.zeros(2 * p - 1)
    for q in range(p):
        c[q] = K_scaled_deriv(q, rB) * (eps_B / rB) ** q / math.factorial(q)
    if p > 1:
        unk = list(range(p, 2 * p - 1))
        A = np.array([[_ff(k, q) for k in unk] for q in range(1, p)])
        rhs = -np.array([sum(c[k] * _ff(k, q) for k in range(p)) for q in range(1, p)])
        c[p:] = np.linalg.solve(A, rhs)
    return c


def K_R(r, prm: Params):
    """The regularized (smoothed, periodizable) kernel as a function of radius."""
    r = np.asarray(r, dtype=np.float64)
    a = inner_coeffs(prm.p, prm.eps_I)
    c = boundary_coeffs(prm.p, prm.eps_B)
    rB = 0.5 - prm.eps_B
    out = np.empty_like(r)
    m_in = r < prm.eps_I
    m_mid = (r >= prm.eps_I) & (r <= rB)
    m_bd = (r > rB) & (r <= 0.5)
    m_out = r > 0.5
    rho2 = (r[m_in] / prm.eps_I) ** 2
    out[m_in] = sum(a[k] * rho2 ** k for k in range(prm.p))
    out[m_mid] = K(r[m_mid])
    t = (r[m_bd] - rB) / prm.eps_B
    out[m_bd] = sum(c[k] * t ** k for k in range(len(c)))
    out[m_out] = c.sum()
    return out


def b_coeffs(prm: Params):
    """b_l, l in I_n (numpy FFT order, n x n): DFT of K_R sampled on the n-grid."""
    n = prm.n
    j = np.fft.fftfreq(n) * n
    J1, J2 = np.meshgrid(j, j, indexing="ij")
    samples = K_R(np.hypot(J1, J2) / n, prm)
    return fft2(samples).real / (n * n)


# ----------------------------------------------------------------------------
# Kaiser-Bessel window
# ----------------------------------------------------------------------------

def kb_psi(t, m, b):
    """Window in grid-cell units, normalized by I0(m b); zero for |t| >= m."""
    t = np.asarray(t, dtype=np.float64)
    z2 = m * m - t * t
    out = np.zeros_like(t)
    ok = z2 > 0
    z = np.sqrt(z2[ok])
    # sinh(bz)/I0(mb) = e^{b(z-m)} (1 - e^{-2bz}) / (2 i0e(mb))
    out[ok] = np.exp(b * (z - m)) * (-np.expm1(-2.0 * b * z)) / (2.0 * np.pi * z * special.i0e(m * b))
    return out


def kb_psi_hat(xi, m, b):
    """Continuous Fourier transform of kb_psi at xi cycles/cell (|2 pi xi| < b)."""
    xi = np.asarray(xi, dtype=np.float64)
    a = m * np.sqrt(b * b - (TWO_PI * xi) ** 2)
    return special.i0e(a) / special.i0e(m * b) * np.exp(a - m * b)


# ----------------------------------------------------------------------------
# S0 torus map
# ----------------------------------------------------------------------------

def torus_map(y, x, eps_B, extra=None):
    """c, s and the mapped points; extra points take part in c and D only."""
    allp = np.concatenate([y, x] + ([np.asarray(extra, np.float64)] if extra is not None else []), axis=0)
    lo, hi = allp.min(0), allp.max(0)
    c = 0.5 * (lo + hi)
    D = 2.0 * np.sqrt(((allp - c) ** 2).sum(1).max())
    if not D > 0:
        raise ValueError("all points coincide")
    s = (0.5 - eps_B) / D
    return c, s, s * (y - c), s * (x - c)


# ----------------------------------------------------------------------------
# S2 / S6 window sums as a sparse matrix
# ----------------------------------------------------------------------------

def window_matrix(pt, prm: Params):
    """B with B[k1*G + k2, j] = psi(G pt_j1 - k1) psi(G pt_j2 - k2) (k mod G)."""
    G, m, b = prm.G, prm.m, prm.kb_b
    N = len(pt)
    a = np.arange(2 * m)
    taps, wts = [], []
    for d in range(2):
        u = pt[:, d] * G
        k = np.floor(u)[:, None] - m + 1 + a[None, :]
        taps.append(np.mod(k, G).astype(np.int64))
        wts.append(kb_psi(u[:, None] - k, m, b))
    rows = (taps[0][:, :, None] * G + taps[1][:, None, :]).ravel()
    vals = (wts[0][:, :, None] * wts[1][:, None, :]).ravel()
    cols = np.repeat(np.arange(N), 4 * m * m)
    return sparse.csr_matrix((vals, (rows, cols)), shape=(G * G, N))


def multiplier(prm: Params, b=None):
    """W_l (G x G, FFT order) and the integer frequencies l1 [G, 1], l2 [1, G] (they
    broadcast to the G x G grid of l = (l1, l2)).  Every factor but b_l depends on one
    component of l only, so it is evaluated once per component value and the two
    factors multiplied per element."""
    G, n, m = prm.G, prm.n, prm.m
    if b is None:
        b = b_coeffs(prm)
    l = np.rint(np.fft.fftfreq(G) * G).astype(np.int64)
    L1, L2 = l[:, None], l[None, :]
    inband = np.abs(l) <= n // 2
    band = inband[:, None] & inband[None, :]
    om1 = np.where(np.abs(l) == n // 2, 0.5, 1.0)
    om = om1[:, None] * om1[None, :]
    bl = b[np.mod(L1, n), np.mod(L2, n)]
    ph1 = kb_psi_hat(l / G, m, prm.kb_b)
    ph = ph1[:, None] * ph1[None, :]
    W = np.where(band, om * bl / (ph * ph), 0.0)
    return W, L1, L2


def near_pairs(yt, xt, eps_I):
    """All (i, j) with |yt_i - xt_j| <= eps_I (boundary pairs contribute zero)."""
    tree = cKDTree(xt)
    lists = tree.query_ball_point(yt, eps_I, return_sorted=False)
    cnt = np.fromiter((len(v) for v in lists), dtype=np.int64, count=len(lists))
    ii = np.repeat(np.arange(len(yt)), cnt)
    jj = np.fromiter((j for v in lists for j in v), dtype=np.int64, count=int(cnt.sum()))
    return ii, jj


def _near_kernels(d, prm: Params, a):
    """(K - T_I)(r) and the scalar f with -grad(K - T_I)(d) = f d, for r > 0."""
    r2 = (d * d).sum(1)
    e2 = prm.eps_I ** 2
    rho2 = r2 / e2
    TI = sum(a[k] * rho2 ** k for k in range(prm.p))
    dTI = sum(2 * k * a[k] * rho2 ** (k - 1) / e2 for k in range(1, prm.p))  # (dT_I/dr)/r
    with np.errstate(divide="ignore", invalid="ignore"):
        kphi = -np.log(r2) / (2.0 * TWO_PI) - TI
        f = 1.0 / (TWO_PI * r2) + dTI
    return kphi, f, r2


class FastSum:
    """One geometry (targets y, sources x, weights w) and one parameter set.

    map_with: further points of the same problem that are not summed here but take
    part in the torus map (S0 is defined over all points of a problem).  The sum is
    linear in the sources, so a problem whose sources are split into classes (say
    volume and surface charges) is the sum of one FastSum per class, each with the
    other classes' points in map_with and its own parameters."""

    def __init__(self, y, x, w, prm: Params, map_with=None):
        self.prm = prm
        self.y = np.asarray(y, np.float64)
        self.x = np.asarray(x, np.float64)
        self.w = np.asarray(w, np.float64)
        self.c, self.s, self.yt, self.xt = torus_map(self.y, self.x, prm.eps_B, map_with)
        self.Bx = window_matrix(self.xt, prm)
        self.By = window_matrix(self.yt, prm)
        self.W, self.L1, self.L2 = multiplier(prm)
        self.a = inner_coeffs(prm.p, prm.eps_I)
        ii, jj = near_pairs(self.yt, self.xt, prm.eps_I)
        d = self.yt[ii] - self.xt[jj]
        self.ni, self.nj, self.nd = ii, jj, d
        self.kphi, self.kf, r2 = _near_kernels(d, prm, self.a)
        self.zero = r2 == 0.0

    # the grid pipeline: spread -> FFT -> multiply -> inverse FFT (no gather)
    def _grid(self, B, vals):
        G = self.prm.G
        return (B @ vals).reshape(G, G)

    def _back(self, spec):
        G = self.prm.G
        return (ifft2(spec) * (G * G)).real.ravel()

    def far_forward(self, s_src):
        gh = fft2(self._grid(self.Bx, s_src))
        W = self.W
        phi = self.By.T @ self._back(W * gh)
        hx = self.By.T @ self._back(-1j * TWO_PI * self.L1 * W * gh)
        hy = self.By.T @ self._back(-1j * TWO_PI * self.L2 * W * gh)
        return phi, np.stack([hx, hy], axis=1)

    def forward(self, q):
        """phi [nt], H [nt, 2] for charges q [ns]."""
        s_src = self.w * np.asarray(q, np.float64)
        phi, H = self.far_forward(s_src)
        sj = s_src[self.nj]
        kphi = np.where(self.zero, -(self.a[0] + np.log(self.s) / TWO_PI), self.kphi)
        kf = np.where(self.zero, 0.0, self.kf)
        nt = len(self.y)
        phi = phi + np.bincount(self.ni, weights=sj * kphi, minlength=nt)
        H = H + np.stack([np.bincount(self.ni, weights=sj * kf * self.nd[:, c], minlength=nt)
                          for c in range(2)], axis=1)
        phi = phi + np.log(self.s) / TWO_PI * s_src.sum()
        return phi, self.s * H

    def adjoint_H(self, V):
        """u_j = w_j sum_i V_i . (-grad G)(y_i - x_j), the transpose of forward()'s H map."""
        V = np.asarray(V, np.float64)
        W = self.W
        vx = fft2(self._grid(self.By, V[:, 0]))
        vy = fft2(self._grid(self.By, V[:, 1]))
        spec = 1j * TWO_PI * (self.L1 * W * vx + self.L2 * W * vy)
        u = self.Bx.T @ self._back(spec)
        kf = np.where(self.zero, 0.0, self.kf)
        dot = (V[self.ni] * self.nd).sum(1)
        u = u + np.bincount(self.nj, weights=kf * dot, minlength=len(self.x))
        return self.w * self.s * u

    def adjoint_phi(self, v):
        """u_j = w_j sum_i v_i G(y_i - x_j), the transpose of forward()'s phi map."""
        v = np.asarray(v, np.float64)
        spec = self.W * fft2(self._grid(self.By, v))
        u = self.Bx.T @ self._back(spec)
        kphi = np.where(self.zero, -(self.a[0] + np.log(self.s) / TWO_PI), self.kphi)
        u = u + np.bincount(self.nj, weights=v[self.ni] * kphi, minlength=len(self.x))
        u = u + np.log(self.s) / TWO_PI * v.sum()
        return self.w * u


def direct_ndft(yt, xt, s_src, prm: Params, b=None):
    """Windowless far field sum_l omega_l b_l sum_j s_j e^{2 pi i l.(y - x_j)} (and its
    -grad) by brute force over l in [-n/2, n/2]^2 -- tiny inputs only."""
    n = prm.n
    if b is None:
        b = b_coeffs(prm)
    l = np.arange(-n // 2, n // 2 + 1)
    L1, L2 = np.meshgrid(l, l, indexing="ij")
    om = np.where(np.abs(L1) == n // 2, 0.5, 1.0) * np.where(np.abs(L2) == n // 2, 0.5, 1.0)
    coef = (om * b[np.mod(L1, n), np.mod(L2, n)]).ravel()
    Lf = np.stack([L1.ravel(), L2.ravel()], axis=1).astype(np.float64)
    ah = np.exp(-1j * TWO_PI * (xt @ Lf.T)).T @ s_src          # sum_j s_j e^{-2 pi i l.x_j}
    E = np.exp(1j * TWO_PI * (yt @ Lf.T))                      # [nt, nl]
    phi = (E @ (coef * ah)).real
    hx = (E @ (-1j * TWO_PI * Lf[:, 0] * coef * ah)).real
    hy = (E @ (-1j * TWO_PI * Lf[:, 1] * coef * ah)).real
    return phi, np.stack([hx, hy], axis=1)
