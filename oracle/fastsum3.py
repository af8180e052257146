"""Oracle O2 in 3D -- the fast summation's steps in plain FP64 numpy for the 3D Green
function of eq. (1), G(r) = 1/(4 pi r).  TEST INFRASTRUCTURE ONLY.

The paper states the method for 2D and 3D alike (the 3D kernel next to the 2D one with
eq. (1); a grid of about p^3 N points in 3D in the NFFT section).  The steps are those of
the 2D module oracle.fastsum, in three dimensions:

  S0  torus map     c = bounding-box midpoint, D = 2 max |p - c| over all points,
                    s = (1/2 - eps_B)/D.  For mapped points t = s (r - c):
                    G(y - x) = s K(|t_y - t_x|) with K(r) = 1/(4 pi r), so
                    phi = s (torus sum) and H = -grad_y phi = s^2 (torus gradient sum).
  S0' plan          K_R = T_I on r < eps_I (even polynomial of degree 2p-2 matching K and
                    its first p-1 derivatives at eps_I), K on [eps_I, 1/2 - eps_B], T_B on
                    (1/2 - eps_B, 1/2] (degree 2p-2, matching K and p-1 derivatives at
                    1/2 - eps_B, derivatives 1..p-1 zero at 1/2), T_B(1/2) beyond.
                    b_l = (1/n^3) sum_{j in I_n^3} K_R(|j|/n) e^{-2 pi i j.l/n}.
                    Kaiser-Bessel window: the product of the 1D windows of oracle.fastsum
                    over the three axes, its transform the product of the 1D transforms.
  S2  spread        g_k = sum_j s_j psi(G t_j1 - k1) psi(G t_j2 - k2) psi(G t_j3 - k3).
  S3  FFT           over the G^3 grid.
  S4  multiply      W_l = omega_l b_l / prod_d psi^(l_d/G)^2 on |l_d| <= n/2 (omega = 1/2
                    per Nyquist index), times -2 pi i l_d for the gradient components.
  S5  inverse FFT;  S6 gather with the same window.
  S7  near field    for |t_y - t_x| < eps_I add s_j (K - T_I)(r) to phi and
                    -s_j grad(K - T_I) to H.  A pair at r = 0 is not part of the exact sum:
                    the far field holds K_R(0) = a_0 for it, so it adds -s_j a_0.
                    phi = s (far + near), H = s^2 (far + near).
  S8  adjoint       the exact transposes with respect to the charges.

Library primitives only (scipy FFT, sparse window matrices, a KD-tree for the near pairs).
direct_ndft() gives the windowless far field for tiny inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import sparse
from scipy.spatial import cKDTree

from .fastsum import _ff, fftn_w, ifftn_w, kb_psi, kb_psi_hat

FOUR_PI = 4.0 * np.pi


@dataclass
class Params3:
    G: int
    m: int
    p: int
    eps_I: float
    eps_B: float = 1.0 / 16.0
    band: int = 0

    @property
    def n(self):
        return self.band if self.band else self.G // 2

    @property
    def kb_b(self):
        return np.pi * (2.0 - 1.0 / (self.G / self.n))


def K(r):
    return 1.0 / (FOUR_PI * r)


def K_scaled_deriv(q, r):
    """r^q K^{(q)}(r) for K = 1/(4 pi r): (-1)^q q! / (4 pi r)."""
    return (-1.0) ** q * math.factorial(q) / (FOUR_PI * r)


def inner_coeffs(p, eps_I):
    """a_k with T_I(r) = sum_{k<p} a_k (r/eps_I)^{2k}, T_I^{(q)}(eps_I) = K^{(q)}(eps_I), q < p."""
    A = np.array([[_ff(2 * k, q) for k in range(p)] for q in range(p)])
    rhs = np.array([K_scaled_deriv(q, eps_I) for q in range(p)])
    return np.linalg.solve(A, rhs)


def boundary_coeffs(p, eps_B):
    """c_k with T_B(r) = sum_{k<=2p-2} c_k t^k, t = (r - r_B)/eps_B, r_B = 1/2 - eps_B."""
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


def K_R(r, prm: Params3):
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


def b_coeffs(prm: Params3):
    """b_l, l in I_n^3 (FFT order, n x n x n): the DFT of K_R sampled on the n-grid."""
    n = prm.n
    j = np.fft.fftfreq(n) * n
    J1, J2, J3 = np.meshgrid(j, j, j, indexing="ij")
    samples = K_R(np.sqrt(J1 ** 2 + J2 ** 2 + J3 ** 2) / n, prm)
    return fftn_w(samples).real / float(n) ** 3


def torus_map(y, x, eps_B, extra=None):
    allp = np.concatenate([y, x] + ([np.asarray(extra, np.float64)] if extra is not None else []), axis=0)
    lo, hi = allp.min(0), allp.max(0)
    c = 0.5 * (lo + hi)
    D = 2.0 * np.sqrt(((allp - c) ** 2).sum(1).max())
    if not D > 0:
        raise ValueError("all points coincide")
    s = (0.5 - eps_B) / D
    return c, s, s * (y - c), s * (x - c)


def window_matrix(pt, prm: Params3):
    """B with B[(k1 G + k2) G + k3, j] = prod_d psi(G pt_jd - k_d) (k mod G)."""
    G, m, b = prm.G, prm.m, prm.kb_b
    N = len(pt)
    a = np.arange(2 * m)
    taps, wts = [], []
    for d in range(3):
        u = pt[:, d] * G
        k = np.floor(u)[:, None] - m + 1 + a[None, :]
        taps.append(np.mod(k, G).astype(np.int64))
        wts.append(kb_psi(u[:, None] - k, m, b))
    rows = ((taps[0][:, :, None, None] * G + taps[1][:, None, :, None]) * G + taps[2][:, None, None, :]).ravel()
    vals = (wts[0][:, :, None, None] * wts[1][:, None, :, None] * wts[2][:, None, None, :]).ravel()
    cols = np.repeat(np.arange(N), (2 * m) ** 3)
    return sparse.csr_matrix((vals, (rows, cols)), shape=(G ** 3, N))


def multiplier(prm: Params3, b=None):
    """W_l on the G^3 grid (FFT order) and the integer frequencies l_d (broadcastable)."""
    G, n, m = prm.G, prm.n, prm.m
    if b is None:
        b = b_coeffs(prm)
    l = np.rint(np.fft.fftfreq(G) * G).astype(np.int64)
    L = (l[:, None, None], l[None, :, None], l[None, None, :])
    inb = np.abs(l) <= n // 2
    om1 = np.where(np.abs(l) == n // 2, 0.5, 1.0)
    ph1 = kb_psi_hat(l / G, m, prm.kb_b)
    band = inb[:, None, None] & inb[None, :, None] & inb[None, None, :]
    om = om1[:, None, None] * om1[None, :, None] * om1[None, None, :]
    ph = ph1[:, None, None] * ph1[None, :, None] * ph1[None, None, :]
    bl = b[np.mod(L[0], n), np.mod(L[1], n), np.mod(L[2], n)]
    W = np.where(band, om * bl / (ph * ph), 0.0)
    return W, L


def _near_kernels(d, prm: Params3, a):
    """(K - T_I)(r) and f with -grad(K - T_I)(d) = f d, for r > 0."""
    r2 = (d * d).sum(1)
    e2 = prm.eps_I ** 2
    rho2 = r2 / e2
    TI = sum(a[k] * rho2 ** k for k in range(prm.p))
    dTI = sum(2 * k * a[k] * rho2 ** (k - 1) / e2 for k in range(1, prm.p))  # (dT_I/dr)/r
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.sqrt(r2)
        kphi = 1.0 / (FOUR_PI * r) - TI
        f = 1.0 / (FOUR_PI * r2 * r) + dTI
    return kphi, f, r2


class FastSum3:
    """One 3D geometry (targets y, sources x, weights w) and one parameter set."""

    def __init__(self, y, x, w, prm: Params3, map_with=None):
        self.prm = prm
        self.y = np.asarray(y, np.float64)
        self.x = np.asarray(x, np.float64)
        self.w = np.asarray(w, np.float64)
        self.c, self.s, self.yt, self.xt = torus_map(self.y, self.x, prm.eps_B, map_with)
        self.Bx = window_matrix(self.xt, prm)
        self.By = window_matrix(self.yt, prm)
        self.W, self.L = multiplier(prm)
        self.a = inner_coeffs(prm.p, prm.eps_I)
        tree = cKDTree(self.xt)
        lists = tree.query_ball_point(self.yt, prm.eps_I, return_sorted=False)
        cnt = np.fromiter((len(v) for v in lists), dtype=np.int64, count=len(lists))
        self.ni = np.repeat(np.arange(len(self.yt)), cnt)
        self.nj = np.fromiter((j for v in lists for j in v), dtype=np.int64, count=int(cnt.sum()))
        self.nd = self.yt[self.ni] - self.xt[self.nj]
        self.kphi, self.kf, r2 = _near_kernels(self.nd, prm, self.a)
        self.zero = r2 == 0.0

    def _grid(self, B, vals):
        G = self.prm.G
        return (B @ vals).reshape(G, G, G)

    def _back(self, spec):
        G = self.prm.G
        return (ifftn_w(spec) * float(G) ** 3).real.ravel()

    def far_forward(self, s_src):
        """S2-S6: the far field of source strengths s_src in torus units (phi, -grad phi)."""
        gh = fftn_w(self._grid(self.Bx, s_src))
        W = self.W
        phi = self.By.T @ self._back(W * gh)
        H = np.stack([self.By.T @ self._back(-1j * 2 * np.pi * self.L[d] * W * gh) for d in range(3)], axis=1)
        return phi, H

    def forward(self, q):
        """phi [nt], H [nt, 3] for charges q [ns]."""
        s_src = self.w * np.asarray(q, np.float64)
        phi, H = self.far_forward(s_src)
        sj = s_src[self.nj]
        kphi = np.where(self.zero, -self.a[0], self.kphi)
        kf = np.where(self.zero, 0.0, self.kf)
        nt = len(self.y)
        phi = phi + np.bincount(self.ni, weights=sj * kphi, minlength=nt)
        H = H + np.stack([np.bincount(self.ni, weights=sj * kf * self.nd[:, c], minlength=nt) for c in range(3)],
                         axis=1)
        return self.s * phi, self.s ** 2 * H

    def adjoint_H(self, V):
        """u_j = w_j sum_i V_i . (-grad G)(y_i - x_j): the transpose of forward()'s H map."""
        V = np.asarray(V, np.float64)
        W = self.W
        spec = 0.0
        for d in range(3):
            spec = spec + 1j * 2 * np.pi * self.L[d] * W * fftn_w(self._grid(self.By, V[:, d]))
        u = self.Bx.T @ self._back(spec)
        kf = np.where(self.zero, 0.0, self.kf)
        dot = (V[self.ni] * self.nd).sum(1)
        u = u + np.bincount(self.nj, weights=kf * dot, minlength=len(self.x))
        return self.w * self.s ** 2 * u

    def adjoint_phi(self, v):
        """u_j = w_j sum_i v_i G(y_i - x_j): the transpose of forward()'s phi map."""
        v = np.asarray(v, np.float64)
        u = self.Bx.T @ self._back(self.W * fftn_w(self._grid(self.By, v)))
        kphi = np.where(self.zero, -self.a[0], self.kphi)
        u = u + np.bincount(self.nj, weights=v[self.ni] * kphi, minlength=len(self.x))
        return self.w * self.s * u


def direct_ndft(yt, xt, s_src, prm: Params3, b=None):
    """Windowless far field sum_l omega_l b_l sum_j s_j e^{2 pi i l.(y - x_j)} and its -grad,
    by brute force over l in [-n/2, n/2]^3 (torus units, before the factors s and s^2) --
    tiny inputs only."""
    n = prm.n
    if b is None:
        b = b_coeffs(prm)
    l = np.arange(-n // 2, n // 2 + 1)
    L1, L2, L3 = np.meshgrid(l, l, l, indexing="ij")
    om = (np.where(np.abs(L1) == n // 2, 0.5, 1.0) * np.where(np.abs(L2) == n // 2, 0.5, 1.0)
          * np.where(np.abs(L3) == n // 2, 0.5, 1.0))
    coef = (om * b[np.mod(L1, n), np.mod(L2, n), np.mod(L3, n)]).ravel()
    Lf = np.stack([L1.ravel(), L2.ravel(), L3.ravel()], axis=1).astype(np.float64)
    ah = np.exp(-1j * 2 * np.pi * (xt @ Lf.T)).T @ s_src
    E = np.exp(1j * 2 * np.pi * (yt @ Lf.T))
    phi = (E @ (coef * ah)).real
    H = np.stack([(E @ (-1j * 2 * np.pi * Lf[:, d] * coef * ah)).real for d in range(3)], axis=1)
    return phi, H
