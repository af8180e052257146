"""Pins of the 3D oracles (O1 direct sum, O2 step-by-step fast sum) for the Green function
G(r) = 1/(4 pi r) given with eq. (1), against what the mathematics fixes:

  * O1: Newton's shell theorem on an exact-to-rounding spherical quadrature (potential and
    field of a uniform shell, inside and outside), the adjoint identities, coincident pairs;
  * O2: the regularization conditions of T_I and T_B (derivatives by mpmath), the b_l
    interpolation property, the windowed pipeline against the brute-force trigonometric sum,
    accuracy against O1 improving with the near radius, a single source against 1/(4 pi r),
    coincident pairs, the adjoint identity, linearity over a partition of the sources.
"""
import math

import mpmath
import numpy as np
import pytest

import synth
from oracle import direct
from oracle import fastsum3 as f3
from tests.conftest import rel_l2


def sphere_rule(R, c, n_theta=40, n_phi=80):
    """Gauss-Legendre in cos(theta) x trapezoid in phi on the sphere |r - c| = R: exact for
    spherical harmonics of degree < min(2 n_theta, n_phi), so the potential of a uniform shell
    at |y - c| = rho R (rho < 1) is reproduced up to ~rho^n_phi."""
    z, wz = np.polynomial.legendre.leggauss(n_theta)
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    Z, P = np.meshgrid(z, ph, indexing="ij")
    S = np.sqrt(1 - Z * Z)
    pts = np.stack([S * np.cos(P), S * np.sin(P), Z], axis=-1).reshape(-1, 3)
    w = (np.repeat(wz, n_phi) * (2 * np.pi / n_phi)) * R * R
    return c + R * pts, w


def test_o1_shell_theorem_potential_and_field():
    R, c = 1.3, np.array([0.2, -0.1, 0.4])
    x, w = sphere_rule(R, c)
    assert abs(w.sum() - 4 * np.pi * R * R) < 1e-12 * 4 * np.pi * R * R
    sigma = 0.7
    q = np.full(len(x), sigma)
    Q = sigma * w.sum()
    rng = np.random.default_rng(5)
    d = rng.standard_normal((60, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    inside = c + d[:30] * (0.5 * R * rng.random(30))[:, None]
    outside = c + d[30:] * (R * (2.0 + 3.0 * rng.random(30)))[:, None]
    y = np.concatenate([inside, outside])
    phi, H = direct.forward3(y, x, w, q)
    # inside: constant potential Q/(4 pi R), no field
    assert np.abs(phi[:30] - Q / (4 * np.pi * R)).max() < 1e-12 * Q / (4 * np.pi * R)
    assert np.abs(H[:30]).max() < 1e-12 * Q / (4 * np.pi * R * R)
    # outside: a point charge Q at the centre
    r = outside - c
    rn = np.linalg.norm(r, axis=1)
    assert np.abs(phi[30:] - Q / (4 * np.pi * rn)).max() < 1e-12 * Q / (4 * np.pi * 2 * R)
    Hex = Q * r / (4 * np.pi * rn[:, None] ** 3)
    assert np.abs(H[30:] - Hex).max() < 1e-12 * Q / (4 * np.pi * 4 * R * R)


def test_o1_adjoint_identities_and_coincident_pairs():
    y, x, w, q = synth.random_cloud3(70, 90, 3)
    y[:5] = x[10:15]  # coincident pairs are left out of the sum
    rng = np.random.default_rng(4)
    v = rng.standard_normal(len(y))
    V = rng.standard_normal((len(y), 3))
    phi, H = direct.forward3(y, x, w, q)
    assert abs(phi @ v - q @ direct.adjoint3(y, x, w, v=v)) < 1e-13 * np.abs(phi * v).sum()
    assert abs((H * V).sum() - q @ direct.adjoint3(y, x, w, V=V)) < 1e-13 * np.abs(H * V).sum()
    # the coincident target 0 sees every source but source 10
    keep = np.arange(len(x)) != 10
    p0, H0 = direct.forward3(y[:1], x[keep], w[keep], q[keep])
    assert abs(phi[0] - p0[0]) < 1e-15 * np.abs(p0).max() * 10 and np.abs(H[0] - H0[0]).max() < 1e-13 * np.abs(H0).max()
    # one pair by hand
    p1, H1 = direct.forward3(np.array([[1.0, 2.0, 2.0]]), np.zeros((1, 3)), np.array([2.0]), np.array([1.5]))
    assert abs(p1[0] - 3.0 / (4 * np.pi * 3.0)) < 1e-16
    assert np.abs(H1[0] - 3.0 * np.array([1.0, 2.0, 2.0]) / (4 * np.pi * 27.0)).max() < 1e-16


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_inner_polynomial_matches_the_kernel_derivatives(p):
    eps = 0.07
    a = f3.inner_coeffs(p, eps)
    mpmath.mp.dps = 40
    T = lambda r: sum(mpmath.mpf(a[k]) * (r / eps) ** (2 * k) for k in range(p))
    K = lambda r: 1 / (4 * mpmath.pi * r)
    for q in range(p):
        dT = mpmath.diff(T, mpmath.mpf(eps), q)
        dK = mpmath.diff(K, mpmath.mpf(eps), q)
        assert abs(float(dT - dK)) < 1e-10 * max(1.0, abs(float(dK)))


@pytest.mark.parametrize("p,epsB", [(3, 1 / 16), (6, 1 / 8), (8, 1 / 8)])
def test_boundary_polynomial_conditions(p, epsB):
    c = f3.boundary_coeffs(p, epsB)
    rB = 0.5 - epsB
    mpmath.mp.dps = 40
    P = lambda r: sum(mpmath.mpf(c[k]) * ((r - rB) / epsB) ** k for k in range(len(c)))
    K = lambda r: 1 / (4 * mpmath.pi * r)
    for q in range(p):
        scale = abs(float(mpmath.diff(K, rB, q)))
        assert abs(float(mpmath.diff(P, rB, q) - mpmath.diff(K, rB, q))) < 1e-12 * max(scale, 1.0)
    for q in range(1, p):
        # rounding scale: the sum of the absolute terms of the q-th derivative at t = 1
        terms = sum(abs(c[k]) * math.perm(k, q) for k in range(q, len(c))) / epsB ** q
        assert abs(float(mpmath.diff(P, mpmath.mpf(0.5), q))) < 1e-14 * terms


def test_regularized_kernel_is_continuous_and_equals_the_kernel_between():
    prm = f3.Params3(G=64, m=6, p=6, eps_I=6 / 32, eps_B=1 / 8)
    r = np.linspace(prm.eps_I, 0.5 - prm.eps_B, 50)
    assert np.allclose(f3.K_R(r, prm), 1 / (4 * np.pi * r), rtol=1e-15, atol=0)
    for r0 in (prm.eps_I, 0.5 - prm.eps_B, 0.5):
        lo, hi = f3.K_R(np.array([r0 - 1e-9, r0 + 1e-9]), prm)
        assert abs(hi - lo) < 1e-6


@pytest.mark.parametrize("G,band", [(16, 0), (32, 0), (16, 12), (32, 24)])
def test_b_coefficients_interpolate_on_the_bandwidth_grid(G, band):
    prm = f3.Params3(G=G, m=3, p=4, eps_I=4 / (band or G // 2), eps_B=1 / 8, band=band)
    n = prm.n
    b = f3.b_coeffs(prm)
    neg = (-np.arange(n)) % n
    assert np.allclose(b, b[neg][:, neg][:, :, neg], atol=1e-17)  # even in l
    rng = np.random.default_rng(1)
    l = np.arange(-n // 2, n // 2 + 1)
    om = np.where(np.abs(l) == n // 2, 0.5, 1.0)
    for _ in range(4):
        j = rng.integers(-n // 2 + 1, n // 2, size=3)
        e = [np.exp(2j * np.pi * l * j[d] / n) * om for d in range(3)]
        bb = b[np.mod(l, n)][:, np.mod(l, n)][:, :, np.mod(l, n)]
        val = np.einsum("i,j,k,ijk->", e[0], e[1], e[2], bb).real
        assert abs(val - f3.K_R(np.array([np.linalg.norm(j) / n]), prm)[0]) < 1e-13


def test_windowed_pipeline_matches_brute_force_ndft():
    """Spread + FFT + deconvolution + multiply + inverse + gather equals the direct
    trigonometric sum up to the window error (Kaiser-Bessel, ~e^{-b m})."""
    y, x, w, q = synth.random_cloud3(30, 40, 2)
    s = w * q
    prm = f3.Params3(G=32, m=7, p=3, eps_I=3 / 16, eps_B=1 / 8)
    F = f3.FastSum3(y, x, w, prm)
    phi, H = F.far_forward(s)
    phi0, H0 = f3.direct_ndft(F.yt, F.xt, s, prm)
    assert rel_l2(phi, phi0) < 1e-11 and rel_l2(H, H0) < 1e-11
    prm4 = f3.Params3(G=32, m=4, p=3, eps_I=3 / 16, eps_B=1 / 8)
    phi4, _ = f3.FastSum3(y, x, w, prm4).far_forward(s)
    assert 1e-12 < rel_l2(phi4, phi0) < 1e-6  # window error grows as m shrinks


def test_windowed_pipeline_at_oversampling_4_3_matches_brute_force_ndft():
    """The same with bandwidth n = 3G/4 (oversampling 4/3, Kaiser-Bessel shape
    b = pi (2 - 1/sigma)): the window error decays like e^{-pi m} instead of e^{-sqrt(2) pi m}."""
    y, x, w, q = synth.random_cloud3(30, 40, 3)
    s = w * q
    errs = {}
    for m in (4, 6, 8):
        prm = f3.Params3(G=32, m=m, p=3, eps_I=3 / 24, eps_B=1 / 8, band=24)
        F = f3.FastSum3(y, x, w, prm)
        phi, H = F.far_forward(s)
        phi0, H0 = f3.direct_ndft(F.yt, F.xt, s, prm)
        errs[m] = max(rel_l2(phi, phi0), rel_l2(H, H0))
    print(errs)
    assert errs[8] < 1e-11 and errs[4] > errs[6] > errs[8]


def test_fast_sum_matches_direct_sum_and_improves_with_the_near_radius():
    y, x, w, q = synth.random_cloud3(1200, 1500, 6)
    phi1, H1 = direct.forward3(y, x, w, q)
    rng = np.random.default_rng(7)
    V = rng.standard_normal((len(y), 3))
    u1 = direct.adjoint3(y, x, w, V=V)
    v = rng.standard_normal(len(y))
    up1 = direct.adjoint3(y, x, w, v=v)
    errs = []
    for c in (2, 3, 4, 5):  # n eps_I with p = n eps_I + 1; at n = 32 the error floors near c = 5
        prm = f3.Params3(G=64, m=6, p=c + 1, eps_I=c / 32, eps_B=1 / 8)
        F = f3.FastSum3(y, x, w, prm)
        phi, H = F.forward(q)
        errs.append((rel_l2(phi, phi1), rel_l2(H, H1), rel_l2(F.adjoint_H(V), u1), rel_l2(F.adjoint_phi(v), up1)))
    assert all(max(a) > max(b) for a, b in zip(errs, errs[1:])), errs
    assert max(errs[-1]) < 3e-5, errs


def test_fast_sum_at_the_bench_parameters_matches_direct_sum():
    y, x, w, q = synth.random_cloud3(1500, 2000, 8)
    prm = f3.Params3(G=128, m=8, p=8, eps_I=8 / 64, eps_B=1 / 8)
    F = f3.FastSum3(y, x, w, prm)
    phi, H = F.forward(q)
    phi1, H1 = direct.forward3(y, x, w, q)
    assert rel_l2(phi, phi1) < 1e-6 and rel_l2(H, H1) < 1e-6
    V = np.random.default_rng(9).standard_normal((len(y), 3))
    assert rel_l2(F.adjoint_H(V), direct.adjoint3(y, x, w, V=V)) < 1e-6


def test_single_source_potential_and_field():
    """One unit source against 1/(4 pi r) and its field, from 0.02 to 0.92 away; the fast
    sum's error is nearly uniform in absolute terms, so it is measured against the largest value."""
    x = np.array([[0.1, -0.2, 0.05]])
    rng = np.random.default_rng(11)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    rr = 0.02 + 0.9 * rng.random(200)
    y = x + d * rr[:, None]
    prm = f3.Params3(G=128, m=8, p=8, eps_I=8 / 64, eps_B=1 / 8)
    F = f3.FastSum3(y, x, np.array([1.0]), prm)
    phi, H = F.forward(np.array([1.0]))
    ex = 1 / (4 * np.pi * rr)
    assert np.abs(phi - ex).max() < 1e-7 * ex.max()
    Hex = d / (4 * np.pi * rr[:, None] ** 2)
    assert np.linalg.norm(H - Hex, axis=1).max() < 1e-7 * np.linalg.norm(Hex, axis=1).max()


def test_coincident_target_and_source_contribute_nothing():
    y, x, w, q = synth.random_cloud3(200, 300, 12)
    y[:20] = x[:20]
    prm = f3.Params3(G=64, m=6, p=7, eps_I=6 / 32, eps_B=1 / 8)
    F = f3.FastSum3(y, x, w, prm)
    phi, H = F.forward(q)
    phi1, H1 = direct.forward3(y, x, w, q)
    sc = np.abs(phi1).max()
    assert np.abs(phi - phi1).max() < 1e-4 * sc and np.abs(H - H1).max() < 1e-4 * np.abs(H1).max()
    # the coincident pair is the one the far field holds at K_R(0): dropping the correction
    # moves exactly those 20 targets by s_j a_0
    delta = F.s * w[:20] * q[:20] * F.a[0]
    assert np.all(np.abs(delta) > 100 * np.abs(phi[:20] - phi1[:20]))


def test_fast_sum_adjoint_identity_and_linearity():
    y, x, w, q = synth.random_cloud3(300, 400, 13)
    prm = f3.Params3(G=32, m=5, p=5, eps_I=4 / 16, eps_B=1 / 8)
    F = f3.FastSum3(y, x, w, prm)
    phi, H = F.forward(q)
    rng = np.random.default_rng(14)
    V = rng.standard_normal((len(y), 3))
    v = rng.standard_normal(len(y))
    assert abs(np.sum(H * V) - np.dot(q, F.adjoint_H(V))) < 1e-12 * np.abs(H * V).sum()
    assert abs(np.dot(phi, v) - np.dot(q, F.adjoint_phi(v))) < 1e-12 * np.abs(phi * v).sum()
    # a partition of the sources, one shared torus map
    a = np.arange(len(x)) < 150
    Fa = f3.FastSum3(y, x[a], w[a], prm, map_with=x[~a])
    Fb = f3.FastSum3(y, x[~a], w[~a], prm, map_with=x[a])
    pa, Ha = Fa.forward(q[a])
    pb, Hb = Fb.forward(q[~a])
    assert rel_l2(pa + pb, phi) < 1e-12 and rel_l2(Ha + Hb, H) < 1e-12


def test_torus_map_puts_every_point_in_the_safe_ball():
    y, x, w, q = synth.random_cloud3(100, 120, 15, shape="cube", R=3.0)
    c, s, yt, xt = f3.torus_map(y, x, 1 / 8)
    allt = np.concatenate([yt, xt])
    assert np.linalg.norm(allt, axis=1).max() <= (0.5 - 1 / 8) / 2 * (1 + 1e-15)
    d = allt[:, None, :] - allt[None, :, :]
    assert np.linalg.norm(d, axis=2).max() <= 0.5 - 1 / 8 + 1e-15
    assert math.isclose(s * 2 * np.linalg.norm(np.concatenate([y, x]) - c, axis=1).max(), 0.5 - 1 / 8)
