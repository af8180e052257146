"""Pins of oracle O2 (the fast summation's steps in FP64 numpy) against independent facts:
the window's Fourier transform by numerical integration, the regularization's derivative
conditions by high-precision differentiation, the trigonometric interpolation property of
b_l, a brute-force NDFT, the direct sum O1, single-source exactness and the adjoint identity."""
import mpmath
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import direct
from oracle import fastsum as fs
from tests.conftest import rel_l2

pytestmark = pytest.mark.cpu


@pytest.mark.parametrize("m", [4, 6, 8])
def test_kaiser_bessel_transform_pair(m):
    """The untruncated window's transform I0(m sqrt(b^2 - (2 pi xi)^2)) vanishes for |2 pi xi| > b,
    so the pair can be checked exactly by inverting over that band: psi(t) for |t| < m."""
    b = np.pi * 1.5
    xmax = b / (2 * np.pi)
    for t in (0.0, 0.37, 1.5, 3.2, m - 0.3):
        num = 2 * integrate.quad(lambda xi: fs.kb_psi_hat(xi, m, b) * np.cos(2 * np.pi * xi * t),
                                 0, xmax, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
        assert abs(num - fs.kb_psi(np.array([t]), m, b)[0]) < 1e-12
    assert np.allclose(fs.kb_psi(np.array([m, -m, m + 0.5]), m, b), 0.0)


def test_truncated_window_transform_gap_shrinks_with_m():
    """Truncating the window to |t| < m makes its transform differ from I0(...) by the window
    error, which must fall fast with m."""
    b = np.pi * 1.5
    gaps = []
    for m in (4, 6, 8):
        g = 0.0
        for xi in (0.0, 0.1, 0.25):
            num = 2 * integrate.quad(lambda t: fs.kb_psi(np.array([t]), m, b)[0] * np.cos(2 * np.pi * xi * t),
                                     0, m, epsabs=1e-16, epsrel=1e-14, limit=400)[0]
            g = max(g, abs(num - fs.kb_psi_hat(xi, m, b)))
        gaps.append(g)
    assert gaps[0] < 1e-7 and gaps[1] < gaps[0] / 100 and gaps[2] < 1e-11


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_inner_polynomial_matches_log_derivatives(p):
    eps = 0.013
    a = fs.inner_coeffs(p, eps)
    mpmath.mp.dps = 40
    T = lambda r: sum(mpmath.mpf(a[k]) * (r / eps) ** (2 * k) for k in range(p))
    K = lambda r: -mpmath.log(r) / (2 * mpmath.pi)
    for q in range(p):
        dT = mpmath.diff(T, mpmath.mpf(eps), q)
        dK = mpmath.diff(K, mpmath.mpf(eps), q)
        assert abs(float(dT - dK)) < 1e-10 * max(1.0, abs(float(dK)))


@pytest.mark.parametrize("p,epsB", [(2, 1 / 16), (4, 1 / 16), (8, 1 / 16), (5, 1 / 32), (5, 1 / 48)])
def test_boundary_polynomial_conditions(p, epsB):
    """In t = (r - r_B)/eps_B: the q-th t-derivative equals eps_B^q K^(q)(r_B) at t = 0 and
    vanishes at t = 1 (q >= 1), relative to the size of the terms summed."""
    c = fs.boundary_coeffs(p, epsB)
    rB = 0.5 - epsB
    mpmath.mp.dps = 40
    P = lambda t: sum(mpmath.mpf(c[k]) * t ** k for k in range(len(c)))
    K = lambda t: -mpmath.log(rB + epsB * t) / (2 * mpmath.pi)
    for q in range(p):
        scale = sum(abs(c[k]) * fs._ff(k, q) for k in range(len(c)))
        assert abs(float(mpmath.diff(P, 0, q) - mpmath.diff(K, 0, q))) < 1e-13 * max(scale, 1.0)
    for q in range(1, p):
        scale = sum(abs(c[k]) * fs._ff(k, q) for k in range(len(c)))
        assert abs(float(mpmath.diff(P, 1, q))) < 1e-13 * max(scale, 1.0)


def test_regularized_kernel_is_continuous_and_equals_log_between():
    prm = fs.Params(G=128, m=6, p=4, eps_I=4 / 64)
    r = np.linspace(0.07, 0.43, 50)
    assert np.allclose(fs.K_R(r, prm), -np.log(r) / (2 * np.pi), rtol=0, atol=1e-15)
    for r0 in (prm.eps_I, 0.5 - prm.eps_B, 0.5):
        e = 1e-9
        lo, hi = fs.K_R(np.array([r0 - e]), prm)[0], fs.K_R(np.array([r0 + e]), prm)[0]
        assert abs(hi - lo) < 1e-7


@pytest.mark.parametrize("band", [0, 48])
def test_b_coefficients_interpolate_on_the_bandwidth_grid(band):
    """b_l is real and even, and its symmetric trigonometric sum reproduces K_R at the n-grid
    points (it is the trigonometric interpolant of the sampled kernel); n = G/2 and n = 3G/4."""
    prm = fs.Params(G=64, m=4, p=3, eps_I=3 / 32, band=band)
    n = prm.n
    b = fs.b_coeffs(prm)
    assert np.allclose(b, b[(-np.arange(n)) % n][:, (-np.arange(n)) % n], atol=1e-17)
    l = np.arange(-n // 2, n // 2 + 1)
    om = np.where(np.abs(l) == n // 2, 0.5, 1.0)
    rng = np.random.default_rng(1)
    for _ in range(6):
        j = rng.integers(-n // 2, n // 2, size=2)
        ph1 = np.exp(2j * np.pi * l * j[0] / n) * om
        ph2 = np.exp(2j * np.pi * l * j[1] / n) * om
        val = (ph1[:, None] * ph2[None, :] * b[np.mod(l, n)][:, np.mod(l, n)]).sum().real
        assert abs(val - fs.K_R(np.array([np.hypot(*j) / n]), prm)[0]) < 1e-13


@pytest.mark.parametrize("band", [0, 48])
def test_windowed_pipeline_matches_brute_force_ndft(band):
    """Spread + FFT + deconvolution + multiply + inverse + gather equals the direct trigonometric
    sum up to the window error (Kaiser-Bessel bound ~e^{-b m}: 4e-14 at m = 8, sigma = 2; 2e-14
    at sigma = 4/3, where b = 1.25 pi)."""
    prm = fs.Params(G=64, m=8, p=3, eps_I=3 / 32, band=band)
    y, x, w, q = synth.random_cloud(40, 50, 2)
    F = fs.FastSum(y, x, w, prm)
    s = w * q
    phi, H = F.far_forward(s)
    phi0, H0 = fs.direct_ndft(F.yt, F.xt, s, prm)
    assert rel_l2(phi, phi0) < 1e-12 and rel_l2(H, H0) < 1e-12
    prm6 = fs.Params(G=64, m=6, p=3, eps_I=3 / 32, band=band)
    F6 = fs.FastSum(y, x, w, prm6)
    phi6, H6 = F6.far_forward(s)
    assert 1e-13 < rel_l2(phi6, phi0) < 1e-8  # window error grows as m shrinks


def test_fast_sum_matches_direct_sum():
    y, x, w, q = synth.random_cloud(500, 700, 3)
    prm = fs.Params(G=512, m=8, p=10, eps_I=10 / 256)
    F = fs.FastSum(y, x, w, prm)
    phi, H = F.forward(q)
    phi1, H1 = direct.forward(y, x, w, q)
    assert rel_l2(phi, phi1) < 1e-8 and rel_l2(H, H1) < 1e-7
    V = np.random.default_rng(4).standard_normal((500, 2))
    assert rel_l2(F.adjoint_H(V), direct.adjoint(y, x, w, V=V)) < 1e-7
    v = V[:, 0].copy()
    assert rel_l2(F.adjoint_phi(v), direct.adjoint(y, x, w, v=v)) < 1e-8


def test_fast_sum_matches_direct_sum_at_lower_oversampling():
    """Bandwidth n = 3G/4 (oversampling 4/3) with n eps_I fixed: same accuracy class, a
    near-field radius 2/3 as large."""
    y, x, w, q = synth.random_cloud(500, 700, 3)
    prm = fs.Params(G=512, m=8, p=10, eps_I=10 / 384, band=384)
    F = fs.FastSum(y, x, w, prm)
    phi, H = F.forward(q)
    phi1, H1 = direct.forward(y, x, w, q)
    assert rel_l2(phi, phi1) < 1e-8 and rel_l2(H, H1) < 1e-7
    V = np.random.default_rng(4).standard_normal((500, 2))
    assert rel_l2(F.adjoint_H(V), direct.adjoint(y, x, w, V=V)) < 1e-7


def test_single_source_potential_and_field():
    """One source: phi = -(s/2pi) ln r and H = (s/2pi) d/r^2 exactly, across the near/far seam
    and including the ln(scale) offset (the sum of charges is not zero here)."""
    x = np.array([[0.3, -0.2]])
    w = np.array([0.7])
    q = np.array([1.3])
    r = np.concatenate([np.geomspace(1e-6, 2.0, 40)])
    ang = np.linspace(0, 2 * np.pi, 40, endpoint=False)
    y = x + np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1)
    y = np.concatenate([y, x + np.array([[-2.0, 0.0]])])
    prm = fs.Params(G=512, m=8, p=10, eps_I=10 / 256)
    F = fs.FastSum(y, x, w, prm)
    phi, H = F.forward(q)
    s = w[0] * q[0]
    d = y - x
    rr = np.hypot(d[:, 0], d[:, 1])
    assert np.abs(phi + s / (2 * np.pi) * np.log(rr)).max() < 1e-8
    Hex = s / (2 * np.pi) * d / rr[:, None] ** 2
    # the largest relative error sits at the largest separation (next to the boundary zone)
    assert (np.linalg.norm(H - Hex, axis=1) / np.linalg.norm(Hex, axis=1)).max() < 1e-6


def test_coincident_target_and_source_contribute_nothing():
    y = np.array([[0.0, 0.0], [0.5, 0.1]])
    x = np.array([[0.0, 0.0], [-0.4, 0.3]])
    w = np.array([1.0, 1.0])
    q = np.array([1.0, -0.5])
    prm = fs.Params(G=512, m=8, p=10, eps_I=10 / 256)
    F = fs.FastSum(y, x, w, prm)
    phi, H = F.forward(q)
    phi1, H1 = direct.forward(y, x, w, q)
    assert np.abs(phi - phi1).max() < 1e-8 and np.abs(H - H1).max() < 1e-7
    v = np.array([0.3, -1.1])
    u1 = direct.adjoint(y, x, w, v=v)
    assert np.abs(F.adjoint_phi(v) - u1).max() < 1e-8


def test_fast_sum_adjoint_identity():
    y, x, w, q = synth.random_cloud(300, 400, 5)
    prm = fs.Params(G=128, m=6, p=4, eps_I=4 / 64)
    F = fs.FastSum(y, x, w, prm)
    rng = np.random.default_rng(6)
    V = rng.standard_normal((300, 2))
    v = rng.standard_normal(300)
    phi, H = F.forward(q)
    assert abs(np.sum(H * V) - np.dot(q, F.adjoint_H(V))) < 1e-12 * np.abs(H * V).sum()
    assert abs(np.dot(phi, v) - np.dot(q, F.adjoint_phi(v))) < 1e-12 * np.abs(phi * v).sum()


def test_accuracy_improves_with_regularization_degree_and_radius():
    """The kernel-truncation error falls with p (at fixed eps_I n) and with eps_I n."""
    d = synth.rounded_square_cloud(N=4096, seed=5)
    y, x, w, q = d["y"], d["x"], d["w"], d["q"]
    phi1, H1 = direct.forward(y, x, w, q)
    e = {}
    for p, c in ((2, 4), (4, 4), (6, 6), (8, 8)):
        phi, H = fs.FastSum(y, x, w, fs.Params(G=256, m=6, p=p, eps_I=c / 128)).forward(q)
        e[(p, c)] = rel_l2(H, H1)
    assert e[(2, 4)] > e[(4, 4)] > e[(6, 6)] > e[(8, 8)]


def test_sum_over_a_partition_of_the_sources_is_the_whole_sum():
    """Eq. (2) is linear in the sources: with the torus map taken over all points (map_with),
    the fast sums over two disjoint source subsets add up to the fast sum over all sources at
    the same parameters, and the adjoints are the restrictions of the whole adjoint."""
    y, x, w, q = synth.random_cloud(300, 400, 7)
    prm = fs.Params(G=128, m=6, p=6, eps_I=5 / 64)
    k = 170
    F = fs.FastSum(y, x, w, prm)
    Fa = fs.FastSum(y, x[:k], w[:k], prm, map_with=x[k:])
    Fb = fs.FastSum(y, x[k:], w[k:], prm, map_with=x[:k])
    assert Fa.s == F.s and Fb.s == F.s and np.all(Fa.c == F.c)
    phi, H = F.forward(q)
    pa, Ha = Fa.forward(q[:k])
    pb, Hb = Fb.forward(q[k:])
    assert rel_l2(pa + pb, phi) < 1e-12 and rel_l2(Ha + Hb, H) < 1e-12
    rng = np.random.default_rng(8)
    V, v = rng.standard_normal((300, 2)), rng.standard_normal(300)
    assert rel_l2(np.concatenate([Fa.adjoint_H(V), Fb.adjoint_H(V)]), F.adjoint_H(V)) < 1e-12
    assert rel_l2(np.concatenate([Fa.adjoint_phi(v), Fb.adjoint_phi(v)]), F.adjoint_phi(v)) < 1e-12


def test_two_source_classes_with_their_own_radius_match_the_direct_sum():
    """The rounded-square workload (jittered lattice of volume charges plus the boundary
    line of surface charges, at the bench's density of about 2.3 points per grid cell):
    each class summed with its own regularization radius and the torus map over all
    points.  Together the two fast sums match the direct sum O1, and giving the line its
    larger radius lowers the H error several times over the one-radius sum (the line's
    truncation error dominates the latter)."""
    d = synth.rounded_square_cloud(N=16384, seed=synth.SEED_BASE + 4)
    y, x, w, q = d["y"], d["x"], d["w"], d["q"]
    ns1 = int(np.sum(w == d["h"] ** 2))
    assert np.all(w[:ns1] == d["h"] ** 2) and not np.any(w[ns1:] == d["h"] ** 2)
    G, n = 256, 192
    prm_v = fs.Params(G=G, m=6, p=8, eps_I=6 / n, band=n)
    prm_s = fs.Params(G=G, m=6, p=8, eps_I=10 / n, band=n)
    Fv = fs.FastSum(y, x[:ns1], w[:ns1], prm_v, map_with=x[ns1:])
    Fs = fs.FastSum(y, x[ns1:], w[ns1:], prm_s, map_with=x[:ns1])
    F1 = fs.FastSum(y, x[ns1:], w[ns1:], prm_v, map_with=x[:ns1])  # line at the volume radius
    pv, Hv = Fv.forward(q[:ns1])
    ps, Hs = Fs.forward(q[ns1:])
    _, H1s = F1.forward(q[ns1:])
    phi1, H1 = direct.forward(y, x, w, q)
    e_phi, e_H, e_one = rel_l2(pv + ps, phi1), rel_l2(Hv + Hs, H1), rel_l2(Hv + H1s, H1)
    assert e_phi < 1e-7 and e_H < 5e-7, (e_phi, e_H)
    assert e_one > 3 * e_H, (e_one, e_H)
    V = d["h"] ** 2 * d["M_tgt"]  # the adjoint input of the energy gradient: nodal mass times M
    u = np.concatenate([Fv.adjoint_H(V), Fs.adjoint_H(V)])
    assert rel_l2(u, direct.adjoint(y, x, w, V=V)) < 5e-7
