"""Pins of oracle O1 (direct FP64 sum) and of the oracle's FEM front against what the
mathematics and the paper fix: closed-form potentials and fields, exact segment
integrals, brute-force quadrature, conservation and symmetry properties."""
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import direct, fem
from tests.conftest import rel_l2

pytestmark = pytest.mark.cpu


def disk_problem(N, R=1.0, M=(1.0, 0.0), seed=1):
    nodes, tris, bedges = synth.disk_mesh_n(N, R=R, seed=seed)
    Mn = synth.M_uniform(nodes, *M)
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, Mn)
    return nodes, tris, bedges, Mn, x, w, q


# ---------------------------------------------------------------- exact polygon potential

def segment_log_integral(y, a, b):
    """int_a^b ln|y - x| ds and its gradient in y, from the antiderivative
    F(u) = u ln(u^2 + eta^2)/2 - u + eta atan(u/eta) along the segment."""
    d = b - a
    L = np.hypot(*d)
    t = d / L
    n = np.array([-t[1], t[0]])
    xi = (y - a) @ t
    eta = (y - a) @ n

    def F(u):
        return 0.5 * u * np.log(u * u + eta * eta) - u + eta * np.arctan(u / eta) if eta != 0 else \
            0.5 * u * np.log(u * u) - u

    val = F(L - xi) - F(-xi)
    g_xi = 0.5 * np.log(xi ** 2 + eta ** 2) - 0.5 * np.log((L - xi) ** 2 + eta ** 2)
    g_eta = np.arctan((L - xi) / eta) + np.arctan(xi / eta) if eta != 0 else 0.0
    return val, g_xi * t + g_eta * n


def test_segment_integral_closed_form_against_quadrature():
    a, b = np.array([0.1, -0.2]), np.array([0.7, 0.3])
    for y in (np.array([0.3, 0.5]), np.array([-0.4, 0.1]), np.array([1.2, -0.6])):
        val, grad = segment_log_integral(y, a, b)
        L = np.hypot(*(b - a))
        num = integrate.quad(lambda s: np.log(np.hypot(*(y - a - s * (b - a) / L))), 0, L, epsabs=1e-14)[0]
        assert abs(val - num) < 1e-12
        h = 1e-6
        fd = [(segment_log_integral(y + h * e, a, b)[0] - segment_log_integral(y - h * e, a, b)[0]) / (2 * h)
              for e in np.eye(2)]
        assert np.allclose(grad, fd, atol=1e-8)


def test_uniform_polygon_matches_exact_segment_integrals():
    """Uniform M: rho = 0 and sigma = M.n per straight edge, so the exact potential is a sum of
    segment integrals; O1 with 2-point Gauss on each edge must converge to it like h^4 at
    interior targets (this pins the edge quadrature, sigma, the sign and scale of G and of H)."""
    targets = np.array([[0.1, 0.2], [-0.3, 0.1], [0.0, -0.4], [0.35, -0.25]])
    M = np.array([0.8, -0.6])
    errs_phi, errs_H = [], []
    for K in (6, 12, 24):
        nodes, tris, bedges = synth.disk_mesh(R=1.0, K=K, seed=2)
        Mn = synth.M_uniform(nodes, *M)
        x, w = fem.sources(nodes, tris, bedges)
        q = fem.charges(nodes, tris, bedges, Mn)
        assert np.abs(q[:3 * len(tris)]).max() < 1e-12  # no volume charge for uniform M
        phi, H = direct.forward(targets, x, w, q)
        ex_phi = np.zeros(len(targets))
        ex_H = np.zeros((len(targets), 2))
        for (ia, ib) in bedges:
            a, b = nodes[ia], nodes[ib]
            d = b - a
            nrm = np.array([d[1], -d[0]]) / np.hypot(*d)
            sig = M @ nrm
            for k, y in enumerate(targets):
                val, grad = segment_log_integral(y, a, b)
                ex_phi[k] += -sig / (2 * np.pi) * val
                ex_H[k] += sig / (2 * np.pi) * grad
        errs_phi.append(np.abs(phi - ex_phi).max())
        errs_H.append(np.abs(H - ex_H).max())
    # h halves each time: 4th-order convergence gives a factor ~16
    assert errs_phi[-1] < 1e-7 and errs_H[-1] < 1e-6
    assert errs_phi[0] / errs_phi[-1] > 64 and errs_H[0] / errs_H[-1] > 64


def test_disk_closed_form_and_convergence():
    """Uniformly magnetized disk: phi = M x / 2 inside (paper, first test case), H = -M/2."""
    errs = []
    for N in (400, 1600, 6400):
        nodes, tris, bedges, Mn, x, w, q = disk_problem(N, R=1.0)
        phi, H = direct.forward(nodes, x, w, q)
        deep = np.hypot(nodes[:, 0], nodes[:, 1]) < 0.8
        errs.append(np.sqrt(np.mean((phi[deep] - 0.5 * nodes[deep, 0]) ** 2)))
        assert np.abs(H[deep] - np.array([-0.5, 0.0])).max() < 5e-3
    assert errs[0] / errs[-1] > 4  # converges (polygon error, O(h^2))
    assert errs[-1] < 1e-4


def test_ellipse_demagnetizing_factors():
    """Uniformly magnetized elliptic cylinder: H = -diag(b/(a+b), a/(a+b)) M inside."""
    a, b = 2.0, 1.0
    nodes, tris, bedges = synth.ellipse_mesh(a, b, N=6000, seed=3)
    ell_r = np.hypot(nodes[:, 0] / a, nodes[:, 1] / b)
    deep = ell_r < 0.6
    for Mv in ((1.0, 0.0), (0.0, 1.0), (0.6, 0.8)):
        Mn = synth.M_uniform(nodes, *Mv)
        x, w = fem.sources(nodes, tris, bedges)
        q = fem.charges(nodes, tris, bedges, Mn)
        _, H = direct.forward(nodes[deep], x, w, q)
        Hex = -np.array([b / (a + b) * Mv[0], a / (a + b) * Mv[1]])
        assert np.abs(H - Hex).max() < 4e-3


def test_magic_cylinder_closed_forms():
    """Magic cylinder (paper, second test case): M at twice the polar angle in R1 < r < R2 gives
    phi = r cos(theta) ln(r/R2) in the annulus and the uniform field (ln(R2/R1), 0) in the hole."""
    R1, R2 = 0.5, 1.0
    nodes, tris, bedges = synth.annulus_mesh(R1, R2, N=8000, seed=4)
    Mn = synth.M_magic_cylinder(nodes)
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, Mn)
    r = np.hypot(nodes[:, 0], nodes[:, 1])
    mid = (r > 0.6) & (r < 0.9)
    phi, _ = direct.forward(nodes[mid], x, w, q)
    ex = nodes[mid, 0] * np.log(r[mid] / R2)
    assert np.sqrt(np.mean((phi - ex) ** 2)) < 2e-3
    rng = np.random.default_rng(0)
    hole = synth._jitter_disk(rng, 50, 0.35)
    _, H = direct.forward(hole, x, w, q)
    assert np.abs(H - np.array([np.log(R2 / R1), 0.0])).max() < 1e-2
    outside = np.array([[1.5, 0.2], [-0.3, 1.8], [2.0, -2.0]])
    phi_out, _ = direct.forward(outside, x, w, q)
    assert np.abs(phi_out).max() < 2e-3  # phi vanishes outside


def test_charge_neutrality():
    """sum_j w_j q_j = 0 for a P1 magnetization: the divergence theorem, exact for these rules."""
    for mk in (lambda: synth.workload_ellipse_c2(N=3000), lambda: synth.workload_annulus_c4(N=3000)):
        d = mk()
        x, w = fem.sources(d["nodes"], d["tris"], d["bedges"])
        q = fem.charges(d["nodes"], d["tris"], d["bedges"], d["M"])
        assert abs(np.dot(w, q)) < 1e-13 * np.abs(w * q).sum()


def test_charge_operator_transpose():
    d = synth.workload_ellipse_c2(N=2000)
    rng = np.random.default_rng(5)
    M = rng.standard_normal(d["M"].shape)
    x, w = fem.sources(d["nodes"], d["tris"], d["bedges"])
    u = rng.standard_normal(len(x))
    lhs = np.dot(fem.charges(d["nodes"], d["tris"], d["bedges"], M), u)
    rhs = np.sum(M * fem.charges_T(d["nodes"], d["tris"], d["bedges"], u))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_hand_computed_charges_one_triangle():
    """One triangle (0,0),(1,0),(0,1) with M = (x, 2y) at its nodes: div M = 3, rho = -3;
    quadrature weights |T|/3 = 1/6 at barycentric (2/3,1/6,1/6)...; edge charges M.n."""
    nodes = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    tris = np.array([[0, 1, 2]], dtype=np.int32)
    bedges = np.array([[0, 1], [1, 2], [2, 0]], dtype=np.int32)  # counter-clockwise
    M = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0]])
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, M)
    assert np.allclose(q[:3], -3.0) and np.allclose(w[:3], 1.0 / 6.0)
    assert np.allclose(x[0], [1 / 6, 1 / 6]) and np.allclose(x[1], [2 / 3, 1 / 6])
    g = 0.5 / np.sqrt(3.0)
    # bottom edge (0,0)->(1,0): n = (0,-1), M.n = 0
    assert np.allclose(q[3:5], 0.0) and np.allclose(w[3:5], 0.5)
    assert np.allclose(x[3], [0.5 - g, 0.0])
    # hypotenuse (1,0)->(0,1): n = (1,1)/sqrt2, M(t) = ((1-t), 2t)
    n = np.array([1.0, 1.0]) / np.sqrt(2.0)
    for k, t in enumerate((0.5 - g, 0.5 + g)):
        assert np.isclose(q[5 + k], ((1 - t) * np.array([1.0, 0.0]) + t * np.array([0.0, 2.0])) @ n)
    assert np.isclose(w[5], np.sqrt(2.0) / 2)
    assert abs(np.dot(w, q)) < 1e-14


def test_volume_quadrature_converges_to_brute_force():
    """A triangle with linear M: O1's 3-point rule on a refined sub-mesh converges to an adaptive
    quadrature of the continuous volume integral at an outside target."""
    P = np.array([[0.0, 0.0], [1.0, 0.2], [0.3, 0.9]])
    y = np.array([1.4, 1.1])
    Mfun = lambda p: np.array([0.5 + p[0] - 0.3 * p[1], 0.2 * p[0] + 0.7 * p[1]])
    rho = -(1.0 + 0.7)  # -div M
    J = np.array([P[1] - P[0], P[2] - P[0]]).T
    detJ = abs(np.linalg.det(J))
    exact = integrate.dblquad(
        lambda v, u: rho * (-np.log(np.hypot(*(y - (P[0] + J @ [u, v])))) / (2 * np.pi)) * detJ,
        0, 1, 0, lambda u: 1 - u, epsabs=1e-13, epsrel=1e-13)[0]
    errs = []
    for k in (1, 2, 3, 4):
        n = 2 ** k
        pts, tri = [], []
        idx = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                idx[(i, j)] = len(pts)
                pts.append(P[0] + J @ [i / n, j / n])
        for i in range(n):
            for j in range(n - i):
                tri.append([idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]])
                if i + j + 1 < n:
                    tri.append([idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]])
        nodes = np.array(pts)
        tris = np.array(tri, dtype=np.int32)
        M = np.array([Mfun(p) for p in nodes])
        x, w = fem.sources(nodes, tris, np.zeros((0, 2), np.int32))
        q = fem.charges(nodes, tris, np.zeros((0, 2), np.int32), M)
        assert np.allclose(q, rho)
        phi, _ = direct.forward(y[None], x, w, q)
        errs.append(abs(phi[0] - exact))
    assert errs[-1] < 1e-7 * abs(exact) and errs[0] / errs[-1] > 50


def test_invariants_linearity_rotation_translation_scale():
    d = synth.workload_ellipse_c2(N=1500)
    nodes, tris, bedges, M = d["nodes"], d["tris"], d["bedges"], d["M"]
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, M)
    phi, H = direct.forward(nodes, x, w, q)
    # oddness / linearity
    phim, Hm = direct.forward(nodes, x, w, fem.charges(nodes, tris, bedges, -M))
    assert rel_l2(phim, -phi) < 1e-13 and rel_l2(Hm, -H) < 1e-13
    # rotation equivariance: rotate mesh and M together
    th = 0.7
    Rm = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    nr, Mr = nodes @ Rm.T, M @ Rm.T
    xr, wr = fem.sources(nr, tris, bedges)
    phir, Hr = direct.forward(nr, xr, wr, fem.charges(nr, tris, bedges, Mr))
    assert rel_l2(phir, phi) < 1e-12 and rel_l2(Hr, H @ Rm.T) < 1e-12
    # translation invariance
    nt = nodes + np.array([3.0, -2.0])
    xt, wt = fem.sources(nt, tris, bedges)
    phit, Ht = direct.forward(nt, xt, wt, fem.charges(nt, tris, bedges, M))
    assert rel_l2(phit, phi) < 1e-12 and rel_l2(Ht, H) < 1e-12
    # scale covariance: coordinates x lam -> phi x lam, H unchanged (neutral charges)
    lam = 2.5
    ns = nodes * lam
    xs, ws = fem.sources(ns, tris, bedges)
    phis, Hs = direct.forward(ns, xs, ws, fem.charges(ns, tris, bedges, M))
    assert rel_l2(phis, lam * phi) < 1e-11 and rel_l2(Hs, H) < 1e-11


def test_adjoint_identities(o1):
    y, x, w, q = synth.random_cloud(300, 400, 6)
    rng = np.random.default_rng(7)
    V = rng.standard_normal((300, 2))
    v = rng.standard_normal(300)
    phi, H = o1.forward(y, x, w, q)
    assert abs(np.sum(H * V) - np.dot(q, o1.adjoint(y, x, w, V=V))) < 1e-12 * np.abs(H * V).sum()
    assert abs(np.dot(phi, v) - np.dot(q, o1.adjoint(y, x, w, v=v))) < 1e-12 * np.abs(phi * v).sum()


def test_coincident_pairs_are_skipped(o1):
    y = np.array([[0.0, 0.0], [1.0, 0.0]])
    x = np.array([[0.0, 0.0], [0.0, 1.0]])
    w = np.array([1.0, 1.0])
    q = np.array([2.0, 3.0])
    phi, H = o1.forward(y, x, w, q)
    # target 0 sees only source 1 at distance 1: ln 1 = 0, H = 3/(2pi) * (0,-1)
    assert abs(phi[0]) < 1e-16 and np.allclose(H[0], [0.0, -3.0 / (2 * np.pi)])


def test_energy_gradient_finite_difference(o1):
    """E(M) = -1/2 sum l_i M_i.H_i is quadratic, so a central difference with any step is exact
    up to rounding; the gradient -1/2 (l H + C^T A^T (l M)) must match it."""
    d = synth.workload_annulus_c4(N=400)
    nodes, tris, bedges, M = d["nodes"], d["tris"], d["bedges"], d["M"]
    x, w = fem.sources(nodes, tris, bedges)
    ell = fem.lumped_mass(nodes, tris)

    def E(Mv):
        _, H = o1.forward(nodes, x, w, fem.charges(nodes, tris, bedges, Mv))
        return fem.energy(Mv, H, ell), H

    E0, H0 = E(M)
    u = o1.adjoint(nodes, x, w, V=ell[:, None] * M)
    grad = fem.energy_grad(H0, ell, fem.charges_T(nodes, tris, bedges, u))
    rng = np.random.default_rng(8)
    for _ in range(3):
        v = rng.standard_normal(M.shape)
        fd = (E(M + v)[0] - E(M - v)[0]) / 2.0
        assert abs(fd - np.sum(grad * v)) < 1e-10 * (abs(fd) + 1e-12)


def test_demag_energy_closed_forms(o1):
    """Disk: pi R^2 M^2 / 4; ellipse (M = x): pi a b b/(2(a+b)); magic cylinder: pi (R2^2 - R1^2)/4.
    The lumped nodal energy converges at O(h) (boundary nodes see the surface charges)."""
    nodes, tris, bedges, M, x, w, q = disk_problem(6000)
    ell = fem.lumped_mass(nodes, tris)
    _, H = o1.forward(nodes, x, w, q)
    assert abs(fem.energy(M, H, ell) - np.pi / 4) < 0.02 * np.pi / 4
    d = synth.workload_annulus_c4(N=6000, magic=True)
    x, w = fem.sources(d["nodes"], d["tris"], d["bedges"])
    q = fem.charges(d["nodes"], d["tris"], d["bedges"], d["M"])
    _, H = o1.forward(d["nodes"], x, w, q)
    ell = fem.lumped_mass(d["nodes"], d["tris"])
    ex = np.pi * (1.0 - 0.25) / 4
    assert abs(fem.energy(d["M"], H, ell) - ex) < 0.05 * ex
