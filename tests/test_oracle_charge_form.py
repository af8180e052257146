"""Pins of the oracle's outputs at the quadrature points and of its FEM-consistent field
(oracle/fem.py: phi_at_sources, charge_energy, charge_energy_grad, p1_gradient,
p1_gradient_nodal) against what the mathematics fixes: closed-form energies of uniformly
magnetized bodies, exactness of the P1 gradient on linear potentials, the closed-form
demagnetizing field of an ellipse, brute force on two charges, and the exact central
difference of a quadratic energy."""
import numpy as np
import pytest

import synth
from oracle import direct, fem

pytestmark = pytest.mark.cpu


def mesh_problem(kind, N, M=(1.0, 0.0), seed=1):
    if kind == "disk":
        nodes, tris, bedges = synth.disk_mesh_n(N, R=1.0, seed=seed)
    else:
        nodes, tris, bedges = synth.ellipse_mesh(2.0, 1.0, N=N, seed=seed)
    Mn = synth.M_uniform(nodes, *M)
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, Mn)
    return nodes, tris, bedges, Mn, x, w, q


def test_phi_at_sources_leaves_each_points_own_charge_out():
    """Two charges by hand: each sees only the other, G = -(1/2pi) ln r; a third point placed
    exactly on the first adds nothing to it (a pair at distance 0 is not part of the sum)."""
    x = np.array([[0.1, -0.2], [0.7, 0.4]])
    w = np.array([0.5, 2.0])
    q = np.array([3.0, -1.5])
    r = np.hypot(0.6, 0.6)
    G = -np.log(r) / (2 * np.pi)
    phi = fem.phi_at_sources(x, w, q)
    assert abs(phi[0] - w[1] * q[1] * G) < 1e-15 and abs(phi[1] - w[0] * q[0] * G) < 1e-15
    x3 = np.concatenate([x, x[:1]])
    phi3 = fem.phi_at_sources(x3, np.append(w, 1.0), np.append(q, 4.0))
    assert abs(phi3[0] - phi[0]) < 1e-15 and abs(phi3[2] - phi[0] + w[0] * q[0] * 0.0) < 1e-15


def test_p1_gradient_is_exact_on_linear_potentials():
    """phi = a.r + b is reproduced by P1 interpolation: -grad is -a on every triangle and at
    every node after the lumped projection (pins the hat gradients and the sign)."""
    nodes, tris, bedges = synth.annulus_mesh(0.5, 1.0, N=3000, seed=5)
    a = np.array([0.7, -1.3])
    phi = nodes @ a + 0.25
    HT = fem.p1_gradient(nodes, tris, phi)
    Hn = fem.p1_gradient_nodal(nodes, tris, phi)
    assert np.abs(HT + a).max() < 1e-12
    assert np.abs(Hn + a).max() < 1e-12


def test_p1_gradient_recovers_the_ellipse_demagnetizing_field():
    """Ellipse a = 2, b = 1, M = (1, 0): the potential inside is linear, phi = N_x x with
    N_x = b/(a+b) = 1/3, so the P1 gradient of the nodal direct-sum potential is
    H = (-1/3, 0) at interior nodes, up to the discretization of the charges."""
    nodes, tris, bedges, M, x, w, q = mesh_problem("ellipse", 8000, seed=3)
    phi, _ = direct.forward(nodes, x, w, q, want_H=False)
    Hn = fem.p1_gradient_nodal(nodes, tris, phi)
    inner = np.hypot(nodes[:, 0] / 2, nodes[:, 1]) < 0.6
    assert inner.sum() > 1000
    assert np.abs(Hn[inner] - [-1.0 / 3.0, 0.0]).max() < 1e-6


def test_charge_energy_converges_to_the_closed_forms():
    """E_q = 1/2 sum_j s_j phi_j: disk (R = 1, M = x) pi/4, ellipse (a = 2, b = 1, M = x)
    pi a b^2 / (2 (a + b)) = pi/3.  The quadrature of the singular self-potential converges
    at about first order: the error falls with N and is a few percent at these sizes."""
    errs = []
    for N in (1500, 6000):
        nodes, tris, bedges, M, x, w, q = mesh_problem("disk", N)
        errs.append(abs(fem.charge_energy(w, q, fem.phi_at_sources(x, w, q)) / (np.pi / 4) - 1))
    assert errs[1] < 0.03 and errs[1] < 0.7 * errs[0], errs
    nodes, tris, bedges, M, x, w, q = mesh_problem("ellipse", 8000, seed=3)
    e = abs(fem.charge_energy(w, q, fem.phi_at_sources(x, w, q)) / (np.pi / 3) - 1)
    assert e < 0.02, e


def test_charge_energy_gradient_is_exact():
    """E_q(M) is quadratic, so the central difference with any step equals grad . v up to
    rounding; grad = C^T (w phi) relies on the symmetry of the potential matrix."""
    d = synth.workload_annulus_c4(N=500)
    nodes, tris, bedges, M = d["nodes"], d["tris"], d["bedges"], d["M"]
    x, w = fem.sources(nodes, tris, bedges)

    def E(Mv):
        q = fem.charges(nodes, tris, bedges, Mv)
        ps = fem.phi_at_sources(x, w, q)
        return fem.charge_energy(w, q, ps), ps

    E0, ps0 = E(M)
    grad = fem.charge_energy_grad(nodes, tris, bedges, w, ps0)
    rng = np.random.default_rng(4)
    for _ in range(3):
        v = rng.standard_normal(M.shape)
        fd = (E(M + v)[0] - E(M - v)[0]) / 2.0
        assert abs(fd - np.sum(grad * v)) < 1e-10 * (abs(fd) + 1e-12)
