"""Pins of the 3D FEM front (oracle/fem3.py) and of the tetrahedral mesh generators.

  * the meshes: positive total volume equal to the boundary flux of r/3 (outward faces);
  * charge neutrality (divergence theorem, exact for P1 with the degree-2 rules) and the
    adjoint identity of C and C^T on random magnetizations;
  * a uniformly magnetized cube: no volume charge, +-M_z on the faces normal to z, the
    potential against the closed form (exact integral of 1/r over a rectangle, checked
    against numerical quadrature) converging as the mesh is refined, the field -M/3 at
    the centre;
  * a uniformly magnetized ball: potential M.r/3 and field -M/3 inside, approached at
    second order as the mesh is refined (the boundary is a polyhedron); its lumped
    energy tends to V M^2 / 6 at first order.
"""
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import direct, fem3


def _F(x, y, z):
    """An antiderivative of 1/sqrt(x^2 + y^2 + z^2) in x and y (d^2 F / dx dy = 1/r)."""
    r = np.sqrt(x * x + y * y + z * z)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(z != 0, z * np.arctan(x * y / (z * r)), 0.0)
    return x * np.log(y + r) + y * np.log(x + r) - t


def rect_integral(x1, x2, y1, y2, z):
    """int_{x1}^{x2} int_{y1}^{y2} dy dx / sqrt(x^2 + y^2 + z^2)."""
    return _F(x2, y2, z) - _F(x1, y2, z) - _F(x2, y1, z) + _F(x1, y1, z)


def cube_potential(r, L=1.0, Mz=1.0):
    """Potential of the cube [-L/2, L/2]^3 magnetized Mz along z: surface charge +Mz on its
    top face and -Mz on its bottom face."""
    h = L / 2
    out = np.zeros(len(r))
    for zf, sg in ((h, 1.0), (-h, -1.0)):
        out += sg * Mz * rect_integral(-h - r[:, 0], h - r[:, 0], -h - r[:, 1], h - r[:, 1], zf - r[:, 2])
    return out / (4 * np.pi)


@pytest.mark.parametrize("box", [(-0.3, 0.7, -0.2, 0.5, 0.4), (-0.3, 0.7, -0.2, 0.5, -0.4),
                                 (0.1, 0.9, 0.2, 0.6, -0.3), (-1.0, 1.0, -1.0, 1.0, 0.05)])
def test_rectangle_integral_against_quadrature(box):
    x1, x2, y1, y2, z = box
    num, _ = integrate.dblquad(lambda y, x: 1 / np.sqrt(x * x + y * y + z * z), x1, x2, y1, y2,
                               epsabs=1e-13, epsrel=1e-13)
    assert abs(rect_integral(x1, x2, y1, y2, z) - num) < 1e-12 * abs(num)


@pytest.mark.parametrize("mesh", ["cube", "ball"])
def test_meshes_are_closed_and_outward(mesh):
    nodes, tets, bf = synth.cube_tet_mesh(n=5, jitter=0.12) if mesh == "cube" else synth.ball_tet_mesh(n=6)
    p = nodes[tets]
    vol = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6
    a, b, c = nodes[bf[:, 0]], nodes[bf[:, 1]], nodes[bf[:, 2]]
    flux = (np.cross(b - a, c - a) / 2 * (a + b + c) / 3).sum() / 3  # oint r.n dA / 3 = volume
    assert np.all(vol != 0) and abs(np.abs(vol).sum() - flux) < 1e-13 * flux
    assert abs(fem3.lumped_mass(nodes, tets).sum() - flux) < 1e-13 * flux


@pytest.mark.parametrize("mesh", ["cube", "ball"])
def test_charge_neutrality_and_adjoint(mesh):
    nodes, tets, bf = synth.cube_tet_mesh(n=5, jitter=0.12) if mesh == "cube" else synth.ball_tet_mesh(n=6)
    rng = np.random.default_rng(4)
    M = rng.standard_normal((len(nodes), 3))
    x, w = fem3.sources(nodes, tets, bf)
    q = fem3.charges(nodes, tets, bf, M)
    assert len(x) == len(w) == len(q) == 4 * len(tets) + 3 * len(bf)
    assert abs(np.dot(w, q)) < 1e-13 * np.abs(w * q).sum()
    u = rng.standard_normal(len(q))
    assert abs(np.dot(u, q) - (fem3.charges_T(nodes, tets, bf, u) * M).sum()) < 1e-12 * np.abs(u * q).sum()


def test_uniform_cube_charges_potential_and_centre_field():
    rng = np.random.default_rng(3)
    tg = np.concatenate([rng.uniform(-0.3, 0.3, (150, 3)),
                         rng.standard_normal((80, 3))])
    tg[150:] *= (rng.uniform(1.0, 2.0, 80) / np.linalg.norm(tg[150:], axis=1))[:, None]
    ex = cube_potential(tg)
    errs = []
    for n in (4, 8, 16):
        nodes, tets, bf = synth.cube_tet_mesh(n=n, jitter=0.1)
        M = np.zeros((len(nodes), 3))
        M[:, 2] = 1.0
        x, w = fem3.sources(nodes, tets, bf)
        q = fem3.charges(nodes, tets, bf, M)
        T = len(tets)
        assert np.abs(q[:4 * T]).max() < 1e-12
        (a, b, c), _, nrm = fem3._face_geom(nodes, bf)
        qs = q[4 * T:].reshape(-1, 3)
        assert np.allclose(qs, nrm[:, 2:3], atol=1e-14)  # M.n: +1 on top, -1 on bottom, 0 on the sides
        phi, _ = direct.forward3(tg, x, w, q, want_H=False)
        errs.append(np.abs(phi - ex).max() / np.abs(ex).max())
        if n == 8:
            _, Hc = direct.forward3(np.zeros((1, 3)), x, w, q, want_phi=False)
            assert np.abs(Hc[0] - np.array([0.0, 0.0, -1.0 / 3.0])).max() < 1e-7
    assert errs[0] > 10 * errs[1] > 10 * errs[2] and errs[2] < 1e-6, errs


def test_uniform_ball_potential_and_field():
    rng = np.random.default_rng(5)
    tb = rng.uniform(-0.5, 0.5, (300, 3))
    tb = tb[np.linalg.norm(tb, axis=1) < 0.5]
    ep, eh = [], []
    for n in (4, 8, 16):
        nodes, tets, bf = synth.ball_tet_mesh(n=n)
        M = np.zeros((len(nodes), 3))
        M[:, 0] = 1.0
        x, w = fem3.sources(nodes, tets, bf)
        q = fem3.charges(nodes, tets, bf, M)
        phi, H = direct.forward3(tb, x, w, q)
        ep.append(np.abs(phi - tb[:, 0] / 3).max())
        eh.append(np.abs(H - np.array([-1 / 3, 0.0, 0.0])).max())
    assert ep[0] > 2.5 * ep[1] > 2.5 * 2.5 * ep[2] and ep[2] < 1e-4, ep
    assert eh[0] > 2.5 * eh[1] > 2.5 * 2.5 * eh[2] and eh[2] < 5e-4, eh


def test_uniform_ball_lumped_energy_converges_at_first_order():
    """E = -1/2 sum l_i M_i.H_i of the uniformly magnetized ball tends to V M^2 / 6 (H = -M/3
    inside); the boundary nodes, where H is the average of the inner and outer fields, make
    the lumped sum's error first order in h: (E/(V/6) - 1) n is constant."""
    devs = []
    for n in (8, 12, 16):
        nodes, tets, bf = synth.ball_tet_mesh(n=n)
        M = np.zeros((len(nodes), 3))
        M[:, 2] = 1.0
        x, w = fem3.sources(nodes, tets, bf)
        q = fem3.charges(nodes, tets, bf, M)
        _, H = direct.forward3(nodes, x, w, q, want_phi=False)
        ell = fem3.lumped_mass(nodes, tets)
        devs.append((fem3.energy(M, H, ell) / (ell.sum() / 6) - 1) * n)
    assert all(d < 0 for d in devs) and max(devs) / min(devs) < 1.03, devs
