"""FEM front of the oracle (FP64 numpy) -- TEST INFRASTRUCTURE ONLY.

Turns a P1 nodal magnetization on a triangle mesh into the point-charge list of
the paper's eq. (2): quadrature points r_j, weights omega_j det J(r_j) and
charge densities (rho = -div M inside, sigma = M.n on the boundary, from the
definitions given with eq. (1)), using the linear interpolation of nodal M
inside each element that the paper describes just before eq. (2).

Readings of the paper (its quadrature footnote is missing):
  * volume: the 3-point interior rule at barycentric (2/3,1/6,1/6) and
    permutations, omega = 1/6 on the reference triangle, det J = 2|T|,
    so w = |T|/3; rho is constant per triangle for P1 M.
  * surface: 2-point Gauss-Legendre on each straight boundary edge,
    t = 1/2 -+ 1/(2 sqrt 3), w = |e|/2 (1D Jacobian |e|); sigma = M_h.n_e with
    the straight edge's outward normal.
  * one merged source list: all volume points (triangle-major, 3 each), then
    all surface points (edge-major, 2 each).

The energy E = -1/2 sum_i l_i M_i.H_i uses the lumped nodal mass
l_i = sum_{T containing i} |T|/3 (the physical demagnetizing energy, mu0 = 1);
its exact gradient for H = A C M is -1/2 (L H + C^T A^T L M).

Outputs at the quadrature points (the charge form of the same energy): with the
potential of eq. (2) taken at the quadrature points themselves, a point's own
charge left out (the pair at distance 0 is not part of the sum, like any
coincident pair),
    phi_j = sum_{k != j} s_k G(r_j - r_k),   s = w q,
the energy of the charges in their own potential is E_q = 1/2 sum_j s_j phi_j
(= 1/2 int rho phi + 1/2 oint sigma phi with both integrals by the same
quadrature: the physical energy of the definitions given with eq. (1), mu0 = 1).
The matrix [G(r_j - r_k)]_{j != k} is symmetric, so dE_q/dq = w phi and
dE_q/dM = C^T (w phi): one potential evaluation gives the energy and its gradient.

FEM-consistent field: the P1 interpolant of the nodal potential has the constant
gradient sum_k phi_{i_k} grad(lambda_k) on each triangle (lambda_k its hat
functions), so H_T = -that; its lumped projection onto the nodes is
H_i = (1/l_i) sum_{T containing i} (|T|/3) H_T.

Pins: charge neutrality (divergence theorem), closed-form potentials of
uniformly magnetized polygons/disks/ellipses and of the magic cylinder,
adjoint identity of C and C^T, finite differences of E (tests/test_oracle_direct.py);
the charge-form energy against the disk and ellipse energies, its exact central
difference, the P1 gradient on linear potentials and on the ellipse's uniform
interior field, the own-charge exclusion by hand (tests/test_oracle_charge_form.py).
"""
from __future__ import annotations

import numpy as np

_G1 = 0.5 - 0.5 / np.sqrt(3.0)
_G2 = 0.5 + 0.5 / np.sqrt(3.0)
_BARY = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])


def _tri_geom(nodes, tris):
    p0, p1, p2 = nodes[tris[:, 0]], nodes[tris[:, 1]], nodes[tris[:, 2]]
    a2 = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0])
    # gradients of the barycentric (P1 hat) functions, constant per triangle
    g0 = np.stack([p1[:, 1] - p2[:, 1], p2[:, 0] - p1[:, 0]], axis=1) / a2[:, None]
    g1 = np.stack([p2[:, 1] - p0[:, 1], p0[:, 0] - p2[:, 0]], axis=1) / a2[:, None]
    g2 = np.stack([p0[:, 1] - p1[:, 1], p1[:, 0] - p0[:, 0]], axis=1) / a2[:, None]
    area = 0.5 * np.abs(a2)
    return (p0, p1, p2), area, (g0, g1, g2)


def _edge_geom(nodes, bedges):
    a, b = nodes[bedges[:, 0]], nodes[bedges[:, 1]]
    d = b - a
    L = np.hypot(d[:, 0], d[:, 1])
    n = np.stack([d[:, 1], -d[:, 0]], axis=1) / L[:, None]  # domain on the left -> outward = right
    return a, b, L, n


def sources(nodes, tris, bedges):
    """Quadrature points x [Ns, 2] and weights w [Ns] (volume first, then surface)."""
    (p0, p1, p2), area, _ = _tri_geom(nodes, tris)
    xv = np.stack([_BARY[k, 0] * p0 + _BARY[k, 1] * p1 + _BARY[k, 2] * p2 for k in range(3)], axis=1)
    wv = np.repeat((area / 3.0)[:, None], 3, axis=1)
    a, b, L, _ = _edge_geom(nodes, bedges)
    xs = np.stack([(1 - t) * a + t * b for t in (_G1, _G2)], axis=1)
    ws = np.repeat((0.5 * L)[:, None], 2, axis=1)
    x = np.concatenate([xv.reshape(-1, 2), xs.reshape(-1, 2)], axis=0)
    w = np.concatenate([wv.ravel(), ws.ravel()])
    return x, w


def charges(nodes, tris, bedges, M):
    """q = C M: rho_T = -div(M_h) at the 3 volume points of T, sigma = M_h.n_e at edge points."""
    _, _, (g0, g1, g2) = _tri_geom(nodes, tris)
    div = (M[tris[:, 0]] * g0).sum(1) + (M[tris[:, 1]] * g1).sum(1) + (M[tris[:, 2]] * g2).sum(1)
    qv = np.repeat(-div[:, None], 3, axis=1)
    _, _, _, n = _edge_geom(nodes, bedges)
    Ma, Mb = M[bedges[:, 0]], M[bedges[:, 1]]
    qs = np.stack([(((1 - t) * Ma + t * Mb) * n).sum(1) for t in (_G1, _G2)], axis=1)
    return np.concatenate([qv.ravel(), qs.ravel()])


def charges_T(nodes, tris, bedges, u):
    """C^T u: nodal 2-vectors, the exact transpose of charges()."""
    N = len(nodes)
    T = len(tris)
    _, _, grads = _tri_geom(nodes, tris)
    uv = u[:3 * T].reshape(T, 3).sum(1)  # the 3 volume points of T share rho_T
    out = np.zeros((N, 2))
    for k in range(3):
        np.add.at(out, tris[:, k], -uv[:, None] * grads[k])
    _, _, _, n = _edge_geom(nodes, bedges)
    us = u[3 * T:].reshape(-1, 2)
    for c, t in enumerate((_G1, _G2)):
        np.add.at(out, bedges[:, 0], ((1 - t) * us[:, c])[:, None] * n)
        np.add.at(out, bedges[:, 1], (t * us[:, c])[:, None] * n)
    return out


def lumped_mass(nodes, tris):
    _, area, _ = _tri_geom(nodes, tris)
    ell = np.zeros(len(nodes))
    for k in range(3):
        np.add.at(ell, tris[:, k], area / 3.0)
    return ell


def energy(M, H, ell):
    """E = -1/2 sum_i l_i M_i . H_i."""
    return -0.5 * float(np.dot(ell, (M * H).sum(1)))


def energy_grad(H, ell, CtATLM):
    """dE/dM = -1/2 (l H + C^T A^T (l M)); the caller supplies C^T A^T (l M)."""
    return -0.5 * (ell[:, None] * H + CtATLM)


def phi_at_sources(x, w, q):
    """phi_j = sum_{k != j} w_k q_k G(r_j - r_k) at the quadrature points, by the plain
    direct sum (oracle O1 with targets = sources: a pair at distance 0 is skipped, so
    each point's own charge is left out)."""
    from . import direct
    phi, _ = direct.forward(np.asarray(x, np.float64), x, w, q, want_H=False)
    return phi


def charge_energy(w, q, phi_s):
    """E_q = 1/2 sum_j w_j q_j phi_j (phi_j from phi_at_sources)."""
    return 0.5 * float(np.dot(np.asarray(w) * np.asarray(q), phi_s))


def charge_energy_grad(nodes, tris, bedges, w, phi_s):
    """dE_q/dM = C^T (w phi): the potential matrix between distinct points is symmetric."""
    return charges_T(nodes, tris, bedges, np.asarray(w) * np.asarray(phi_s))


def p1_gradient(nodes, tris, phi):
    """H_T = -grad of the P1 interpolant of the nodal potential phi [N], per triangle [T, 2]."""
    _, _, grads = _tri_geom(nodes, tris)
    return -sum(phi[tris[:, k]][:, None] * grads[k] for k in range(3))


def p1_gradient_nodal(nodes, tris, phi):
    """Lumped projection of p1_gradient onto the nodes: H_i = (1/l_i) sum_{T at i} (|T|/3) H_T."""
    _, area, _ = _tri_geom(nodes, tris)
    HT = p1_gradient(nodes, tris, phi)
    out = np.zeros((len(nodes), 2))
    for k in range(3):
        np.add.at(out, tris[:, k], (area / 3.0)[:, None] * HT)
    return out / lumped_mass(nodes, tris)[:, None]
