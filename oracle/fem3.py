"""FEM front of the oracle in 3D (FP64 numpy) -- TEST INFRASTRUCTURE ONLY.

The tetrahedral counterpart of oracle.fem: a P1 nodal magnetization on a tetrahedral
mesh becomes the point-charge list of the paper's eq. (2) with the 3D Green function
given with eq. (1): quadrature points r_j, weights omega_j det J(r_j) and charge
densities (rho = -div M inside, sigma = M.n on the boundary, the definitions given
with eq. (1)), using the linear interpolation of nodal M inside each element that the
paper describes before eq. (2).

Readings of the paper (its quadrature footnote is missing; it describes 2D and
states the method for 3D alike):
  * volume: the 4-point degree-2 rule on each tetrahedron, barycentric
    (a, b, b, b) and permutations with a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20,
    weight |T|/4 each; rho is constant per tetrahedron for P1 M;
  * surface: the 3-point degree-2 rule on each boundary triangle, barycentric
    (2/3, 1/6, 1/6) and permutations, weight |F|/3 each; sigma = M_h.n_F with the
    flat face's outward unit normal;
  * one merged source list: all volume points (tetrahedron-major, 4 each), then all
    surface points (face-major, 3 each).
Lumped nodal mass l_i = sum_{T containing i} |T|/4; E = -1/2 sum_i l_i M_i.H_i as in 2D.

Pins (tests/test_oracle_fem3.py): charge neutrality (divergence theorem: both rules
integrate the P1 integrands exactly), the adjoint identity of C and C^T, a uniformly
magnetized cube (no volume charge, +-M_z on the faces normal to z; its potential in
closed form from the exact integral of 1/r over a rectangle, itself checked against
numerical quadrature; the field -M/3 at the centre), a uniformly magnetized ball
(potential M.r/3 inside) approached as the mesh is refined.
"""
from __future__ import annotations

import numpy as np

_A = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
_B = (5.0 - np.sqrt(5.0)) / 20.0
_TBARY = np.array([[_A, _B, _B, _B], [_B, _A, _B, _B], [_B, _B, _A, _B], [_B, _B, _B, _A]])
_FBARY = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])


def _tet_geom(nodes, tets):
    """Corner points, volumes |T| and the gradients of the four barycentric functions [4][T, 3]."""
    p = nodes[tets]                                     # [T, 4, 3]
    J = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)  # columns
    vol = np.abs(np.linalg.det(J)) / 6.0
    Jinv = np.linalg.inv(J)                             # lambda_{1..3} = Jinv (x - p0)
    g = [Jinv[:, 0, :], Jinv[:, 1, :], Jinv[:, 2, :]]
    return p, vol, [-(g[0] + g[1] + g[2])] + g


def _face_geom(nodes, bfaces):
    a, b, c = nodes[bfaces[:, 0]], nodes[bfaces[:, 1]], nodes[bfaces[:, 2]]
    cr = np.cross(b - a, c - a)
    area2 = np.linalg.norm(cr, axis=1)
    return (a, b, c), 0.5 * area2, cr / area2[:, None]


def sources(nodes, tets, bfaces):
    """Quadrature points x [S, 3] and weights w [S] (volume first, then surface)."""
    p, vol, _ = _tet_geom(nodes, tets)
    xv = np.einsum("qk,tkd->tqd", _TBARY, p)
    wv = np.repeat((vol / 4.0)[:, None], 4, axis=1)
    (a, b, c), area, _ = _face_geom(nodes, bfaces)
    xs = np.stack([l[0] * a + l[1] * b + l[2] * c for l in _FBARY], axis=1)
    ws = np.repeat((area / 3.0)[:, None], 3, axis=1)
    return (np.concatenate([xv.reshape(-1, 3), xs.reshape(-1, 3)]),
            np.concatenate([wv.ravel(), ws.ravel()]))


def charges(nodes, tets, bfaces, M):
    """q = C M: rho_T = -div(M_h) at the 4 volume points of T, sigma = M_h.n_F at face points."""
    _, _, g = _tet_geom(nodes, tets)
    div = sum((M[tets[:, k]] * g[k]).sum(1) for k in range(4))
    qv = np.repeat(-div[:, None], 4, axis=1)
    _, _, n = _face_geom(nodes, bfaces)
    Mf = [M[bfaces[:, k]] for k in range(3)]
    qs = np.stack([((l[0] * Mf[0] + l[1] * Mf[1] + l[2] * Mf[2]) * n).sum(1) for l in _FBARY], axis=1)
    return np.concatenate([qv.ravel(), qs.ravel()])


def charges_T(nodes, tets, bfaces, u):
    """C^T u: nodal 3-vectors, the exact transpose of charges()."""
    T = len(tets)
    _, _, g = _tet_geom(nodes, tets)
    uv = u[:4 * T].reshape(T, 4).sum(1)
    out = np.zeros((len(nodes), 3))
    for k in range(4):
        np.add.at(out, tets[:, k], -uv[:, None] * g[k])
    _, _, n = _face_geom(nodes, bfaces)
    us = u[4 * T:].reshape(-1, 3)
    for q, l in enumerate(_FBARY):
        for k in range(3):
            np.add.at(out, bfaces[:, k], (l[k] * us[:, q])[:, None] * n)
    return out


def lumped_mass(nodes, tets):
    _, vol, _ = _tet_geom(nodes, tets)
    ell = np.zeros(len(nodes))
    for k in range(4):
        np.add.at(ell, tets[:, k], vol / 4.0)
    return ell


def energy(M, H, ell):
    """E = -1/2 sum_i l_i M_i . H_i."""
    return -0.5 * float(np.dot(ell, (M * H).sum(1)))
