"""Seeded synthetic workloads for the FEM-NFFT fast summation.

This module only builds inputs: point sets (2D and 3D), 2D triangle meshes,
boundary edge lists and magnetization fields, all from seeded random
generators.  It holds none of the fast summation's arithmetic (no Green
function, no regularization, no window, no FFT, no near-field correction), so
that the CPU oracle and the GPU path can both be fed from it without sharing any
code with each other.  Two point-cloud workloads carry their own charges: the
rounded-square cloud writes -div M analytically at its cell points and M.n at
2-point Gauss points of its boundary, the 3D ball lattice a smooth random field.
Both paths take those charges as plain inputs; the FEM charge operators under
test (oracle/fem.py and the library's mesh calls) are separate code.

Mesh conventions shared by every consumer:
  nodes  float64 [N, 2]
  tris   int32   [T, 3]   vertex indices, any orientation
  bedges int32   [E, 2]   boundary edges (a, b) oriented so that the domain
                          lies to the LEFT of a->b (outer boundaries run
                          counter-clockwise, hole boundaries clockwise)
  M      float64 [N, 2]   nodal magnetization

The paper's own meshes (a uniformly magnetized disk and a "magic cylinder"
annulus, 400 to 38k nodes) are not available; the generators below stand in
for them with polar-ring meshes of the same shapes.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Delaunay

SEED_BASE = 8072387  # per-workload seeds are SEED_BASE + k


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def _ring(n, r, phase):
    a = phase + 2.0 * np.pi * np.arange(n) / n
    return np.stack([r * np.cos(a), r * np.sin(a)], axis=1)


def _jitter_disk(rng, n, radius):
    """n offsets uniform in a disk of the given radius."""
    rad = radius * np.sqrt(rng.random(n))
    ang = 2.0 * np.pi * rng.random(n)
    return np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)


def _clean_tris(nodes, tris):
    """Drop zero-area triangles (can only appear from exactly collinear nodes)."""
    p = nodes[tris]
    a2 = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - \
         (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0])
    return tris[np.abs(a2) > 1e-14 * np.max(np.abs(a2))]


def disk_mesh(R=1.0, K=30, ring_nodes=None, jitter=0.1, seed=SEED_BASE):
    """Polar-ring disk mesh.

    Centre node plus K rings at radius kR/K; ring k holds ring_nodes(k) nodes
    (default round(2*pi*k), i.e. isotropic spacing h = R/K).  Interior nodes are
    jittered uniformly in a disk of radius jitter*h; the outer ring lies exactly
    on the circle.  Delaunay triangulation (the domain is convex).
    """
    rng = np.random.default_rng(seed)
    h = R / K
    if ring_nodes is None:
        ring_nodes = lambda k: int(round(2.0 * np.pi * k))
    pts = [np.zeros((1, 2))]
    starts = []
    for k in range(1, K + 1):
        n = ring_nodes(k)
        starts.append(sum(len(q) for q in pts))
        pts.append(_ring(n, k * h, rng.random() * 2.0 * np.pi / n))
    nodes = np.concatenate(pts, axis=0)
    nb = ring_nodes(K)
    interior = np.arange(len(nodes) - nb)
    nodes[interior] += _jitter_disk(rng, len(interior), jitter * h)
    tris = Delaunay(nodes).simplices.astype(np.int32)
    tris = _clean_tris(nodes, tris)
    b0 = starts[-1]
    ring = np.arange(b0, b0 + nb)
    bedges = np.stack([ring, np.roll(ring, -1)], axis=1).astype(np.int32)  # CCW
    return nodes, tris, bedges


def disk_mesh_n(N, R=1.0, jitter=0.1, seed=SEED_BASE):
    """Disk mesh with about N nodes (isotropic ring spacing)."""
    K = max(2, int(round(np.sqrt(N / np.pi))))
    return disk_mesh(R=R, K=K, jitter=jitter, seed=seed)


def ellipse_mesh(a=2.0, b=1.0, N=50_000, jitter=0.1, seed=SEED_BASE + 1):
    """Ellipse mesh: a unit-disk ring mesh with about N nodes mapped by (x, y) -> (a x, b y).

    An affine map keeps the triangulation valid and the boundary orientation.
    """
    nodes, tris, bedges = disk_mesh_n(N, R=1.0, jitter=jitter, seed=seed)
    nodes = nodes * np.array([a, b])
    return nodes, tris, bedges


def annulus_mesh(R1=0.5, R2=1.0, N=20_000, jitter=0.1, seed=SEED_BASE + 3):
    """Annulus R1 < r < R2 from rings at radii R1 + k h, k = 0..K.

    Ring k holds round(2 pi r_k / h) nodes; interior rings are jittered by
    jitter*h.  Delaunay triangles whose centroid lies in the hole are removed.
    Outer boundary counter-clockwise, inner boundary clockwise.
    """
    rng = np.random.default_rng(seed)
    K = max(2, int(round(np.sqrt(N * (R2 - R1) / (np.pi * (R1 + R2))))))
    h = (R2 - R1) / K
    pts, starts, counts = [], [], []
    off = 0
    for k in range(K + 1):
        r = R1 + k * h
        n = int(round(2.0 * np.pi * r / h))
        starts.append(off)
        counts.append(n)
        pts.append(_ring(n, r, rng.random() * 2.0 * np.pi / n))
        off += n
    nodes = np.concatenate(pts, axis=0)
    inner = np.arange(starts[1], starts[K])
    nodes[inner] += _jitter_disk(rng, len(inner), jitter * h)
    tris = Delaunay(nodes).simplices.astype(np.int32)
    cen = nodes[tris].mean(axis=1)
    tris = tris[np.hypot(cen[:, 0], cen[:, 1]) > R1]
    tris = _clean_tris(nodes, tris)
    outer = np.arange(starts[K], starts[K] + counts[K])
    ring0 = np.arange(starts[0], starts[0] + counts[0])
    e_out = np.stack([outer, np.roll(outer, -1)], axis=1)
    e_in = np.stack([np.roll(ring0, -1), ring0], axis=1)  # clockwise: hole on the right
    bedges = np.concatenate([e_out, e_in], axis=0).astype(np.int32)
    return nodes, tris, bedges


def rounded_rect_boundary(Lx, Ly, rc, h):
    """Counter-clockwise points on a rounded rectangle centred at 0, spacing about h."""
    ax, ay = Lx / 2 - rc, Ly / 2 - rc
    segs = []
    # straight sides and quarter arcs, counter-clockwise from (Lx/2, -ay)
    def line(p0, p1):
        L = np.hypot(*(np.asarray(p1) - np.asarray(p0)))
        n = max(1, int(round(L / h)))
        t = np.arange(n) / n
        return np.asarray(p0)[None] + t[:, None] * (np.asarray(p1) - np.asarray(p0))[None]

    def arc(cx, cy, a0):
        n = max(1, int(round(0.5 * np.pi * rc / h)))
        a = a0 + 0.5 * np.pi * np.arange(n) / n
        return np.stack([cx + rc * np.cos(a), cy + rc * np.sin(a)], axis=1)

    segs.append(line((Lx / 2, -ay), (Lx / 2, ay)))
    segs.append(arc(ax, ay, 0.0))
    segs.append(line((ax, Ly / 2), (-ax, Ly / 2)))
    segs.append(arc(-ax, ay, 0.5 * np.pi))
    segs.append(line((-Lx / 2, ay), (-Lx / 2, -ay)))
    segs.append(arc(-ax, -ay, np.pi))
    segs.append(line((-ax, -Ly / 2), (ax, -Ly / 2)))
    segs.append(arc(ax, -ay, 1.5 * np.pi))
    return np.concatenate(segs, axis=0)


def rounded_rect_sdf(p, Lx, Ly, rc):
    """Signed distance to a rounded rectangle centred at 0 (negative inside)."""
    q = np.abs(p) - np.array([Lx / 2 - rc, Ly / 2 - rc])
    out = np.hypot(np.maximum(q[:, 0], 0), np.maximum(q[:, 1], 0))
    ins = np.minimum(np.maximum(q[:, 0], q[:, 1]), 0)
    return out + ins - rc


def rounded_rect_mesh(Lx=2.0, Ly=1.0, rc=0.2, N=20_000, jitter=0.1, seed=SEED_BASE + 2):
    """Rounded-rectangle mesh: boundary polygon + jittered interior lattice, Delaunay."""
    rng = np.random.default_rng(seed)
    area = Lx * Ly - (4.0 - np.pi) * rc * rc
    h = np.sqrt(area / N)
    bnd = rounded_rect_boundary(Lx, Ly, rc, h)
    xs = np.arange(-Lx / 2 + h / 2, Lx / 2, h)
    ys = np.arange(-Ly / 2 + h / 2, Ly / 2, h)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    lat = np.stack([X.ravel(), Y.ravel()], axis=1)
    lat = lat + _jitter_disk(rng, len(lat), jitter * h)
    lat = lat[rounded_rect_sdf(lat, Lx, Ly, rc) < -0.5 * h]
    nodes = np.concatenate([bnd, lat], axis=0)
    tris = Delaunay(nodes).simplices.astype(np.int32)
    tris = _clean_tris(nodes, tris)
    nb = len(bnd)
    ring = np.arange(nb)
    bedges = np.stack([ring, np.roll(ring, -1)], axis=1).astype(np.int32)
    return nodes, tris, bedges


# --------------------------------------------------------------------------
# magnetization fields (unit norm unless stated)
# --------------------------------------------------------------------------

def M_uniform(nodes, Mx=1.0, My=0.0):
    M = np.empty_like(nodes)
    M[:, 0] = Mx
    M[:, 1] = My
    return M


def M_magic_cylinder(nodes):
    """Angle of M with the x axis equal to twice the polar angle."""
    th = np.arctan2(nodes[:, 1], nodes[:, 0])
    return np.stack([np.cos(2 * th), np.sin(2 * th)], axis=1)


def _modes(rng, count, kmax, exclude_zero=True):
    ks = []
    while len(ks) < count:
        k = rng.integers(-kmax, kmax + 1, size=2)
        if exclude_zero and k[0] == 0 and k[1] == 0:
            continue
        ks.append(k)
    return np.array(ks, dtype=np.float64)


def M_vortex_modes(nodes, a, b, seed, n_modes=8, amp=0.3, centre=None):
    """Vortex angle plus seeded Fourier modes in the ellipse's scaled coordinates."""
    rng = np.random.default_rng(seed)
    if centre is None:
        centre = rng.uniform(-0.25, 0.25, size=2) * np.array([a, b]) / 30.0
    kap = _modes(rng, n_modes, 3)
    ph = rng.uniform(0, 2 * np.pi, size=n_modes)
    xs = np.stack([nodes[:, 0] / a, nodes[:, 1] / b], axis=1)
    th = np.arctan2(nodes[:, 1] - centre[1], nodes[:, 0] - centre[0]) + 0.5 * np.pi
    th = th + amp * np.cos(np.pi * xs @ kap.T + ph).sum(axis=1)
    return np.stack([np.cos(th), np.sin(th)], axis=1)


def smooth_angle_params(seed, n_modes=8, amp=0.5, kmax=3, L=2.0):
    rng = np.random.default_rng(seed)
    u0 = rng.random()
    kap = _modes(rng, n_modes, kmax)
    ph = rng.uniform(0, 2 * np.pi, size=n_modes)
    return dict(u0=u0, kap=kap, ph=ph, amp=np.full(n_modes, amp), L=L)


def smooth_angle(x, prm):
    """theta(x) = 2 pi u0 + sum_k amp_k cos(2 pi kappa_k . x / L + phi_k) and its gradient."""
    arg = 2 * np.pi * (x @ prm["kap"].T) / prm["L"] + prm["ph"]
    th = 2 * np.pi * prm["u0"] + (prm["amp"] * np.cos(arg)).sum(axis=1)
    dth = -(prm["amp"] * np.sin(arg)) @ (2 * np.pi * prm["kap"] / prm["L"])
    return th, dth


def M_smooth(nodes, seed, n_modes=8, amp=0.5, L=2.0):
    prm = smooth_angle_params(seed, n_modes=n_modes, amp=amp, L=L)
    th, _ = smooth_angle(nodes, prm)
    return np.stack([np.cos(th), np.sin(th)], axis=1)


# --------------------------------------------------------------------------
# point clouds for the fast summation alone
# --------------------------------------------------------------------------

def random_cloud(n_tgt, n_src, seed, shape="disk", R=1.0, neutral=True):
    """Uniform random targets and sources in a disk or square, positive weights,
    charges of both signs (zero weighted sum if neutral)."""
    rng = np.random.default_rng(seed)

    def pts(n):
        if shape == "disk":
            return _jitter_disk(rng, n, R)
        return rng.uniform(-R, R, size=(n, 2))

    y = pts(n_tgt)
    x = pts(n_src)
    w = rng.uniform(0.5, 1.5, size=n_src) / max(n_src, 1)
    q = rng.standard_normal(n_src)
    if neutral and n_src > 1:
        q -= np.dot(w, q) / w.sum()
    return y, x, w, q


def random_cloud3(n_tgt, n_src, seed, shape="ball", R=1.0, neutral=True):
    """3D: uniform random targets and sources in a ball or cube, positive weights,
    charges of both signs (zero weighted sum if neutral)."""
    rng = np.random.default_rng(seed)

    def pts(n):
        if shape == "ball":
            v = rng.standard_normal((n, 3))
            v /= np.linalg.norm(v, axis=1)[:, None]
            return v * (R * rng.random(n) ** (1.0 / 3.0))[:, None]
        return rng.uniform(-R, R, size=(n, 3))

    y = pts(n_tgt)
    x = pts(n_src)
    w = rng.uniform(0.5, 1.5, size=n_src) / max(n_src, 1)
    q = rng.standard_normal(n_src)
    if neutral and n_src > 1:
        q -= np.dot(w, q) / w.sum()
    return y, x, w, q


# --------------------------------------------------------------------------
# tetrahedral meshes (3D)
# --------------------------------------------------------------------------
#   nodes  float64 [N, 3]
#   tets   int32   [T, 4]   vertex indices, any orientation
#   bfaces int32   [F, 3]   boundary triangles (a, b, c) with (b - a) x (c - a) pointing
#                           out of the domain
#   M      float64 [N, 3]   nodal magnetization

# the six tetrahedra of a unit cube cell around its main diagonal v000 -> v111 (corner
# k = x + 2 y + 4 z); every cell uses the same diagonal, so neighbouring cells share faces
_KUHN = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7], [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7]])


def boundary_faces(nodes, tets):
    """Faces that belong to one tetrahedron only, oriented outward (away from the fourth vertex)."""
    tets = np.asarray(tets, np.int64)
    loc = np.array([[1, 2, 3, 0], [0, 2, 3, 1], [0, 1, 3, 2], [0, 1, 2, 3]])  # face (3), opposite (1)
    faces = np.concatenate([tets[:, l[:3]] for l in loc])
    opp = np.concatenate([tets[:, l[3]] for l in loc])
    key = np.sort(faces, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    once = cnt[inv.ravel()] == 1
    f, d = faces[once], opp[once]
    a, b, c = nodes[f[:, 0]], nodes[f[:, 1]], nodes[f[:, 2]]
    flip = (np.cross(b - a, c - a) * (nodes[d] - a)).sum(1) > 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return f.astype(np.int32)


def cube_tet_mesh(n=8, L=1.0, jitter=0.0, seed=SEED_BASE + 6):
    """Cube [-L/2, L/2]^3 cut into n^3 cells of six tetrahedra each; interior nodes jittered by
    up to jitter*h per axis.  Returns nodes, tets, bfaces."""
    rng = np.random.default_rng(seed)
    h = L / n
    g = np.arange(n + 1) * h - L / 2
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    idx = lambda i, j, k: (i * (n + 1) + j) * (n + 1) + k
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    corner = np.stack([idx(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)) for c in range(8)], axis=1)
    tets = corner[:, _KUHN].reshape(-1, 4).astype(np.int32)
    if jitter:
        inner = np.all(np.abs(nodes) < L / 2 - 0.5 * h, axis=1)
        nodes[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    return nodes, tets, boundary_faces(nodes, tets)


def ball_tet_mesh(n=8, R=1.0):
    """Ball of radius R: the cube mesh of [-1, 1]^3 pushed radially onto the ball
    (p -> R p |p|_inf / |p|_2).  The boundary is the polyhedron of the mapped cube surface,
    its vertices on the sphere.  The map keeps every tetrahedron's orientation but flattens
    the cells along the cube's diagonals (smallest volume ~1e-3 of the mean at n = 16), so
    the nodes are not jittered: a jitter of 0.1 h already inverts some of them."""
    nodes, tets, _ = cube_tet_mesh(n=n, L=2.0)
    r2 = np.linalg.norm(nodes, axis=1)
    rinf = np.abs(nodes).max(axis=1)
    sc = np.where(r2 > 0, rinf / np.where(r2 > 0, r2, 1.0), 0.0)
    nodes = R * nodes * sc[:, None]
    return nodes, tets, boundary_faces(nodes, tets)


def _smooth3(rng, pts, n_modes, kmax, L):
    """A smooth random scalar field on 3D points: a sum of cosine modes of wavelength >= L/kmax."""
    ks = rng.integers(-kmax, kmax + 1, size=(n_modes, 3)).astype(np.float64)
    ph = rng.uniform(0.0, 2 * np.pi, n_modes)
    amp = rng.standard_normal(n_modes) / np.sqrt(n_modes)
    out = np.zeros(len(pts))
    for k, f, a in zip(ks, ph, amp):
        out += a * np.cos(2 * np.pi * (pts @ k) / L + f)
    return out


def ball_lattice3(K=64, R=1.0, spc=4, jitter=0.1, n_modes=16, kmax=3, seed=SEED_BASE + 5):
    """3D workload: a ball of radius R on a lattice of spacing h = 2R/K.  Targets: the lattice
    nodes inside the ball, interior ones jittered by up to jitter*h per axis (mesh-node-like);
    sources: spc uniform random points in every lattice cell whose centre lies inside the ball
    (quadrature-point-like), weight h^3/spc; charges a smooth random field with zero weighted
    sum; V a smooth random 3-vector field times h^3 (an adjoint input like l_i M_i)."""
    rng = np.random.default_rng(seed)
    h = 2.0 * R / K
    g = np.arange(K + 1) * h - R
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    r = np.linalg.norm(nodes, axis=1)
    nodes = nodes[r <= R]
    inner = np.linalg.norm(nodes, axis=1) <= R - 1.75 * h
    nodes[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    c = np.arange(K) * h - R + 0.5 * h
    CX, CY, CZ = np.meshgrid(c, c, c, indexing="ij")
    cent = np.stack([CX.ravel(), CY.ravel(), CZ.ravel()], axis=1)
    cent = cent[np.linalg.norm(cent, axis=1) <= R]
    x = (np.repeat(cent, spc, axis=0) + rng.uniform(-0.5 * h, 0.5 * h, size=(len(cent) * spc, 3)))
    w = np.full(len(x), h ** 3 / spc)
    q = _smooth3(rng, x, n_modes, kmax, 2 * R)
    q -= np.dot(w, q) / w.sum()
    V = np.stack([_smooth3(rng, nodes, n_modes, kmax, 2 * R) for _ in range(3)], axis=1) * h ** 3
    return dict(y=nodes, x=x, w=w, q=q, V=V, h=h)


def rounded_square_cloud(N=1 << 24, side=4.0, rc=0.5, n_modes=32, kmax=4,
                         jitter=0.1, seed=SEED_BASE + 4, with_boundary=True):
    """Jittered-lattice targets and sources in a rounded square with smooth M.

    Targets: lattice nodes of spacing h (about N of them inside the shape),
    each jittered uniformly in a disk of radius jitter*h.
    Sources: one point per lattice cell (the cell centre, jittered likewise) with
    weight h^2 and charge -div M evaluated analytically there; plus two points
    per boundary segment (spacing about h) at the 2-point Gauss-Legendre
    abscissae with weight |e|/2 and charge M.n.  The theta(x) field is a sum of
    n_modes cosines with N(0,1)/sqrt(n_modes) amplitudes and |kappa| <= kmax.

    Returns dict(y, x, w, q, M_tgt, h, prm).
    """
    rng = np.random.default_rng(seed)
    area = side * side - (4.0 - np.pi) * rc * rc
    h = np.sqrt(area / N)
    prm = dict(u0=0.0, kap=_modes(rng, n_modes, kmax),
               ph=rng.uniform(0, 2 * np.pi, size=n_modes),
               amp=rng.standard_normal(n_modes) / np.sqrt(n_modes), L=side)
    nx = int(np.ceil(side / h)) + 1
    g = -side / 2 + h * np.arange(nx)
    out = {}
    for name, shift in (("y", 0.0), ("x", 0.5)):
        gx = g + shift * h
        X, Y = np.meshgrid(gx, gx, indexing="ij")
        p = np.stack([X.ravel(), Y.ravel()], axis=1)
        del X, Y
        p += _jitter_disk(rng, len(p), jitter * h)
        p = p[rounded_rect_sdf(p, side, side, rc) < 0.0]
        out[name] = np.ascontiguousarray(p)
    y, xv = out["y"], out["x"]
    th, dth = smooth_angle(xv, prm)
    # rho = -div M with M = (cos th, sin th): div M = -sin th dth/dx + cos th dth/dy
    qv = np.sin(th) * dth[:, 0] - np.cos(th) * dth[:, 1]
    wv = np.full(len(xv), h * h)
    thy, _ = smooth_angle(y, prm)
    M_tgt = np.stack([np.cos(thy), np.sin(thy)], axis=1)
    if with_boundary:
        bp = rounded_rect_boundary(side, side, rc, h)
        a, b = bp, np.roll(bp, -1, axis=0)
        d = b - a
        L = np.hypot(d[:, 0], d[:, 1])
        nrm = np.stack([d[:, 1], -d[:, 0]], axis=1) / L[:, None]
        xs, ws, qs = [], [], []
        for t in (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)):
            pt = a + t * d
            tb, _ = smooth_angle(pt, prm)
            xs.append(pt)
            ws.append(0.5 * L)
            qs.append(np.cos(tb) * nrm[:, 0] + np.sin(tb) * nrm[:, 1])
        xv = np.concatenate([xv] + xs, axis=0)
        wv = np.concatenate([wv] + ws)
        qv = np.concatenate([qv] + qs)
    return dict(y=y, x=np.ascontiguousarray(xv), w=wv, q=qv, M_tgt=M_tgt, h=h, prm=prm)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def workload_disk_c1(seed=SEED_BASE):
    """~2,000-node disk, 30 rings, 128 boundary edges, uniform M=(1,0)."""
    nodes, tris, bedges = disk_mesh(R=1.0, K=30, ring_nodes=lambda k: int(round(128 * k / 30)),
                                    jitter=0.1, seed=seed)
    return dict(nodes=nodes, tris=tris, bedges=bedges, M=M_uniform(nodes))


def workload_ellipse_c2(N=50_000, seed=SEED_BASE + 1):
    nodes, tris, bedges = ellipse_mesh(2.0, 1.0, N=N, seed=seed)
    M = M_vortex_modes(nodes, 2.0, 1.0, seed=seed + 100)
    return dict(nodes=nodes, tris=tris, bedges=bedges, M=M)


def workload_annulus_c4(N=1_000_000, seed=SEED_BASE + 3, magic=False):
    nodes, tris, bedges = annulus_mesh(0.5, 1.0, N=N, seed=seed)
    M = M_magic_cylinder(nodes) if magic else M_smooth(nodes, seed=seed + 100, L=2.0)
    return dict(nodes=nodes, tris=tris, bedges=bedges, M=M)


def batch_meshes(count=64, nmin=5_000, nmax=200_000, seed=8072390):
    """Meshes of uneven size for batching: disk, ellipse, annulus, rounded rectangle in turn."""
    ss = np.random.SeedSequence(seed).spawn(count)
    out = []
    for k, s in enumerate(ss):
        rng = np.random.default_rng(s)
        N = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        sd = int(rng.integers(1 << 30))
        kind = k % 4
        if kind == 0:
            nodes, tris, bedges = disk_mesh_n(N, seed=sd)
        elif kind == 1:
            asp = rng.uniform(1, 4)
            nodes, tris, bedges = ellipse_mesh(asp, 1.0, N=N, seed=sd)
        elif kind == 2:
            nodes, tris, bedges = annulus_mesh(rng.uniform(0.3, 0.7), 1.0, N=N, seed=sd)
        else:
            asp = rng.uniform(1, 4)
            Ly = 1.0
            rc = rng.uniform(0.1, 0.3) * min(asp, Ly)
            nodes, tris, bedges = rounded_rect_mesh(asp, Ly, rc, N=N, seed=sd)
        M = M_smooth(nodes, seed=sd + 1, L=2.0 * float(np.max(np.abs(nodes))))
        out.append(dict(nodes=nodes, tris=tris, bedges=bedges, M=M))
    return out
