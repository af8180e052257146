"""The 3D FEM front on the GPU (fn3_mesh_*, fn3_bind_mesh, fn3_energy) through the C-ABI.

  * sources, charges C M, C^T u and the lumped mass against oracle/fem3.py, element by
    element (bound 1e-12) on a jittered cube mesh and a ball mesh;
  * the demagnetizing energy and its gradient against the step-by-step 3D oracle
    (oracle.fastsum3 on the oracle's sources, FP64 bound 1e-10), and an exact central
    difference of the quadratic energy along a random direction;
  * a uniformly magnetized ball: the fast energy equals the direct-sum energy (O1) within
    the fast summation's error, and lies where the lumped energy's first-order approach to
    V M^2 / 6 puts it at that mesh;
  * bad meshes (index out of range, a flat tetrahedron) and calls out of order.
"""
import numpy as np
import pytest

import synth
from oracle import direct, fem3
from oracle import fastsum3 as f3
from tests.conftest import parity_err, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a HIP device"
    return _t


@pytest.fixture(scope="module")
def fn():
    import paper_0807_2387_amd as _fn
    return _fn


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


MESHES = {"cube": lambda: synth.cube_tet_mesh(n=6, jitter=0.12), "ball": lambda: synth.ball_tet_mesh(n=8)}


@pytest.mark.parametrize("name", list(MESHES))
def test_fem3_operators_match_oracle(torch, fn, name):
    nodes, tets, bf = MESHES[name]()
    rng = np.random.default_rng(7)
    M = rng.standard_normal((len(nodes), 3))
    mesh = fn.Mesh3(dev(torch, nodes), dev(torch, tets, torch.int32), dev(torch, bf, torch.int32))
    x, w = mesh.sources()
    q = mesh.charges(dev(torch, M))
    u = rng.standard_normal(mesh.n_sources)
    ct = mesh.charges_T(dev(torch, u))
    ell = mesh.lumped_mass()
    torch.cuda.synchronize()
    x0, w0 = fem3.sources(nodes, tets, bf)
    got = dict(x=x.cpu().numpy(), w=w.cpu().numpy(), q=q.cpu().numpy(), ct=ct.cpu().numpy(), ell=ell.cpu().numpy())
    ref = dict(x=x0, w=w0, q=fem3.charges(nodes, tets, bf, M), ct=fem3.charges_T(nodes, tets, bf, u),
               ell=fem3.lumped_mass(nodes, tets))
    errs = {k: parity_err(got[k], ref[k]) for k in got}
    print(name, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) < 1e-12, errs


def test_fem3_energy_and_gradient_match_oracle(torch, fn):
    nodes, tets, bf = synth.cube_tet_mesh(n=6, jitter=0.12)
    rng = np.random.default_rng(8)
    M = rng.standard_normal((len(nodes), 3))
    G, m, p, c = 64, 6, 6, 5
    prm = f3.Params3(G=G, m=m, p=p, eps_I=c / (G // 2), eps_B=1 / 8)
    x, w = fem3.sources(nodes, tets, bf)
    q = fem3.charges(nodes, tets, bf, M)
    ell = fem3.lumped_mass(nodes, tets)
    F = f3.FastSum3(nodes, x, w, prm)
    _, H = F.forward(q)
    E_ref = fem3.energy(M, H, ell)
    g_ref = -0.5 * (ell[:, None] * H + fem3.charges_T(nodes, tets, bf, F.adjoint_H(ell[:, None] * M)))
    mesh = fn.Mesh3(dev(torch, nodes), dev(torch, tets, torch.int32), dev(torch, bf, torch.int32))
    S = fn.Solver3(grid=G, m=m, p=p, eps_I=c / (G // 2), eps_B=1 / 8)
    mesh.bind(S)
    E, g = mesh.energy(S, dev(torch, M))
    torch.cuda.synchronize()
    e_E = abs(E.item() - E_ref) / abs(E_ref)
    e_g = parity_err(g.cpu().numpy(), g_ref)
    print(f"energy {E.item():.12e} vs {E_ref:.12e}: {e_E:.1e}; gradient {e_g:.1e}", flush=True)
    assert e_E < 1e-10 and e_g < 1e-10
    # exact central difference of the quadratic energy
    D = rng.standard_normal(M.shape)
    h = 1e-3
    Ep, _ = mesh.energy(S, dev(torch, M + h * D), grad=False)
    Em, _ = mesh.energy(S, dev(torch, M - h * D), grad=False)
    torch.cuda.synchronize()
    fd = (Ep.item() - Em.item()) / (2 * h)
    an = float((g.cpu().numpy() * D).sum())
    print(f"central difference {fd:.12e} vs gradient . D {an:.12e}", flush=True)
    assert abs(fd - an) < 1e-9 * abs(an)


def test_fem3_uniform_ball_energy(torch, fn):
    nodes, tets, bf = synth.ball_tet_mesh(n=12)
    M = np.zeros((len(nodes), 3))
    M[:, 2] = 1.0
    mesh = fn.Mesh3(dev(torch, nodes), dev(torch, tets, torch.int32), dev(torch, bf, torch.int32))
    S = fn.Solver3(grid=128, m=8, p=8, eps_I=8 / 64, eps_B=1 / 8)
    mesh.bind(S)
    E, _ = mesh.energy(S, dev(torch, M), grad=False)
    torch.cuda.synchronize()
    x, w = fem3.sources(nodes, tets, bf)
    q = fem3.charges(nodes, tets, bf, M)
    _, H1 = direct.forward3(nodes, x, w, q, want_phi=False)
    ell = fem3.lumped_mass(nodes, tets)
    E1 = fem3.energy(M, H1, ell)
    V = ell.sum()
    print(f"ball energy: fast {E.item():.8f}, direct {E1:.8f}, V/6 = {V / 6:.8f}", flush=True)
    assert abs(E.item() - E1) < 1e-6 * abs(E1)
    # the lumped nodal energy approaches V/6 at first order (boundary nodes see the surface
    # charge's average field; tests/test_oracle_fem3.py): 12% low at n = 12
    assert -0.15 < E1 / (V / 6) - 1 < -0.08


def test_fem3_bad_meshes_and_order(torch, fn):
    nodes, tets, bf = synth.cube_tet_mesh(n=2)
    bad = tets.copy()
    bad[3, 2] = len(nodes)
    with pytest.raises(fn.FemNfftError, match="out of range"):
        fn.Mesh3(dev(torch, nodes), dev(torch, bad, torch.int32), dev(torch, bf, torch.int32))
    flat = nodes.copy()
    flat[tets[0]] = flat[tets[0][0]] + np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]]) * 1e-3
    with pytest.raises(fn.FemNfftError, match="degenerate"):
        fn.Mesh3(dev(torch, flat), dev(torch, tets, torch.int32), dev(torch, bf, torch.int32))
    mesh = fn.Mesh3(dev(torch, nodes), dev(torch, tets, torch.int32), dev(torch, bf, torch.int32))
    S = fn.Solver3(grid=32, m=4, p=4, eps_I=3 / 16)
    with pytest.raises(fn.FemNfftError, match="fn3_bind_mesh"):
        mesh.energy(S, dev(torch, np.ones((len(nodes), 3))))
    mesh.bind(S)
    y, x, w, q = synth.random_cloud3(10, 12, 3)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))  # the binding is stale now
    with pytest.raises(fn.FemNfftError, match="fn3_bind_mesh"):
        mesh.energy(S, dev(torch, np.ones((len(nodes), 3))))
