"""The P1 front on the GPU (fn_mesh_*, fn_energy) against the oracle's FEM module.

Tolerances: quadrature points, weights, charges, C^T and the lumped mass are the
same FP64 formulas evaluated in a different summation order -> 1e-13 relative.
Energy and gradient: FP64 path vs the oracle's step-by-step fast sum (O2) 1e-10,
FP32-mixed path 1e-6; vs the direct sum (O1) at the bench parameters 1e-6.  The
energy is a quadratic form in M, so a central difference of it is exact up to
rounding for any step: it must match the gradient to 1e-9 (FP64 path).
"""
import numpy as np
import pytest

import synth
from oracle import direct, fem
from oracle import fastsum as fs
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
    import torch as _t
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype or _t.float64).cuda()


def annulus(N=3000, seed=0):
    nodes, tris, bedges = synth.annulus_mesh(R1=0.5, R2=1.0, N=N, seed=synth.SEED_BASE + 3 + seed)
    M = synth.M_smooth(nodes, seed=synth.SEED_BASE + 10 + seed)
    return nodes, tris, bedges, M


def make_mesh(torch, fn, nodes, tris, bedges):
    return fn.Mesh(dev(torch, nodes), dev(torch, tris, torch.int32), dev(torch, bedges, torch.int32))


def test_mesh_operators_match_oracle(torch, fn):
    nodes, tris, bedges, M = annulus()
    print(f"fem operators: {len(nodes)} nodes, {len(tris)} triangles, {len(bedges)} edges", flush=True)
    mesh = make_mesh(torch, fn, nodes, tris, bedges)
    x, w = mesh.sources()
    x0, w0 = fem.sources(nodes, tris, bedges)
    assert mesh.n_sources == len(w0)
    np.testing.assert_allclose(x.cpu().numpy(), x0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w.cpu().numpy(), w0, rtol=1e-14, atol=0)
    ell = mesh.lumped_mass().cpu().numpy()
    np.testing.assert_allclose(ell, fem.lumped_mass(nodes, tris), rtol=1e-13, atol=0)
    q = mesh.charges(dev(torch, M)).cpu().numpy()
    q0 = fem.charges(nodes, tris, bedges, M)
    assert parity_err(q, q0) < 1e-13
    u = np.random.default_rng(5).standard_normal(len(w0))
    ct = mesh.charges_T(dev(torch, u)).cpu().numpy()
    assert parity_err(ct, fem.charges_T(nodes, tris, bedges, u)) < 1e-13
    # C^T is the transpose of C on the device too
    lhs = float(np.dot(q, u))
    rhs = float(np.sum(M * ct))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(q) * np.linalg.norm(u))


def oracle_energy(nodes, tris, bedges, M, prm):
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, M)
    ell = fem.lumped_mass(nodes, tris)
    F = fs.FastSum(nodes, x, w, prm)
    _, H = F.forward(q)
    E = fem.energy(M, H, ell)
    u = F.adjoint_H(ell[:, None] * M)
    g = fem.energy_grad(H, ell, fem.charges_T(nodes, tris, bedges, u))
    return E, g


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_energy_and_gradient_vs_step_by_step_oracle(torch, fn, precision):
    nodes, tris, bedges, M = annulus()
    print(f"energy vs O2 {precision}", flush=True)
    prm = fs.Params(G=256, m=6, p=6, eps_I=6 / 128)
    E0, g0 = oracle_energy(nodes, tris, bedges, M, prm)
    P = fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED
    S = fn.Solver(grid=prm.G, m=prm.m, p=prm.p, eps_I=prm.eps_I, eps_B=prm.eps_B, precision=P)
    mesh = make_mesh(torch, fn, nodes, tris, bedges)
    S.bind_mesh(mesh)
    E, g = S.energy(dev(torch, M))
    tol = 1e-10 if precision == "fp64" else 1e-6
    assert abs(float(E) - E0) <= tol * abs(E0)
    assert parity_err(g.cpu().numpy(), g0) < tol


def test_energy_vs_direct_sum_at_bench_parameters(torch, fn):
    nodes, tris, bedges, M = annulus(N=20000, seed=1)
    print(f"energy vs O1: {len(nodes)} nodes", flush=True)
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, M)
    ell = fem.lumped_mass(nodes, tris)
    _, H1 = direct.forward(nodes, x, w, q, want_phi=False)
    E1 = fem.energy(M, H1, ell)
    u1 = direct.adjoint(nodes, x, w, V=ell[:, None] * M)
    g1 = fem.energy_grad(H1, ell, fem.charges_T(nodes, tris, bedges, u1))
    G = 1 << int(np.ceil(np.log2(2 * np.sqrt(len(x)))))  # about 4 grid cells per source
    S = fn.Solver(grid=G, precision=fn.FN_FP32_MIXED)
    mesh = make_mesh(torch, fn, nodes, tris, bedges)
    S.bind_mesh(mesh)
    E, g = S.energy(dev(torch, M))
    assert abs(float(E) - E1) <= 1e-6 * abs(E1)
    assert rel_l2(g.cpu().numpy(), g1) < 1e-6


def test_energy_central_difference_is_the_gradient(torch, fn):
    nodes, tris, bedges, M = annulus(N=2000, seed=2)
    print("energy finite difference", flush=True)
    S = fn.Solver(grid=256, m=6, p=6, eps_I=6 / 128, precision=fn.FN_FP64)
    mesh = make_mesh(torch, fn, nodes, tris, bedges)
    S.bind_mesh(mesh)
    D = np.random.default_rng(7).standard_normal(M.shape)
    _, g = S.energy(dev(torch, M))
    Ep, _ = S.energy(dev(torch, M + D), grad=False)
    Em, _ = S.energy(dev(torch, M - D), grad=False)
    fd = (float(Ep) - float(Em)) / 2.0
    an = float(np.sum(g.cpu().numpy() * D))
    assert abs(fd - an) <= 1e-9 * (abs(float(Ep)) + abs(float(Em)))


def test_autograd_function(torch, fn):
    nodes, tris, bedges, M = annulus(N=2000, seed=3)
    S = fn.Solver(grid=256, m=6, p=6, eps_I=6 / 128, precision=fn.FN_FP64)
    mesh = make_mesh(torch, fn, nodes, tris, bedges)
    S.bind_mesh(mesh)
    Mt = dev(torch, M).requires_grad_(True)
    E = fn.DemagEnergy.apply(Mt, S, mesh)
    (gM,) = torch.autograd.grad(3.0 * E, Mt)
    E2, g2 = S.energy(dev(torch, M))
    assert float(E.detach()) == float(E2)
    assert torch.equal(gM, 3.0 * g2)


def test_energy_is_deterministic(torch, fn):
    nodes, tris, bedges, M = annulus(N=3000, seed=4)
    S = fn.Solver(grid=256, m=6, p=6, eps_I=6 / 128, precision=fn.FN_FP32_MIXED)
    mesh = make_mesh(torch, fn, nodes, tris, bedges)
    S.bind_mesh(mesh)
    Md = dev(torch, M)
    E1, g1 = S.energy(Md)
    E2, g2 = S.energy(Md)
    assert float(E1) == float(E2) and torch.equal(g1, g2)


def test_mesh_errors(torch, fn):
    nodes, tris, bedges, M = annulus(N=500, seed=5)
    bad = tris.copy()
    bad[3, 1] = len(nodes)
    with pytest.raises(fn.FemNfftError) as ei:
        make_mesh(torch, fn, nodes, bad, bedges)
    assert ei.value.code == 1
    deg = tris.copy()
    deg[0, 2] = deg[0, 1]
    with pytest.raises(fn.FemNfftError) as ei:
        make_mesh(torch, fn, nodes, deg, bedges)
    assert ei.value.code == 3
    S = fn.Solver(grid=256, precision=fn.FN_FP64)
    mesh = make_mesh(torch, fn, nodes, tris, bedges)
    S.set_geometry(dev(torch, nodes), dev(torch, nodes), dev(torch, np.ones(len(nodes))))
    S._mesh = mesh  # bypass the Python-side binding: the library must refuse
    with pytest.raises(fn.FemNfftError) as ei:
        S.energy(dev(torch, M))
    assert ei.value.code == 2


def test_energy_under_capture_with_and_without_the_overlapped_stream(torch, fn):
    """fn_energy with the gradient runs H and the H adjoint at once once the context has
    its second stream; captured before that, it runs them one after the other.  Both
    give the eager result."""
    import ctypes
    print("energy capture, fresh context then overlapped", flush=True)
    nodes, tris, bedges, M = annulus(N=3000, seed=6)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        S = fn.Solver(grid=256, m=6, p=6, eps_I=6 / 128, precision=fn.FN_FP32_MIXED)
        mesh = make_mesh(torch, fn, nodes, tris, bedges)
        S.bind_mesh(mesh)
        Md = dev(torch, M)
        E = torch.empty((), dtype=torch.float64, device="cuda")
        g = torch.empty(len(nodes), 2, dtype=torch.float64, device="cuda")
        L = fn._lib.lib()
        args = (S._ctx, mesh._mesh, ctypes.c_void_p(Md.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                ctypes.c_void_p(g.data_ptr()))
        G1 = fn.Graph()
        with G1.capture(st):
            assert L.fn_energy(*args) == 0  # no second stream yet: one after the other
        G1.launch(st)
        st.synchronize()
        E1, g1 = E.clone(), g.clone()
        E2, g2 = S.energy(Md)  # eager: creates the stream, overlapped
        st.synchronize()
        rel = lambda a, b: parity_err(a.cpu().numpy(), b.cpu().numpy())
        assert abs(float(E1) - float(E2)) <= 1e-12 * abs(float(E2)) and rel(g1, g2) < 1e-12
        G2 = fn.Graph()
        with G2.capture(st):
            assert L.fn_energy(*args) == 0  # overlapped, captured across both streams
        for rep in range(3):
            E.zero_()
            g.zero_()
            G2.launch(st)
            st.synchronize()
            assert abs(float(E) - float(E2)) <= 1e-12 * abs(float(E2)) and rel(g, g2) < 1e-12, rep
