"""Outputs at the quadrature points on the GPU (fn_bind_mesh_sources, fn_energy_charge) and the
P1-gradient field (fn_mesh_p1_gradient), against the oracle's FEM module.

  * phi at the quadrature points, each point's own charge left out (the pair at distance 0
    is not part of the sum), all sources in one class at eps_I (the binding's choice, which
    keeps the fast potential matrix symmetric): FP64 path vs the step-by-step oracle (O2,
    targets = sources) 1e-10, FP32-mixed path 1e-6, relative L2 and per element; both
    against the direct sum (O1) 1e-6.
  * Charge-form energy E_q = 1/2 sum_j s_j phi_j and its gradient C^T (w phi): against the
    oracle's charge_energy / charge_energy_grad on the O2 potential (FP64 1e-10, FP32 1e-6)
    and on the O1 potential (1e-6); the central difference of the quadratic E_q (FP64 path)
    equals the gradient to 1e-9.
  * P1 gradient of a nodal potential, per triangle and lumped to the nodes: the oracle's
    formulas evaluated in another order, 1e-13.
"""
import numpy as np
import pytest

import synth
from oracle import fem
from oracle import fastsum as fs
from tests.conftest import parity_err, rel_l2

pytestmark = pytest.mark.gpu

P_DEG, C_VOL, C_SURF, EPS_B, M_WIN = 8, 7.0, 11.0, 1.0 / 32.0, 6  # eps_S is set but not used by this binding


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


_CASE = {}


def case():
    """Annulus mesh, its quadrature points and the oracle potentials at them (once)."""
    if _CASE:
        return _CASE
    nodes, tris, bedges = synth.annulus_mesh(R1=0.5, R2=1.0, N=12_000, seed=synth.SEED_BASE + 21)
    M = synth.M_smooth(nodes, seed=synth.SEED_BASE + 22)
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, M)
    ns1 = 3 * len(tris)
    G = 512
    band = 3 * G // 4
    pv = fs.Params(G=G, m=M_WIN, p=P_DEG, eps_I=C_VOL / band, band=band, eps_B=EPS_B)
    # one source class (the binding's): every source at eps_I
    phi2 = fs.FastSum(x, x, w, pv).forward(q)[0]
    phi1 = fem.phi_at_sources(x, w, q)
    _CASE.update(nodes=nodes, tris=tris, bedges=bedges, M=M, x=x, w=w, q=q, G=G, band=band, phi1=phi1, phi2=phi2)
    return _CASE


def solver(fn, c, precision):
    return fn.Solver(grid=c["G"], m=M_WIN, p=P_DEG, eps_I=C_VOL / c["band"], eps_S=C_SURF / c["band"],
                     eps_B=EPS_B, n=c["band"], precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_potential_and_charge_energy_at_the_quadrature_points(torch, fn, precision):
    c = case()
    print(f"charge form {precision}: {len(c['nodes'])} nodes, {len(c['x'])} quadrature points", flush=True)
    P = fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED
    S = solver(fn, c, P)
    mesh = fn.Mesh(dev(torch, c["nodes"]), dev(torch, c["tris"], torch.int32), dev(torch, c["bedges"], torch.int32))
    S.bind_mesh_sources(mesh)
    E, g, phi = S.energy_charge(dev(torch, c["M"]))
    phi, g, E = phi.cpu().numpy(), g.cpu().numpy(), float(E)
    tol = 1e-10 if precision == "fp64" else 1e-6
    e2, e1 = parity_err(phi, c["phi2"]), rel_l2(phi, c["phi1"])
    print(f"  phi vs O2 {e2:.2e}, vs O1 {e1:.2e}", flush=True)
    assert e2 < tol and e1 < 1e-6
    nodes, tris, bedges, w, q = c["nodes"], c["tris"], c["bedges"], c["w"], c["q"]
    for ref, t in ((c["phi2"], tol), (c["phi1"], 1e-6)):
        E0 = fem.charge_energy(w, q, ref)
        g0 = fem.charge_energy_grad(nodes, tris, bedges, w, ref)
        print(f"  E_q {E:.12e} vs {E0:.12e}; gradient {parity_err(g, g0):.2e}", flush=True)
        assert abs(E - E0) <= t * abs(E0)
        assert parity_err(g, g0) < t


def test_charge_energy_central_difference_is_the_gradient(torch, fn):
    c = case()
    S = solver(fn, c, fn.FN_FP64)
    mesh = fn.Mesh(dev(torch, c["nodes"]), dev(torch, c["tris"], torch.int32), dev(torch, c["bedges"], torch.int32))
    S.bind_mesh_sources(mesh)
    D = np.random.default_rng(23).standard_normal(c["M"].shape)
    _, g, _ = S.energy_charge(dev(torch, c["M"]))
    Ep, _, _ = S.energy_charge(dev(torch, c["M"] + D), grad=False)
    Em, _, _ = S.energy_charge(dev(torch, c["M"] - D), grad=False)
    fd = (float(Ep) - float(Em)) / 2.0
    an = float(np.sum(g.cpu().numpy() * D))
    print(f"charge-form central difference {fd:.12e}, gradient . D {an:.12e}", flush=True)
    assert abs(fd - an) <= 1e-9 * (abs(float(Ep)) + abs(float(Em)))


def test_p1_gradient_field(torch, fn):
    c = case()
    nodes, tris = c["nodes"], c["tris"]
    mesh = fn.Mesh(dev(torch, nodes), dev(torch, tris, torch.int32), dev(torch, c["bedges"], torch.int32))
    phi = np.random.default_rng(24).standard_normal(len(nodes)) + nodes @ np.array([0.3, -0.8])
    HT, Hn = mesh.p1_gradient(dev(torch, phi))
    assert parity_err(HT.cpu().numpy(), fem.p1_gradient(nodes, tris, phi)) < 1e-13
    assert parity_err(Hn.cpu().numpy(), fem.p1_gradient_nodal(nodes, tris, phi)) < 1e-13
