"""Parity of the HIP path with the oracle, through the C-ABI.

Tolerances (relative L2 per output kind, FP64 reference):
  * FP64 path vs O2 (same parameters, same algorithm): 1e-10 -- rounding only.
  * FP32-mixed path vs O2: 1e-6.
  * FP32-mixed path vs O1 (the exact discrete sum) on the paper-shaped workloads, at the
    parameters the bench uses (m = 6, p = 8, eps_I = 7/n): 1e-6.
"""
import ctypes

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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run_gpu(torch, fn, y, x, w, q, V, v, prm, precision):
    S = fn.Solver(grid=prm.G, m=prm.m, p=prm.p, eps_I=prm.eps_I, eps_B=prm.eps_B, precision=precision,
                  n=prm.band)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
    S.set_charges(dev(torch, q))
    phi, H = S.eval()
    u = S.adjoint_H(dev(torch, V))
    up = S.adjoint_phi(dev(torch, v))
    torch.cuda.synchronize()
    return phi.cpu().numpy(), H.cpu().numpy(), u.cpu().numpy(), up.cpu().numpy(), S


CASES = [
    # name, nt, ns, G, m, p, c, seed
    ("tiny", 7, 9, 64, 4, 2, 2.0, 1),
    ("ragged", 1000, 1531, 128, 6, 4, 4.0, 2),
    ("m8", 3000, 2000, 256, 8, 6, 6.0, 4),
    ("multi_tile", 20000, 30011, 512, 6, 8, 7.0, 3),
    # bandwidth 3G/4 (oversampling 4/3): a length-3*2^k plan transform; eps_I = c/n
    ("band_3G4", 20000, 30011, 512, 6, 8, 7.0, 5, 384),
    ("band_3G4_small", 1000, 1531, 128, 6, 4, 4.0, 6, 96),
    # the bench's regularization: p = 5, a narrower boundary zone eps_B = 1/32
    ("p5_epsB32", 20000, 30011, 512, 6, 5, 4.0, 7, 384, 1 / 32),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_parity_with_step_by_step_oracle(torch, fn, case, precision):
    name, nt, ns, G, m, p, c, seed = case[:8]
    band = case[8] if len(case) > 8 else 0
    eps_B = case[9] if len(case) > 9 else 1 / 16
    print(f"case {name} {precision}", flush=True)
    y, x, w, q = synth.random_cloud(nt, ns, seed)
    rng = np.random.default_rng(seed + 100)
    V = rng.standard_normal((nt, 2))
    v = rng.standard_normal(nt)
    prm = fs.Params(G=G, m=m, p=p, eps_I=c / (band or G // 2), band=band, eps_B=eps_B)
    F = fs.FastSum(y, x, w, prm)
    phi2, H2 = F.forward(q)
    u2, up2 = F.adjoint_H(V), F.adjoint_phi(v)
    P = fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED
    phi, H, u, up, _ = run_gpu(torch, fn, y, x, w, q, V, v, prm, P)
    tol = 1e-10 if precision == "fp64" else 1e-6
    errs = dict(phi=parity_err(phi, phi2), H=parity_err(H, H2), HT=parity_err(u, u2), phiT=parity_err(up, up2))
    print(errs, flush=True)
    assert max(errs.values()) < tol, errs


def fem_workload(d):
    x, w = fem.sources(d["nodes"], d["tris"], d["bedges"])
    q = fem.charges(d["nodes"], d["tris"], d["bedges"], d["M"])
    return d["nodes"], x, w, q


def test_disk_c1_fp64(torch, fn):
    """~2,000-node disk, M = (1,0), surface charges only; FP64, grid 64, m = 4, eps_I = 4/64, p = 2
    (the paper's smoothness degree)."""
    y, x, w, q = fem_workload(synth.workload_disk_c1())
    assert len(y) == 1985
    prm = fs.Params(G=64, m=4, p=2, eps_I=4 / 64)
    rng = np.random.default_rng(1)
    V = rng.standard_normal((len(y), 2))
    v = rng.standard_normal(len(y))
    F = fs.FastSum(y, x, w, prm)
    phi2, H2 = F.forward(q)
    phi, H, u, up, _ = run_gpu(torch, fn, y, x, w, q, V, v, prm, fn.FN_FP64)
    assert parity_err(phi, phi2) < 1e-10 and parity_err(H, H2) < 1e-10
    assert parity_err(u, F.adjoint_H(V)) < 1e-10 and parity_err(up, F.adjoint_phi(v)) < 1e-10
    phi1, H1 = direct.forward(y, x, w, q)
    # at these pinned parameters the fast method's error stays below the discretization error
    # (closed form phi = x/2); the ratio is printed for the record
    ex = 0.5 * y[:, 0]
    assert rel_l2(phi, phi1) < 1e-3
    approx = np.sqrt(np.mean((phi - phi1) ** 2))
    discr = np.sqrt(np.mean((phi1 - ex) ** 2))
    print(f"C1: approximation RMS {approx:.3e}, discretization RMS {discr:.3e}, ratio {approx / discr:.2f}")
    assert approx < 0.5 * discr


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ellipse_c2(torch, fn, precision):
    """Ellipse a=2, b=1, 50k nodes, vortex + 8 modes, volume + surface charges, grid 512."""
    y, x, w, q = fem_workload(synth.workload_ellipse_c2())
    prm = fs.Params(G=512, m=6, p=8, eps_I=7 / 256)
    ell = fem.lumped_mass(synth.workload_ellipse_c2()["nodes"], synth.workload_ellipse_c2()["tris"])
    V = ell[:, None] * synth.workload_ellipse_c2()["M"]
    v = ell.copy()
    P = fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED
    phi, H, u, up, _ = run_gpu(torch, fn, y, x, w, q, V, v, prm, P)
    rng = np.random.default_rng(2)
    it = rng.choice(len(y), 2000, replace=False)
    js = rng.choice(len(x), 2000, replace=False)
    phi1, H1 = direct.forward(y[it], x, w, q)
    u1 = direct.adjoint(y, x[js], w[js], V=V)
    e1 = dict(phi=rel_l2(phi[it], phi1), H=rel_l2(H[it], H1), HT=rel_l2(u[js], u1))
    print("vs O1", e1, flush=True)
    assert max(e1.values()) < 1e-6, e1
    if precision == "fp64":
        F = fs.FastSum(y, x, w, prm)
        phi2, H2 = F.forward(q)
        e2 = dict(phi=parity_err(phi, phi2), H=parity_err(H, H2), HT=parity_err(u, F.adjoint_H(V)))
        print("vs O2", e2, flush=True)
        assert max(e2.values()) < 1e-10, e2


@pytest.mark.slow
def test_rounded_square_full_size_sampled(torch, fn):
    """The bench workload at full size (about 2^24 targets and sources, grid 8192, m = 6):
    FP32-mixed vs the FP64 direct sum on sampled targets and sources."""
    d = synth.rounded_square_cloud(N=1 << 24, seed=synth.SEED_BASE + 4)
    y, x, w, q = d["y"], d["x"], d["w"], d["q"]
    V = (d["h"] ** 2) * d["M_tgt"]
    S = fn.Solver(grid=8192, m=6, p=8, eps_I=7 / 4096, precision=fn.FN_FP32_MIXED)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
    S.set_charges(dev(torch, q))
    phi, H = S.eval()
    u = S.adjoint_H(dev(torch, V))
    rng = np.random.default_rng(3)
    it = np.sort(rng.choice(len(y), 200, replace=False))
    js = np.sort(rng.choice(len(x), 200, replace=False))
    phi = phi.cpu().numpy()[it]
    H = H.cpu().numpy()[it]
    u = u.cpu().numpy()[js]
    del S
    torch.cuda.empty_cache()
    phi1, H1 = direct.forward(y[it], x, w, q)
    u1 = direct.adjoint(y, x[js], w[js], V=V)
    e = dict(phi=rel_l2(phi, phi1), H=rel_l2(H, H1), HT=rel_l2(u, u1))
    print(e, flush=True)
    assert max(e.values()) < 1e-6, e


# ------------------------------------------------------------------------- edge cases

def test_targets_equal_sources(torch, fn):
    """Every target coincides with a source: those pairs are excluded from the sum."""
    _, x, w, q = synth.random_cloud(0, 2000, 9)
    y = x.copy()
    prm = fs.Params(G=256, m=6, p=6, eps_I=6 / 128)
    rng = np.random.default_rng(9)
    V = rng.standard_normal((len(y), 2))
    v = rng.standard_normal(len(y))
    F = fs.FastSum(y, x, w, prm)
    phi2, H2 = F.forward(q)
    phi, H, u, up, _ = run_gpu(torch, fn, y, x, w, q, V, v, prm, fn.FN_FP64)
    assert parity_err(phi, phi2) < 1e-10 and parity_err(H, H2) < 1e-10
    assert parity_err(u, F.adjoint_H(V)) < 1e-10 and parity_err(up, F.adjoint_phi(v)) < 1e-10
    phi1, H1 = direct.forward(y, x, w, q)
    assert rel_l2(phi, phi1) < 1e-5 and rel_l2(H, H1) < 1e-4


def test_dense_cluster_exercises_near_field_chunking(torch, fn):
    """Thousands of sources inside a few grid cells plus scattered points: a near-field block
    then stages far more points than one LDS chunk holds."""
    rng = np.random.default_rng(11)
    clus = 0.2 + 1e-4 * rng.standard_normal((6000, 2))
    y = np.concatenate([clus[:3000], rng.uniform(-1, 1, size=(2000, 2))])
    x = np.concatenate([clus[3000:], rng.uniform(-1, 1, size=(2000, 2))])
    w = rng.uniform(0.5, 1.5, len(x)) / len(x)
    q = rng.standard_normal(len(x))
    V = rng.standard_normal((len(y), 2))
    v = rng.standard_normal(len(y))
    prm = fs.Params(G=256, m=6, p=6, eps_I=6 / 128)
    F = fs.FastSum(y, x, w, prm)
    phi2, H2 = F.forward(q)
    for P, tol in ((fn.FN_FP64, 1e-10), (fn.FN_FP32_MIXED, 1e-6)):
        phi, H, u, up, _ = run_gpu(torch, fn, y, x, w, q, V, v, prm, P)
        e = dict(phi=parity_err(phi, phi2), H=parity_err(H, H2), HT=parity_err(u, F.adjoint_H(V)),
                 phiT=parity_err(up, F.adjoint_phi(v)))
        assert max(e.values()) < tol, (P, e)


def test_no_sources_and_no_targets(torch, fn):
    y, x, w, q = synth.random_cloud(50, 60, 12)
    S = fn.Solver(grid=64, m=4, p=2, eps_I=2 / 32, precision=fn.FN_FP64)
    S.set_geometry(dev(torch, y), dev(torch, x[:0]), dev(torch, w[:0]))
    S.set_charges(dev(torch, q[:0]))
    phi, H = S.eval()
    assert torch.all(phi == 0) and torch.all(H == 0)
    phi, H, u = S.eval_with_H_adjoint(dev(torch, np.ones((50, 2))))
    torch.cuda.synchronize()
    assert torch.all(phi == 0) and torch.all(H == 0) and u.shape[0] == 0
    S.set_geometry(dev(torch, y[:0]), dev(torch, x), dev(torch, w))
    S.set_charges(dev(torch, q))
    u = S.adjoint_H(dev(torch, np.zeros((0, 2))))
    assert torch.all(u == 0) and u.shape[0] == 60
    phi, H = S.eval()
    assert phi.shape[0] == 0 and H.shape[0] == 0
    phi, H, u = S.eval_with_H_adjoint(dev(torch, np.zeros((0, 2))))
    torch.cuda.synchronize()
    assert torch.all(u == 0) and u.shape[0] == 60 and phi.shape[0] == 0


def test_single_source_against_closed_form(torch, fn):
    x = np.array([[0.3, -0.2]])
    w = np.array([0.7])
    q = np.array([1.3])
    r = np.geomspace(1e-6, 2.0, 40)
    ang = np.linspace(0, 2 * np.pi, 40, endpoint=False)
    y = x + np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1)
    prm = fs.Params(G=512, m=8, p=10, eps_I=10 / 256)
    phi, H, _, _, _ = run_gpu(torch, fn, y, x, w, q, np.zeros_like(y), np.zeros(len(y)), prm, fn.FN_FP64)
    s = w[0] * q[0]
    d = y - x
    rr = np.hypot(d[:, 0], d[:, 1])
    assert np.abs(phi + s / (2 * np.pi) * np.log(rr)).max() < 1e-8
    Hex = s / (2 * np.pi) * d / rr[:, None] ** 2
    assert (np.linalg.norm(H - Hex, axis=1) / np.linalg.norm(Hex, axis=1)).max() < 1e-6


def test_adjoint_dot_product_identity(torch, fn):
    y, x, w, q = synth.random_cloud(3000, 4000, 13)
    rng = np.random.default_rng(13)
    V = rng.standard_normal((3000, 2))
    v = rng.standard_normal(3000)
    prm = fs.Params(G=256, m=6, p=6, eps_I=6 / 128)
    phi, H, u, up, _ = run_gpu(torch, fn, y, x, w, q, V, v, prm, fn.FN_FP64)
    assert abs(np.sum(H * V) - np.dot(q, u)) < 1e-12 * np.abs(H * V).sum()
    assert abs(np.dot(phi, v) - np.dot(q, up)) < 1e-12 * np.abs(phi * v).sum()
    phi, H, u, up, _ = run_gpu(torch, fn, y, x, w, q, V, v, prm, fn.FN_FP32_MIXED)
    assert abs(np.sum(H * V) - np.dot(q, u)) < 1e-6 * np.abs(H * V).sum()


def test_repeat_runs_are_bitwise_identical(torch, fn):
    y, x, w, q = synth.random_cloud(20000, 20000, 14)
    V = np.random.default_rng(14).standard_normal((20000, 2))
    for P in (fn.FN_FP32_MIXED, fn.FN_FP64):
        S = fn.Solver(grid=512, m=6, p=8, eps_I=7 / 256, precision=P)
        S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
        S.set_charges(dev(torch, q))
        a = S.eval()
        ua = S.adjoint_H(dev(torch, V))
        b = S.eval()
        ub = S.adjoint_H(dev(torch, V))
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(ua, ub)


def test_error_codes(torch, fn):
    from paper_0807_2387_amd import _lib
    L = _lib.lib()
    y, x, w, q = synth.random_cloud(10, 10, 15)
    S = fn.Solver(grid=64, m=4, p=2, eps_I=2 / 32, precision=fn.FN_FP64)
    # evaluation before geometry / charges
    with pytest.raises(fn.FemNfftError) as ei:
        S.eval()
    assert ei.value.code == _lib.FN_E_STATE
    # all points coincide
    same = np.zeros((10, 2))
    with pytest.raises(fn.FemNfftError) as ei:
        S.set_geometry(dev(torch, same), dev(torch, same), dev(torch, w))
    assert ei.value.code == _lib.FN_E_DOMAIN
    # non-finite coordinate
    bad = y.copy()
    bad[3, 1] = np.nan
    with pytest.raises(fn.FemNfftError) as ei:
        S.set_geometry(dev(torch, bad), dev(torch, x), dev(torch, w))
    assert ei.value.code == _lib.FN_E_INVAL
    # workspace too small
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    assert L.fn_set_workspace(S._ctx, ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(1024)) == 0
    ty, tx, tw = dev(torch, y), dev(torch, x), dev(torch, w)
    rc = L.fn_set_geometry(S._ctx, 10, ctypes.c_void_p(ty.data_ptr()), 10, ctypes.c_void_p(tx.data_ptr()),
                           ctypes.c_void_p(tw.data_ptr()))
    assert rc == _lib.FN_E_NOMEM
    # the context recovers with a proper workspace
    S._ws = None
    S.set_geometry(ty, tx, tw)
    S.set_charges(dev(torch, q))
    phi, _ = S.eval()
    assert torch.isfinite(phi).all()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", ["disk", "magic_cylinder"])
def test_paper_tables_claim_on_gpu(torch, fn, shape, precision):
    """The claim of the paper's Tables 1 and 2 (fast summation error within 3.5% of the
    direct FEM sum's error against the analytic potential), for the HIP path at the
    paper's p = 2 on the tables' smallest meshes."""
    from tests import test_golden_tables as gt
    N = 400 if shape == "disk" else 1192
    nodes, tris, bedges, M, exact = (gt.disk_case if shape == "disk" else gt.magic_case)(N)
    print(f"paper-table case {shape} N={N} {precision}", flush=True)
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, M)
    phi1, _ = direct.forward(nodes, x, w, q, want_H=False)
    G = gt.grid_rule(len(nodes))
    prm = fs.Params(G=G, m=4, p=2, eps_I=4 / (G // 2))
    P = fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED
    z = np.zeros((len(nodes), 2))
    phi, _, _, _, _ = run_gpu(torch, fn, nodes, x, w, q, z, z[:, 0], prm, P)
    rms = lambda a: float(np.sqrt(np.mean((a - exact) ** 2)))
    bound = max(gt.max_printed_gap(gt.load_table("paper_table1_disk.txt")),
                gt.max_printed_gap(gt.load_table("paper_table2_magic_cylinder.txt")))
    assert abs(rms(phi) - rms(phi1)) <= bound * rms(phi1)


def test_adjoint_input_at_an_8_byte_offset(torch, fn):
    """V [n][2] that is 8- but not 16-byte aligned takes the scalar-load path of the value
    kernel; the result equals that of an aligned copy."""
    print("adjoint input alignment", flush=True)
    y, x, w, q = synth.random_cloud(5000, 7000, 21)
    V = np.random.default_rng(22).standard_normal((len(y), 2))
    S = fn.Solver(grid=256, m=6, p=6, eps_I=6 / 128, precision=fn.FN_FP32_MIXED)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
    S.set_charges(dev(torch, q))
    Va = dev(torch, V)
    buf = torch.empty(2 * len(y) + 1, dtype=torch.float64, device="cuda")
    Vo = buf[1:].view(len(y), 2)
    Vo.copy_(Va)
    assert Vo.data_ptr() % 16 == 8 and Va.data_ptr() % 16 == 0
    ua = S.adjoint_H(Va)
    uo = S.adjoint_H(Vo)
    torch.cuda.synchronize()
    assert torch.equal(ua, uo)
