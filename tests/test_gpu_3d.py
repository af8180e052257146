"""The 3D fast summation (fn3_*, G = 1/(4 pi r)) through the C-ABI against the 3D oracles.

  * parity with the step-by-step oracle O2 (oracle.fastsum3) element by element: phi, H and
    the H adjoint, FP64, bound 1e-10 (relative L2 and per element, tests.conftest.parity_err),
    on ball and cube clouds at G = 32, 64, 128 (several cells per near radius, ragged point
    counts, targets coinciding with sources, window half-widths 4 to 7), at bandwidths G/2
    and 3G/4;
  * a dense cluster (more near-field candidates per home block than the kernel's row table);
  * accuracy against the direct sum O1 at the tested parameters (the oracle's own bounds);
  * empty source or target sets, degenerate geometry and the parameter checks.
"""
import numpy as np
import pytest

import synth
from oracle import direct
from oracle import fastsum3 as f3
from tests.conftest import max_rel, parity_err, rel_l2

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


# name, n_tgt, n_src, shape, G, m, p, n eps_I, seed, coincident targets, bandwidth (0: G/2)
CASES = [
    ("G32-ball", 701, 903, "ball", 32, 5, 5, 4, 31, 0, 0),
    ("G64-cube", 2999, 4001, "cube", 64, 6, 6, 5, 32, 50, 0),
    ("G128-ball", 9001, 12003, "ball", 128, 7, 8, 8, 33, 100, 0),
    ("G64-ball-m4", 2501, 3307, "ball", 64, 4, 6, 5, 34, 30, 0),  # 2m <= 8: 8-lane gather groups
    ("G64-ball-n48", 2999, 4001, "ball", 64, 5, 6, 5.5, 37, 20, 48),   # oversampling 4/3
    ("G128-cube-n96", 9001, 12003, "cube", 128, 6, 6, 5.5, 38, 60, 96),
    ("G32-ball-n20", 701, 903, "ball", 32, 4, 5, 3, 39, 5, 20),      # n/2 = 10, not a power of two
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_3d_matches_step_by_step_oracle(torch, fn, case):
    name, nt, ns, shape, G, m, p, c, seed, nco, band = case
    n = band or G // 2
    print(f"3D case {name}: oracle", flush=True)
    y, x, w, q = synth.random_cloud3(nt, ns, seed, shape=shape)
    y[:nco] = x[:nco]
    prm = f3.Params3(G=G, m=m, p=p, eps_I=c / n, eps_B=1 / 8, band=band)
    F = f3.FastSum3(y, x, w, prm)
    rng = np.random.default_rng(seed + 1)
    V = rng.standard_normal((nt, 3))
    ref = dict(phi=None, H=None)
    ref["phi"], ref["H"] = F.forward(q)
    ref["HT"] = F.adjoint_H(V)
    del F
    print("  GPU", flush=True)
    S = fn.Solver3(grid=G, m=m, p=p, eps_I=c / n, eps_B=1 / 8, n=band)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
    info = S.info()
    assert info["near_cells"] == int(np.ceil(c / n * G)) and abs(info["scale"] - f3.torus_map(y, x, 1 / 8)[1]) < 1e-15
    S.set_charges(dev(torch, q))
    phi, H = S.eval()
    u = S.adjoint_H(dev(torch, V))
    torch.cuda.synchronize()
    got = dict(phi=phi.cpu().numpy(), H=H.cpu().numpy(), HT=u.cpu().numpy())
    errs = {k: (rel_l2(got[k], ref[k]), max_rel(got[k], ref[k])) for k in got}
    print("  rel L2, per-element max:", {k: f"{a:.2e}, {b:.2e}" for k, (a, b) in errs.items()}, flush=True)
    assert max(parity_err(got[k], ref[k]) for k in got) < 1e-10, errs
    # phi only and H only give the same values
    p2, _ = S.eval(H=False)
    _, H2 = S.eval(phi=False)
    torch.cuda.synchronize()
    assert np.array_equal(p2.cpu().numpy(), got["phi"]) and np.array_equal(H2.cpu().numpy(), got["H"])


def test_3d_dense_cluster_matches_step_by_step_oracle(torch, fn):
    """10,000 sources and 300 targets inside a ball of radius 0.02: the home blocks at the
    cluster see more candidates than the kernel tabulates rows for, so the forward near
    field takes its row-search path there (FP64 parity bound as above)."""
    y, x, w, q = synth.random_cloud3(2001, 12003, 35, shape="ball")
    x[:10000] *= 0.02
    y[:300] *= 0.02
    prm = f3.Params3(G=32, m=5, p=6, eps_I=4 / 16, eps_B=1 / 8)
    F = f3.FastSum3(y, x, w, prm)
    V = np.random.default_rng(36).standard_normal((len(y), 3))
    ref = dict(zip(("phi", "H"), F.forward(q)))
    ref["HT"] = F.adjoint_H(V)
    S = fn.Solver3(grid=32, m=5, p=6, eps_I=4 / 16, eps_B=1 / 8)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
    S.set_charges(dev(torch, q))
    phi, H = S.eval()
    u = S.adjoint_H(dev(torch, V))
    torch.cuda.synchronize()
    got = dict(phi=phi.cpu().numpy(), H=H.cpu().numpy(), HT=u.cpu().numpy())
    errs = {k: parity_err(got[k], ref[k]) for k in got}
    print("3D cluster parity:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) < 1e-10, errs


def test_3d_accuracy_against_the_direct_sum(torch, fn):
    y, x, w, q = synth.random_cloud3(3000, 4000, 41)
    S = fn.Solver3(grid=128, m=8, p=8, eps_I=8 / 64, eps_B=1 / 8)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
    S.set_charges(dev(torch, q))
    phi, H = S.eval()
    V = np.random.default_rng(42).standard_normal((len(y), 3))
    u = S.adjoint_H(dev(torch, V))
    torch.cuda.synchronize()
    phi1, H1 = direct.forward3(y, x, w, q)
    u1 = direct.adjoint3(y, x, w, V=V)
    e = (rel_l2(phi.cpu().numpy(), phi1), rel_l2(H.cpu().numpy(), H1), rel_l2(u.cpu().numpy(), u1))
    print("3D vs direct sum (rel L2 phi, H, H^T):", [f"{v:.2e}" for v in e], flush=True)
    assert max(e) < 1e-6, e


def test_3d_empty_sets_and_errors(torch, fn):
    y, x, w, q = synth.random_cloud3(50, 60, 43)
    # no sources: zero outputs; no targets: nothing to do, the adjoint is zero
    S = fn.Solver3(grid=32, m=4, p=4, eps_I=3 / 16)
    S.set_geometry(dev(torch, y), dev(torch, x[:0]), dev(torch, w[:0]))
    S.set_charges(dev(torch, q[:0]))
    phi, H = S.eval()
    torch.cuda.synchronize()
    assert not phi.cpu().numpy().any() and not H.cpu().numpy().any()
    S.set_geometry(dev(torch, y[:0]), dev(torch, x), dev(torch, w))
    S.set_charges(dev(torch, q))
    phi, H = S.eval()
    u = S.adjoint_H(dev(torch, np.zeros((0, 3))))
    torch.cuda.synchronize()
    assert phi.numel() == 0 and not u.cpu().numpy().any()
    # one target, one source
    S.set_geometry(dev(torch, y[:1]), dev(torch, x[:1]), dev(torch, w[:1]))
    S.set_charges(dev(torch, q[:1]))
    phi, H = S.eval()
    torch.cuda.synchronize()
    p1, H1 = direct.forward3(y[:1], x[:1], w[:1], q[:1])
    assert abs(phi.item() - p1[0]) < 1e-3 * abs(p1[0])
    # every point at one place
    with pytest.raises(fn.FemNfftError, match="coincide"):
        S.set_geometry(dev(torch, np.zeros((3, 3))), dev(torch, np.zeros((2, 3))), dev(torch, np.ones(2)))
    # non-finite input
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(fn.FemNfftError, match="non-finite"):
        S.set_geometry(dev(torch, y), dev(torch, bad), dev(torch, w))
    # parameters the 3D path does not take
    for kw, msg in ((dict(grid=48), "power of two"), (dict(grid=16, m=4), "grid/4"), (dict(grid=512), "power of two"),
                    (dict(grid=64, n=50), "G/2 <= n"), (dict(grid=64, n=30), "G/2 <= n"),
                    (dict(grid=64, n=41), "G/2 <= n")):
        with pytest.raises(fn.FemNfftError, match=msg):
            fn.Solver3(**dict(dict(m=3, p=4, eps_I=0.1), **kw))


def test_3d_stage_profile_records_every_stage(torch, fn):
    y, x, w, q = synth.random_cloud3(2000, 3000, 44)
    S = fn.Solver3(grid=64, m=6, p=6, eps_I=5 / 32, eps_B=1 / 8)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
    V = dev(torch, np.random.default_rng(45).standard_normal((len(y), 3)))
    S.set_profiling(True)
    for _ in range(2):
        S.set_charges(dev(torch, q))
        S.eval()
        S.adjoint_H(V)
    torch.cuda.synchronize()
    prof = S.profile()
    S.set_profiling(False)
    print({k: f"{v[0]:.3f} ms x {v[1]}" for k, v in prof.items()}, flush=True)
    assert all(n == 2 and ms > 0 for ms, n in prof.values()), prof
