"""Parity with the step-by-step oracle (O2) at the grid sizes the bench runs, through the C-ABI.

The small parity cases stop at G = 512, where an FFT block holds several short lines.  These
cases run the shapes of the timed configuration itself: G = 2048 (m = 6, and m = 5 with tuned
shapes) and G = 8192 (one line of G points per FFT block; the bench's m = 6 and the
autotuner's kernel shapes),
bandwidth 3G/4, p = 5, n eps_I = 3.25 for the volume
sources and n eps_S = 11 for the boundary Gauss points, eps_B = 1/32, two source classes,
forward and H adjoint in one overlapped call (as timed) plus the phi adjoint.  The points
are the bench workload's recipe (rounded square, jittered lattice, boundary Gauss points)
at 6e4 / 1.5e5 points, so the data window is the timed one (about 0.36 G cells a side):
every tile of the spread and gather, every FFT line and every near-field home block runs.

Bounds: FP64 path 1e-10, FP32-mixed path 1e-6, each as relative L2 per output kind AND
per element (max |a_i - b_i| below 10x the tolerance times max |b|; tests.conftest.parity_err).
The expected values are two per-class O2 fast sums (the sum of eq. (2) is linear in the
sources; the torus map is taken over all points).
"""
import numpy as np
import pytest

import synth
from oracle import fastsum as fs
from tests.conftest import max_rel, parity_err, rel_l2

pytestmark = pytest.mark.gpu

# name, lattice points, G, window half-width m, seed, tuned shapes
GRIDS = [("G2048", 60_000, 2048, 6, 91, False), ("G2048-m5", 60_000, 2048, 5, 93, True),
         ("G8192", 150_000, 8192, 6, 92, True)]
P_DEG, C_VOL, C_SURF, EPS_B = 5, 3.25, 11.0, 1.0 / 32.0


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


_CACHE = {}


def expected(name, N, G, m, seed):
    """Inputs and the O2 outputs of one grid case (computed once per module)."""
    if name in _CACHE:
        return _CACHE[name]
    d = synth.rounded_square_cloud(N=N, seed=seed)
    y, x, w, q = d["y"], d["x"], d["w"], d["q"]
    ns1 = int(np.sum(w == d["h"] ** 2))
    assert 0 < ns1 < len(x) and np.all(w[:ns1] == d["h"] ** 2)  # boundary points come last
    rng = np.random.default_rng(seed + 1)
    V = rng.standard_normal((len(y), 2))
    v = rng.standard_normal(len(y))
    band = 3 * G // 4
    pv = fs.Params(G=G, m=m, p=P_DEG, eps_I=C_VOL / band, band=band, eps_B=EPS_B)
    ps = fs.Params(G=G, m=m, p=P_DEG, eps_I=C_SURF / band, band=band, eps_B=EPS_B)
    out = []
    phi, H = 0.0, 0.0
    for sl, prm, other in ((slice(0, ns1), pv, slice(ns1, None)), (slice(ns1, None), ps, slice(0, ns1))):
        F = fs.FastSum(y, x[sl], w[sl], prm, map_with=x[other])
        p_, H_ = F.forward(q[sl])
        phi, H = phi + p_, H + H_
        out.append((F.adjoint_H(V), F.adjoint_phi(v)))
        del F
    u = np.concatenate([o[0] for o in out])
    up = np.concatenate([o[1] for o in out])
    _CACHE[name] = dict(y=y, x=x, w=w, q=q, ns1=ns1, V=V, v=v, band=band,
                        ref=dict(phi=phi, H=H, HT=u, phiT=up))
    return _CACHE[name]


@pytest.mark.parametrize("case", GRIDS, ids=[c[0] for c in GRIDS])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bench_grid_matches_step_by_step_oracle(torch, fn, case, precision, tmp_path, monkeypatch):
    name, N, G, m, seed, tuned = case
    print(f"bench-grid case {name} m={m} {precision}: oracle", flush=True)
    e = expected(name, N, G, m, seed)
    print(f"  {len(e['y'])} targets, {len(e['x'])} sources ({len(e['x']) - e['ns1']} surface); GPU", flush=True)
    P = fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED
    band = e["band"]
    S = fn.Solver(grid=G, m=m, p=P_DEG, eps_I=C_VOL / band, eps_S=C_SURF / band, eps_B=EPS_B, n=band,
                  precision=P)
    S.set_geometry(dev(torch, e["y"]), dev(torch, e["x"]), dev(torch, e["w"]), n_surf=len(e["x"]) - e["ns1"])
    if tuned:  # the autotuner's shapes, as the bench runs them (searched here on this data)
        from paper_0807_2387_amd import tune
        monkeypatch.setenv("FEMNFFT_TUNE_CACHE", str(tmp_path / "tune.json"))
        shapes, _, _ = tune.apply(S, dev(torch, e["q"]), dev(torch, e["V"]), reps=2)
        print(f"  tuned shapes {shapes}", flush=True)
    info = S.info()
    # the data window of the timed configuration (about 0.36 G cells) and the FFT size
    assert 0.3 * G < info["win_ext"][0] < 0.4 * G, info["win_ext"]
    S.set_charges(dev(torch, e["q"]))
    phi, H, u = S.eval_with_H_adjoint(dev(torch, e["V"]))
    up = S.adjoint_phi(dev(torch, e["v"]))
    torch.cuda.synchronize()
    got = dict(phi=phi.cpu().numpy(), H=H.cpu().numpy(), HT=u.cpu().numpy(), phiT=up.cpu().numpy())
    del S
    torch.cuda.empty_cache()
    tol = 1e-10 if precision == "fp64" else 1e-6
    errs = {k: (rel_l2(got[k], e["ref"][k]), max_rel(got[k], e["ref"][k])) for k in got}
    print("  rel L2, per-element max:", {k: f"{a:.2e}, {b:.2e}" for k, (a, b) in errs.items()}, flush=True)
    worst = {k: parity_err(got[k], e["ref"][k]) for k in got}
    assert max(worst.values()) < tol, errs
