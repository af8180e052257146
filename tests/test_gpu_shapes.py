"""Kernel work shapes (fn_set_shapes) and the autotuner (paper_0807_2387_amd.tune) on the GPU.

Shapes change speed only: at every supported tile edge, spread row grouping and near-field
home block / staging capacity the results match the step-by-step oracle (O2, per source
class) to the usual bounds (FP64 1e-10, FP32-mixed 1e-6; relative L2 and per element).  The
tuner's pick is applied, cached under its key, found again, and its results match O2 too.
"""
import numpy as np
import pytest

import synth
from oracle import fastsum as fs
from tests.conftest import parity_err

pytestmark = pytest.mark.gpu

G, BAND, M_WIN, P_DEG, CV, CS = 256, 192, 5, 5, 3.25, 11.0


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


_REF = {}


def reference(N=20_000, seed=51, grid=G, band=BAND):
    key = (N, seed, grid)
    if key in _REF:
        return _REF[key]
    d = synth.rounded_square_cloud(N=N, seed=seed)
    y, x, w, q = d["y"], d["x"], d["w"], d["q"]
    ns1 = int(np.sum(w == d["h"] ** 2))
    V = np.random.default_rng(seed + 1).standard_normal((len(y), 2))
    pv = fs.Params(G=grid, m=M_WIN, p=P_DEG, eps_I=CV / band, band=band, eps_B=1 / 32)
    ps = fs.Params(G=grid, m=M_WIN, p=P_DEG, eps_I=CS / band, band=band, eps_B=1 / 32)
    Fv = fs.FastSum(y, x[:ns1], w[:ns1], pv, map_with=x[ns1:])
    Fs = fs.FastSum(y, x[ns1:], w[ns1:], ps, map_with=x[:ns1])
    pv_, Hv = Fv.forward(q[:ns1])
    ps_, Hs = Fs.forward(q[ns1:])
    u = np.concatenate([Fv.adjoint_H(V), Fs.adjoint_H(V)])
    _REF[key] = dict(y=y, x=x, w=w, q=q, ns1=ns1, V=V, phi=pv_ + ps_, H=Hv + Hs, u=u)
    return _REF[key]


def solver(fn, r, precision, grid=G, band=BAND):
    S = fn.Solver(grid=grid, m=M_WIN, p=P_DEG, eps_I=CV / band, eps_S=CS / band, eps_B=1 / 32, n=band,
                  precision=precision)
    return S


def run(torch, S, r, out=None):
    S.set_charges(dev(torch, r["q"]))
    phi, H, u = S.eval_with_H_adjoint(dev(torch, r["V"]))
    torch.cuda.synchronize()
    return dict(phi=phi.cpu().numpy(), H=H.cpu().numpy(), u=u.cpu().numpy())


SHAPES = [
    dict(tile=16),
    dict(spread_groups=2),
    dict(spread_groups=3, tile=16),
    dict(near_fwd_bx=16, near_fwd_by=16, near_fwd_cap=384, near_adj_bx=64, near_adj_by=4, near_adj_cap=128),
    dict(near_fwd_bx=64, near_fwd_by=4, near_fwd_cap=2048, near_adj_bx=16, near_adj_by=16, near_adj_cap=1536),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[str(i) for i in range(len(SHAPES))])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_results_do_not_depend_on_shapes(torch, fn, shape, precision):
    r = reference()
    print(f"shapes {shape} {precision}", flush=True)
    S = solver(fn, r, fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED)
    S.set_shapes(**shape)
    got = S.shapes()
    for k, v in shape.items():
        assert got[k] == v
    S.set_geometry(dev(torch, r["y"]), dev(torch, r["x"]), dev(torch, r["w"]), n_surf=len(r["x"]) - r["ns1"])
    o = run(torch, S, r)
    tol = 1e-10 if precision == "fp64" else 1e-6
    errs = {k: parity_err(o[k], r[k]) for k in o}
    print(errs, flush=True)
    assert max(errs.values()) < tol, errs


def test_unsupported_shapes_are_rejected(torch, fn):
    S = solver(fn, None, fn.FN_FP32_MIXED)
    before = S.shapes()
    for bad in (dict(tile=24), dict(near_fwd_bx=128, near_fwd_by=2), dict(near_adj_cap=100), dict(spread_groups=4)):
        with pytest.raises(fn.FemNfftError):
            S.set_shapes(**bad)
        assert S.shapes() == before


def test_tuner_picks_caches_and_keeps_parity(torch, fn, tmp_path, monkeypatch):
    from paper_0807_2387_amd import tune
    monkeypatch.setenv("FEMNFFT_TUNE_CACHE", str(tmp_path / "tune.json"))
    r = reference(N=120_000, seed=52, grid=1024, band=768)
    S = solver(fn, r, fn.FN_FP32_MIXED, grid=1024, band=768)
    S.set_geometry(dev(torch, r["y"]), dev(torch, r["x"]), dev(torch, r["w"]), n_surf=len(r["x"]) - r["ns1"])
    q, V = dev(torch, r["q"]), dev(torch, r["V"])
    shapes, key, tuned = tune.apply(S, q, V, reps=2, log=lambda s: print(s, flush=True))
    print("tuned", key, shapes, flush=True)
    assert tuned and tune.lookup(key) == shapes
    assert S.shapes() == shapes
    S2 = solver(fn, r, fn.FN_FP32_MIXED, grid=1024, band=768)
    S2.set_geometry(dev(torch, r["y"]), dev(torch, r["x"]), dev(torch, r["w"]), n_surf=len(r["x"]) - r["ns1"])
    shapes2, key2, tuned2 = tune.apply(S2, q, V)
    assert key2 == key and shapes2 == shapes and not tuned2
    o = run(torch, S2, r)
    errs = {k: parity_err(o[k], r[k]) for k in o}
    print(errs, flush=True)
    assert max(errs.values()) < 1e-6, errs
