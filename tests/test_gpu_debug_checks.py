"""The binning debug checks (FEMNFFT_DEBUG_CHECKS, read when a context is created): after
set_geometry the library validates every binned point set on the device -- keys sorted and
inside the cell table, cell starts consistent with the keys, fractions in [0, 1] (2D) or packed
positions inside their key's cell (3D), the permutation a permutation -- and fails with
FN_E_DEVICE on a violation.  Here every geometry of the usual kinds passes them, and the results
equal a context's without the checks bit for bit."""
import numpy as np
import pytest

import synth

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


def _run2(fn, torch, y, x, w, q, n_surf, precision):
    S = fn.Solver(grid=128, m=6, p=6, eps_I=5 / 64, eps_S=(10 / 64 if n_surf else 0.0), precision=precision)
    S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w), n_surf=n_surf)
    S.set_charges(dev(torch, q))
    phi, H = S.eval()
    torch.cuda.synchronize()
    return phi.cpu().numpy(), H.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_debug_checks_pass_and_change_nothing_2d(torch, fn, monkeypatch, precision):
    P = fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED
    y, x, w, q = synth.random_cloud(3000, 4000, 51)
    y[:40] = x[:40]  # coincident points
    d = synth.rounded_square_cloud(N=20_000, seed=52)
    ns1 = int(np.sum(d["w"] == d["h"] ** 2))
    cases = [(y, x, w, q, 0), (d["y"], d["x"], d["w"], d["q"], len(d["x"]) - ns1)]
    for yy, xx, ww, qq, ns in cases:
        monkeypatch.delenv("FEMNFFT_DEBUG_CHECKS", raising=False)
        ref = _run2(fn, torch, yy, xx, ww, qq, ns, P)
        monkeypatch.setenv("FEMNFFT_DEBUG_CHECKS", "1")
        got = _run2(fn, torch, yy, xx, ww, qq, ns, P)
        assert all(np.array_equal(a, b) for a, b in zip(got, ref))


def test_debug_checks_pass_and_change_nothing_3d(torch, fn, monkeypatch):
    y, x, w, q = synth.random_cloud3(2000, 3000, 53)
    y[:30] = x[:30]
    out = []
    for flag in (None, "1"):
        if flag:
            monkeypatch.setenv("FEMNFFT_DEBUG_CHECKS", flag)
        else:
            monkeypatch.delenv("FEMNFFT_DEBUG_CHECKS", raising=False)
        S = fn.Solver3(grid=64, m=6, p=6, eps_I=5 / 32, eps_B=1 / 8)
        S.set_geometry(dev(torch, y), dev(torch, x), dev(torch, w))
        S.set_charges(dev(torch, q))
        phi, H = S.eval()
        torch.cuda.synchronize()
        out.append((phi.cpu().numpy(), H.cpu().numpy()))
    assert all(np.array_equal(a, b) for a, b in zip(out[0], out[1]))
