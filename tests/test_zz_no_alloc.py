"""fn_eval_noalloc (the entry point for callers that cannot allocate device memory) through
the C-ABI, against the same evaluation on a context with its own workspace
(fn_set_geometry_split + fn_set_charges + fn_eval).

Both run the same kernels on the same inputs, each summing in a fixed order, so the results
agree to rounding (bitwise in practice); the bound is 1e-12 relative, per output kind and per
element.  Two calls in a row share the library's static buffer, the second with a smaller
problem, and the context's own workspace and geometry must be untouched by them.
"""
import ctypes

import numpy as np
import pytest

import synth
from tests.conftest import parity_err

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


def problem(nt, nv, nsurf, seed):
    y, x, w, q = synth.random_cloud(nt, nv, seed)
    t = 2 * np.pi * (np.arange(nsurf) + 0.5) / nsurf
    xs = np.stack([np.cos(t), np.sin(t)], axis=1)
    ws = np.full(nsurf, 2 * np.pi / nsurf)
    qs = np.cos(t)
    return y, np.concatenate([x, xs]), np.concatenate([w, ws]), np.concatenate([q, qs]), nsurf


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_workspace_path_on_two_calls(torch, fn, precision):
    P = fn.FN_FP64 if precision == "fp64" else fn.FN_FP32_MIXED
    kw = dict(grid=512, m=6, p=6, eps_I=4 / 384, eps_S=9 / 384, n=384, precision=P)
    ref = fn.Solver(**kw)      # context with its own workspace (the existing path)
    na = fn.Solver(**kw)       # context that only lends parameters and stream to fn_eval_noalloc
    # a geometry of its own on `na`, to check that the no-allocation calls leave it alone
    y0, x0, w0, q0, s0 = problem(3000, 3500, 300, 70)
    na.set_geometry(dev(torch, y0), dev(torch, x0), dev(torch, w0), n_surf=s0)
    na.set_charges(dev(torch, q0))
    phi_before, H_before = na.eval()
    for call, (nt, nv, ns, seed) in enumerate([(40_000, 52_000, 900, 71), (9_000, 11_000, 200, 72)]):
        print(f"no-alloc call {call} {precision}: {nt} targets, {nv + ns} sources", flush=True)
        y, x, w, q, nsurf = problem(nt, nv, ns, seed)
        assert ref.workspace_bytes(nt, nv + ns) <= fn._lib.FN_NOALLOC_SCRATCH_BYTES
        Y, X, Wt, Q = dev(torch, y), dev(torch, x), dev(torch, w), dev(torch, q)
        ref.set_geometry(Y, X, Wt, n_surf=nsurf)
        ref.set_charges(Q)
        pr, hr = ref.eval()
        pn = torch.empty(nt, dtype=torch.float64, device="cuda")
        hn = torch.empty(nt, 2, dtype=torch.float64, device="cuda")
        na.eval_noalloc(Y, X, Wt, Q, pn, hn, n_surf=nsurf)
        torch.cuda.synchronize()
        e = dict(phi=parity_err(pn.cpu().numpy(), pr.cpu().numpy()), H=parity_err(hn.cpu().numpy(), hr.cpu().numpy()))
        print(e, flush=True)
        assert max(e.values()) < 1e-12, (call, e)
    # the context's own workspace, geometry and charges are as before
    assert na.info()["n_tgt"] == len(y0)
    phi_after, H_after = na.eval()
    torch.cuda.synchronize()
    assert parity_err(phi_after.cpu().numpy(), phi_before.cpu().numpy()) < 1e-14
    assert parity_err(H_after.cpu().numpy(), H_before.cpu().numpy()) < 1e-14


def test_noalloc_rejects_problems_beyond_its_buffer(torch, fn):
    """The size check comes before anything is read: huge counts with a small dummy buffer."""
    S = fn.Solver(grid=2048, m=6, p=6, eps_I=4 / 1024)
    big = 4_000_000
    assert S.workspace_bytes(big, big) > fn._lib.FN_NOALLOC_SCRATCH_BYTES
    d = torch.zeros(16, dtype=torch.float64, device="cuda")
    L = fn._lib.lib()
    p = ctypes.c_void_p(d.data_ptr())
    rc = L.fn_eval_noalloc(S._ctx, big, p, big, p, p, 0, p, p, p)
    assert rc == fn._lib.FN_E_NOMEM
    assert b"static buffer" in L.fn_last_error(S._ctx)
