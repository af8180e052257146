"""The C-ABI library loads on the host and exports every function include/femnfft.h declares;
parameter validation runs before any device call."""
import ctypes
import os
import re

import pytest

pytestmark = pytest.mark.cpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "femnfft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fn3?_[A-Za-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fn_create", "fn_set_geometry", "fn_set_charges", "fn_eval", "fn_eval_phi", "fn_eval_H",
                 "fn_eval_H_adjoint", "fn_eval_phi_adjoint", "fn_workspace_size", "fn_set_workspace"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_0807_2387_amd import _lib
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(_lib.SYMBOLS) == set(declared_functions())


def test_params_default_and_validation():
    from paper_0807_2387_amd import _lib
    L = _lib.lib()
    p = _lib.Params()
    assert L.fn_params_default(ctypes.byref(p), 8192) == 0
    assert (p.grid, p.m, p.p, p.precision) == (8192, 6, 8, _lib.FN_FP32_MIXED)
    assert abs(p.eps_I - 7.0 / 4096) < 1e-18 and p.eps_B == 1.0 / 16
    ctx = ctypes.c_void_p()
    bad = []
    for field, val in (("grid", 100), ("grid", 16384), ("m", 1), ("m", 9), ("p", 0), ("p", 13),
                       ("eps_I", 0.0), ("eps_I", 0.1), ("eps_B", 0.3), ("precision", 7)):
        q = _lib.Params()
        L.fn_params_default(ctypes.byref(q), 512)
        setattr(q, field, val)
        rc = L.fn_create(ctypes.byref(q), None, ctypes.byref(ctx))
        bad.append((field, val, rc))
        assert rc == _lib.FN_E_INVAL, (field, val, rc, L.fn_last_error(None))
    q = _lib.Params()
    L.fn_params_default(ctypes.byref(q), 512)
    q.flags = 1
    assert L.fn_create(ctypes.byref(q), None, ctypes.byref(ctx)) == _lib.FN_E_UNSUPPORTED
    assert L.fn_create(None, None, ctypes.byref(ctx)) == _lib.FN_E_INVAL
    assert b"NULL" in L.fn_last_error(None)


def test_null_context_is_rejected():
    from paper_0807_2387_amd import _lib
    L = _lib.lib()
    for f in (L.fn_set_charges, L.fn_eval_phi, L.fn_eval_H):
        assert f(None, None) == _lib.FN_E_INVAL
    assert L.fn_eval(None, None, None) == _lib.FN_E_INVAL
    assert L.fn_set_geometry(None, 1, None, 1, None, None) == _lib.FN_E_INVAL


def test_params_auto_rule():
    """fn_params_auto as the header states it: n = 3G/4, eps_I = 7/n, m = 6; p = 8 with
    G^2 >= 2N from 2^22 points up, p = 9 with G^2 >= 4N below (N = targets + sources)."""
    from paper_0807_2387_amd import _lib
    L = _lib.lib()

    def grid_for(c, N):
        G = 64
        while G < 8192 and G * G < c * N:
            G *= 2
        return G

    for nt, ns in ((2_000, 12_000), (100_000, 600_000), (200_000, 1_200_000), (1 << 21, (1 << 21) - 1),
                   (1 << 21, 1 << 21), (1_000_000, 6_000_000), (1 << 24, 1 << 24), (1 << 26, 1 << 26)):
        p = _lib.Params()
        assert L.fn_params_auto(nt, ns, _lib.FN_FP32_MIXED, ctypes.byref(p)) == 0
        N = nt + ns
        small = N < (1 << 22)
        G = grid_for(4.0 if small else 2.0, N)
        assert p.grid == G, (nt, ns, p.grid, G)
        n = 3 * G // 4 if G >= 128 else 0
        assert p.n == n and p.m == 6 and p.p == (9 if small else 8), (nt, ns, p.n, p.m, p.p)
        assert abs(p.eps_I - 7.0 / (n or G // 2)) < 1e-18 and p.precision == _lib.FN_FP32_MIXED
    p = _lib.Params()
    assert L.fn_params_auto(-1, 5, _lib.FN_FP64, ctypes.byref(p)) == _lib.FN_E_INVAL


def test_3d_bandwidth_is_checked_before_any_device_call():
    from paper_0807_2387_amd import _lib
    L = _lib.lib()
    ctx = ctypes.c_void_p()
    for n in (50, 30, 41):  # above 3G/4, below G/2, odd (G = 64)
        q = _lib.Params(grid=64, m=4, p=6, precision=_lib.FN_FP64, eps_I=5.5 / 48, eps_B=0.125, flags=0, n=n,
                        eps_S=0.0)
        assert L.fn3_create(ctypes.byref(q), None, ctypes.byref(ctx)) == _lib.FN_E_INVAL, n
        assert b"G/2 <= n <= 3G/4" in L.fn3_last_error(None)
