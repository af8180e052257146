"""ctypes binding of oracle O1 (oracle/direct.c, 2D; oracle/direct3.c, 3D) -- TEST
INFRASTRUCTURE ONLY.

build() compiles both with gcc (-O2 -fopenmp, no fast-math, no FMA contraction) into
oracle/_o1.so.  The loader builds it on first use if absent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "direct.c"), os.path.join(_HERE, "direct3.c")]
_SO = os.path.join(_HERE, "_o1.so")
_lib = None


def build(force=True):
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-o", _SO + ".tmp", *_SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.o1_forward.argtypes = [I64, P, I64, P, P, P, P, P]
        lib.o1_forward.restype = ctypes.c_int
        lib.o1_adjoint.argtypes = [I64, P, I64, P, P, P, P, P]
        lib.o1_adjoint.restype = ctypes.c_int
        lib.o1_threads.restype = ctypes.c_int
        for f in (lib.o1_3d_forward, lib.o1_3d_adjoint):
            f.argtypes = [I64, P, I64, P, P, P, P, P]
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, shape_last=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def threads():
    return int(_load().o1_threads())


def forward(y, x, w, q, want_phi=True, want_H=True):
    """phi [nt], H [nt, 2] of sum_j w_j q_j G(y_i - x_j), G = -(1/2pi) ln r."""
    lib = _load()
    y, x, w, q = _c(y), _c(x), _c(w), _c(q)
    nt, ns = len(y), len(x)
    phi = np.empty(nt) if want_phi else None
    H = np.empty((nt, 2)) if want_H else None
    rc = lib.o1_forward(nt, _p(y), ns, _p(x), _p(w), _p(q), _p(phi), _p(H))
    if rc:
        raise ValueError("o1_forward: bad arguments")
    return phi, H


def adjoint(y, x, w, v=None, V=None):
    """u_j = w_j sum_i (v_i G(y_i - x_j) + V_i . (-grad G)(y_i - x_j))."""
    lib = _load()
    y, x, w = _c(y), _c(x), _c(w)
    v, V = _c(v), _c(V)
    u = np.empty(len(x))
    rc = lib.o1_adjoint(len(y), _p(y), len(x), _p(x), _p(w), _p(v), _p(V), _p(u))
    if rc:
        raise ValueError("o1_adjoint: bad arguments")
    return u


def forward3(y, x, w, q, want_phi=True, want_H=True):
    """3D: phi [nt], H [nt, 3] of sum_j w_j q_j G(y_i - x_j), G = 1/(4 pi r)."""
    lib = _load()
    y, x, w, q = _c(y), _c(x), _c(w), _c(q)
    nt, ns = len(y), len(x)
    phi = np.empty(nt) if want_phi else None
    H = np.empty((nt, 3)) if want_H else None
    if lib.o1_3d_forward(nt, _p(y), ns, _p(x), _p(w), _p(q), _p(phi), _p(H)):
        raise ValueError("o1_3d_forward: bad arguments")
    return phi, H


def adjoint3(y, x, w, v=None, V=None):
    """3D: u_j = w_j sum_i (v_i G(y_i - x_j) + V_i . (-grad G)(y_i - x_j)), G = 1/(4 pi r)."""
    lib = _load()
    y, x, w = _c(y), _c(x), _c(w)
    v, V = _c(v), _c(V)
    u = np.empty(len(x))
    if lib.o1_3d_adjoint(len(y), _p(y), len(x), _p(x), _p(w), _p(v), _p(V), _p(u)):
        raise ValueError("o1_3d_adjoint: bad arguments")
    return u
