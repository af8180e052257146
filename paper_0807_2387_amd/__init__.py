"""MI355X-native FEM-NFFT fast summation of 2D magnetostatic potentials and fields.

Python face of libfemnfft.so (include/femnfft.h).  Every computation runs in the
library's HIP kernels; this module only marshals torch device tensors (device
memory and the current stream) into the C calls.

    s = Solver(grid=8192, m=6, p=8, eps_I=7/4096)           # FN_FP32_MIXED by default
    s.set_geometry(tgt_xy, src_xy, src_w)                   # cuda float64 tensors
    s.set_charges(q)
    phi, H = s.eval()
    u = s.adjoint_H(V)                                       # u_j = w_j sum_i V_i.(-grad G)(r_i - r_j)
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import FN_FP32_MIXED, FN_FP64, FemNfftError  # noqa: F401

__all__ = ["Solver", "default_params", "FN_FP64", "FN_FP32_MIXED", "FemNfftError"]


def default_params(grid):
    p = _lib.Params()
    _lib.check(_lib.lib().fn_params_default(ctypes.byref(p), int(grid)))
    return dict(grid=p.grid, m=p.m, p=p.p, eps_I=p.eps_I, eps_B=p.eps_B, precision=p.precision)


def _torch():
    import torch
    return torch


def _dev_ptr(t, name, shape_tail=()):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One fast-summation context bound to the current device and torch stream."""

    def __init__(self, grid, m=None, p=None, eps_I=None, eps_B=None, precision=FN_FP32_MIXED, stream=None):
        torch = _torch()
        L = _lib.lib()
        d = default_params(grid)
        prm = _lib.Params(grid=int(grid), m=int(m if m is not None else d["m"]),
                          p=int(p if p is not None else d["p"]), precision=int(precision),
                          eps_I=float(eps_I if eps_I is not None else d["eps_I"]),
                          eps_B=float(eps_B if eps_B is not None else d["eps_B"]), flags=0, reserved=0)
        self.params = prm
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        _lib.check(L.fn_create(ctypes.byref(prm), ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(ctx)))
        self._ctx = ctx
        self._ws = None
        self.n_tgt = self.n_src = 0

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx:
            try:
                _lib.lib().fn_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    def _check(self, rc):
        _lib.check(rc, self._ctx)

    def workspace_bytes(self, n_tgt, n_src):
        b = ctypes.c_size_t()
        self._check(_lib.lib().fn_workspace_size(self._ctx, int(n_tgt), int(n_src), ctypes.byref(b)))
        return b.value

    def set_geometry(self, tgt_xy, src_xy, src_w):
        torch = _torch()
        L = _lib.lib()
        nt, ns = int(tgt_xy.shape[0]), int(src_xy.shape[0])
        need = self.workspace_bytes(nt, ns)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._check(L.fn_set_workspace(self._ctx, ctypes.c_void_p(self._ws.data_ptr()), ctypes.c_size_t(need)))
        pt = _dev_ptr(tgt_xy, "tgt_xy", (2,)) if nt else None
        ps = _dev_ptr(src_xy, "src_xy", (2,)) if ns else None
        pw = _dev_ptr(src_w, "src_w") if ns else None
        self._check(L.fn_set_geometry(self._ctx, nt, pt, ns, ps, pw))
        self.n_tgt, self.n_src = nt, ns
        self._geom_refs = (tgt_xy, src_xy, src_w)  # inputs must outlive the enqueued work
        return self

    def set_charges(self, q):
        self._q = q
        self._check(_lib.lib().fn_set_charges(self._ctx, _dev_ptr(q, "q") if self.n_src else None))
        return self

    def eval(self, phi=True, H=True, out_phi=None, out_H=None):
        torch = _torch()
        p = out_phi if out_phi is not None else (
            torch.empty(self.n_tgt, dtype=torch.float64, device=self.device) if phi else None)
        h = out_H if out_H is not None else (
            torch.empty(self.n_tgt, 2, dtype=torch.float64, device=self.device) if H else None)
        self._check(_lib.lib().fn_eval(self._ctx, _dev_ptr(p, "phi") if p is not None else None,
                                       _dev_ptr(h, "H", (2,)) if h is not None else None))
        return p, h

    def adjoint_H(self, V, out=None):
        torch = _torch()
        u = out if out is not None else torch.empty(self.n_src, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_eval_H_adjoint(self._ctx, _dev_ptr(V, "V", (2,)), _dev_ptr(u, "u")))
        return u

    def adjoint_phi(self, v, out=None):
        torch = _torch()
        u = out if out is not None else torch.empty(self.n_src, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_eval_phi_adjoint(self._ctx, _dev_ptr(v, "v"), _dev_ptr(u, "u")))
        return u

    def set_profiling(self, enable=True):
        self._check(_lib.lib().fn_set_profiling(self._ctx, int(bool(enable))))

    def profile(self):
        """Per-stage event time (ms) and launch counts since profiling was enabled."""
        pr = _lib.Profile()
        self._check(_lib.lib().fn_get_profile(self._ctx, ctypes.byref(pr)))
        return {name: (pr.ms[i], pr.count[i]) for i, name in enumerate(_lib.STAGES)}

    def info(self):
        i = _lib.Info()
        self._check(_lib.lib().fn_get_info(self._ctx, ctypes.byref(i)))
        return dict(centre=tuple(i.centre), scale=i.scale, n_tgt=i.n_tgt, n_src=i.n_src,
                    win_lo=tuple(i.win_lo), win_ext=tuple(i.win_ext), tiles=tuple(i.tiles),
                    near_cells=i.near_cells, workspace_bytes=i.workspace_bytes, near_pairs=i.near_pairs)
