"""MI355X-native FEM-NFFT fast summation of 2D magnetostatic potentials and fields.

Python face of libfemnfft.so (include/femnfft.h).  Every computation runs in the
library's HIP kernels; this module only marshals torch device tensors (device
memory and the current stream) into the C calls.

    s = Solver(grid=8192, m=6, p=8, eps_I=7/4096)           # FN_FP32_MIXED by default
    s.set_geometry(tgt_xy, src_xy, src_w)                   # cuda float64 tensors
    s.set_charges(q)
    phi, H = s.eval()
    u = s.adjoint_H(V)                                       # u_j = w_j sum_i V_i.(-grad G)(r_i - r_j)
    phi, H, u = s.eval_with_H_adjoint(V)                     # both at once, on two streams

    s = Solver(grid=8192, m=6, p=5, eps_I=3.25/6144, eps_S=11/6144, eps_B=1/32, n=6144)
    s.set_geometry(tgt_xy, src_xy, src_w, n_surf=k)          # last k sources: surface charges at eps_S

    mesh = Mesh(nodes, tris, bedges)                         # P1 triangle mesh (float64 / int32 tensors)
    s.bind_mesh(mesh)                                        # targets = nodes, sources = quadrature points
    E, dE = s.energy(M)                                      # demagnetizing energy and dE/dM
    E = DemagEnergy.apply(M, s, mesh)                        # the same as a torch autograd function

    b = Batch([dict(grid=512), dict(grid=1024)])             # independent problems on one stream
    b.set_geometry(tgt_off, tgt_xy, src_off, src_xy, src_w)  # CSR offsets, concatenated arrays
    b.set_shapes(1, tile=16)                                 # kernel work shapes of member 1
    tune.apply_batch(b, tgt_off, tgt_xy, src_off, src_xy, src_w, q, V)   # tuned shapes per member
    g = Graph()
    with g.capture(stream):                                  # record library calls issued on `stream`
        b.set_charges(q); b.eval(out_phi=phi, out_H=H)
    g.launch(stream)                                         # replay them with one launch
"""
from __future__ import annotations

import contextlib
import ctypes

from . import _lib
from ._lib import FN_FP32_MIXED, FN_FP64, FemNfftError  # noqa: F401

__all__ = ["Solver", "Solver3", "Mesh", "Mesh3", "Batch", "Graph", "DemagEnergy", "default_params", "auto_params",
           "FN_FP64", "FN_FP32_MIXED",
           "FemNfftError"]


def default_params(grid):
    p = _lib.Params()
    _lib.check(_lib.lib().fn_params_default(ctypes.byref(p), int(grid)))
    return dict(grid=p.grid, m=p.m, p=p.p, eps_I=p.eps_I, eps_B=p.eps_B, precision=p.precision, n=p.n,
                eps_S=p.eps_S)


def auto_params(n_tgt, n_src, precision=FN_FP32_MIXED):
    """Grid and regularization for a problem size (fn_params_auto)."""
    p = _lib.Params()
    _lib.check(_lib.lib().fn_params_auto(int(n_tgt), int(n_src), int(precision), ctypes.byref(p)))
    return dict(grid=p.grid, m=p.m, p=p.p, eps_I=p.eps_I, eps_B=p.eps_B, precision=p.precision, n=p.n,
                eps_S=p.eps_S)


def _torch():
    import torch
    return torch


def _dev_ptr(t, name, shape_tail=(), dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    want = dtype if dtype is not None else torch.float64
    if t.dtype != want:
        raise TypeError(f"{name} must be {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")
    return ctypes.c_void_p(t.data_ptr())


SHAPE_KEYS = ("spread_groups", "near_fwd_bx", "near_fwd_by", "near_fwd_cap", "near_adj_bx", "near_adj_by",
              "near_adj_cap", "tile")


def _set_shapes(ctx, shapes):
    bad = set(shapes) - set(SHAPE_KEYS)
    if bad:
        raise ValueError(f"unknown shape fields {sorted(bad)}")
    sh = _lib.Shapes(**{k: int(v) for k, v in shapes.items()})
    _lib.check(_lib.lib().fn_set_shapes(ctx, ctypes.byref(sh)), ctx)


def _get_shapes(ctx):
    sh = _lib.Shapes()
    _lib.check(_lib.lib().fn_get_shapes(ctx, ctypes.byref(sh)), ctx)
    return {k: int(getattr(sh, k)) for k in SHAPE_KEYS}


class Solver:
    """One fast-summation context bound to the current device and torch stream."""

    def __init__(self, grid, m=None, p=None, eps_I=None, eps_B=None, precision=FN_FP32_MIXED, stream=None, n=0,
                 eps_S=0.0):
        torch = _torch()
        L = _lib.lib()
        d = default_params(grid)
        prm = _lib.Params(grid=int(grid), m=int(m if m is not None else d["m"]),
                          p=int(p if p is not None else d["p"]), precision=int(precision),
                          eps_I=float(eps_I if eps_I is not None else d["eps_I"]),
                          eps_B=float(eps_B if eps_B is not None else d["eps_B"]), flags=0, n=int(n or 0),
                          eps_S=float(eps_S or 0.0))
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

    def set_geometry(self, tgt_xy, src_xy, src_w, n_surf=0):
        """Targets, sources and weights (device tensors); the last n_surf sources are
        surface quadrature points (fn_set_geometry_split)."""
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
        if n_surf:
            self._check(L.fn_set_geometry_split(self._ctx, nt, pt, ns, ps, pw, int(n_surf)))
        else:
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

    def eval_with_H_adjoint(self, V, out_phi=None, out_H=None, out_u=None):
        """phi, H = eval() and u = adjoint_H(V) in one call that runs the two at once on
        two streams; returns (phi, H, u)."""
        torch = _torch()
        p = out_phi if out_phi is not None else torch.empty(self.n_tgt, dtype=torch.float64, device=self.device)
        h = out_H if out_H is not None else torch.empty(self.n_tgt, 2, dtype=torch.float64, device=self.device)
        u = out_u if out_u is not None else torch.empty(self.n_src, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_eval_with_H_adjoint(self._ctx, _dev_ptr(p, "phi"), _dev_ptr(h, "H", (2,)),
                                                      _dev_ptr(V, "V", (2,)), _dev_ptr(u, "u")))
        return p, h, u

    def eval_noalloc(self, tgt_xy, src_xy, src_w, q, out_phi, out_H, n_surf=0):
        """fn_eval_noalloc: geometry + charges + eval on the library's static scratch (no
        device allocation; the outputs are the caller's tensors).  The context's own
        workspace and state are untouched."""
        nt, ns = int(tgt_xy.shape[0]), int(src_xy.shape[0])
        self._check(_lib.lib().fn_eval_noalloc(
            self._ctx, nt, _dev_ptr(tgt_xy, "tgt_xy", (2,)) if nt else None, ns,
            _dev_ptr(src_xy, "src_xy", (2,)) if ns else None, _dev_ptr(src_w, "src_w") if ns else None,
            int(n_surf), _dev_ptr(q, "q") if ns else None,
            _dev_ptr(out_phi, "phi") if out_phi is not None else None,
            _dev_ptr(out_H, "H", (2,)) if out_H is not None else None))
        return out_phi, out_H

    def adjoint_phi(self, v, out=None):
        torch = _torch()
        u = out if out is not None else torch.empty(self.n_src, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_eval_phi_adjoint(self._ctx, _dev_ptr(v, "v"), _dev_ptr(u, "u")))
        return u

    def bind_mesh(self, mesh):
        """Targets = the mesh's nodes, sources = its quadrature points (fn_bind_mesh)."""
        torch = _torch()
        L = _lib.lib()
        need = self.workspace_bytes(mesh.n_nodes, mesh.n_sources)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._check(L.fn_set_workspace(self._ctx, ctypes.c_void_p(self._ws.data_ptr()), ctypes.c_size_t(need)))
        self._check(L.fn_bind_mesh(self._ctx, mesh._mesh))
        self.n_tgt, self.n_src = mesh.n_nodes, mesh.n_sources
        self._mesh = mesh
        return self

    def bind_mesh_sources(self, mesh):
        """Targets = sources = the mesh's quadrature points (fn_bind_mesh_sources)."""
        torch = _torch()
        L = _lib.lib()
        need = self.workspace_bytes(mesh.n_sources, mesh.n_sources)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._check(L.fn_set_workspace(self._ctx, ctypes.c_void_p(self._ws.data_ptr()), ctypes.c_size_t(need)))
        self._check(L.fn_bind_mesh_sources(self._ctx, mesh._mesh))
        self.n_tgt = self.n_src = mesh.n_sources
        self._mesh = mesh
        return self

    def energy_charge(self, M, grad=True):
        """Charge-form energy E_q = 1/2 sum_j s_j phi_j (0-d tensor), dE_q/dM [n_nodes, 2] if grad,
        and phi at the quadrature points [S] (fn_energy_charge; needs bind_mesh_sources)."""
        torch = _torch()
        mesh = self._mesh
        E = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty(mesh.n_nodes, 2, dtype=torch.float64, device=self.device) if grad else None
        phi = torch.empty(mesh.n_sources, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_energy_charge(self._ctx, mesh._mesh, _dev_ptr(M, "M", (2,)),
                                                ctypes.c_void_p(E.data_ptr()),
                                                _dev_ptr(g, "grad", (2,)) if g is not None else None,
                                                _dev_ptr(phi, "phi_s")))
        return E, g, phi

    def energy(self, M, grad=True):
        """E = -1/2 sum_i l_i M_i . H_i (0-d tensor) and, if grad, dE/dM [n_nodes, 2] (fn_energy)."""
        torch = _torch()
        mesh = self._mesh
        E = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty(mesh.n_nodes, 2, dtype=torch.float64, device=self.device) if grad else None
        self._check(_lib.lib().fn_energy(self._ctx, mesh._mesh, _dev_ptr(M, "M", (2,)), ctypes.c_void_p(E.data_ptr()),
                                         _dev_ptr(g, "grad", (2,)) if g is not None else None))
        return E, g

    SHAPE_KEYS = SHAPE_KEYS

    def set_shapes(self, **shapes):
        """Kernel work shapes (fn_set_shapes); unnamed fields keep the library default."""
        _set_shapes(self._ctx, shapes)
        return self

    def shapes(self):
        return _get_shapes(self._ctx)

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
                    near_cells=i.near_cells, workspace_bytes=i.workspace_bytes, near_pairs=i.near_pairs,
                    n_surf=i.n_surf, near_pairs_surf=i.near_pairs_surf, near_cells_surf=i.near_cells_surf)


class Solver3:
    """The 3D fast summation (fn3_*): G = 1/(4 pi r), FP64, points as [n, 3] device tensors."""

    def __init__(self, grid, m=6, p=8, eps_I=None, eps_B=0.125, stream=None, n=0):
        """n: bandwidth, 0 for G/2 (oversampling 2), or even in [G/2, 3G/4]."""
        torch = _torch()
        prm = _lib.Params(grid=int(grid), m=int(m), p=int(p), precision=FN_FP64,
                          eps_I=float(eps_I if eps_I is not None else 6.0 / (n or grid // 2)), eps_B=float(eps_B),
                          flags=0, n=int(n), eps_S=0.0)
        self.params = prm
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        _lib.check3(_lib.lib().fn3_create(ctypes.byref(prm), ctypes.c_void_p(self._stream.cuda_stream),
                                          ctypes.byref(ctx)))
        self._ctx = ctx
        self._ws = None
        self.n_tgt = self.n_src = 0

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx:
            try:
                _lib.lib().fn3_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    def _check(self, rc):
        _lib.check3(rc, self._ctx)

    def set_geometry(self, tgt_xyz, src_xyz, src_w):
        torch = _torch()
        L = _lib.lib()
        nt, ns = int(tgt_xyz.shape[0]), int(src_xyz.shape[0])
        if src_w.dim() != 1 or src_w.shape[0] != ns:
            raise ValueError(f"src_w must have shape [{ns}]")
        self._ensure_ws(nt, ns)
        self._check(L.fn3_set_geometry(self._ctx, nt, _dev_ptr(tgt_xyz, "tgt_xyz", (3,)) if nt else None, ns,
                                       _dev_ptr(src_xyz, "src_xyz", (3,)) if ns else None,
                                       _dev_ptr(src_w, "src_w") if ns else None))
        self.n_tgt, self.n_src = nt, ns
        self._geom_refs = (tgt_xyz, src_xyz, src_w)
        return self

    def _ensure_ws(self, nt, ns):
        torch = _torch()
        L = _lib.lib()
        need = ctypes.c_size_t()
        self._check(L.fn3_workspace_size(self._ctx, nt, ns, ctypes.byref(need)))
        if self._ws is None or self._ws.numel() < need.value:
            self._ws = None
            self._ws = torch.empty(need.value, dtype=torch.uint8, device=self.device)
            self._check(L.fn3_set_workspace(self._ctx, ctypes.c_void_p(self._ws.data_ptr()), need))

    def set_charges(self, q):
        if q.dim() != 1 or q.shape[0] != self.n_src:
            raise ValueError(f"q must have shape [{self.n_src}]")
        self._q = q
        self._check(_lib.lib().fn3_set_charges(self._ctx, _dev_ptr(q, "q") if self.n_src else None))
        return self

    def eval(self, phi=True, H=True, out_phi=None, out_H=None):
        """phi [n_tgt] and H [n_tgt, 3] (either may be skipped); out_* are optional preallocated outputs."""
        torch = _torch()
        for t, nm in ((out_phi, "out_phi"), (out_H, "out_H")):
            if t is not None and (t.dim() < 1 or t.shape[0] != self.n_tgt):
                raise ValueError(f"{nm} must have {self.n_tgt} rows")
        p = (out_phi if out_phi is not None else torch.empty(self.n_tgt, dtype=torch.float64, device=self.device)) \
            if phi else None
        h = (out_H if out_H is not None else torch.empty(self.n_tgt, 3, dtype=torch.float64, device=self.device)) \
            if H else None
        self._check(_lib.lib().fn3_eval(self._ctx, _dev_ptr(p, "phi") if p is not None else None,
                                        _dev_ptr(h, "H", (3,)) if h is not None else None))
        return p, h

    def adjoint_H(self, V, out=None):
        """u [n_src] = the transpose of the H map applied to V [n_tgt, 3]."""
        torch = _torch()
        if V.dim() != 2 or V.shape[0] != self.n_tgt:
            raise ValueError(f"V must have shape [{self.n_tgt}, 3]")
        if out is not None and (out.dim() != 1 or out.shape[0] != self.n_src):
            raise ValueError(f"out must have shape [{self.n_src}]")
        u = out if out is not None else torch.empty(self.n_src, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn3_eval_H_adjoint(self._ctx, _dev_ptr(V, "V", (3,)), _dev_ptr(u, "u")))
        return u

    def set_profiling(self, enable=True):
        self._check(_lib.lib().fn3_set_profiling(self._ctx, int(bool(enable))))

    def profile(self):
        """Per-stage event time (ms) and launch counts since profiling was enabled."""
        pr = _lib.Profile()
        self._check(_lib.lib().fn3_get_profile(self._ctx, ctypes.byref(pr)))
        return {name: (pr.ms[i], pr.count[i]) for i, name in enumerate(_lib.STAGES3)}

    def info(self):
        nt, ns, ne, nc = ctypes.c_int64(), ctypes.c_int64(), (ctypes.c_int32 * 3)(), ctypes.c_int32()
        sc = ctypes.c_double()
        self._check(_lib.lib().fn3_get_info(self._ctx, ctypes.byref(nt), ctypes.byref(ns), ctypes.byref(sc), ne,
                                            ctypes.byref(nc)))
        return dict(n_tgt=nt.value, n_src=ns.value, scale=sc.value, win_ext=tuple(ne), near_cells=nc.value)


class Mesh:
    """A P1 triangle mesh on the device (fn_mesh_*): nodes [N, 2] float64, tris [T, 3] int32,
    bedges [E, 2] int32 (domain on the left of each boundary edge)."""

    def __init__(self, nodes, tris, bedges, stream=None):
        torch = _torch()
        L = _lib.lib()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n_nodes, self.n_tris, self.n_bedges = int(nodes.shape[0]), int(tris.shape[0]), int(bedges.shape[0])
        self.n_sources = 3 * self.n_tris + 2 * self.n_bedges
        m = ctypes.c_void_p()
        _lib.check_mesh(L.fn_mesh_create(self.n_nodes, self.n_tris, self.n_bedges,
                                         ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(m)))
        self._mesh = m
        b = ctypes.c_size_t()
        self._check(L.fn_mesh_workspace_size(m, ctypes.byref(b)))
        self._ws = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self._check(L.fn_mesh_set_workspace(m, ctypes.c_void_p(self._ws.data_ptr()), b))
        self._check(L.fn_mesh_set(m, _dev_ptr(nodes, "nodes", (2,)), _dev_ptr(tris, "tris", (3,), torch.int32),
                                  _dev_ptr(bedges, "bedges", (2,), torch.int32) if self.n_bedges else None))

    def __del__(self):
        m = getattr(self, "_mesh", None)
        if m:
            try:
                _lib.lib().fn_mesh_destroy(m)
            except Exception:
                pass
            self._mesh = None

    def _check(self, rc):
        _lib.check_mesh(rc, self._mesh)

    def sources(self):
        torch = _torch()
        x = torch.empty(self.n_sources, 2, dtype=torch.float64, device=self.device)
        w = torch.empty(self.n_sources, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_mesh_sources(self._mesh, _dev_ptr(x, "x", (2,)), _dev_ptr(w, "w")))
        return x, w

    def lumped_mass(self):
        torch = _torch()
        ell = torch.empty(self.n_nodes, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_mesh_lumped_mass(self._mesh, _dev_ptr(ell, "ell")))
        return ell

    def charges(self, M):
        torch = _torch()
        q = torch.empty(self.n_sources, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_mesh_charges(self._mesh, _dev_ptr(M, "M", (2,)), _dev_ptr(q, "q")))
        return q

    def charges_T(self, u):
        torch = _torch()
        out = torch.empty(self.n_nodes, 2, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_mesh_charges_T(self._mesh, _dev_ptr(u, "u"), _dev_ptr(out, "out", (2,))))
        return out

    def p1_gradient(self, phi):
        """Field of the P1 interpolant of nodal phi: per triangle [T, 2] and lumped to the
        nodes [N, 2] (fn_mesh_p1_gradient)."""
        torch = _torch()
        HT = torch.empty(self.n_tris, 2, dtype=torch.float64, device=self.device)
        Hn = torch.empty(self.n_nodes, 2, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_mesh_p1_gradient(self._mesh, _dev_ptr(phi, "phi"), _dev_ptr(HT, "H_tri", (2,)),
                                                   _dev_ptr(Hn, "H_node", (2,))))
        return HT, Hn


class Mesh3:
    """A P1 tetrahedral mesh on the device (fn3_mesh_*): nodes [N, 3] float64, tets [T, 4] int32,
    bfaces [F, 3] int32 with (b - a) x (c - a) pointing out of the domain."""

    def __init__(self, nodes, tets, bfaces, stream=None):
        torch = _torch()
        L = _lib.lib()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n_nodes, self.n_tets, self.n_bfaces = int(nodes.shape[0]), int(tets.shape[0]), int(bfaces.shape[0])
        self.n_sources = 4 * self.n_tets + 3 * self.n_bfaces
        m = ctypes.c_void_p()
        _lib.check_mesh3(L.fn3_mesh_create(self.n_nodes, self.n_tets, self.n_bfaces,
                                           ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(m)))
        self._mesh = m
        b = ctypes.c_size_t()
        self._check(L.fn3_mesh_workspace_size(m, ctypes.byref(b)))
        self._ws = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self._check(L.fn3_mesh_set_workspace(m, ctypes.c_void_p(self._ws.data_ptr()), b))
        self._check(L.fn3_mesh_set(m, _dev_ptr(nodes, "nodes", (3,)), _dev_ptr(tets, "tets", (4,), torch.int32),
                                   _dev_ptr(bfaces, "bfaces", (3,), torch.int32) if self.n_bfaces else None))

    def __del__(self):
        m = getattr(self, "_mesh", None)
        if m:
            try:
                _lib.lib().fn3_mesh_destroy(m)
            except Exception:
                pass
            self._mesh = None

    def _check(self, rc):
        _lib.check_mesh3(rc, self._mesh)

    def sources(self):
        torch = _torch()
        x = torch.empty(self.n_sources, 3, dtype=torch.float64, device=self.device)
        w = torch.empty(self.n_sources, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn3_mesh_sources(self._mesh, _dev_ptr(x, "x", (3,)), _dev_ptr(w, "w")))
        return x, w

    def lumped_mass(self):
        torch = _torch()
        ell = torch.empty(self.n_nodes, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn3_mesh_lumped_mass(self._mesh, _dev_ptr(ell, "ell")))
        return ell

    def charges(self, M):
        torch = _torch()
        if M.dim() != 2 or M.shape[0] != self.n_nodes:
            raise ValueError(f"M must have shape [{self.n_nodes}, 3]")
        q = torch.empty(self.n_sources, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn3_mesh_charges(self._mesh, _dev_ptr(M, "M", (3,)), _dev_ptr(q, "q")))
        return q

    def charges_T(self, u):
        torch = _torch()
        if u.dim() != 1 or u.shape[0] != self.n_sources:
            raise ValueError(f"u must have shape [{self.n_sources}]")
        out = torch.empty(self.n_nodes, 3, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn3_mesh_charges_T(self._mesh, _dev_ptr(u, "u"), _dev_ptr(out, "out", (3,))))
        return out

    def bind(self, solver):
        """Targets = this mesh's nodes, sources = its quadrature points, on the 3D solver."""
        solver._ensure_ws(self.n_nodes, self.n_sources)
        self._check(_lib.lib().fn3_bind_mesh(solver._ctx, self._mesh))
        solver.n_tgt, solver.n_src = self.n_nodes, self.n_sources
        solver._geom_refs = (self,)
        return solver

    def energy(self, solver, M, grad=True):
        """E (a device scalar) and dE/dM [N, 3] (or None) of nodal M through the bound 3D solver."""
        torch = _torch()
        if M.dim() != 2 or M.shape[0] != self.n_nodes:
            raise ValueError(f"M must have shape [{self.n_nodes}, 3]")
        E = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty(self.n_nodes, 3, dtype=torch.float64, device=self.device) if grad else None
        self._check(_lib.lib().fn3_energy(solver._ctx, self._mesh, _dev_ptr(M, "M", (3,)), _dev_ptr(E, "E"),
                                          _dev_ptr(g, "grad", (3,)) if g is not None else None))
        return E, g


def _params(d):
    base = default_params(int(d["grid"]))
    base.update({k: v for k, v in d.items() if v is not None})
    return _lib.Params(grid=int(base["grid"]), m=int(base["m"]), p=int(base["p"]), precision=int(base["precision"]),
                       eps_I=float(base["eps_I"]), eps_B=float(base["eps_B"]), flags=0, n=int(base.get("n") or 0),
                       eps_S=float(base.get("eps_S") or 0.0))


class Batch:
    """Independent problems (fn_batch_*): members' arrays are concatenated; offsets are host
    sequences of B + 1 point counts (CSR).  Calls are ordered on one stream; inside an
    evaluation the members' tasks run over a few lanes (set_lanes)."""

    def __init__(self, params, stream=None):
        torch = _torch()
        L = _lib.lib()
        self.count = len(params)
        arr = (_lib.Params * self.count)(*[_params(dict(d)) for d in params])
        self.params = list(arr)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = ctypes.c_void_p()
        _lib.check_batch(L.fn_batch_create(self.count, arr, ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(b)))
        self._b = b
        self._ws = None

    def __del__(self):
        b = getattr(self, "_b", None)
        if b:
            try:
                _lib.lib().fn_batch_destroy(b)
            except Exception:
                pass
            self._b = None

    def _check(self, rc):
        _lib.check_batch(rc, self._b)

    def set_geometry(self, tgt_off, tgt_xy, src_off, src_xy, src_w, n_surf=None):
        """n_surf: per-member counts of trailing surface sources (None: none)."""
        torch = _torch()
        L = _lib.lib()
        to = (ctypes.c_int64 * (self.count + 1))(*[int(v) for v in tgt_off])
        so = (ctypes.c_int64 * (self.count + 1))(*[int(v) for v in src_off])
        need = ctypes.c_size_t()
        self._check(L.fn_batch_workspace_size(self._b, to, so, ctypes.byref(need)))
        if self._ws is None or self._ws.numel() < need.value:
            self._ws = None
            self._ws = torch.empty(need.value, dtype=torch.uint8, device=self.device)
            self._check(L.fn_batch_set_workspace(self._b, ctypes.c_void_p(self._ws.data_ptr()), need))
        if n_surf is not None:
            nsf = (ctypes.c_int64 * self.count)(*[int(v) for v in n_surf])
            self._check(L.fn_set_geometry_batch_split(self._b, to, _dev_ptr(tgt_xy, "tgt_xy", (2,)), so,
                                                      _dev_ptr(src_xy, "src_xy", (2,)), _dev_ptr(src_w, "src_w"), nsf))
        else:
            self._check(L.fn_set_geometry_batch(self._b, to, _dev_ptr(tgt_xy, "tgt_xy", (2,)), so,
                                                _dev_ptr(src_xy, "src_xy", (2,)), _dev_ptr(src_w, "src_w")))
        self.n_tgt, self.n_src = int(tgt_off[-1]), int(src_off[-1])
        return self

    def _member(self, i):
        if not 0 <= int(i) < self.count:
            raise IndexError(f"member {i} of a batch of {self.count}")
        ctx = ctypes.c_void_p()
        self._check(_lib.lib().fn_batch_member(self._b, int(i), ctypes.byref(ctx)))
        return ctx

    def set_shapes(self, i, **shapes):
        """Kernel work shapes of member i (fn_set_shapes on its context, borrowed with
        fn_batch_member); unnamed fields keep the library default."""
        _set_shapes(self._member(i), shapes)
        return self

    def shapes(self, i):
        """The shapes in effect for member i."""
        return _get_shapes(self._member(i))

    def set_lanes(self, lanes):
        """Streams an evaluation spreads the members' tasks over (fn_batch_set_lanes)."""
        self._check(_lib.lib().fn_batch_set_lanes(self._b, int(lanes)))
        return self

    def set_charges(self, q):
        self._check(_lib.lib().fn_batch_set_charges(self._b, _dev_ptr(q, "q")))
        return self

    def eval(self, out_phi=None, out_H=None):
        torch = _torch()
        p = out_phi if out_phi is not None else torch.empty(self.n_tgt, dtype=torch.float64, device=self.device)
        h = out_H if out_H is not None else torch.empty(self.n_tgt, 2, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_batch_eval(self._b, _dev_ptr(p, "phi"), _dev_ptr(h, "H", (2,))))
        return p, h

    def adjoint_H(self, V, out=None):
        torch = _torch()
        u = out if out is not None else torch.empty(self.n_src, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_batch_eval_H_adjoint(self._b, _dev_ptr(V, "V", (2,)), _dev_ptr(u, "u")))
        return u

    def eval_with_H_adjoint(self, V, out_phi=None, out_H=None, out_u=None):
        """phi, H = eval() and u = adjoint_H(V) in one call, every member's two directions
        in one schedule over the lanes (fn_batch_eval_with_H_adjoint); returns (phi, H, u)."""
        torch = _torch()
        p = out_phi if out_phi is not None else torch.empty(self.n_tgt, dtype=torch.float64, device=self.device)
        h = out_H if out_H is not None else torch.empty(self.n_tgt, 2, dtype=torch.float64, device=self.device)
        u = out_u if out_u is not None else torch.empty(self.n_src, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_batch_eval_with_H_adjoint(self._b, _dev_ptr(p, "phi"), _dev_ptr(h, "H", (2,)),
                                                            _dev_ptr(V, "V", (2,)), _dev_ptr(u, "u")))
        return p, h, u

    def adjoint_phi(self, v, out=None):
        torch = _torch()
        u = out if out is not None else torch.empty(self.n_src, dtype=torch.float64, device=self.device)
        self._check(_lib.lib().fn_batch_eval_phi_adjoint(self._b, _dev_ptr(v, "v"), _dev_ptr(u, "u")))
        return u


class Graph:
    """A HIP graph of library calls recorded on one (non-default) stream (fn_graph_*)."""

    def __init__(self):
        self._g = None

    def __del__(self):
        g = getattr(self, "_g", None)
        if g:
            try:
                _lib.lib().fn_graph_destroy(g)
            except Exception:
                pass
            self._g = None

    @contextlib.contextmanager
    def capture(self, stream):
        L = _lib.lib()
        if self._g:
            L.fn_graph_destroy(self._g)
            self._g = None
        sp = ctypes.c_void_p(stream.cuda_stream)
        _lib.check_graph(L.fn_graph_begin(sp))
        ok = False
        try:
            yield self
            ok = True
        finally:
            g = ctypes.c_void_p()
            rc = L.fn_graph_end(sp, ctypes.byref(g))
            if ok:
                _lib.check_graph(rc)
                self._g = g
            elif g:
                L.fn_graph_destroy(g)

    def launch(self, stream):
        if not self._g:
            raise FemNfftError(2, "nothing captured")
        _lib.check_graph(_lib.lib().fn_graph_launch(self._g, ctypes.c_void_p(stream.cuda_stream)))


def _demag_energy_class():
    torch = _torch()

    class DemagEnergy(torch.autograd.Function):
        """E(M) = -1/2 sum_i l_i M_i . H_i(M) with its exact gradient from the library
        (fn_energy); the solver must be bound to the mesh (Solver.bind_mesh)."""

        @staticmethod
        def forward(ctx, M, solver, mesh):
            if getattr(solver, "_mesh", None) is not mesh:
                raise FemNfftError(2, "solver is not bound to this mesh (Solver.bind_mesh)")
            Mc = M.detach().contiguous()
            E, g = solver.energy(Mc, grad=ctx.needs_input_grad[0])
            ctx.save_for_backward(g if g is not None else E)
            return E

        @staticmethod
        def backward(ctx, gE):
            (g,) = ctx.saved_tensors
            return gE * g, None, None

    return DemagEnergy


def __getattr__(name):
    if name == "DemagEnergy":
        cls = _demag_energy_class()
        globals()["DemagEnergy"] = cls
        return cls
    raise AttributeError(name)
