"""ctypes declarations for libfemnfft.so (argument marshalling only).

The library is built in-tree by paper_0807_2387_amd.build; importing this module
raises if it is missing, so no code path can silently run without it.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfemnfft.so")

FN_OK, FN_E_INVAL, FN_E_STATE, FN_E_DOMAIN, FN_E_NOMEM, FN_E_DEVICE, FN_E_UNSUPPORTED = range(7)
FN_FP64, FN_FP32_MIXED = 0, 1
FN_NOALLOC_SCRATCH_BYTES = 64 << 20  # static scratch of fn_eval_noalloc per device
ERR_NAMES = {0: "FN_OK", 1: "FN_E_INVAL", 2: "FN_E_STATE", 3: "FN_E_DOMAIN", 4: "FN_E_NOMEM",
             5: "FN_E_DEVICE", 6: "FN_E_UNSUPPORTED"}

# exported C-ABI symbols (include/femnfft.h)
SYMBOLS = (
    "fn_params_default", "fn_params_auto", "fn_create", "fn_destroy", "fn_workspace_size", "fn_set_workspace",
    "fn_set_geometry", "fn_set_geometry_split", "fn_set_charges", "fn_eval", "fn_eval_phi", "fn_eval_H",
    "fn_eval_phi_adjoint", "fn_eval_H_adjoint", "fn_eval_with_H_adjoint", "fn_eval_noalloc", "fn_get_info",
    "fn_last_error",
    "fn_set_profiling", "fn_get_profile", "fn_set_shapes", "fn_get_shapes",
    "fn_mesh_create", "fn_mesh_destroy", "fn_mesh_workspace_size", "fn_mesh_set_workspace", "fn_mesh_set",
    "fn_mesh_sources", "fn_mesh_lumped_mass", "fn_mesh_charges", "fn_mesh_charges_T", "fn_bind_mesh",
    "fn_energy", "fn_bind_mesh_sources", "fn_energy_charge", "fn_mesh_p1_gradient", "fn_mesh_last_error",
    "fn_batch_create", "fn_batch_destroy", "fn_batch_workspace_size", "fn_batch_set_workspace",
    "fn_set_geometry_batch", "fn_set_geometry_batch_split", "fn_batch_set_lanes", "fn_batch_set_charges", "fn_batch_eval", "fn_batch_eval_H_adjoint", "fn_batch_eval_with_H_adjoint",
    "fn_batch_eval_phi_adjoint", "fn_batch_member", "fn_batch_last_error",
    "fn_graph_begin", "fn_graph_end", "fn_graph_launch", "fn_graph_destroy", "fn_graph_last_error",
    "fn3_create", "fn3_destroy", "fn3_workspace_size", "fn3_set_workspace", "fn3_set_geometry", "fn3_set_charges",
    "fn3_eval", "fn3_eval_H_adjoint", "fn3_get_info", "fn3_set_profiling", "fn3_get_profile", "fn3_last_error",
    "fn3_mesh_create", "fn3_mesh_destroy", "fn3_mesh_workspace_size", "fn3_mesh_set_workspace", "fn3_mesh_set",
    "fn3_mesh_sources", "fn3_mesh_lumped_mass", "fn3_mesh_charges", "fn3_mesh_charges_T", "fn3_bind_mesh",
    "fn3_energy", "fn3_mesh_last_error",
)

STAGES = ("charges", "spread", "fold", "rows_fwd", "cols", "rows_inv", "gather", "near",
          "a_values", "a_spread", "a_fold", "a_rows_fwd", "a_cols", "a_rows_inv", "a_gather", "a_near",
          "near_surf", "a_near_surf")
STAGES3 = ("charges", "spread", "fft", "multiply", "ifft", "gather", "near",
           "a_values", "a_spread", "a_fft", "a_multiply", "a_ifft", "a_gather", "a_near")


class Params(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("m", ctypes.c_int32), ("p", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("eps_I", ctypes.c_double), ("eps_B", ctypes.c_double),
                ("flags", ctypes.c_int32), ("n", ctypes.c_int32), ("eps_S", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("centre", ctypes.c_double * 2), ("scale", ctypes.c_double),
                ("n_tgt", ctypes.c_int64), ("n_src", ctypes.c_int64),
                ("win_lo", ctypes.c_int32 * 2), ("win_ext", ctypes.c_int32 * 2),
                ("tiles", ctypes.c_int32 * 2), ("near_cells", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t), ("near_pairs", ctypes.c_int64),
                ("n_surf", ctypes.c_int64), ("near_pairs_surf", ctypes.c_int64),
                ("near_cells_surf", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Shapes(ctypes.Structure):
    _fields_ = [("spread_groups", ctypes.c_int32),
                ("near_fwd_bx", ctypes.c_int32), ("near_fwd_by", ctypes.c_int32), ("near_fwd_cap", ctypes.c_int32),
                ("near_adj_bx", ctypes.c_int32), ("near_adj_by", ctypes.c_int32), ("near_adj_cap", ctypes.c_int32),
                ("tile", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(STAGES)), ("count", ctypes.c_int64 * len(STAGES)),
                ("dropped", ctypes.c_int64)]


class FemNfftError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_0807_2387_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    sig = {
        "fn_params_default": ([ctypes.POINTER(Params), I32], ctypes.c_int),
        "fn_params_auto": ([I64, I64, I32, ctypes.POINTER(Params)], ctypes.c_int),
        "fn_create": ([ctypes.POINTER(Params), P, ctypes.POINTER(P)], ctypes.c_int),
        "fn_destroy": ([P], ctypes.c_int),
        "fn_workspace_size": ([P, I64, I64, ctypes.POINTER(SZ)], ctypes.c_int),
        "fn_set_workspace": ([P, P, SZ], ctypes.c_int),
        "fn_set_geometry": ([P, I64, P, I64, P, P], ctypes.c_int),
        "fn_set_geometry_split": ([P, I64, P, I64, P, P, I64], ctypes.c_int),
        "fn_set_charges": ([P, P], ctypes.c_int),
        "fn_eval": ([P, P, P], ctypes.c_int),
        "fn_eval_phi": ([P, P], ctypes.c_int),
        "fn_eval_H": ([P, P], ctypes.c_int),
        "fn_eval_phi_adjoint": ([P, P, P], ctypes.c_int),
        "fn_eval_H_adjoint": ([P, P, P], ctypes.c_int),
        "fn_eval_with_H_adjoint": ([P, P, P, P, P], ctypes.c_int),
        "fn_eval_noalloc": ([P, I64, P, I64, P, P, I64, P, P, P], ctypes.c_int),
        "fn_get_info": ([P, ctypes.POINTER(Info)], ctypes.c_int),
        "fn_last_error": ([P], ctypes.c_char_p),
        "fn_set_profiling": ([P, ctypes.c_int], ctypes.c_int),
        "fn_get_profile": ([P, ctypes.POINTER(Profile)], ctypes.c_int),
        "fn_set_shapes": ([P, ctypes.POINTER(Shapes)], ctypes.c_int),
        "fn_get_shapes": ([P, ctypes.POINTER(Shapes)], ctypes.c_int),
        "fn_mesh_create": ([I64, I64, I64, P, ctypes.POINTER(P)], ctypes.c_int),
        "fn_mesh_destroy": ([P], ctypes.c_int),
        "fn_mesh_workspace_size": ([P, ctypes.POINTER(SZ)], ctypes.c_int),
        "fn_mesh_set_workspace": ([P, P, SZ], ctypes.c_int),
        "fn_mesh_set": ([P, P, P, P], ctypes.c_int),
        "fn_mesh_sources": ([P, P, P], ctypes.c_int),
        "fn_mesh_lumped_mass": ([P, P], ctypes.c_int),
        "fn_mesh_charges": ([P, P, P], ctypes.c_int),
        "fn_mesh_charges_T": ([P, P, P], ctypes.c_int),
        "fn_bind_mesh": ([P, P], ctypes.c_int),
        "fn_energy": ([P, P, P, P, P], ctypes.c_int),
        "fn_bind_mesh_sources": ([P, P], ctypes.c_int),
        "fn_energy_charge": ([P, P, P, P, P, P], ctypes.c_int),
        "fn_mesh_p1_gradient": ([P, P, P, P], ctypes.c_int),
        "fn_mesh_last_error": ([P], ctypes.c_char_p),
        "fn_batch_create": ([I32, ctypes.POINTER(Params), P, ctypes.POINTER(P)], ctypes.c_int),
        "fn_batch_destroy": ([P], ctypes.c_int),
        "fn_batch_workspace_size": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(SZ)], ctypes.c_int),
        "fn_batch_set_workspace": ([P, P, SZ], ctypes.c_int),
        "fn_set_geometry_batch": ([P, ctypes.POINTER(I64), P, ctypes.POINTER(I64), P, P], ctypes.c_int),
        "fn_set_geometry_batch_split": ([P, ctypes.POINTER(I64), P, ctypes.POINTER(I64), P, P, ctypes.POINTER(I64)],
                                        ctypes.c_int),
        "fn_batch_set_lanes": ([P, I32], ctypes.c_int),
        "fn_batch_set_charges": ([P, P], ctypes.c_int),
        "fn_batch_eval": ([P, P, P], ctypes.c_int),
        "fn_batch_eval_H_adjoint": ([P, P, P], ctypes.c_int),
        "fn_batch_eval_with_H_adjoint": ([P, P, P, P, P], ctypes.c_int),
        "fn_batch_eval_phi_adjoint": ([P, P, P], ctypes.c_int),
        "fn_batch_member": ([P, I32, ctypes.POINTER(P)], ctypes.c_int),
        "fn_batch_last_error": ([P], ctypes.c_char_p),
        "fn_graph_begin": ([P], ctypes.c_int),
        "fn_graph_end": ([P, ctypes.POINTER(P)], ctypes.c_int),
        "fn_graph_launch": ([P, P], ctypes.c_int),
        "fn_graph_destroy": ([P], ctypes.c_int),
        "fn_graph_last_error": ([], ctypes.c_char_p),
        "fn3_create": ([ctypes.POINTER(Params), P, ctypes.POINTER(P)], ctypes.c_int),
        "fn3_destroy": ([P], ctypes.c_int),
        "fn3_workspace_size": ([P, I64, I64, ctypes.POINTER(SZ)], ctypes.c_int),
        "fn3_set_workspace": ([P, P, SZ], ctypes.c_int),
        "fn3_set_geometry": ([P, I64, P, I64, P, P], ctypes.c_int),
        "fn3_set_charges": ([P, P], ctypes.c_int),
        "fn3_eval": ([P, P, P], ctypes.c_int),
        "fn3_eval_H_adjoint": ([P, P, P], ctypes.c_int),
        "fn3_get_info": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(I32), ctypes.POINTER(I32)], ctypes.c_int),
        "fn3_set_profiling": ([P, ctypes.c_int], ctypes.c_int),
        "fn3_get_profile": ([P, ctypes.POINTER(Profile)], ctypes.c_int),
        "fn3_last_error": ([P], ctypes.c_char_p),
        "fn3_mesh_create": ([I64, I64, I64, P, ctypes.POINTER(P)], ctypes.c_int),
        "fn3_mesh_destroy": ([P], ctypes.c_int),
        "fn3_mesh_workspace_size": ([P, ctypes.POINTER(SZ)], ctypes.c_int),
        "fn3_mesh_set_workspace": ([P, P, SZ], ctypes.c_int),
        "fn3_mesh_set": ([P, P, P, P], ctypes.c_int),
        "fn3_mesh_sources": ([P, P, P], ctypes.c_int),
        "fn3_mesh_lumped_mass": ([P, P], ctypes.c_int),
        "fn3_mesh_charges": ([P, P, P], ctypes.c_int),
        "fn3_mesh_charges_T": ([P, P, P], ctypes.c_int),
        "fn3_bind_mesh": ([P, P], ctypes.c_int),
        "fn3_energy": ([P, P, P, P, P], ctypes.c_int),
        "fn3_mesh_last_error": ([P], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(rc, ctx=None):
    if rc != FN_OK:
        msg = lib().fn_last_error(ctx)
        raise FemNfftError(rc, msg.decode() if msg else "")


def check_batch(rc, batch=None):
    if rc != FN_OK:
        msg = lib().fn_batch_last_error(batch)
        raise FemNfftError(rc, msg.decode() if msg else "")


def check_graph(rc):
    if rc != FN_OK:
        msg = lib().fn_graph_last_error()
        raise FemNfftError(rc, msg.decode() if msg else "")


def check_mesh(rc, mesh=None):
    if rc != FN_OK:
        msg = lib().fn_mesh_last_error(mesh)
        raise FemNfftError(rc, msg.decode() if msg else "")


def check_mesh3(rc, mesh=None):
    if rc != FN_OK:
        msg = lib().fn3_mesh_last_error(mesh)
        raise FemNfftError(rc, msg.decode() if msg else "")


def check3(rc, ctx=None):
    if rc != FN_OK:
        msg = lib().fn3_last_error(ctx)
        raise FemNfftError(rc, msg.decode() if msg else "")
