"""Autotuner of the kernel work shapes (fn_set_shapes), with a JSON cache.

The library's kernels take their tile and bin shapes at run time: the spread/gather tile
edge, the register row groups of the FP32 spread, and the near field's home block shape and
LDS staging capacity per direction.  tune() times candidates on the caller's own data with
the library's stage events (fn_set_profiling / fn_get_profile) and keeps the fastest, one
kernel family at a time (coordinate search; the families touch different stages):

    family          candidates                                    stages timed
    tile            16, 32                                        spread, fold, gather (both directions)
    spread_groups   1, 2, 3 (at most 144 register sums a group)   spread, a_spread
    near_fwd        32 x 8, 16 x 16, 64 x 4 home cells;           near
                    staging 512, 768, 1024, 1536 points
    near_adj        the same shapes; staging 384, 512, 768, 1024  a_near

Every candidate runs set_charges + eval + H adjoint `reps` times one direction after the
other; the median of its stage times decides.  The result is keyed by what sets the best
shape -- grid, window half-width, regularization degree, precision, bandwidth, near radius
in cells, points per grid cell of the data window and the GPU architecture -- and stored in
a JSON file: $FEMNFFT_TUNE_CACHE, else ~/.cache/femnfft/tune.json.  Entries measured on
MI355X for the bench workloads (the square and the 64-mesh batch's members) ship with the
package (tune_cache.json) and are read first.

    shapes = tune.apply(solver, q, V)       # cached shapes, or tune now and cache them

A batch's members are tuned one distinct key at a time, each on a standalone solver holding
that member's points, and the winners are set on every member with that key (apply_batch).
"""
from __future__ import annotations

import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
PACKAGED = os.path.join(HERE, "tune_cache.json")

NEAR_DIMS = ((32, 8), (16, 16), (64, 4))
CAPS_FWD = (512, 768, 1024, 1536)
CAPS_ADJ = (384, 512, 768, 1024)


def cache_path():
    p = os.environ.get("FEMNFFT_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "femnfft", "tune.json")


def _load(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def lookup(key):
    """Cached shapes for key: the user cache first, then the packaged entries."""
    for path in (cache_path(), PACKAGED):
        ent = _load(path).get(key)
        if ent:
            return ent.get("shapes")
    return None


def store(key, shapes, record=None, path=None):
    path = path or cache_path()
    d = _load(path)
    d[key] = {"shapes": shapes, **(record or {})}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def arch():
    import torch
    try:
        return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def key_of(solver):
    """Cache key of a solver whose geometry is set."""
    prm = solver.params
    info = solver.info()
    ex, ey = info["win_ext"]
    ppc = (info["n_tgt"] + info["n_src"]) / max(1, ex * ey)
    # points per cell in steps of 2^(1/4): shapes change slowly with density
    ppc_b = round(4 * math.log2(ppc)) / 4 if ppc > 0 else -99
    n = prm.n or prm.grid // 2
    return (f"{arch()}|G{prm.grid}|n{n}|m{prm.m}|p{prm.p}|"
            f"{'fp64' if prm.precision == 0 else 'fp32'}|rn{info['near_cells']}|"
            f"ppc2^{ppc_b:g}|surf{1 if info['n_surf'] else 0}")


def _stage_times(solver, q, V, reps):
    import torch
    torch.cuda.synchronize()
    runs = []
    for _ in range(reps):
        solver.set_profiling(True)
        solver.set_charges(q)
        solver.eval()
        solver.adjoint_H(V)
        torch.cuda.synchronize()
        runs.append({k: v[0] for k, v in solver.profile().items()})
        solver.set_profiling(False)
    out = {}
    for k in runs[0]:
        vals = sorted(r[k] for r in runs)
        out[k] = vals[len(vals) // 2]
    return out


def _score(times, stages):
    return sum(times.get(s, 0.0) for s in stages)


def tune(solver, q, V, reps=3, log=None):
    """Search the shapes on the solver's current geometry with charges q and adjoint input V
    (device tensors).  Leaves the best shapes set on the solver and returns them."""
    best = dict(solver.shapes())
    m = solver.params.m
    trace = []
    import torch
    for _ in range(2):  # first launches of the pipeline (module load, LDS attributes) are not timed
        solver.set_charges(q)
        solver.eval()
        solver.adjoint_H(V)
    torch.cuda.synchronize()

    def trial(cand, stages):
        solver.set_shapes(**cand)
        solver.set_charges(q)  # warm-up of the new kernels
        solver.eval()
        solver.adjoint_H(V)
        t = _score(_stage_times(solver, q, V, reps), stages)
        trace.append((dict(cand), stages[0], round(t, 4)))
        if log:
            log(f"tune {stages[0]:8s} {cand} -> {t:.4f} ms")
        return t

    # each family's candidates vary its own fields around the winners so far
    fams = [
        (lambda b: [dict(b, tile=t) for t in (32, 16)],
         ("spread", "fold", "gather", "a_spread", "a_fold", "a_gather")),
        (lambda b: [dict(b, spread_groups=g) for g in (1, 2, 3) if 2 * -(-m // g) * 2 * m <= 144],
         ("spread", "a_spread")),
        (lambda b: [dict(b, near_fwd_bx=bx, near_fwd_by=by, near_fwd_cap=c) for bx, by in NEAR_DIMS
                    for c in CAPS_FWD], ("near",)),
        (lambda b: [dict(b, near_adj_bx=bx, near_adj_by=by, near_adj_cap=c) for bx, by in NEAR_DIMS
                    for c in CAPS_ADJ], ("a_near",)),
    ]
    for cands, stages in fams:
        results = [(trial(c, stages), c) for c in cands(best)]
        best = min(results, key=lambda r: r[0])[1]
    solver.set_shapes(**best)
    return best, trace


def apply(solver, q, V, reps=3, log=None, retune=False):
    """Set the cached shapes for this solver's geometry, or tune and cache them.
    Returns (shapes, key, tuned_now)."""
    key = key_of(solver)
    shapes = None if retune else lookup(key)
    if shapes:
        solver.set_shapes(**shapes)
        return shapes, key, False
    shapes, trace = tune(solver, q, V, reps=reps, log=log)
    store(key, shapes, {"trials": len(trace)})
    return shapes, key, True


def apply_batch(batch, tgt_off, tgt_xy, src_off, src_xy, src_w, q, V, n_surf=None, reps=3, log=None,
                retune=False):
    """Set cached or freshly tuned shapes on every member of a Batch whose geometry is set
    from these arrays (its concatenated inputs, host offsets).  Members that share a cache key
    share one search.  Returns [(key, shapes, tuned_now)] per member."""
    from . import Solver
    done, out = {}, []
    for i, prm in enumerate(batch.params):
        t0, t1, s0, s1 = int(tgt_off[i]), int(tgt_off[i + 1]), int(src_off[i]), int(src_off[i + 1])
        S = Solver(grid=prm.grid, m=prm.m, p=prm.p, eps_I=prm.eps_I, eps_B=prm.eps_B, precision=prm.precision,
                   n=prm.n, eps_S=prm.eps_S)
        S.set_geometry(tgt_xy[t0:t1], src_xy[s0:s1], src_w[s0:s1], n_surf=int(n_surf[i]) if n_surf is not None else 0)
        key = key_of(S)
        if key in done:
            shapes, now = done[key], False
        else:
            shapes, _, now = apply(S, q[s0:s1], V[t0:t1], reps=reps, log=log, retune=retune)
            done[key] = shapes
        del S
        batch.set_shapes(i, **shapes)
        out.append((key, shapes, now))
        if log:
            log(f"member {i}: {key} {'searched' if now else 'cached'} {shapes}")
    return out
