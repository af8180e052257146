#!/usr/bin/env python3
"""Throughput of the FEM-NFFT fast summation, forward + adjoint, on one MI355X.

One step = set_charges(q) + eval(phi, H) + H adjoint(V) over the whole point set
(every stage of the hot path: spread, FFTs with the kernel multiply, gather,
FP64 near field and final sum, and the transposed pipeline).  The forward and the
adjoint run at the same time on two streams (fn_eval_with_H_adjoint; --no-overlap
runs them one after the other).  Inputs are resident in HBM before the timed region.

Workload (default): rounded square of side 4 (corner radius 1/2), about 2^24
jittered-lattice targets and 2^24 + 31k sources (cell points with charge
-div M, boundary Gauss points with M.n), M a unit field whose angle is a sum of
32 random cosine modes; FP32-mixed path, FFT grid 8192^2, bandwidth n = 6144,
Kaiser-Bessel m = 5, regularization degree p = 5; the volume sources use the
near radius eps_I = 3.25/n, the 31k boundary Gauss points (surface sources) their
own eps_S = 11/n (fn_set_geometry_split); boundary regularization zone eps_B = 1/32
(the torus map scales the workload to a distance of at most 1/2 - eps_B).

Prints ONE JSON line (rank 0).  `value` = (N_src + N_tgt) / (seconds per step).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP64_VEC_TFLOPS = 78.6
FP32_VEC_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 24, help="about this many targets (and sources)")
    ap.add_argument("--grid", type=int, default=8192)
    ap.add_argument("--m", type=int, default=6)
    ap.add_argument("--p", type=int, default=5)
    ap.add_argument("--c", type=float, default=3.25,
                    help="eps_I = c / n for the volume sources (all sources when --cs 0)")
    ap.add_argument("--cs", type=float, default=11.0,
                    help="surface sources (the boundary Gauss points) get eps_S = cs / n; 0: one class")
    ap.add_argument("--eps-b", type=float, default=1 / 32,
                    help="width of the boundary regularization zone in torus units (the library's default is 1/16)")
    ap.add_argument("--band", type=int, default=None,
                    help="bandwidth n (default 3 grid/4, oversampling 4/3; 0 means grid/2)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 GPU path comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg and the sampled accuracy check")
    ap.add_argument("--no-c3", action="store_true",
                    help="square2d: skip the 64-mesh batch record that the default run adds to its line")
    ap.add_argument("--samples", type=int, default=1536, help="sampled targets/sources for the O1 check")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the forward and the H adjoint one after the other on one stream instead of "
                         "at the same time (fn_eval_with_H_adjoint)")
    ap.add_argument("--shapes", type=str, default=None,
                    help="kernel work shapes as JSON (fn_set_shapes fields), e.g. '{\"spread_groups\": 1}'; "
                         "default: the autotuner's cache entry for this workload, else the library defaults")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default shapes instead of the autotuner's (cached, or tuned before the timed region)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one elementwise kernel over 256 MiB (read and write) before the timed region, "
                         "as the byte-counter calibration for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--workload", choices=("square2d", "ball3d", "disk_c1", "ellipse_c2", "batch_c3", "annulus_c4"),
                    default="square2d",
                    help="square2d: the 2D rounded square (default); ball3d: the 3D path (fn3_*, G = 1/(4 pi r)) "
                         "on a ball lattice, options --K, --grid3, --m3, --p3, --c3; disk_c1, ellipse_c2, batch_c3, "
                         "annulus_c4: the other configurations (a disk of 2k nodes, an ellipse of 50k nodes, a batch "
                         "of 64 meshes, an annulus of 1M nodes), each through the GPU FEM front")
    ap.add_argument("--K", type=int, default=64, help="ball3d: lattice cells across the ball")
    ap.add_argument("--grid3", type=int, default=256)
    ap.add_argument("--m3", type=int, default=4)
    ap.add_argument("--p3", type=int, default=6)
    ap.add_argument("--band3", type=int, default=176, help="ball3d: bandwidth n (0: grid3/2)")
    ap.add_argument("--c3", type=float, default=5.5, help="ball3d: eps_I = c3 / n")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library evaluates one point set per device and has "
              "no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_0807_2387_amd as fn

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload == "ball3d":
        return main_3d(args, torch, synth, fn, dev)
    if args.workload != "square2d":
        return main_configs(args, torch, synth, fn, dev)
    t0 = time.time()
    d = synth.rounded_square_cloud(N=args.n, seed=synth.SEED_BASE + 4)
    y, x, w, q = d["y"], d["x"], d["w"], d["q"]
    V = (d["h"] ** 2) * d["M_tgt"]          # l_i M_i with the lattice cell area as nodal mass
    nt, ns = len(y), len(x)
    log(f"workload: {nt} targets, {ns} sources (synth {time.time() - t0:.1f}s)")
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ty, tx, tw, tq, tV = tt(y), tt(x), tt(w), tt(q), tt(V)
    if args.band is None:
        args.band = 3 * args.grid // 4
    nband = args.band or args.grid // 2
    eps_I = args.c / nband
    eps_S = args.cs / nband if args.cs else 0.0
    n_surf = int(np.sum(w != d["h"] ** 2)) if args.cs else 0  # boundary points come last
    if n_surf:
        assert np.all(w[ns - n_surf:] != d["h"] ** 2)

    def run(precision, steps, warmup, profile):
        S = fn.Solver(grid=args.grid, m=args.m, p=args.p, eps_I=eps_I, precision=precision, n=args.band,
                      eps_S=eps_S, eps_B=args.eps_b)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        S.set_geometry(ty, tx, tw, n_surf=n_surf)
        torch.cuda.synchronize()
        t_geom = time.perf_counter() - g0
        # kernel work shapes: given, or the autotuner's (a cache hit, or a search on this data
        # before the timed region)
        tune_rec = {"source": "library defaults"}
        if args.shapes:
            S.set_shapes(**json.loads(args.shapes))
            tune_rec = {"source": "--shapes"}
        elif not args.no_tune:
            from paper_0807_2387_amd import tune
            t1 = time.perf_counter()
            _, key, now = tune.apply(S, tq, tV, log=log)
            tune_rec = {"source": "autotuner, searched now" if now else "autotuner cache", "key": key,
                        "search_s": round(time.perf_counter() - t1, 2) if now else 0.0}
        phi = torch.empty(nt, dtype=torch.float64, device=dev)
        H = torch.empty(nt, 2, dtype=torch.float64, device=dev)
        u = torch.empty(ns, dtype=torch.float64, device=dev)

        def step():
            S.set_charges(tq)
            if args.no_overlap:
                S.eval(out_phi=phi, out_H=H)
                S.adjoint_H(tV, out=u)
            else:
                S.eval_with_H_adjoint(tV, out_phi=phi, out_H=H, out_u=u)

        for _ in range(warmup):
            step()
        if args.calib_copy and profile:
            src = torch.ones(64 << 20, dtype=torch.float32, device=dev)  # 256 MiB
            dst = torch.empty_like(src)
            torch.add(src, 1.0, out=dst)
            del src, dst
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - a
        prof = None
        if profile:
            # kernel durations: HIP events around every stage, recorded on the stream the
            # stage runs on, over `steps` steps with the two directions one after the other
            # (with the directions overlapped an event span would also hold the wait for CUs
            # that the other direction's kernels occupy)
            S.set_profiling(True)
            for _ in range(steps):
                S.set_charges(tq)
                S.eval(out_phi=phi, out_H=H)
                S.adjoint_H(tV, out=u)
            torch.cuda.synchronize()
            prof = S.profile()
            S.set_profiling(False)
        info = S.info()
        return dict(sec=el / steps, t_geom=t_geom, prof=prof, info=info, phi=phi, H=H, u=u, S=S,
                    shapes=S.shapes(), tune=tune_rec)

    r = run(fn.FN_FP32_MIXED, args.steps, args.warmup, True)
    r["info"]["tile"] = r["shapes"]["tile"]
    ms = r["sec"] * 1e3
    value = (nt + ns) / r["sec"]
    log(f"FP32-mixed: {ms:.3f} ms/step, {value:.4e} points/s, set_geometry {r['t_geom'] * 1e3:.1f} ms")
    stages = {k: v[0] / max(args.steps, 1) for k, v in r["prof"].items() if v[1]}
    log(f"  kernel time per step, the two directions one after the other: {sum(stages.values()):.3f} ms")
    for k, v in sorted(stages.items(), key=lambda kv: -kv[1]):
        log(f"  {k:12s} {v:9.3f} ms/step")

    # dominant kernel (the largest kernel time per step) and the roofline of every stage
    dom = max(stages, key=stages.get)
    per_launch = lambda k: stages[k] / (r["prof"][k][1] / max(args.steps, 1))
    roof = roofline(dom, per_launch(dom), None, args, r["info"], nt, ns)
    roof_stages = {k: {kk: vv for kk, vv in roofline(k, per_launch(k), None, args, r["info"], nt, ns).items()
                       if kk in ("bound", "achieved", "unit", "frac", "ms_per_launch")}
                   for k in stages if k not in ("near_surf", "a_near_surf")}
    sg = [k for k in ("spread", "gather", "a_spread", "a_gather") if k in stages]
    sg_bytes = sum(roofline(k, per_launch(k), None, args, r["info"], nt, ns)["algorithmic_bytes_per_launch"]
                   * r["prof"][k][1] / max(args.steps, 1) for k in sg)
    sg_ms = sum(stages[k] for k in sg)
    spread_gather = {"stages": sg, "algorithmic_bytes_per_step": sg_bytes, "ms_per_step": sg_ms,
                     "achieved": sg_bytes / (sg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sg_bytes / (sg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    out = {
        "metric": "source+target points/s for forward+adjoint fast summation at <=1e-6 rel L2 vs FP64",
        "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "rounded square side 4, jittered lattice, 32-mode smooth M",
                   "n_tgt": nt, "n_src": ns, "grid": args.grid, "bandwidth": nband, "m": args.m, "p": args.p,
                   "eps_I": eps_I, "eps_S": eps_S, "n_surf": n_surf, "precision": "fp32_mixed",
                   "eps_B": args.eps_b,
                   "overlap": not args.no_overlap,
                   "parallelism": "single_gpu",
                   "near_field": "FP64 offsets, polynomial and sums; FP32 ln x and 1/x per pair",
                   "shapes": r["shapes"], "shapes_from": r["tune"]},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "stages_ms_from": "HIP events per stage on its stream, the two directions one after the other",
        "set_geometry_ms": r["t_geom"] * 1e3,
        "roofline": roof,
        "roofline_stages": roof_stages,
        "spread_gather_hbm": spread_gather,
    }

    if not args.no_cpu:
        err, cpu = accuracy_and_cpu(d, r, args, nt, ns)
        out["rel_l2_vs_fp64_oracle"] = err
        out["cpu_baseline"] = cpu
        out["cpu_fastsum"] = cpu_fastsum(args)
    else:
        out["cpu_baseline"] = None

    phi32, H32, u32 = r["phi"], r["H"], r["u"]
    del r
    if not args.no_fp64:
        torch.cuda.empty_cache()
        f = run(fn.FN_FP64, max(2, args.steps // 3), 1, False)
        out["fp64_path"] = {"ms_per_step": f["sec"] * 1e3, "points_per_s": (nt + ns) / f["sec"],
                            "speedup_of_fp32_mixed": f["sec"] / (ms * 1e-3)}
        rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        out["fp32_vs_fp64_path_rel_l2"] = {"phi": rel(phi32, f["phi"]), "H": rel(H32, f["H"]),
                                           "HT": rel(u32, f["u"])}
        del f
    if not args.no_c3:
        # the batch configuration beside the headline one (its own record, not part of value)
        del ty, tx, tw, tq, tV, phi32, H32, u32
        torch.cuda.empty_cache()
        c3_ms, c3_pts, c3_cfg = batch_c3_step(args, torch, synth, fn, dev)
        out["batch_c3"] = {"metric": "nodes + quadrature points per second, one step", "value": c3_pts / (c3_ms * 1e-3),
                           "unit": "points/s", "ms_per_step": c3_ms, "steps": args.steps, "config": c3_cfg}
        log(f"batch_c3: {c3_ms:.3f} ms per step, {c3_pts / (c3_ms * 1e-3):.3e} points/s")
    print(json.dumps(out), flush=True)


# Near-field flops per interacting pair (FMA = 2 flops; an FP32 log2 or reciprocal = 1;
# integer work, conversions, compares and selects are not counted):
#   forward (phi and H): offsets 4, r^2 3, x 1, U and U' by synthetic division
#     2(p-1) + 2(p-2), ln x, 1/x, phi share and its sum 4, field factor 3, H sums 4;
#   adjoint (H^T): offsets 4, r^2 3, x 1, U' by Horner 2(p-2), 1/x, factor 2, V.d 3, sum 2.
# In the FP64 path ln x costs 38 (reduction, a Newton-refined reciprocal, 9-term series)
# and 1/x costs 9 (estimate and two Newton steps).
def near_flops_per_pair(stage, p, f32=True):
    ln, rc = (1, 1) if f32 else (38, 9)
    if stage == "near":
        return 4 + 3 + 1 + 2 * (p - 1) + 2 * (p - 2) + ln + rc + 4 + 3 + 4
    return 4 + 3 + 1 + 2 * (p - 2) + rc + 2 + 3 + 2


def roofline(stage, ms_per_launch, calls, args, info, nt, ns):
    """Roofline of the dominant stage.  Near field: FP64 flops per interacting pair times the
    pair count, against the FP64 vector peak.  Grid stages: the bytes they must move at least
    (points' cell, fractions and values once, grid cells once per field), against HBM peak."""
    G, m = args.grid, args.m
    ex, ey = info["win_ext"]
    cells = ex * ey
    sec = ms_per_launch * 1e-3
    nh = (args.band or G // 2) // 2
    if stage in ("near", "a_near"):
        pairs = info["near_pairs"]
        fl = near_flops_per_pair(stage, args.p, f32=True)
        ach = pairs * fl / sec / 1e12
        nb = args.band or G // 2
        traffic = counter_traffic("k_near<0" if stage == "near" else "k_near<1", nb, args.c / nb, args.eps_b,
                                  args.n)
        return {"kernel": stage, "bound": "alu", "achieved": ach, "peak": FP64_VEC_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_VEC_TFLOPS, "traffic": traffic, "ms_per_launch": ms_per_launch,
                "pairs_per_launch": pairs, "flops_per_pair": fl}
    if stage in ("spread", "a_spread"):
        npt, nf = (ns, 1) if stage == "spread" else (nt, 2)
        byts = npt * (12 + 4 * nf) + cells * 4 * nf
    elif stage in ("gather", "a_gather"):
        npt, nf = (nt, 3) if stage == "gather" else (ns, 1)
        byts = npt * (12 + 8 * nf) + cells * 4 * nf
    elif stage in ("rows_fwd", "a_rows_fwd"):
        nf = 1 if stage == "rows_fwd" else 2
        byts = nf * (cells * 4 + (nh + 1) * ey * 8)
    elif stage in ("cols", "a_cols"):
        nin, nout = (1, 2) if stage == "cols" else (2, 1)
        byts = (nin + nout) * (nh + 1) * ey * 8
    elif stage in ("rows_inv", "a_rows_inv"):
        nin, nout = (2, 3) if stage == "rows_inv" else (1, 1)
        byts = nin * (nh + 1) * ey * 8 + nout * cells * 4
    elif stage == "charges":
        byts = ns * 32          # permutation 4, charge 8, weight 8 in; FP32 and FP64 values out
    elif stage == "a_values":
        byts = nt * 44          # permutation 4, V 16 in; FP32 and FP64 pairs out
    elif stage in ("fold", "a_fold"):
        nf = 2 if args.cs else 1
        if stage == "a_fold":
            nf = 2
        t = 32 if not info.get("tile") else info["tile"]
        pt = t + 2 * m - 1
        ntl = -(-ex // t) * -(-ey // t)
        byts = nf * (ntl * pt * pt * 8 + cells * 4)  # padded tile sums in, grid out
    else:
        byts = (nt + ns) * 16
    ach = byts / sec / 1e9
    return {"kernel": stage, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "ms_per_launch": ms_per_launch,
            "algorithmic_bytes_per_launch": byts}


def counter_traffic(kernel_prefix, bandwidth, eps_I, eps_B, n_points):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source (its sha256 prefix is stored with the numbers) and on this
    workload: size, bandwidth, near radius and boundary zone (which sets the points per cell)."""
    path = os.path.join(HERE, "profiles", "counters.json")
    src = os.path.join(HERE, "paper_0807_2387_amd", "csrc", "fn_near.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(kernel_prefix)
    if not ent or ent.get("source_sha256_16") != src_hash(src) or ent.get("bandwidth") != bandwidth:
        return None
    if ent.get("eps_I") is None or abs(ent["eps_I"] - eps_I) > 1e-12 * eps_I:
        return None
    if ent.get("eps_B") is None or abs(ent["eps_B"] - eps_B) > 1e-12 or ent.get("n_points") != n_points:
        return None
    return ent.get("hbm_bytes_per_launch")


def stratified_sample(mask, k, rng):
    """k indices, half drawn from the points where mask holds and half from the rest, with the
    weight (stratum size / stratum sample size) that makes weighted sums unbiased."""
    idx, wts = [], []
    for sel in (np.flatnonzero(mask), np.flatnonzero(~mask)):
        kk = min(len(sel), k // 2)
        if kk == 0:
            continue
        idx.append(rng.choice(sel, kk, replace=False))
        wts.append(np.full(kk, len(sel) / kk))
    idx, wts = np.concatenate(idx), np.concatenate(wts)
    o = np.argsort(idx)
    return idx[o], wts[o]


def accuracy_and_cpu(d, r, args, nt, ns):
    """Sampled check against the FP64 direct-sum oracle, and the oracle's own rate.

    The fast sum's error is not spread evenly: most of the H error sits on targets about
    eps_I from the boundary line charges, a layer holding about 1% of the points.  Targets
    and sources are therefore sampled in two strata (within side/80 of the boundary, and the
    rest; every boundary quadrature point counts as near), half the sample in each, and the
    relative L2 errors are the stratum-weighted estimates of the all-points values."""
    import synth
    from oracle import direct
    y, x, w, q = d["y"], d["x"], d["w"], d["q"]
    V = (d["h"] ** 2) * d["M_tgt"]
    side, rc = 4.0, 0.5
    band = side / 80
    rng = np.random.default_rng(12345)
    it, wt = stratified_sample(synth.rounded_rect_sdf(y, side, side, rc) > -band, args.samples, rng)
    near_s = synth.rounded_rect_sdf(x, side, side, rc) > -band
    near_s[w != d["h"] ** 2] = True  # boundary quadrature points
    js, wsr = stratified_sample(near_s, args.samples, rng)
    a = time.perf_counter()
    phi1, H1 = direct.forward(y[it], x, w, q)
    t_f = time.perf_counter() - a
    a = time.perf_counter()
    u1 = direct.adjoint(y, x[js], w[js], V=V)
    t_a = time.perf_counter() - a
    phi, H, u = r["phi"].cpu().numpy()[it], r["H"].cpu().numpy()[it], r["u"].cpu().numpy()[js]

    def rel(a_, b_, wgt):
        e2 = ((a_ - b_) ** 2).reshape(len(wgt), -1).sum(axis=1)
        r2 = (b_ ** 2).reshape(len(wgt), -1).sum(axis=1)
        return float(np.sqrt(np.dot(wgt, e2) / np.dot(wgt, r2)))

    err = {"phi": rel(phi, phi1, wt), "H": rel(H, H1, wt), "HT": rel(u, u1, wsr),
           "samples": f"{len(it)} targets and {len(js)} sources, stratified by distance to the boundary"}
    # whole-job CPU time extrapolated linearly from the sample (the direct sum is exactly O(N_t N_s))
    t_full = t_f * nt / len(it) + t_a * ns / len(js)
    cpu = {"value": (nt + ns) / t_full, "unit": "points/s", "cores": direct.threads(), "kind": "oracle",
           "sample": f"O1 direct FP64 sum for {len(it)} targets x {ns} sources (phi, H) and "
                     f"{len(js)} sources x {nt} targets (H adjoint), extrapolated linearly; "
                     f"{t_f + t_a:.1f} s of CPU work"}
    log(f"vs O1 (sampled): {err}; CPU oracle {cpu['value']:.3e} points/s on {cpu['cores']} threads")
    return err, cpu


def cpu_fastsum(args):
    """The step-by-step fast-summation oracle (O2, numpy/scipy FP64) timed on the host on the
    same workload recipe at 1/64 of the points (2^18 + 2^18), the grid scaled with sqrt(N)
    (G/8 = 1024, bandwidth 3G/4, the same m, p, n eps_I, n eps_S and eps_B): a fair N log N CPU
    figure beside the O(N^2) direct sum.  The construction (window matrices, near-pair search,
    the counterpart of set_geometry) is not timed; forward (phi, H) + H adjoint is."""
    import synth
    from oracle import fastsum as fs
    n = args.n // 64
    G = max(64, args.grid // 8)
    band = 3 * G // 4
    d = synth.rounded_square_cloud(N=n, seed=synth.SEED_BASE + 4)
    y, x, w, q = d["y"], d["x"], d["w"], d["q"]
    V = (d["h"] ** 2) * d["M_tgt"]
    ns1 = int(np.sum(w == d["h"] ** 2))
    parts = ((slice(0, ns1), args.c, slice(ns1, None)), (slice(ns1, None), args.cs, slice(0, ns1)))
    t_set, t_run = 0.0, 0.0
    for sl, c, other in parts:
        prm = fs.Params(G=G, m=args.m, p=args.p, eps_I=c / band, band=band, eps_B=args.eps_b)
        a = time.perf_counter()
        F = fs.FastSum(y, x[sl], w[sl], prm, map_with=x[other])
        t_set += time.perf_counter() - a
        a = time.perf_counter()
        F.forward(q[sl])
        F.adjoint_H(V)
        t_run += time.perf_counter() - a
        del F
    npts = len(y) + len(x)
    rec = {"value": npts / t_run, "unit": "points/s", "cores": fs._WORKERS, "kind": "oracle O2 (fast sum)",
           "sample": f"forward + H adjoint of {len(y)} targets and {len(x)} sources (the workload recipe at 1/64 "
                     f"of the points), G = {G}, n = {band}; {t_run:.1f} s (construction {t_set:.1f} s, not timed); "
                     f"the FFTs use {fs._WORKERS} threads, the sparse window products and the near field one"}
    log(f"CPU fast sum (O2): {rec['value']:.3e} points/s ({rec['sample']})")
    return rec


# ---------------------------------------------------------------------------- other configurations

def _timed(torch, f, steps, warmup):
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(steps):
        f()
    torch.cuda.synchronize()
    return (time.perf_counter() - a) / steps


def main_configs(args, torch, synth, fn, dev):
    """The smaller configurations, every step through the library's GPU FEM front:
    disk_c1    disk of ~2k nodes, uniform M = (1, 0) (surface charges only), FP64, G = 64, m = 4,
               eps_I = 4/64; step = set_charges + phi, H + H adjoint (V = l M)
    ellipse_c2 ellipse a = 2, b = 1, 50k nodes, vortex M with 8 random modes, G = 512 at
               bandwidth 384, p = 8, n eps_I = 7, FP32-mixed and FP64; the same step
    batch_c3   64 meshes of 5k-200k nodes in one batch (fn_params_auto per member, FP32-mixed),
               4 lanes, forward and H adjoint at once, replayed from a HIP graph
    annulus_c4 annulus of 1M nodes, smooth M, fn_params_auto, FP32-mixed; step = energy and
               gradient (set charges, H and the H adjoint at once, C^T)
    Prints one JSON line per precision (rank 0); value = (nodes + quadrature points)/s."""
    tt = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).to(dt or torch.float64).to(dev)
    out_lines = []

    def mesh_of(d):
        return fn.Mesh(tt(d["nodes"]), tt(d["tris"], torch.int32), tt(d["bedges"], torch.int32))

    def record(name, precision, ms, npts, cfg, extra=None):
        rec = {"metric": f"{name}: nodes + quadrature points per second, one step", "value": npts / (ms * 1e-3),
               "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64" if precision == fn.FN_FP64 else "f32+f64", "data": "synthetic", "config": cfg}
        rec.update(extra or {})
        out_lines.append(rec)
        log(f"{name} ({rec['dtype']}): {ms:.3f} ms per step, {rec['value']:.3e} points/s")

    if args.workload in ("disk_c1", "ellipse_c2"):
        d = synth.workload_disk_c1() if args.workload == "disk_c1" else synth.workload_ellipse_c2()
        mesh = mesh_of(d)
        Md = tt(d["M"])
        q = mesh.charges(Md)
        V = mesh.lumped_mass()[:, None] * Md
        nt, ns = mesh.n_nodes, mesh.n_sources
        precs = (fn.FN_FP64,) if args.workload == "disk_c1" else (fn.FN_FP32_MIXED, fn.FN_FP64)
        for P in precs:
            if args.workload == "disk_c1":
                S = fn.Solver(grid=64, m=4, eps_I=4 / 64, precision=P)
                cfg = {"workload": "disk radius 1, 30 polar rings, 128 boundary edges, M = (1, 0)", "grid": 64,
                       "m": 4, "eps_I": 4 / 64, "n_nodes": nt, "n_src": ns}
            else:
                # the configuration's 512^2 grid at bandwidth 3G/4 (oversampling 4/3): the near
                # radius eps_I = 7/n shrinks by 2/3 at the same n eps_I
                S = fn.Solver(grid=512, n=384, eps_I=7 / 384, p=8, precision=P)
                cfg = {"workload": "ellipse a = 2, b = 1, vortex M + 8 modes", "grid": 512, "bandwidth": 384,
                       "p": 8, "eps_I": 7 / 384, "n_nodes": nt, "n_src": ns}
            S.bind_mesh(mesh)
            phi = torch.empty(nt, dtype=torch.float64, device=dev)
            H = torch.empty(nt, 2, dtype=torch.float64, device=dev)
            u = torch.empty(ns, dtype=torch.float64, device=dev)

            def step():
                S.set_charges(q)
                S.eval_with_H_adjoint(V, out_phi=phi, out_H=H, out_u=u)

            ms = _timed(torch, step, args.steps, args.warmup) * 1e3
            extra = {}
            if not args.no_cpu:
                extra = _configs_vs_direct(d, phi, H, u, args)
            record(args.workload, P, ms, nt + ns, cfg, extra)
            del S
    elif args.workload == "annulus_c4":
        d = synth.workload_annulus_c4()
        mesh = mesh_of(d)
        Md = tt(d["M"])
        a = fn.auto_params(mesh.n_nodes, mesh.n_sources, fn.FN_FP32_MIXED)
        S = fn.Solver(grid=a["grid"], m=a["m"], p=a["p"], eps_I=a["eps_I"], eps_B=a["eps_B"], n=a["n"],
                      eps_S=a["eps_S"], precision=fn.FN_FP32_MIXED)
        S.bind_mesh(mesh)
        ms = _timed(torch, lambda: S.energy(Md), args.steps, args.warmup) * 1e3
        record("annulus_c4", fn.FN_FP32_MIXED, ms, mesh.n_nodes + mesh.n_sources,
               {"workload": "annulus r in [0.5, 1], smooth M, energy and gradient", "n_nodes": mesh.n_nodes,
                "n_src": mesh.n_sources, "grid": a["grid"], "params": "fn_params_auto"})
    else:  # batch_c3
        ms, npts, cfg = batch_c3_step(args, torch, synth, fn, dev)
        record("batch_c3", fn.FN_FP32_MIXED, ms, npts, cfg)
    for rec in out_lines:
        print(json.dumps(rec), flush=True)


def batch_c3_step(args, torch, synth, fn, dev):
    """The 64-mesh batch (C3): every mesh through the library's GPU FEM front, one Batch of
    fn_params_auto members (FP32-mixed), shapes per member from the autotuner (cached, or
    searched on each distinct member before the timed region; --no-tune: library defaults),
    set_charges + forward + H adjoint at once over 4 lanes, replayed from a HIP graph.
    Returns (ms per step, points, config)."""
    tt = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).to(dt or torch.float64).to(dev)
    meshes = synth.batch_meshes()
    xs, ws, qs, Vs, ys = [], [], [], [], []
    for m in meshes:
        me = fn.Mesh(tt(m["nodes"]), tt(m["tris"], torch.int32), tt(m["bedges"], torch.int32))
        x, w = me.sources()
        Md = tt(m["M"])
        ys.append(tt(m["nodes"]))
        xs.append(x), ws.append(w), qs.append(me.charges(Md)), Vs.append(me.lumped_mass()[:, None] * Md)
    toff = np.cumsum([0] + [len(y) for y in ys])
    soff = np.cumsum([0] + [len(x) for x in xs])
    Y, X, W, Q, V = (torch.cat(a) for a in (ys, xs, ws, qs, Vs))
    del xs, ws, qs, Vs, ys
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        B = fn.Batch([fn.auto_params(int(toff[i + 1] - toff[i]), int(soff[i + 1] - soff[i]), fn.FN_FP32_MIXED)
                      for i in range(len(meshes))])
        B.set_geometry(toff, Y, soff, X, W)
        shapes_from = "library defaults"
        if not args.no_tune:
            # per-member shapes: cached, or searched now on each distinct member (not timed)
            from paper_0807_2387_amd import tune
            res = tune.apply_batch(B, toff, Y, soff, X, W, Q, V, log=log)
            shapes_from = (f"autotuner per member: {len({r[0] for r in res})} keys, "
                           f"{sum(r[2] for r in res)} searched now")
            log(f"batch_c3: {shapes_from}")
        phi = torch.empty(len(Y), dtype=torch.float64, device=dev)
        H = torch.empty(len(Y), 2, dtype=torch.float64, device=dev)
        u = torch.empty(len(X), dtype=torch.float64, device=dev)

        def step():
            B.set_charges(Q)
            B.eval_with_H_adjoint(V, out_phi=phi, out_H=H, out_u=u)

        step()
        st.synchronize()
        g = fn.Graph()
        with g.capture(st):
            step()
        st.synchronize()
        ms = _timed(torch, lambda: g.launch(st), args.steps, args.warmup) * 1e3
    cfg = {"workload": "64 meshes, 5k-200k nodes (disks, ellipses, annuli, rounded rectangles)",
           "n_nodes": len(Y), "n_src": len(X), "lanes": 4, "graph": True, "params": "fn_params_auto per member",
           "shapes_from": shapes_from}
    return ms, len(Y) + len(X), cfg


def _configs_vs_direct(d, phi, H, u, args):
    """The step's outputs against the FP64 direct sum (O1) on the oracle's own FEM sources, at
    up to --samples targets and sources, and the direct sum's own rate (CPU leg only)."""
    from oracle import direct, fem
    nodes, tris, bedges, M = d["nodes"], d["tris"], d["bedges"], d["M"]
    x, w = fem.sources(nodes, tris, bedges)
    q = fem.charges(nodes, tris, bedges, M)
    V = fem.lumped_mass(nodes, tris)[:, None] * M
    rng = np.random.default_rng(7)
    it = np.sort(rng.choice(len(nodes), min(args.samples, len(nodes)), replace=False))
    js = np.sort(rng.choice(len(x), min(args.samples, len(x)), replace=False))
    a = time.perf_counter()
    phi1, H1 = direct.forward(nodes[it], x, w, q)
    t_f = time.perf_counter() - a
    a = time.perf_counter()
    u1 = direct.adjoint(nodes, x[js], w[js], V=V)
    t_a = time.perf_counter() - a
    rel = lambda g, r: float(np.linalg.norm(g - r) / np.linalg.norm(r))
    err = {"phi": rel(phi.cpu().numpy()[it], phi1), "H": rel(H.cpu().numpy()[it], H1),
           "HT": rel(u.cpu().numpy()[js], u1), "samples": f"{len(it)} nodes and {len(js)} sources"}
    t_full = t_f * len(nodes) / len(it) + t_a * len(x) / len(js)
    cpu = {"value": (len(nodes) + len(x)) / t_full, "unit": "points/s", "cores": direct.threads(), "kind": "oracle",
           "sample": f"O1 direct FP64 sum on {len(it)} nodes and {len(js)} sources, extrapolated linearly"}
    log(f"  vs O1: {err}")
    return {"rel_l2_vs_fp64_oracle": err, "cpu_baseline": cpu}


# ---------------------------------------------------------------------------- 3D path

def near3_flops_per_pair(stage, p):
    """3D near field, FP64 flops per interacting pair (FMA = 2; sqrt, division = 1 each):
    forward: offsets 6, r^2 5, x 1, T_I and T_I'/r by Horner 2(p-1) + 2(p-2), sqrt 1, 1/r 1,
    phi share 2, field factor 4, phi sum 2, H sums 7; adjoint: offsets 6, r^2 5, x 1,
    T_I'/r 2(p-2), sqrt 1, field factor 5, V.d 5, sum 2."""
    if stage == "near":
        return 6 + 5 + 1 + 2 * (p - 1) + 2 * (p - 2) + 1 + 1 + 2 + 4 + 2 + 7
    return 6 + 5 + 1 + 2 * (p - 2) + 1 + 5 + 5 + 2


def fft3_bytes(G, n, ext, forward):
    """Bytes the pruned 3D transform must move: each pass reads the elements its lines hold
    (the data window or the band |l| <= n/2) and writes the ones the next step keeps."""
    nb = 2 * (n // 2) + 1
    ex, ey, ez = ext
    if forward:  # x lines of the window's rows, y lines of band x window-z, z lines of band x band
        el = ey * ez * (ex + nb) + nb * ez * (ey + nb) + nb * nb * (ez + nb)
    else:        # z lines of band x band, y lines of band x window-z, x lines of the window's rows
        el = nb * nb * (nb + ez) + nb * ez * (nb + ey) + ey * ez * (nb + ex)
    return el * 16


def roofline3(stage, ms_per_launch, G, n, m, p, info, nt, ns, pairs):
    """Roofline of one 3D stage: algorithmic HBM bytes (points' cell, fractions and values once,
    every grid value a pass needs read and written once), or near-field flops, per launch."""
    sec = ms_per_launch * 1e-3
    ext = tuple(info["win_ext"])
    win = int(np.prod(ext)) * 16
    band3 = (2 * (n // 2) + 1) ** 3 * 16
    if stage in ("near", "a_near"):
        fl = near3_flops_per_pair(stage, p)
        ach = pairs[stage] * fl / sec / 1e12
        return {"kernel": stage, "bound": "alu", "achieved": ach, "peak": FP64_VEC_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_VEC_TFLOPS, "traffic": None, "ms_per_launch": ms_per_launch,
                "pairs_per_launch": pairs[stage], "flops_per_pair": fl}
    byts = {
        "charges": ns * 28, "a_values": nt * 52,
        "spread": ns * 36 + win, "a_spread": nt * 60 + 3 * win,
        "fft": fft3_bytes(G, n, ext, True), "a_fft": 3 * fft3_bytes(G, n, ext, True),
        "multiply": 3 * band3, "a_multiply": 4 * band3,
        "ifft": 2 * fft3_bytes(G, n, ext, False), "a_ifft": fft3_bytes(G, n, ext, False),
        "gather": nt * 60 + 2 * win, "a_gather": ns * 36 + win,
    }[stage]
    ach = byts / sec / 1e9
    return {"kernel": stage, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "ms_per_launch": ms_per_launch,
            "algorithmic_bytes_per_launch": byts}


def main_3d(args, torch, synth, fn, dev):
    """The 3D fast summation on a ball lattice: one step = set_charges + eval (phi, H) + H
    adjoint, FP64, inputs resident before the timed region."""
    from scipy.spatial import cKDTree
    G, m, p = args.grid3, args.m3, args.p3
    n = args.band3 or G // 2
    eps_I, eps_B = args.c3 / n, 1.0 / 8.0
    d = synth.ball_lattice3(K=args.K)
    y, x, w, q, V = d["y"], d["x"], d["w"], d["q"], d["V"]
    nt, ns = len(y), len(x)
    log(f"3D workload: {nt} targets, {ns} sources; G = {G}, n = {n}, m = {m}, p = {p}, eps_I = {eps_I:.5f}")
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ty, tx, tw, tq, tV = tt(y), tt(x), tt(w), tt(q), tt(V)
    S = fn.Solver3(grid=G, m=m, p=p, eps_I=eps_I, eps_B=eps_B, n=n)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    S.set_geometry(ty, tx, tw)
    torch.cuda.synchronize()
    t_geom = time.perf_counter() - g0
    info = S.info()
    phi = torch.empty(nt, dtype=torch.float64, device=dev)
    H = torch.empty(nt, 3, dtype=torch.float64, device=dev)
    u = torch.empty(ns, dtype=torch.float64, device=dev)

    def step():
        S.set_charges(tq)
        S.eval(out_phi=phi, out_H=H)
        S.adjoint_H(tV, out=u)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - a) / args.steps
    # stage times: HIP events recorded on the context's stream around every stage
    S.set_profiling(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = S.profile()
    S.set_profiling(False)
    stages = {k: v[0] / args.steps for k, v in prof.items() if v[1]}
    per_launch = {k: prof[k][0] / prof[k][1] for k in stages}
    # in-zone pairs (|t_y - t_x| < eps_I in torus units, i.e. eps_I / s physically)
    r_phys = eps_I / info["scale"]
    tree = cKDTree(x)
    npairs = int(tree.query_ball_point(y, r_phys, return_length=True).sum())
    pairs = {"near": npairs, "a_near": npairs}  # the adjoint visits the same pairs from the sources
    ms = sec * 1e3
    value = (nt + ns) / sec
    log(f"3D: {ms:.3f} ms/step, {value:.4e} points/s, set_geometry {t_geom * 1e3:.1f} ms, "
        f"{pairs['near']} near pairs")
    for k, v in sorted(stages.items(), key=lambda kv: -kv[1]):
        log(f"  {k:12s} {v:9.3f} ms/step")
    dom = max(stages, key=stages.get)
    roof = roofline3(dom, per_launch[dom], G, n, m, p, info, nt, ns, pairs)
    roof_stages = {k: {kk: vv for kk, vv in roofline3(k, per_launch[k], G, n, m, p, info, nt, ns, pairs).items()
                       if kk in ("bound", "achieved", "unit", "frac", "ms_per_launch")} for k in stages}
    out = {
        "metric": "source+target points/s for 3D forward+adjoint fast summation (G = 1/(4 pi r), FP64)",
        "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"ball radius 1, lattice K = {args.K}: jittered nodes as targets, "
                               f"4 random points per lattice cell as sources, smooth random charges",
                   "n_tgt": nt, "n_src": ns, "grid": G, "bandwidth": n, "m": m, "p": p, "eps_I": eps_I,
                   "eps_B": eps_B, "precision": "fp64", "parallelism": "single_gpu"},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "stages_ms_from": "HIP events per stage on the context's stream (one stream, stages in order)",
        "set_geometry_ms": t_geom * 1e3,
        "roofline": roof,
        "roofline_stages": roof_stages,
    }
    if not args.no_cpu:
        from oracle import direct
        rng = np.random.default_rng(321)
        it = np.sort(rng.choice(nt, min(args.samples, nt), replace=False))
        js = np.sort(rng.choice(ns, min(args.samples, ns), replace=False))
        a = time.perf_counter()
        phi1, H1 = direct.forward3(y[it], x, w, q)
        t_f = time.perf_counter() - a
        a = time.perf_counter()
        u1 = direct.adjoint3(y, x[js], w[js], V=V)
        t_a = time.perf_counter() - a
        rel = lambda g, r: float(np.linalg.norm(g - r) / np.linalg.norm(r))
        out["rel_l2_vs_fp64_oracle"] = {"phi": rel(phi.cpu().numpy()[it], phi1), "H": rel(H.cpu().numpy()[it], H1),
                                        "HT": rel(u.cpu().numpy()[js], u1),
                                        "samples": f"{len(it)} targets and {len(js)} sources, uniform"}
        t_full = t_f * nt / len(it) + t_a * ns / len(js)
        out["cpu_baseline"] = {"value": (nt + ns) / t_full, "unit": "points/s", "cores": direct.threads(),
                               "kind": "oracle",
                               "sample": f"O1 direct FP64 3D sum for {len(it)} targets x {ns} sources (phi, H) and "
                                         f"{len(js)} sources x {nt} targets (H adjoint), extrapolated linearly; "
                                         f"{t_f + t_a:.1f} s of CPU work"}
        log(f"vs O1 (sampled): {out['rel_l2_vs_fp64_oracle']}")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
