"""Host-side logic of bench.py (no GPU): the one-GPU guard, the stratified sample's
weights, the near-field flop accounting and the roofline record."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_stratified_sample_weights_sum_to_the_strata():
    rng = np.random.default_rng(0)
    mask = rng.random(10000) < 0.03
    idx, w = bench.stratified_sample(mask, 400, rng)
    assert np.all(np.diff(idx) > 0)  # sorted, no repeats
    assert abs(w[mask[idx]].sum() - mask.sum()) < 1e-9
    assert abs(w[~mask[idx]].sum() - (~mask).sum()) < 1e-9
    # a weighted mean of any per-point quantity is unbiased: here exact for a constant
    assert abs(np.dot(w, np.ones(len(idx))) - len(mask)) < 1e-9


def test_near_flop_accounting():
    # forward: offsets 4, r^2 3, x 1, U and U' 2(p-1) + 2(p-2), ln 1, 1/x 1, phi 4, field 3, H 4
    assert bench.near_flops_per_pair("near", 6) == 39
    assert bench.near_flops_per_pair("near", 5) == 35
    # adjoint of H: offsets 4, r^2 3, x 1, U' 2(p-2), 1/x 1, factor 2, V.d 3, sum 2
    assert bench.near_flops_per_pair("a_near", 5) == 22
    # FP64 path: ln 38 and 1/x 9 instead of one instruction each
    assert bench.near_flops_per_pair("near", 5, f32=False) == 35 - 2 + 38 + 9


def test_counter_traffic_only_for_the_setting_it_was_taken_on():
    import json
    rec = json.load(open(os.path.join(ROOT, "profiles", "counters.json")))
    ent = rec["kernels"]["k_near<0"]
    args = (ent["bandwidth"], ent["eps_I"], ent["eps_B"], ent["n_points"])
    current = ent["source_sha256_16"] == bench.src_hash(
        os.path.join(ROOT, "paper_0807_2387_amd", "csrc", "fn_near.hip"))
    # counters taken on another near-field source are not reported
    assert bench.counter_traffic("k_near<0", *args) == (ent["hbm_bytes_per_launch"] if current else None)
    assert bench.counter_traffic("k_near<0", args[0], args[1] * 1.1, args[2], args[3]) is None
    assert bench.counter_traffic("k_near<0", args[0], args[1], args[2] * 2, args[3]) is None
    assert bench.counter_traffic("k_near<0", args[0], args[1], args[2], args[3] // 2) is None
    assert bench.counter_traffic("k_near<0", args[0] // 2, args[1], args[2], args[3]) is None


def test_3d_near_flop_accounting_and_roofline_record():
    # forward: offsets 6, r^2 5, x 1, T and D by Horner 2(p-1) + 2(p-2), sqrt 1, 1/r 1,
    # phi share 2, field factor 4, phi sum 2, H sums 7
    assert bench.near3_flops_per_pair("near", 6) == 6 + 5 + 1 + 10 + 8 + 1 + 1 + 2 + 4 + 2 + 7
    # adjoint: offsets 6, r^2 5, x 1, D 2(p-2), sqrt 1, field factor 5, V.d 5, sum 2
    assert bench.near3_flops_per_pair("a_near", 6) == 6 + 5 + 1 + 8 + 1 + 5 + 5 + 2
    info = {"win_ext": (110, 110, 110)}
    pairs = {"near": 10 ** 9, "a_near": 10 ** 9}
    r = bench.roofline3("near", 2.0, 256, 128, 6, 6, info, 1000, 4000, pairs)
    assert r["bound"] == "alu" and abs(r["achieved"] - 1e9 * 47 / 2e-3 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / bench.FP64_VEC_TFLOPS) < 1e-15
    # the pruned transform: window rows in, band out, per pass
    nb = 2 * 64 + 1
    fwd = (110 * 110 * (110 + nb) + nb * 110 * (110 + nb) + nb * nb * (110 + nb)) * 16
    r = bench.roofline3("fft", 1.0, 256, 128, 6, 6, info, 1000, 4000, pairs)
    assert r["algorithmic_bytes_per_launch"] == fwd
    assert r["bound"] == "hbm" and abs(r["achieved"] - fwd / 1e-3 / 1e9) < 1e-6
    # an unpruned transform of the whole cube would move 6 G^3 complex values: far more
    assert fwd < 6 * 256 ** 3 * 16 / 4
    assert bench.fft3_bytes(256, 128, (110, 110, 110), False) == fwd
    # bandwidth 3G/4: the band holds 2 * 96 + 1 frequencies per axis
    nb = 2 * 96 + 1
    assert bench.fft3_bytes(256, 192, (110, 110, 110), True) == (
        110 * 110 * (110 + nb) + nb * 110 * (110 + nb) + nb * nb * (110 + nb)) * 16
