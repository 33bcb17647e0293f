#!/usr/bin/env python3
"""Far-zone MVM throughput on one MI355X.

One step is one far-zone matrix-vector product y = T G S x (aggregation,
translation over the interaction list, disaggregation) of one right-hand
side, on the 3,338-box spherical shell (radius 4, thickness 0.25, boxes of
0.25 wavelength, 3x3x3 dipoles = 81 coefficients per box, 81 synthetic
basis functions per box), as an iterative solver would issue it. Inputs
(50 seeded vectors, cycled) and the basis matrices are resident in HBM
before timing starts; the plan (far set, operator table) is built once.

The headline form is the split-precision translation in FP16 (operands as
FP16 hi/lo pairs with power-of-two scales, three products, FP32
accumulation), whose error against the FP64 oracle is that of the plain
FP32 form; the plain FP32 form is timed after it and reported under
"compare" with the speedup. ``--precision`` selects split-bf16, fp16 (one
FP16 product, about 3e-4) or fp32 instead.

``--workload 5`` runs the serving workload: a Poisson stream of GMRES
solves (tolerance 1e-4) on random-occupancy grids of 500 to 50k boxes with
1 to 8 right-hand sides, served with continuous batching; the value counts
every far-zone product (per right-hand side) over the wall time from the
first arrival to the last completion.

``--workload 4`` times the batching workload instead: 64 scatterers of
200 to 20k boxes, four right-hand sides each, in one plan, one captured HIP
graph of three kernels per step (20 steps by default); a step counts
64 x 4 MVMs.

Prints one JSON line with the throughput, latency percentiles, the
roofline position of the dominant kernel (timed with HIP events on the
stream it runs on) and the FP64 CPU oracle timed on a bounded sample,
with the relative l2 error of both forms against it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0           # MI355X HBM3E peak
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
KERNEL_SOURCE = os.path.join(ROOT, "paper_2501_04684_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "far_mvm_shell3338_hbm_traffic.json")
# Stage times come from a loop of their own after the timed one (at least
# PROFILE_CALLS products, --steps if larger), with the kernels' own dispatch
# recording start and stop on one product in PROFILE_EVERY: a recorded
# product takes about 14 us longer, so recording stays out of the timed loop.
PROFILE_EVERY = 8
PROFILE_CALLS = 200
# Calls of each latency loop (at least; --steps if larger).
LATENCY_CALLS = 200
NETWORK_FILE = os.path.join(ROOT, "paper_2501_04684_amd", "data", "networks_nd4_h50_a0.125.npz")
# Stage-2 forms: (dtype label, BF16/FP16 products per pair or 0 for FP32)
FORMS = {"split-bf16": ("f32 (stage 2 bf16 hi/lo x3, f32 accumulation)", 3),
         "split-fp16": ("f32 (stage 2 fp16 hi/lo x3, scaled, f32 accumulation)", 3),
         "fp16": ("f32 (stage 2 fp16 x1, scaled, f32 accumulation)", 1),
         "fp32": ("f32", 0)}


def issued_16bit_flops(form, nu, n_pairs, nrhs):
    """MFMA flops a 16-bit form issues: products x 2 x (rows padded to 32-row
    blocks) x (K = 2 halves padded to 8) per pair and RHS."""
    khb = (nu + 7) // 8 * 8
    return FORMS[form][1] * 2 * (-(-2 * nu // 32) * 32) * (2 * khb) * n_pairs * nrhs


STAGE_KERNELS = {"aggregate": "::aggregate_kernel",  # not disaggregate_kernel
                 "translate_mfma": "translate_mfma_kernel",
                 "translate_split": "translate_split_kernel",
                 "disaggregate": "disaggregate_"}  # the per-box or the per-wavefront kernel


def source_hash(path=KERNEL_SOURCE):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_key(name, basis, nrhs, far_mode):
    """The workload a counter summary was taken on."""
    return f"{name}/{basis}/nrhs{nrhs}/{far_mode}"


def summarize_pmc(fetch_csv, write_csv, copy_bytes, workload):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the three stage kernels,
    with the scale factors read off the plain device copy of copy_bytes."""
    import csv
    import statistics

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        out = {}
        for stage, name in STAGE_KERNELS.items():
            vals = [float(r["Counter_Value"]) for r in rows if name in r["Kernel_Name"]]
            out[stage] = statistics.median(vals) if vals else None
        copies = [float(r["Counter_Value"]) for r in rows
                  if "copyBuffer" in r["Kernel_Name"]]
        return out, max(copies)

    fetch, fetch_copy = per_kernel(fetch_csv, "FETCH_SIZE")
    write, write_copy = per_kernel(write_csv, "WRITE_SIZE")
    return {
        "source_sha256": source_hash(),
        "workload": workload,
        "copy_bytes": copy_bytes,
        "copy_fetch_kib": fetch_copy, "copy_write_kib": write_copy,
        "fetch_scale": copy_bytes / 1024.0 / fetch_copy,
        "write_scale": copy_bytes / 1024.0 / write_copy,
        "fetch_kib": fetch, "write_kib": write,
    }


def measured_traffic(stage, workload):
    """HBM bytes per launch of `stage` from the committed counter summary,
    or None when it is missing, was taken on another workload, or the
    kernel source changed since."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_hash() or t.get("workload") != workload:
        return None
    f, w = t["fetch_kib"].get(stage), t["write_kib"].get(stage)
    if f is None or w is None:
        return None
    return 1024.0 * (f * t["fetch_scale"] + w * t["write_scale"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    argv = sys.argv[1:]
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--basis", choices=["synthetic", "identity"], default="synthetic")
    ap.add_argument("--rate", type=float, default=200.0,
                    help="serving workload: Poisson arrival rate (requests/s)")
    ap.add_argument("--requests", type=int, default=48,
                    help="serving workload: number of requests")
    ap.add_argument("--far-mode", choices=["ilist", "full"], default="ilist",
                    help="far set of workloads 1-3: the interaction list, or every pair "
                         "with Chebyshev offset >= 2 (FULL)")
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 5, 6],
                    help="synthetic workload index (2 = 3,338-box shell; 6 = the "
                         "2-wavelength sphere with trained translation networks)")
    ap.add_argument("--variant", choices=["shell", "plate"], default="shell",
                    help="workload 3: the shell or the 0.5 x 2 x 8 plate at a = 0.125")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="time budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=list(FORMS), default="split-fp16",
                    help="form timed for the headline value (the other form is "
                         "timed after it for comparison unless --no-compare)")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--operators", choices=["table", "generated"], default="table",
                    help="operator source of the chosen 16-bit form (the FP32 form always "
                         "reads a table)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the counter summary of two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) made with --copy-mb, and exit")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing "
                         "(reference kernel for scaling hardware byte counters)")
    args = ap.parse_args(argv)
    args.steps_given = any(a.startswith("--steps") for a in argv)
    args.warmup_given = any(a.startswith("--warmup") for a in argv)
    return args


def error_stats(errs):
    import numpy as np

    e = np.asarray(errs, dtype=np.float64)
    return {"n_vectors": int(len(e)), "median": float(np.median(e)), "max": float(e.max()),
            "min": float(e.min())}


def cpu_baseline(w, nb_ptr, S, X, budget_s, min_vectors=20):
    """Time the FP64 oracle on the same workload (bounded sample): one call
    per input vector, cycling through the seeded vectors the GPU ran, for
    the time budget (and at least ``min_vectors`` vectors). Returns the
    baseline record and the oracle results per vector (for the error of
    every vector the oracle ran, Eq. 18)."""
    import numpy as np
    import oracle as O
    from threadpoolctl import threadpool_info

    S128 = None if S is None else S.astype(np.complex128)
    refs = []
    t0 = time.perf_counter()
    n = 0
    while True:
        v = n % len(X)
        y = O.far_mvm(X[v].astype(np.complex128), w.boxes, w.a, w.k, w.n_d, nb_ptr, S128,
                      mode=w.far_mode)
        if n < len(X):
            refs.append(y)
        n += 1
        if time.perf_counter() - t0 >= budget_s and n >= min(min_vectors, len(X)):
            break
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()
                   if p.get("user_api") == "blas"] or [1])
    # the same oracle on one BLAS thread, half the time budget
    from threadpoolctl import threadpool_limits
    x = X[0].astype(np.complex128)
    with threadpool_limits(limits=1, user_api="blas"):
        t1 = time.perf_counter()
        n1 = 0
        while True:
            O.far_mvm(x, w.boxes, w.a, w.k, w.n_d, nb_ptr, S128, mode=w.far_mode)
            n1 += 1
            if time.perf_counter() - t1 >= budget_s / 2:
                break
        dt1 = time.perf_counter() - t1
    return {
        "value": n * X.shape[1] / dt, "unit": "MVM/s", "cores": int(threads), "kind": "oracle",
        "sample": f"{n} full far-zone MVMs of the same workload ({len(refs)} distinct seeded "
                  f"vectors) in {dt:.1f} s (NumPy FP64, grouped by offset; "
                  f"{len(os.sched_getaffinity(0))} host cores visible, {cpu_model()})",
        "single_thread": {"value": n1 * X.shape[1] / dt1, "unit": "MVM/s", "cores": 1,
                          "sample": f"{n1} MVMs in {dt1:.1f} s on one BLAS thread"},
    }, refs


def vector_errors(Y, refs):
    """Relative l2 error (Eq. 18) of every (vector, RHS) the oracle ran."""
    import numpy as np

    errs = []
    for v, ref in enumerate(refs):
        for r in range(ref.shape[0]):
            errs.append(float(np.linalg.norm(Y[v, r] - ref[r]) / np.linalg.norm(ref[r])))
    return errs


def cpu_baseline_networks(w, weights, offsets, x0, y0_net, y0_table, budget_s):
    """Oracle leg of the network workload: the oracle's network translation
    (the same expanded weights) timed on the host, parity of the GPU result
    with it, and the error of networks and operator table against the
    oracle's FP64 DGFA product (the networks' approximation error, Eq. 18)."""
    import numpy as np
    import oracle as O
    from oracle import cvfcnn as C

    nets = {tuple(int(c) for c in offsets[o]): tuple(t[o] for t in weights)
            for o in range(len(offsets))}
    P = x0.reshape(1, w.n_box, w.n_u).astype(np.complex128)
    t0 = time.perf_counter()
    n = 0
    y_par = None
    while True:
        y = C.translate_cvfcnn(P, w.boxes, nets, w.far_mode).reshape(1, -1)
        if y_par is None:
            y_par = y
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    y_dgfa = O.far_mvm(x0.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, mode=w.far_mode)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    cb = {"value": n / dt, "unit": "MVM/s", "cores": len(os.sched_getaffinity(0)),
          "kind": "oracle",
          "sample": f"{n} network-translation MVMs of the same workload in {dt:.1f} s "
                    "(NumPy FP64, one matmul pair per offset)"}
    acc = {"rel_l2_vs_oracle": rel(y0_net, y_par),
           "network_rel_l2_vs_dgfa": rel(y0_net, y_dgfa),
           "table_rel_l2_vs_dgfa": rel(y0_table, y_dgfa)}
    return cb, acc


def bench_networks(args, U, W, torch):
    """Stage 2 by trained networks (Sec. 3; 192 -> 50 -> 192, one network per
    offset from the 16 orbit networks) on the 2-wavelength sphere at a =
    0.125, identity basis, then the operator table on the same plan."""
    import numpy as np
    from paper_2501_04684_amd import training as T

    w = W.config(6)
    if not os.path.exists(NETWORK_FILE):
        print(f"{NETWORK_FILE} is missing: train it with python -m "
              "paper_2501_04684_amd.training --n-d 4 --a 0.125 --hidden 50 --out ...",
              file=sys.stderr)
        return 1
    orbit, meta = T.load(NETWORK_FILE)
    hidden = int(meta["hidden"])
    if int(meta["n_d"]) != w.n_d or abs(float(meta["a"]) - w.a) > 1e-12:
        raise ValueError("network file does not match the workload's n_d and a")
    dev = torch.device("cuda:0")
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode)
    offsets = U.plan_offsets(ff.plan)
    weights = T.networks_for_plan(ff.plan, orbit, w.n_d)
    n = w.n_box * w.n_u
    n_vec = 50
    X = torch.from_numpy(W.complex_normal((n_vec, 1, n), seed=1000)).to(dev)
    Y = torch.empty((1, n), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream

    def timed():
        for s in range(args.warmup):
            U.far_mvm(ff.plan, X[s % n_vec], Y, 1, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            U.far_mvm(ff.plan, X[s % n_vec], Y, 1, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stage_ms, call_ms = profiled_loop(U, torch, ff.plan, X, Y, 1, stream,
                                          max(PROFILE_CALLS, args.steps))
        lat = latency_loops(U, torch, ff.plan, X, Y, 1, stream, max(LATENCY_CALLS, args.steps))
        U.far_mvm(ff.plan, X[0], Y, 1, stream)
        torch.cuda.synchronize()
        return dt, stage_ms / len(call_ms) * 1e3, lat, Y.cpu().numpy()

    ff.set_networks(*weights)
    dt, avg_us, lat, y_net = timed()
    ff.set_networks()
    dt_t, avg_t, lat_t, y_table = timed()
    # the same operator table in split FP16 (three products on the 16-bit
    # matrix cores, box vectors staged in LDS)
    ff_fp32 = ff
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, precision="split-fp16")
    dt_s, avg_s, lat_s, y_split = timed()
    ff.close()
    ff = ff_fp32
    info = ff.info
    n_pairs, nu = info["n_pairs"], info["n_u"]
    flops = 16.0 * hidden * nu * n_pairs          # two complex layers per pair
    hp = 32 if hidden <= 32 else 64
    hk = 4 * (-(-hidden // 4))          # layer 2's k loop ends at the last group of 4 units
    issued = 2.0 * (2 * hp) * (2 * nu) * n_pairs + 2.0 * (2 * nu) * (2 * hk) * n_pairs
    tr = flops / (avg_us[1] * 1e-6) / 1e12
    stage_names = ["aggregate", "translate", "disaggregate"]
    dom = int(np.argmax(avg_us))
    byt = 2 * n * 8
    if dom == 1:
        roof = {"kernel": "translate_cvfcnn", "bound": "mfma", "achieved": tr,
                "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": tr / PEAK_FP32_MFMA_TFLOPS, "traffic": None}
    else:
        ach = byt / (avg_us[dom] * 1e-6) / 1e9
        roof = {"kernel": stage_names[dom], "bound": "hbm", "achieved": ach,
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                "traffic": None}
    out = {
        "metric": "far-zone MVMs/s", "value": args.steps / dt, "unit": "MVM/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (network translation, FP32 matrix cores)", "data": "synthetic",
        "config": {"workload": w.name, "n_boxes": w.n_box, "n_pairs": n_pairs,
                   "n_offsets": info["n_offsets"], "n_u": nu, "hidden": hidden,
                   "far_mode": w.far_mode, "basis": "identity", "nrhs": 1,
                   "translation": "trained networks (first training stage)",
                   "network_test_error_mean": float(np.mean([v["err_mean"]
                                                             for v in orbit.values()]))},
        **latency_fields(lat),
        "stages": {name: {"avg_us": float(avg_us[i])} for i, name in enumerate(stage_names)},
        "roofline": roof,
        "compare": {"translation": "operator table (FP32 matrix cores, box vectors staged in LDS)",
                    "value": args.steps / dt_t, "translate_us": float(avg_t[1]),
                    "speedup_of_networks": dt_t / dt,
                    "translate_speedup_of_networks": float(avg_t[1] / avg_us[1])},
        "compare_split_fp16": {
            "translation": "operator table, split FP16 (three products on the FP16 matrix "
                           "cores, box vectors staged in LDS)",
            "value": args.steps / dt_s, "translate_us": float(avg_s[1]),
            "stages_us": [float(v) for v in avg_s],
            "speedup_over_fp32_table": dt_t / dt_s,
            "translate_speedup_over_fp32_table": float(avg_t[1] / avg_s[1])},
    }
    out["stages"]["translate"].update(kernel="translate_cvfcnn", algorithmic_flops=flops,
                                      tflops=tr, issued_flops=issued,
                                      frac_fp32_mfma_peak=tr / PEAK_FP32_MFMA_TFLOPS)
    if not args.no_cpu_baseline:
        x0 = X[0].cpu().numpy()
        cb, acc = cpu_baseline_networks(w, weights, offsets, x0, y_net, y_table,
                                        args.cpu_seconds)
        out["cpu_baseline"] = cb
        out.update(acc)
        import oracle as O
        y_dgfa = O.far_mvm(x0.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, mode=w.far_mode)
        out["compare_split_fp16"]["rel_l2_vs_oracle"] = float(
            np.linalg.norm(y_split - y_dgfa) / np.linalg.norm(y_dgfa))
    ff.close()
    print(json.dumps(out))
    return 0


def cpu_baseline_sampled(w, nb_ptr, S, x0, y0_gpu, budget_s, n_pairs, n_sample=4):
    """FULL far sets (O(N^2) pairs over ~10^5 offsets) are beyond a whole
    oracle product in the time budget: time the oracle's stage 1 on every
    box and stages 2-3 on ``n_sample`` test boxes, and scale stage 2 by the
    far-pair count and stage 3 by the box count."""
    import numpy as np
    import oracle as O

    S128 = None if S is None else S.astype(np.complex128)
    x = x0.astype(np.complex128)
    rng = np.random.default_rng(17)
    sample = np.sort(rng.choice(w.n_box, size=n_sample, replace=False))
    t0 = time.perf_counter()
    P = O.aggregate(x, nb_ptr, S128, w.n_u) if S128 is not None else x.reshape(1, w.n_box, w.n_u)
    t1 = time.perf_counter()
    E = O.translate(P, w.boxes, w.a, w.k, w.n_d, mode=w.far_mode, test_boxes=sample)
    t2 = time.perf_counter()
    y = O.disaggregate(E, nb_ptr, S128)
    t3 = time.perf_counter()
    j, _, _ = O.far_pairs(w.boxes, w.far_mode)
    pairs_sample = int(np.isin(j, sample).sum())
    est = (t1 - t0) + (t2 - t1) * n_pairs / pairs_sample + (t3 - t2)
    if nb_ptr is None:
        rows = np.concatenate([np.arange(b * w.n_u, (b + 1) * w.n_u) for b in sample])
    else:
        rows = np.concatenate([np.arange(nb_ptr[b], nb_ptr[b + 1]) for b in sample])
    ref = y[:, rows]
    rel = float(np.linalg.norm(y0_gpu[:, rows] - ref) / np.linalg.norm(ref))
    cores = len(os.sched_getaffinity(0))
    return {
        "value": 1.0 / est, "unit": "MVM/s", "cores": cores, "kind": "oracle",
        "sample": (f"stage 1 on all boxes ({t1 - t0:.1f} s), stages 2-3 on {n_sample} test "
                   f"boxes ({pairs_sample} far pairs, {t2 - t1:.1f} s), scaled to "
                   f"{n_pairs} pairs: {est:.0f} s per product (NumPy FP64, {cores} host "
                   f"cores visible, {cpu_model()})"),
    }, rel


def run_form(U, W, torch, w, precision, basis, nrhs, warmup, steps, copy_mb=0,
             operators="table"):
    """Build the plan for one precision form (operators from a table, or
    evaluated by the stage-2 kernel), time `steps` MVMs after `warmup`
    untimed ones, and return the measurements."""
    import numpy as np

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, max_nrhs=nrhs,
                    precision=precision, operators=operators)
    plan_ms = (time.perf_counter() - t0) * 1e3
    nb_ptr = S = S_dev = None
    if basis == "synthetic":
        nb = np.full(w.n_box, w.n_u)
        nb_ptr, S = W.random_basis(nb, w.n_u, seed=w.seed)
        S_dev = torch.from_numpy(S).to(dev)
        ff.set_basis(nb_ptr, S_dev)
    nb_total = ff.nb_total
    # the persistent stage-2 grid as the library's autotuner sizes it
    tune = tune_with_report(ff, nrhs, 3)
    n_vec = 50
    X = torch.from_numpy(W.complex_normal((n_vec, nrhs, nb_total), seed=1000)).to(dev)
    Y = torch.empty((nrhs, nb_total), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream

    if copy_mb > 0:  # reference kernel for scaling hardware byte counters
        src = torch.ones(copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for s in range(warmup):
        U.far_mvm(ff.plan, X[s % n_vec], Y, nrhs, stream)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for s in range(steps):
        U.far_mvm(ff.plan, X[s % n_vec], Y, nrhs, stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stage_ms, call_ms = profiled_loop(U, torch, ff.plan, X, Y, nrhs, stream,
                                      max(PROFILE_CALLS, steps))

    lat = latency_loops(U, torch, ff.plan, X, Y, nrhs, stream, max(LATENCY_CALLS, steps))

    # every input vector once more, for the error distribution against the oracle
    Ys = np.empty((n_vec, nrhs, nb_total), dtype=np.complex64)
    for v in range(n_vec):
        U.far_mvm(ff.plan, X[v], Y, nrhs, stream)
        Ys[v] = Y.cpu().numpy()
    torch.cuda.synchronize()
    out = {"info": ff.info, "plan_ms": plan_ms, "dt": dt, "value": steps * nrhs / dt,
           "avg_us": stage_ms / len(call_ms) * 1e3, "call_ms": call_ms, "latency": lat,
           "Y": Ys, "X": X.cpu().numpy(), "nb_ptr": nb_ptr, "S": S, "nb_total": nb_total,
           "tune": tune}
    ff.close()
    del S_dev
    return out


KERNEL_NAMES = {0: "chunks", 1: "chunks+rhs-walk", 2: "rounds", 3: "rounds-double-buffer"}


def tune_with_report(ff, nrhs, reps):
    """Run the library's stage-2 autotuner and return what it timed: the
    chosen kernel and grid and every candidate's time per launch (read back
    from a transient tuner cache file unless UBF_TUNE_CACHE is set)."""
    import tempfile

    own = not os.environ.get("UBF_TUNE_CACHE")
    path = None
    if own:
        fd, path = tempfile.mkstemp(prefix="ubf_tune_", suffix=".txt")
        os.close(fd)
        os.environ["UBF_TUNE_CACHE"] = path
    try:
        groups = ff.tune(nrhs=nrhs, reps=reps)
        out = {"kernel": KERNEL_NAMES.get(ff.info["translate_kernel"]), "groups": groups}
        cache = os.environ["UBF_TUNE_CACHE"]
        try:
            lines = [l for l in open(cache).read().splitlines() if "\t" in l]
        except OSError:
            lines = []
        if lines:
            fields = lines[-1].split("\t")[1].split()
            cands = {}
            for c in fields[3:]:
                k, g, us = c.split(":")
                cands[f"{KERNEL_NAMES.get(int(k), k)}/{g}"] = round(float(us), 2)
            out["candidates_us"] = cands
        return out
    finally:
        if own:
            del os.environ["UBF_TUNE_CACHE"]
            os.remove(path)


def profiled_loop(U, torch, plan, X, Y, nrhs, stream, n_calls):
    """Per-stage kernel times (ms summed over the recorded products) and the
    recorded products' times: n_calls products over the inputs X in turn,
    one in PROFILE_EVERY recorded."""
    n_rec = -(-n_calls // PROFILE_EVERY)
    U.profile_begin(plan, n_rec, PROFILE_EVERY)
    torch.cuda.synchronize()
    for s in range(n_calls):
        U.far_mvm(plan, X[s % len(X)], Y, nrhs, stream)
    torch.cuda.synchronize()
    return U.profile_end(plan, n_rec)


def latency_loops(U, torch, plan, X, Y, nrhs, stream, n_calls):
    """Per-call latency of the product, apart from the throughput loop.

    device: every one of n_calls back-to-back calls recorded through the
    kernels' own dispatch events (start of stage 1 to end of stage 3);
    host: n_calls calls each waited for (launch to completion on the host
    clock, what a caller that needs the result at once sees)."""
    import numpy as np

    n_vec = X.shape[0]
    U.profile_begin(plan, n_calls, 1)
    for s in range(n_calls):
        U.far_mvm(plan, X[s % n_vec], Y, nrhs, stream)
    torch.cuda.synchronize()
    _, dev_ms = U.profile_end(plan, n_calls)
    host_ms = np.empty(n_calls)
    for s in range(n_calls):
        t0 = time.perf_counter()
        U.far_mvm(plan, X[s % n_vec], Y, nrhs, stream)
        torch.cuda.synchronize()
        host_ms[s] = (time.perf_counter() - t0) * 1e3
    return {"device_ms": np.asarray(dev_ms, dtype=np.float64), "host_ms": host_ms}


def latency_fields(lat):
    """p50/p99 of both latency loops, with their sample counts."""
    import numpy as np

    d, h = lat["device_ms"], lat["host_ms"]
    return {"p50_ms": float(np.percentile(d, 50)), "p99_ms": float(np.percentile(d, 99)),
            "latency": {"device_calls": int(len(d)),
                        "device_p50_ms": float(np.percentile(d, 50)),
                        "device_p99_ms": float(np.percentile(d, 99)),
                        "device_max_ms": float(d.max()),
                        "host_sync_calls": int(len(h)),
                        "host_sync_p50_ms": float(np.percentile(h, 50)),
                        "host_sync_p99_ms": float(np.percentile(h, 99)),
                        "what": "device: kernel dispatch events of every call in a "
                                "back-to-back loop (stage 1 start to stage 3 end); "
                                "host_sync: each call launched and waited for"}}


def batch_form(U, W, torch, w, precision, warmup, steps):
    """One batched plan over all scatterers of `w` (identity basis, w.nrhs
    right-hand sides each): tune the stage-2 grid, time eager calls per
    stage, then time `steps` replays of the captured graph."""
    import numpy as np

    parts = w.extra["scatterers"]
    nrhs = w.nrhs
    t0 = time.perf_counter()
    ff = U.FarField(None, w.a, w.k, w.n_d, w.far_mode, max_nrhs=nrhs,
                    precision=precision, scatterers=parts)
    plan_ms = (time.perf_counter() - t0) * 1e3
    tune = tune_with_report(ff, nrhs, 2)
    groups = tune["groups"]
    x = torch.from_numpy(w.coefficients()).to("cuda:0")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(2):
        U.far_mvm(ff.plan, x, y, nrhs, stream)
    n_prof = max(3, min(steps, 10))
    U.profile_begin(ff.plan, n_prof)
    for _ in range(n_prof):
        U.far_mvm(ff.plan, x, y, nrhs, stream)
    stage_ms, _ = U.profile_end(ff.plan, n_prof)
    ff.capture(x, y)
    for _ in range(warmup):
        ff.replay()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        ff.replay()
        b.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    call_ms = np.array([a.elapsed_time(b) for a, b in ev])
    out = {"info": ff.info, "plan_ms": plan_ms, "dt": dt, "groups": groups, "tune": tune,
           "value": steps * nrhs * len(parts) / dt, "avg_us": stage_ms / n_prof * 1e3,
           "call_ms": call_ms, "y": y.cpu().numpy(), "x": x.cpu().numpy()}
    ff.close()
    return out


def batch_cpu_baseline(w, x, y_gpu, budget_s, n_pairs_total):
    """The oracle on whole scatterers (smallest first) until the budget is
    spent; its rate is scaled to the whole batch by far-pair count, which
    sets the oracle's cost."""
    import numpy as np
    import oracle as O

    parts = w.extra["scatterers"]
    offs = np.cumsum([0] + [len(b) for b in parts]) * w.n_u
    order = np.argsort([len(b) for b in parts])
    done, pairs_done, t_used, errs = 0, 0, 0.0, []
    for s in order:
        b = parts[s]
        sl = slice(offs[s], offs[s + 1])
        t0 = time.perf_counter()
        ref = O.far_mvm(x[:, sl].astype(np.complex128), b, w.a, w.k, w.n_d,
                        mode=w.far_mode)
        t_used += time.perf_counter() - t0
        j, _, _ = O.far_pairs(b, O.FAR_ILIST if w.far_mode == "ilist" else O.FAR_FULL)
        pairs_done += len(j)
        done += 1
        errs.append(float(np.linalg.norm(y_gpu[:, sl] - ref) / np.linalg.norm(ref)))
        if t_used >= budget_s:
            break
    est_total_s = t_used * n_pairs_total / max(pairs_done, 1)
    cores = len(os.sched_getaffinity(0))
    return ({"value": w.nrhs * len(parts) / est_total_s, "unit": "MVM/s", "cores": cores,
             "kind": "oracle",
             "sample": (f"{done} whole scatterers (smallest first, {pairs_done} far pairs, "
                        f"{w.nrhs} RHS each) in {t_used:.1f} s, scaled to the batch's "
                        f"{n_pairs_total} far pairs (NumPy FP64, {cores} host cores "
                        f"visible, {cpu_model()})")},
            max(errs))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def bench_batch(args, U, W, torch):
    import numpy as np

    w = W.config(4)
    chosen = args.precision
    steps = args.steps if args.steps_given else 20
    warmup = args.warmup if args.warmup_given else 3
    res = batch_form(U, W, torch, w, chosen, warmup, steps)
    other = None
    if not args.no_compare:
        other = batch_form(U, W, torch, w, "fp32" if chosen != "fp32" else "split-bf16",
                           warmup, steps)
    info, avg_us = res["info"], res["avg_us"]
    n_pairs, n_box, nu, nrhs = info["n_pairs"], info["n_boxes"], info["n_u"], w.nrhs
    split = FORMS[chosen][1] > 0
    flops = info["translate_flops"] * nrhs
    issued = issued_16bit_flops(chosen, nu, n_pairs, nrhs) if split else flops
    ach = (issued if split else flops) / (avg_us[1] * 1e-6) / 1e12
    peak = PEAK_BF16_MFMA_TFLOPS if split else PEAK_FP32_MFMA_TFLOPS
    box_bytes = nrhs * n_box * nu * 8
    stages = {"aggregate": {"avg_us": float(avg_us[0]), "algorithmic_bytes": 2 * box_bytes},
              "translate": {"avg_us": float(avg_us[1]), "algorithmic_flops": flops,
                            "tflops": flops / (avg_us[1] * 1e-6) / 1e12,
                            "issued_flops": issued if split else flops},
              "disaggregate": {"avg_us": float(avg_us[2]),
                               "algorithmic_bytes": 2 * box_bytes}}
    kinds = w.extra["kinds"]
    out = {
        "metric": "far-zone MVMs/s", "value": res["value"], "unit": "MVM/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": res["dt"] / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": FORMS[chosen][0],
        "data": "synthetic",
        "config": {"workload": w.name, "scatterers": len(kinds),
                   "kinds": {k: kinds.count(k) for k in sorted(set(kinds))},
                   "n_boxes": n_box, "n_pairs": n_pairs, "n_u": nu,
                   "far_mode": w.far_mode, "basis": "identity", "nrhs": nrhs,
                   "precision": chosen, "launch": "one HIP graph (3 kernels) per step",
                   "translate_groups": res["groups"]},
        "tune": res["tune"],
        "p50_ms": float(np.percentile(res["call_ms"], 50)),
        "p99_ms": float(np.percentile(res["call_ms"], 99)),
        "plan_ms": res["plan_ms"], "stages": stages,
        "roofline": {"kernel": "translate_split" if split else "translate_mfma",
                     "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": None},
    }
    if other is not None:
        out["compare"] = {"precision": "fp32" if chosen != "fp32" else "split-bf16",
                          "value": other["value"],
                          "translate_us": float(other["avg_us"][1]),
                          "speedup_of_chosen": res["value"] / other["value"],
                          "rel_l2_diff_vs_chosen": float(np.linalg.norm(other["y"] - res["y"])
                                                         / np.linalg.norm(other["y"]))}
    if not args.no_cpu_baseline:
        cb, err = batch_cpu_baseline(w, res["x"], res["y"], args.cpu_seconds, n_pairs)
        out["cpu_baseline"] = cb
        out["rel_l2_vs_oracle_sampled_scatterers_max"] = err
    print(json.dumps(out))
    return 0


def bench_serve(args, U, W, torch):
    import numpy as np
    import paper_2501_04684_amd.serve as S

    tol, restart, max_steps = 1e-4, 30, 300
    specs = W.serving_requests(args.requests, args.rate, seed=5)
    reqs = [S.Request(i, d["boxes"], W.complex_normal((d["nrhs"], len(d["boxes"]) * 81),
                                                      d["b_seed"]),
                      arrival=d["arrival"], precision=args.precision, tol=tol,
                      restart=restart, max_steps=max_steps)
            for i, d in enumerate(specs)]
    total = torch.cuda.get_device_properties(0).total_memory
    budget = int(min(200 << 30, 0.7 * total))
    srv = S.Server(hbm_budget=budget, max_active=16, steps_per_tick=2, profile=True,
                   profile_every=PROFILE_EVERY)
    # warm-up request (not counted): loads kernels, fills the operator cache
    wb = W.mask_boxes(600, 0.5, 1)
    warm = S.Request(-1, wb, W.complex_normal((1, len(wb) * 81), 1), tol=tol,
                     restart=restart, precision=args.precision)
    srv.run([warm], realtime=False)
    res = srv.run(reqs, realtime=True)
    srv.close()
    ok = [r for r in res if r.error is None]
    t_first = min(r.t_arrival for r in res)
    wall = max(r.t_done for r in ok) - t_first
    solve_mvms = sum(r.products * r.nrhs for r in ok)
    setup_mvms = sum(r.setup_products for r in ok)
    mvms = solve_mvms + setup_mvms
    lat = np.array([r.latency for r in ok]) * 1e3
    wait = np.array([r.t_admit - r.t_arrival for r in ok]) * 1e3
    # time-weighted number of active requests
    log = sorted(srv.log)
    area = sum((t1 - t0) * n for (t0, n, _), (t1, _, _) in zip(log, log[1:]))
    conc = area / max(log[-1][0] - log[0][0], 1e-9) if len(log) > 1 else 0.0
    # dominant kernel: stage-2 launches of every product, HIP events per stage
    split = FORMS[args.precision][1] > 0
    flops = issued = t_tr = t_all = 0.0
    nu = 81
    khb = (nu + 7) // 8 * 8
    for r in ok:
        if r.stage_ms is None:
            continue
        per = r.products_timed * r.nrhs
        flops += r.translate_flops * per
        issued += (issued_16bit_flops(args.precision, nu, r.n_pairs, per) if split
                   else r.translate_flops * per)
        t_tr += r.stage_ms[1] * 1e-3
        t_all += r.stage_ms.sum() * 1e-3
    ach = (issued if split else flops) / t_tr / 1e12
    peak = PEAK_BF16_MFMA_TFLOPS if split else PEAK_FP32_MFMA_TFLOPS
    out = {
        "metric": "far-zone MVMs/s", "value": mvms / wall, "unit": "MVM/s", "n_gpus": 1,
        "steps": len(ok), "warmup": 1, "ms_per_step": wall / max(len(ok), 1) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": FORMS[args.precision][0],
        "data": "synthetic",
        "config": {"workload": f"serving_poisson{args.rate:g}_masks500-50k",
                   "requests": len(reqs), "offered_rate_per_s": args.rate,
                   "boxes_mean": float(np.mean([len(q.boxes) for q in reqs])),
                   "nrhs_mean": float(np.mean([q.nrhs for q in reqs])),
                   "solver": f"GMRES({restart}), tol {tol:g}, FP64 orthogonalisation",
                   "system": "sigma I + Z^F, sigma = 2 ||Z^F||_2 e^{j pi/4} (power iteration)",
                   "precision": args.precision, "hbm_budget_gb": budget / 2 ** 30,
                   "max_active": srv.max_active},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "serving": {"completed": len(ok), "rejected": len(res) - len(ok),
                    "converged": sum(r.converged for r in ok),
                    "requests_per_s": len(ok) / wall, "wall_s": wall,
                    "admission_wait_p50_ms": float(np.percentile(wait, 50)),
                    "admission_wait_p99_ms": float(np.percentile(wait, 99)),
                    "mean_active": conc, "peak_active": srv.peak_active,
                    "mean_steps": float(np.mean([r.steps for r in ok])),
                    "products": mvms, "solve_products": solve_mvms,
                    "shift_estimate_products": setup_mvms,
                    "stage_time_share_translate": t_tr / max(t_all, 1e-12)},
        "roofline": {"kernel": "translate_split" if split else "translate_mfma",
                     "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": None},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        # the oracle's product on whole requests (smallest first), scaled to
        # the stream's products by far-pair count
        by = {r.rid: r for r in ok}
        order = [i for i in np.argsort([len(q.boxes) for q in reqs]) if reqs[i].rid in by]
        pairs_all = sum(r.n_pairs * (r.products * r.nrhs + r.setup_products) for r in ok)
        t_used, pairs_done, n_done = 0.0, 0, 0
        for i in order:
            q = reqs[i]
            x = q.b[:1].astype(np.complex128)
            t0 = time.perf_counter()
            O.far_mvm(x, q.boxes, q.a, q.k, q.n_d)
            t_used += time.perf_counter() - t0
            pairs_done += by[q.rid].n_pairs
            n_done += 1
            if t_used >= args.cpu_seconds:
                break
        rate_pairs = pairs_done / t_used            # far pairs per second, one RHS
        cores = len(os.sched_getaffinity(0))
        out["cpu_baseline"] = {
            "value": mvms / (pairs_all / rate_pairs), "unit": "MVM/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"one product on each of the {n_done} smallest requests "
                       f"({pairs_done} far pairs) in {t_used:.1f} s, scaled by far-pair "
                       f"count to the stream's {mvms} products (NumPy FP64, {cores} host "
                       f"cores visible, {cpu_model()})")}
    print(json.dumps(out))
    return 0


def main():
    args = parse()
    if args.summarize_pmc:
        import workloads as W
        key = traffic_key(W.config(args.workload).name, args.basis, args.nrhs, args.far_mode)
        print(json.dumps(summarize_pmc(*args.summarize_pmc,
                                       (args.copy_mb or 256) << 20, key), indent=1))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not a build)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_2501_04684_amd as U
    import workloads as W

    torch.cuda.set_device(0)
    if args.workload == 4:
        return bench_batch(args, U, W, torch)
    if args.workload == 5:
        return bench_serve(args, U, W, torch)
    if args.workload == 6:
        return bench_networks(args, U, W, torch)
    extra = {"variant": args.variant} if args.workload == 3 else {}
    w = W.config(args.workload, far_mode=args.far_mode, **extra)
    if args.far_mode == "full":
        w.name += "_full"
        args.steps = args.steps if args.steps_given else 100
        args.warmup = args.warmup if args.warmup_given else 3
    nrhs = args.nrhs
    chosen = args.precision
    operators = args.operators
    if chosen == "fp32":
        operators = "table"
    res = run_form(U, W, torch, w, chosen, args.basis, nrhs, args.warmup, args.steps,
                   args.copy_mb, operators)
    other = None
    if not args.no_compare:
        other_form = "fp32" if chosen != "fp32" else "split-bf16"
        other = run_form(U, W, torch, w, other_form, args.basis, nrhs, args.warmup,
                         args.steps)

    info, avg_us, S = res["info"], res["avg_us"], res["S"]
    tkey = traffic_key(w.name, args.basis, nrhs, w.far_mode)
    nb_total, K, dt = res["nb_total"], args.steps, res["dt"]
    n_pairs, n_box, nu = info["n_pairs"], info["n_boxes"], info["n_u"]
    s_bytes = 0 if S is None else S.nbytes
    stage_names = ["aggregate", "translate", "disaggregate"]
    split = FORMS[chosen][1] > 0
    translate_kernel = "translate_split" if split else "translate_mfma"
    # algorithmic work per launch
    flops = info["translate_flops"] * nrhs
    bytes_agg = s_bytes + nrhs * (nb_total + n_box * nu) * 8
    bytes_dis = s_bytes + nrhs * (n_box * nu + nb_total) * 8
    trans_tflops = flops / (avg_us[1] * 1e-6) / 1e12
    # split form: three BF16 products over 32-row blocks and 8-wide k-steps
    khb = (nu + 7) // 8 * 8
    issued = issued_16bit_flops(chosen, nu, n_pairs, nrhs) if split else flops
    dom = int(np.argmax(avg_us))
    if dom == 1:
        peak = PEAK_BF16_MFMA_TFLOPS if split else PEAK_FP32_MFMA_TFLOPS
        ach = (issued if split else flops) / (avg_us[1] * 1e-6) / 1e12
        roof = {"kernel": translate_kernel, "bound": "mfma", "achieved": ach,
                "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": measured_traffic(translate_kernel, tkey)}
    else:
        b = bytes_agg if dom == 0 else bytes_dis
        ach = b / (avg_us[dom] * 1e-6) / 1e9
        roof = {"kernel": stage_names[dom], "bound": "hbm", "achieved": ach,
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                "traffic": measured_traffic(stage_names[dom], tkey)}
    stages = {name: {"avg_us": float(avg_us[i])} for i, name in enumerate(stage_names)}
    stages["translate"].update(
        kernel=translate_kernel, algorithmic_flops=flops,
        tflops=trans_tflops, frac_fp32_mfma_peak=trans_tflops / PEAK_FP32_MFMA_TFLOPS,
        traffic=measured_traffic(translate_kernel, tkey))
    if split:
        itf = issued / (avg_us[1] * 1e-6) / 1e12
        stages["translate"].update(issued_bf16_flops=issued, issued_tflops=itf,
                                   frac_bf16_mfma_peak=itf / PEAK_BF16_MFMA_TFLOPS)
    for i, (name, b) in enumerate((("aggregate", bytes_agg), ("disaggregate", bytes_dis))):
        st = stages[name]
        st["algorithmic_bytes"] = b
        st["gbs"] = b / (st["avg_us"] * 1e-6) / 1e9
        st["traffic"] = measured_traffic(name, tkey)

    out = {
        "metric": "far-zone MVMs/s", "value": res["value"], "unit": "MVM/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": FORMS[chosen][0],
        "data": "synthetic",
        "config": {"workload": w.name, "n_boxes": n_box, "n_pairs": n_pairs,
                   "n_offsets": info["n_offsets"], "n_u": nu, "far_mode": w.far_mode,
                   "basis": (f"synthetic, {w.n_u} functions per box"
                             if S is not None else "identity"),
                   "nrhs": nrhs, "precision": chosen, "operators": operators,
                   "translate_groups": info["translate_groups"]},
        "tune": res["tune"],
        **latency_fields(res["latency"]),
        "plan_ms": res["plan_ms"],
        "stages": stages,
        "roofline": roof,
    }
    if other is not None:
        ot = other["avg_us"]
        out["compare"] = {
            "precision": "fp32" if chosen != "fp32" else "split-bf16",
            "value": other["value"], "translate_us": float(ot[1]),
            "p50_ms": float(np.percentile(other["latency"]["device_ms"], 50)),
            "p99_ms": float(np.percentile(other["latency"]["device_ms"], 99)),
            "speedup_of_chosen": res["value"] / other["value"],
            "translate_speedup_of_chosen": float(ot[1] / avg_us[1]),
        }
    if not args.no_cpu_baseline:
        if w.far_mode == "full":
            cb, rel = cpu_baseline_sampled(w, res["nb_ptr"], S, res["X"][0], res["Y"][0],
                                           args.cpu_seconds, n_pairs)
            out["cpu_baseline"] = cb
            out["rel_l2_vs_oracle_sampled"] = rel
            if other is not None:
                _, orel = cpu_baseline_sampled(w, other["nb_ptr"], other["S"], other["X"][0],
                                               other["Y"][0], args.cpu_seconds, n_pairs)
                out["compare"]["rel_l2_vs_oracle_sampled"] = orel
        else:
            # the oracle runs each seeded vector once; both forms ran the same
            # vectors and basis, so its results serve both
            cb, refs = cpu_baseline(w, res["nb_ptr"], S, res["X"], args.cpu_seconds)
            out["cpu_baseline"] = cb
            st = error_stats(vector_errors(res["Y"], refs))
            out["rel_l2_vs_oracle"] = st["max"]
            out["rel_l2_vs_oracle_per_vector"] = st
            if other is not None:
                ost = error_stats(vector_errors(other["Y"], refs))
                out["compare"]["rel_l2_vs_oracle"] = ost["max"]
                out["compare"]["rel_l2_vs_oracle_per_vector"] = ost
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
