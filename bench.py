#!/usr/bin/env python3
"""Benchmark of the EDAA hot path on one MI355X.

Workload (one "step"): the batched ensemble on the Urban-shaped synthetic scene
-- L = 162 bands, N = 307 x 307 = 94249 pixels, p = 6, M = 50 runs (10 seeds x
gamma in {0.25, 0.5, 1, 2, 4}), T = 100 outer iterations, K1 = K2 = 5 --
including the per-pixel normalisation of the raw scene, B0/A0 initialisation,
step sizes, the 100 x (1 + 5) passes over X, the closing pass, coherence and
the Algorithm 2 selection.  Inputs are resident in device memory before the
timed region starts.

Printed: one JSON line with run-iterations/s (M * T per step), the
algorithmic HBM rate, the roofline of the dominant kernel (the B-pass, timed
with HIP events recorded around each of its launches on its launch stream),
the error of the headline runs against stored float64 traces, the plain path
(single runs on the same data, at equal final loss, with its own HBM roofline
on the Urban-shaped scene and on the large L=224, N=512x614, p=12 scene), the
Samson- and Jasper-shaped single runs, the BF16-X ensemble on the large scene
with its error against float64, the ragged batch against per-image launches,
and the float64 oracle timed on this host's cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_MFMA_TFLOPS = 157.3          # MI355X dense FP32 matrix peak (v_mfma_f32_16x16x4f32: 32 cycles/SIMD)
BF16_MFMA_TFLOPS = 2500.0         # MI355X dense bf16 matrix peak (v_mfma_f32_16x16x32_bf16: 16 cycles/SIMD)
HBM_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "k_bpass_urban_ensemble_traffic.txt")
PLAIN_TRAFFIC_FILE = os.path.join(PROFILES, "k_bpass_large_single_traffic.txt")
GOLDEN = os.path.join(ROOT, "tests", "golden")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2209_11002_amd", "csrc", f)
                  for f in ("edaa_device.h", "edaa_inst.hip", "edaa_kernels.hip")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_sha256():
    """SHA-256 over the pass-kernel sources (the device code and its
    launchers), which the stored counter summaries record."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(path, shape=None):
    """HBM bytes per launch of the profiled kernel from a committed counter
    summary, or None when it is missing, was taken from another version of
    the kernels, or (shape given) at another launch shape."""
    try:
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        if fields.get("kernel_source_sha256") != kernel_source_sha256():
            return None
        if shape is not None and fields.get("launch_shape") != shape:
            return None
        return int(float(fields["traffic_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def parse_shape(text):
    """'R,npg' -> (runs per chunk, pixel groups)."""
    r, n = (int(v) for v in text.split(","))
    return r, n


def profile_run(T, workload, shape=None, tiles_per_item=0):
    """Workload for rocprofv3 passes: a plain device copy of known size (the
    calibration of FETCH_SIZE / WRITE_SIZE) and then T outer iterations of
    'urban_ensemble' (the headline ensemble, at the launch shape `shape` if
    given), 'urban_single' (one run on the same scene), 'large_single' (one
    run on the L=224, N=512x614, p=12 scene, float32 X), 'large_bf16' (the
    M=20 ensemble on that scene with bf16 X, bf16 matrix-core passes) or
    'ragged' (the 64-image ragged batch, persistent kernel, work items of
    `tiles_per_item` tiles, 0 for the default)."""
    import torch
    from paper_2209_11002_amd import api, synth
    dev = torch.device("cuda:0")
    nbytes = 256 << 20
    src = torch.ones(nbytes // 4, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)          # reads and writes exactly nbytes
    torch.cuda.synchronize()
    del src, dst
    log(f"calibration copy: {nbytes} bytes read, {nbytes} bytes written")
    if workload == "ragged":
        scenes, _ = synth.ragged_images(64)
        X = [api.normalize_pixels(torch.from_numpy(sc.X).to(dev)) for sc in scenes]
        ps = [sc.M.shape[1] for sc in scenes]
        api.fit_ragged(X, ps, list(range(64)), [1.0] * 64, T=T, tiles_per_item=tiles_per_item)
        torch.cuda.synchronize()
        log(f"profile run done ({workload}, T={T})")
        return
    if workload in ("large_single", "large_bf16"):
        scene, cfg = synth.large_smooth()
        p = 12
    else:
        scene, cfg = synth.urban_ensemble()
        p = 6
    X = api.normalize_pixels(torch.from_numpy(scene.X).to(dev),
                             out_dtype=torch.bfloat16 if workload == "large_bf16" else torch.float32)
    if workload == "large_bf16":
        api.ensemble(X, p, cfg["seeds"], cfg["gammas"], T=T, K1=cfg["K1"], K2=cfg["K2"])
    elif workload == "urban_ensemble":
        R, npg = shape if shape else (0, 0)
        api.ensemble(X, p, cfg["seeds"], cfg["gammas"], T=T, K1=cfg["K1"], K2=cfg["K2"], runs_per_chunk=R,
                     pixel_groups=npg)
    else:
        api.fit(X, p, T=T, K1=cfg["K1"], K2=cfg["K2"], gamma=1.0, seed=0)
    torch.cuda.synchronize()
    log(f"profile run done ({workload}, T={T})")


def summarize(paths):
    """Per-kernel means of rocprofv3 CSV output: counter collections (one row
    per dispatch and counter) or kernel traces (durations)."""
    import csv
    import collections
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        with open(path) as f:
            for row in csv.DictReader(f):
                name = row["Kernel_Name"].replace("edaa::(anonymous namespace)::", "")
                if "Counter_Name" in row:
                    acc[name][row["Counter_Name"]].append(float(row["Counter_Value"]))
                elif "Start_Timestamp" in row:
                    acc[name]["duration_us"].append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3)
    for name, d in acc.items():
        print(name)
        for c, v in sorted(d.items()):
            print(f"    {c:24s} mean {sum(v) / len(v):16.6g}   dispatches {len(v)}")


def pass_bytes(L, N, Q, x_bytes=4):
    """Algorithmic HBM bytes of one pass: X read once, Q rows of pixel
    weights (or abundances) read and written in float32."""
    return L * N * x_bytes + 2 * Q * N * 4


def time_single_runs(X, p, T, runs, gammas, seeds, out):
    """run-iterations/s of `runs` single fits replayed from one captured
    graph (outputs preallocated, so every call replays the same graph)."""
    import torch
    from paper_2209_11002_amd import api
    api.fit(X, p, T=T, gamma=gammas[0], seed=seeds[0], graph=True, out=out)      # capture
    torch.cuda.synchronize()
    losses = []
    t0 = time.perf_counter()
    for m in range(runs):
        r = api.fit(X, p, T=T, gamma=gammas[m % len(gammas)], seed=seeds[m % len(seeds)], graph=True, out=out)
        losses.append(r["loss"][-1])
    torch.cuda.synchronize()
    return runs * T / (time.perf_counter() - t0), losses


def measured_stream_ceiling(dev, gib=2, reps=5):
    """Streaming ceilings measured on this GPU, to state beside the 8 TB/s
    spec: a read-only pass (torch's sum over gib GiB of float32) and a device
    copy of the same size (read + write), each the best of reps after a
    warm-up, timed with HIP events on torch's stream."""
    import torch
    n = gib * (1 << 30) // 4
    src = torch.ones(n, device=dev)
    dst = torch.empty_like(src)
    best = {}
    for name, fn in (("read", lambda: src.sum()), ("copy", lambda: dst.copy_(src))):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        best[name] = min(ts)
    del src, dst
    torch.cuda.empty_cache()
    nb = n * 4
    return dict(read_gbs=round(nb / best["read"] / 1e9, 1), copy_gbs=round(2 * nb / best["copy"] / 1e9, 1),
                bytes=nb, method=f"torch sum and copy over {gib} GiB of float32, best of {reps}")


def plain_pass_roofline(X, p, T, label, traffic_path=None):
    """Pass durations of one eager single run (HIP events around each launch)
    and the B-pass HBM roofline: algorithmic bytes per launch / its mean
    duration against 8 TB/s."""
    import torch
    from paper_2209_11002_amd import api
    dev = X.device
    L, N = X.shape
    api.fit(X, p, T=T, gamma=1.0, seed=0, time_passes=True)
    nb, bms = api.pass_times(dev, 1)
    na, ams = api.pass_times(dev, 0)
    torch.cuda.synchronize()
    b_s, a_s = bms / nb / 1e3, ams / na / 1e3
    nbytes = pass_bytes(L, N, p, 2 if X.dtype == torch.bfloat16 else 4)
    gbs = nbytes / b_s / 1e9
    return dict(bound="hbm", kernel=f"k_bpass<{p}, 1, true> (B-pass, one run)", workload=label,
                achieved=round(gbs, 1), peak=HBM_GBS, unit="GB/s", frac=round(gbs / HBM_GBS, 4),
                traffic=stored_traffic(traffic_path) if traffic_path else None,
                algorithmic_bytes_per_launch=nbytes, avg_launch_us=round(b_s * 1e6, 2),
                apass_avg_launch_us=round(a_s * 1e6, 2),
                apass_achieved_gbs=round(nbytes / a_s / 1e9, 1))


def bench_ragged(n_images, T):
    """Ragged batch: single runs (gamma 1, seed = image index) on n_images
    images of different (L, N, p): the persistent kernel (one launch for the
    whole batch), the launch-per-kernel path (one launch per kernel and group
    of equal p) and per-image fits, each replayed from HIP graphs captured
    before the timed region (outputs preallocated).  Returns
    image-iterations/s of the three, the persistent kernel's HBM rate and the
    largest final-objective difference between the paths (they split their
    sums into different pixel groups)."""
    import numpy as np
    import torch
    from paper_2209_11002_amd import api, synth
    scenes, _ = synth.ragged_images(n_images)
    dev = torch.device("cuda:0")
    X = [api.normalize_pixels(torch.from_numpy(sc.X).to(dev)) for sc in scenes]
    ps = [sc.M.shape[1] for sc in scenes]
    seeds = list(range(n_images))
    gammas = [1.0] * n_images
    api.set_graph_cache(dev, n_images + 8)
    tpi, tuned_us = api.autotune_ragged(X, ps, seeds, gammas)      # recorded for this batch's class
    log(f"ragged: tuned {tpi} tiles per work item ({tuned_us:.0f} us per outer iteration)")

    def timed(fn):
        fn()                                                          # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    tb, rb = timed(lambda: api.fit_ragged(X, ps, seeds, gammas, T=T, graph=True))
    tg, rg = timed(lambda: api.fit_ragged(X, ps, seeds, gammas, T=T, graph=True, grouped=True))
    outs = [dict(A=torch.empty((ps[k], x.shape[1]), device=dev), B=torch.empty((x.shape[1], ps[k]), device=dev),
                 E=torch.empty((x.shape[0], ps[k]), device=dev)) for k, x in enumerate(X)]
    for k in range(n_images):                                         # capture every per-image graph
        api.fit(X[k], ps[k], T=T, gamma=1.0, seed=k, graph=True, out=outs[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [api.fit(X[k], ps[k], T=T, gamma=1.0, seed=k, graph=True, out=outs[k]) for k in range(n_images)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    fin = lambda r: np.array([x["loss"][-1] for x in r])  # noqa: E731
    diff = float(max(np.max(np.abs(fin(rb) - fin(rs)) / fin(rs)), np.max(np.abs(fin(rg) - fin(rs)) / fin(rs))))
    pixels = sum(sc.X.shape[1] for sc in scenes)
    nbytes = sum(pass_bytes(sc.X.shape[0], sc.X.shape[1], ps[k]) for k, sc in enumerate(scenes))
    per_outer = 6 * nbytes
    gbs = per_outer * T / tb / 1e9
    return dict(unit="image-iterations/s", images=n_images, T=T, pixels=pixels,
                batched=round(n_images * T / tb, 2), grouped=round(n_images * T / tg, 2),
                per_image=round(n_images * T / ts, 2), speedup=round(ts / tb, 3),
                final_loss_max_rel_diff_between_paths=float(f"{diff:.3g}"), tuned_tiles_per_item=tpi,
                pixel_groups_first_images=[r["pixel_groups"] for r in rb][:4],
                algorithmic_bytes_per_outer_iteration=per_outer, batched_gbs=round(gbs, 1),
                batched_hbm_frac=round(gbs / HBM_GBS, 4))


def rel_err(a, b):
    import numpy as np
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))))


def errors_vs_reference(r, ref, runs, T, idx, suffix, gammas, ref32=None):
    """Max errors of GPU runs against the stored float64 results, for the runs
    with gamma <= 1 and those with gamma >= 2 separately: objective (relative,
    whole trace), E (max-abs), A and N*B (max-abs on the sampled pixels), and
    the objective drift of the float32 oracle on the same runs when stored."""
    import numpy as np
    N = r["A"].shape[2]
    groups = {}
    for k, m in enumerate(runs):
        key = "gamma_le_1" if gammas[m] <= 1.0 else "gamma_ge_2"
        out = groups.setdefault(key, dict(runs=0, loss_rel=0.0, E_abs=0.0, A_abs=0.0, NB_abs=0.0))
        out["runs"] += 1
        out["loss_rel"] = max(out["loss_rel"], rel_err(r["loss"][m][:T + 1], ref[f"loss{suffix}"][k]))
        out["E_abs"] = max(out["E_abs"], float(np.max(np.abs(r["E"][m].cpu().numpy() - ref[f"E{suffix}"][k]))))
        A = r["A"][m][:, idx].cpu().numpy()
        B = r["B"][m][idx, :].cpu().numpy()
        out["A_abs"] = max(out["A_abs"], float(np.max(np.abs(A - ref[f"A{suffix}"][k]))))
        out["NB_abs"] = max(out["NB_abs"], float(N * np.max(np.abs(B - ref[f"B{suffix}"][k]))))
        if ref32 is not None:
            out["float32_oracle_loss_rel"] = max(out.get("float32_oracle_loss_rel", 0.0),
                                                 rel_err(ref32[f"loss{suffix}"][k], ref[f"loss{suffix}"][k]))
    return {g: {k: (float(f"{v:.3g}") if isinstance(v, float) else v) for k, v in d.items()}
            for g, d in groups.items()}


def bench_large(T, error_T=10):
    """The large smooth scene (L=224, N=512x614, p=12, M=20): the batched
    ensemble with bf16 X (bf16 matrix cores, and widened to the float32
    ones) and with float32 X (run-iterations/s), their errors against the
    stored float64 results (every run at T = 10; runs 0 and 4 at T = 100),
    the per-launch pass times of the bf16 ensemble, plus the plain
    single-run path on float32 X with its B-pass HBM roofline."""
    import numpy as np
    import torch
    from paper_2209_11002_amd import api, synth
    scene, cfg = synth.large_smooth()
    dev = torch.device("cuda:0")
    Xraw = torch.from_numpy(scene.X).to(dev)
    del scene
    X32 = api.normalize_pixels(Xraw)
    X16 = api.normalize_pixels(Xraw, out_dtype=torch.bfloat16)
    del Xraw
    seeds, gammas = cfg["seeds"], cfg["gammas"]
    M, p = len(seeds), 12
    L, N = X32.shape
    ref_path = os.path.join(GOLDEN, "large_fp64_ref.npz")
    ref = dict(np.load(ref_path)) if os.path.exists(ref_path) else None
    ref32_path = os.path.join(GOLDEN, "large_fp32_ref.npz")
    ref32 = dict(np.load(ref32_path)) if os.path.exists(ref32_path) else None
    res, errs, plans = {}, {}, {}
    for name, X in (("bf16", X16), ("f32", X32)):                  # launch shapes for both classes
        plans[name], tuned_us = api.autotune(X, p, M, K1=cfg["K1"], K2=cfg["K2"])
        log(f"large scene {name}: tuned launch shape {plans[name]} ({tuned_us:.0f} us per outer iteration)")
    for name, X, widen in (("bf16", X16, False), ("bf16_widen", X16, True), ("f32", X32, False)):
        api.ensemble(X, p, seeds, gammas, T=T, graph=True, bf16_widen=widen)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.ensemble(X, p, seeds, gammas, T=T, graph=True, bf16_widen=widen)
        torch.cuda.synchronize()
        res[name] = (M * T / (time.perf_counter() - t0), r["loss"][:, -1].copy())
        if ref is not None and not widen:
            e = {}
            long_runs = [int(m) for m in ref["long_runs"]]
            if T >= 100:
                e["T100_runs_0_4"] = errors_vs_reference(r, ref, long_runs, 100, ref["idx"], "100", gammas, ref32)
            r10 = api.ensemble(X, p, seeds, gammas, T=error_T)
            e["T10_all_runs"] = errors_vs_reference(r10, ref, list(range(M)), error_T, ref["idx"], "10", gammas,
                                                    ref32)
            errs[name] = e
        log(f"large scene {name}: {res[name][0]:.1f} run-it/s")
    rel = float(np.max(np.abs(res["bf16"][1] - res["f32"][1]) / res["f32"][1]))
    Q = M * p
    per_outer_bf16 = 6 * pass_bytes(L, N, Q, 2)
    api.ensemble(X16, p, seeds, gammas, T=3, time_passes=True)
    nb, bms = api.pass_times(dev, 1)
    na, ams = api.pass_times(dev, 0)
    b_us, a_us = 1e3 * bms / nb, 1e3 * ams / na
    passes = dict(bpass_avg_launch_us=round(b_us, 2), apass_avg_launch_us=round(a_us, 2),
                  bpass_algorithmic_gbs=round(pass_bytes(L, N, Q, 2) / b_us / 1e3, 1),
                  bpass_flops_per_launch=4.0 * L * N * Q,
                  bpass_fp32_equivalent_tflops=round(4.0 * L * N * Q / b_us / 1e6, 2))
    out = dict(unit="run-iterations/s", L=L, N=N, p=p, M=M, T=T, bf16=round(res["bf16"][0], 2),
               bf16_widen=round(res["bf16_widen"][0], 2), bf16_passes=passes, launch_shapes=plans,
               f32=round(res["f32"][0], 2), final_loss_max_rel_diff_bf16_vs_f32=rel,
               bf16_gbs=round(per_outer_bf16 * res["bf16"][0] / M / 1e9, 1),
               bf16_hbm_frac=round(per_outer_bf16 * res["bf16"][0] / M / 1e9 / HBM_GBS, 4),
               error_vs_fp64=errs or None)
    del X16
    plain = plain_pass_roofline(X32, p, 5, f"one run, L={L} N={N} p={p}, float32 X (X > 256 MB MALL)",
                                PLAIN_TRAFFIC_FILE)
    outp = dict(A=torch.empty((p, N), device=dev), B=torch.empty((N, p), device=dev),
                E=torch.empty((L, p), device=dev))
    v, _ = time_single_runs(X32, p, 10, 3, [1.0], [0], outp)
    plain["run_iterations_per_s"] = round(v, 2)
    return out, plain


def bench_small_plain(which):
    """Samson-shaped (T=200) or Jasper-shaped (T=100) single runs, replayed
    from a captured graph: run-iterations/s."""
    import torch
    from paper_2209_11002_amd import api, synth
    scene, cfg = (synth.samson_like() if which == "samson" else synth.jasper_like())
    dev = torch.device("cuda:0")
    X = api.normalize_pixels(torch.from_numpy(scene.X).to(dev))
    L, N = X.shape
    p = scene.M.shape[1]
    out = dict(A=torch.empty((p, N), device=dev), B=torch.empty((N, p), device=dev),
               E=torch.empty((L, p), device=dev))
    v, _ = time_single_runs(X, p, cfg["T"], 5, cfg["gammas"], cfg["seeds"], out)
    per_outer = 6 * pass_bytes(L, N, p)
    return dict(unit="run-iterations/s", L=L, N=N, p=p, T=cfg["T"], value=round(v, 2),
                algorithmic_gbs=round(per_outer * v / 1e9, 1))


def cpu_baseline(Xraw, p, seed, gamma, T_all, T_one):
    """The float64 oracle as it stands, on the same scene: T_all outer
    iterations of one run with every host thread, then T_one with one BLAS
    thread; run-iterations/s of both."""
    import platform
    import numpy as np
    from oracle import edaa as O
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    X, _ = O.normalize_pixels(Xraw.astype(np.float64))
    t0 = time.perf_counter()
    O.edaa_fit(X, p, T=T_all, gamma=gamma, seed=seed)
    dt_all = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        O.edaa_fit(X, p, T=T_one, gamma=gamma, seed=seed)
        dt_one = time.perf_counter() - t0
    return dict(all_threads=T_all / dt_all, threads=threads, one_thread=T_one / dt_one,
                s_all=dt_all, s_one=dt_one, cpu_model=model, cpu_count=os.cpu_count())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-runs", type=int, default=5, help="single runs timed for the plain path (0: skip)")
    ap.add_argument("--cpu-sample-T", type=int, default=20,
                    help="oracle outer iterations timed with all threads (0: skip); a quarter with one thread")
    ap.add_argument("--n-seeds", type=int, default=10)
    ap.add_argument("--ragged-images", type=int, default=64, help="images of the ragged batch (0: skip)")
    ap.add_argument("--large-T", "--bf16-T", dest="large_T", type=int, default=100,
                    help="outer iterations of the large-scene ensembles (0: skip the large scene)")
    ap.add_argument("--small-plain", type=int, default=1, help="time the Samson- and Jasper-shaped runs (0: skip)")
    ap.add_argument("--tune", type=int, default=1, help="autotune the headline launch shape first (0: default shape)")
    ap.add_argument("--shape", default=None, metavar="R,NPG",
                    help="pin the headline launch shape (runs per chunk, pixel groups) instead of tuning")
    ap.add_argument("--profile-run", type=int, default=0, metavar="T",
                    help="run a counter-profiling workload with T outer iterations and exit")
    ap.add_argument("--profile-workload", default="urban_ensemble",
                    choices=("urban_ensemble", "urban_single", "large_single", "large_bf16", "ragged"))
    ap.add_argument("--tiles-per-item", type=int, default=0,
                    help="--profile-workload ragged: work-item size of the persistent kernel (0: default)")
    ap.add_argument("--summarize", nargs="+", metavar="CSV", help="summarise rocprofv3 CSV files and exit")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run it with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.profile_run > 0:
        profile_run(args.profile_run, args.profile_workload, parse_shape(args.shape) if args.shape else None,
                    args.tiles_per_item)
        return

    import numpy as np
    import torch
    from paper_2209_11002_amd import api, synth

    dev = torch.device("cuda:0")
    scene, cfg = synth.urban_ensemble(n_seeds=args.n_seeds)
    L, N = scene.X.shape
    p, T, K1, K2 = 6, cfg["T"], cfg["K1"], cfg["K2"]
    seeds, gammas = cfg["seeds"], cfg["gammas"]
    M = len(seeds)
    Xraw = torch.from_numpy(scene.X).to(dev)
    shape = parse_shape(args.shape) if args.shape else (0, 0)
    if args.tune and not args.shape:
        best, us = api.autotune(api.normalize_pixels(Xraw), p, M, K1=K1, K2=K2)
        log(f"tuned launch shape {best}: {us:.0f} us per outer iteration")
    plan = api.plan(L, N, p, M, runs_per_chunk=shape[0], pixel_groups=shape[1])
    log(f"scene L={L} N={N} p={p} M={M} T={T}, plan {plan}")
    out = dict(A=torch.empty((M, p, N), device=dev), B=torch.empty((M, N, p), device=dev),
               E=torch.empty((M, L, p), device=dev))

    def step(graph=False, time_passes=False):
        Xn = api.normalize_pixels(Xraw)
        return api.ensemble(Xn, p, seeds, gammas, T=T, K1=K1, K2=K2, graph=graph, out=out,
                            time_passes=time_passes, runs_per_chunk=shape[0], pixel_groups=shape[1])

    for w in range(args.warmup):
        step(time_passes=True)
        step(graph=True)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    # Kernel timing: eager launches, with HIP events recorded around every
    # pass launch on the library's stream (events inside a replayed graph
    # carry no timestamps on this runtime); these give the roofline's
    # per-launch durations.
    b_ms, b_n, a_ms, a_n = 0.0, 0, 0.0, 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = step(time_passes=True)
        n, ms = api.pass_times(dev, 1)
        b_n += n
        b_ms += ms
        n, ms = api.pass_times(dev, 0)
        a_n += n
        a_ms += ms
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value_eager = M * T * args.steps / dt

    # Timed region (value): the same steps as the workload runs them, the
    # ensemble replayed from its captured HIP graph (bit-identical results)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rg = step(graph=True)
        log(f"graph step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    gdt = time.perf_counter() - t0
    value = M * T * args.steps / gdt
    ms_per_step = 1e3 * gdt / args.steps
    assert np.array_equal(rg["loss"], r["loss"]), "graph replay differs from eager launches"
    log(f"graph replay: {value:.1f} run-it/s (eager launches with pass events: {value_eager:.1f})")

    # algorithmic bytes and flops (float32 state, X read once per pass)
    Q = M * p
    xb = L * N * 4
    bpass_bytes = pass_bytes(L, N, Q)
    bpass_flops = 4.0 * L * N * Q
    step_bytes = (2 * xb                       # normalisation
                  + xb + 2 * Q * N * 4         # A0 fill + init pass (writes B)
                  + T * (1 + K2) * bpass_bytes
                  + xb + Q * N * 4             # closing pass
                  + 2 * Q * N * 4)             # B output
    b_avg_s = b_ms / max(b_n, 1) / 1e3
    a_avg_s = a_ms / max(a_n, 1) / 1e3
    achieved = bpass_flops / b_avg_s / 1e12
    R = plan["runs_per_chunk"]
    split_b, split_a = bool(plan["bf16_passes"] & 1), bool(plan["bf16_passes"] & 2)
    roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=FP32_MFMA_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / FP32_MFMA_TFLOPS, 4),
                    traffic=stored_traffic(TRAFFIC_FILE, f"{plan['runs_per_chunk']},{plan['pixel_groups']}"),
                    kernel=(f"k_bpass_xs<{p}, {R}, true> (B-pass; float32 products as six bf16 matrix-core products)"
                            if split_b else f"k_bpass<{p}, {R}, true> (B-pass on the float32 matrix cores)"),
                    avg_launch_us=round(b_avg_s * 1e6, 2),
                    algorithmic_bytes_per_launch=bpass_bytes, flops_per_launch=bpass_flops,
                    achieved_gbs=round(bpass_bytes / b_avg_s / 1e9, 1),
                    apass_kernel=f"k_apass_xs<{p}, {R}>" if split_a else f"k_apass<{p}, {R}>",
                    apass_avg_launch_us=round(a_avg_s * 1e6, 2))
    if split_b:
        # the same float32 work priced at the kernel's own matrix-core
        # ceiling: six bf16 products per float32 product
        roofline["bf16x6_peak_tflops"] = round(BF16_MFMA_TFLOPS / 6, 1)
        roofline["frac_of_bf16x6_peak"] = round(achieved / (BF16_MFMA_TFLOPS / 6), 4)
    final_loss_batched = r["loss"][:, -1].copy()
    log(f"batched: {value:.1f} run-it/s, {ms_per_step:.1f} ms/step, B-pass {b_avg_s * 1e6:.1f} us")

    # error of the headline runs 0 (gamma 0.25) and 4 (gamma 4) against the
    # stored float64 traces (input normalised on the GPU)
    gold = np.loadtxt(os.path.join(GOLDEN, "urban_fp64_traces.txt"))
    headline_err = None
    if args.n_seeds >= 1:
        headline_err = {f"run_{m}_gamma_{gammas[m]}_loss_rel_max_over_trace": float(f"{rel_err(r['loss'][m], gold[:, c]):.3g}")
                        for c, m in ((1, 0), (2, 4))}

    plain = None
    if args.plain_runs > 0:
        Xn = api.normalize_pixels(Xraw)
        outp = dict(A=torch.empty((p, N), device=dev), B=torch.empty((N, p), device=dev),
                    E=torch.empty((L, p), device=dev))
        pval, losses = time_single_runs(Xn, p, T, args.plain_runs, gammas, seeds, outp)
        diffs = np.abs(np.array(losses) - final_loss_batched[:args.plain_runs]) / final_loss_batched[:args.plain_runs]
        plain = dict(value=round(pval, 2), unit="run-iterations/s", runs=args.plain_runs,
                     batched_speedup=round(value / pval, 2),
                     final_loss_rel_diff_per_run={f"gamma_{gammas[m]}": float(f"{d:.3g}") for m, d in enumerate(diffs)},
                     roofline_urban=plain_pass_roofline(Xn, p, 5, f"one run, L={L} N={N} p={p} (X fits the MALL)"))
        log(f"plain: {pval:.1f} run-it/s (speedup {value / pval:.2f}x, final-loss rel diffs {diffs})")

    small = None
    if args.small_plain:
        small = dict(samson_shaped=bench_small_plain("samson"), jasper_shaped=bench_small_plain("jasper"))
        log(f"small plain: {small}")

    large, plain_large = None, None
    if args.large_T > 0:
        log("large smooth scene: bf16 and float32 X ensembles, plain single run")
        large, plain_large = bench_large(args.large_T)
        log(f"large: {large}")
        log(f"plain large: {plain_large}")

    ragged = None
    if args.ragged_images > 0:
        log(f"ragged batch: {args.ragged_images} images")
        ragged = bench_ragged(args.ragged_images, T)
        log(f"ragged: persistent {ragged['batched']}, grouped {ragged['grouped']}, "
            f"per-image {ragged['per_image']} image-it/s")

    cpu = None
    if args.cpu_sample_T > 0:
        log("timing the float64 oracle on the host")
        t_one = max(1, args.cpu_sample_T // 4)
        c = cpu_baseline(scene.X, p, seeds[0], gammas[0], args.cpu_sample_T, t_one)
        cpu = dict(value=round(c["all_threads"], 4), unit="run-iterations/s", cores=c["threads"], kind="oracle",
                   sample=f"1 run x {args.cpu_sample_T} outer iterations (K1=K2=5) of the float64 oracle "
                          f"on the full {L}x{N} scene with {c['threads']} BLAS threads, {c['s_all']:.1f} s; "
                          f"{t_one} outer iterations with 1 thread, {c['s_one']:.1f} s",
                   one_thread=round(c["one_thread"], 4), cpu_model=c["cpu_model"], cpu_count=c["cpu_count"])
        log(f"oracle: {c['all_threads']:.4f} run-it/s on {c['threads']} threads, {c['one_thread']:.4f} on 1")

    if plain is not None and plain_large is not None:
        plain["roofline"] = plain_large

    stream = measured_stream_ceiling(dev)
    log(f"measured streaming ceilings: read {stream['read_gbs']} GB/s, copy {stream['copy_gbs']} GB/s")
    ceiling = max(stream["read_gbs"], stream["copy_gbs"])
    for rl in ([plain.get("roofline_urban"), plain.get("roofline")] if plain else []) + \
            ([ragged] if ragged else []):
        if rl is not None:
            gbs = rl.get("achieved", rl.get("batched_gbs"))
            rl["frac_of_measured_stream"] = round(gbs / ceiling, 4)

    line = {
        "metric": "EDAA run-iterations/sec + HBM GB/s; batched vs plain at equal loss",
        "value": round(value, 2),
        "unit": "run-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched EDAA ensemble, Urban-shaped synthetic scene L={L} N={N} (307x307) "
                               f"p={p}, M={M} runs (seeds x gamma 0.25..4), T={T}, K1={K1}, K2={K2}, "
                               f"Dirichlet(0.7) abundances, noise sigma 0.02",
                   "L": L, "N": N, "p": p, "M": M, "T": T, "K1": K1, "K2": K2, "launch_shape": plan},
        "hbm_gbs": round(step_bytes / (ms_per_step / 1e3) / 1e9, 1),
        "hbm_measured": stream,
        "value_eager": round(value_eager, 2),
        "roofline": roofline,
        "error_vs_fp64": headline_err,
        "plain": plain,
        "small_plain": small,
        "large_scene": large,
        "ragged": ragged,
        "cpu_baseline": cpu,
        "selected_run": int(r["selected"]),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
