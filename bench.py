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
the plain path (single runs on the same data, at equal final loss) and the
float64 oracle timed on this host's cores on a bounded sample.
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
HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bpass_urban_ensemble_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2209_11002_amd", "csrc", "edaa_kernels.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_sha256():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stored_traffic():
    """HBM bytes per B-pass launch from the committed counter summary, or None
    when it is missing or was taken from another version of the kernels."""
    try:
        fields = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        if fields.get("kernel_source_sha256") != kernel_source_sha256():
            return None
        return int(float(fields["traffic_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def profile_run(T):
    """Workload for rocprofv3 counter passes: a plain device copy of known size
    (the calibration of FETCH_SIZE / WRITE_SIZE) and then a short ensemble on
    the bench scene (T outer iterations, so 5 T B-pass launches)."""
    import torch
    from paper_2209_11002_amd import api, synth
    dev = torch.device("cuda:0")
    nbytes = 256 << 20
    src = torch.ones(nbytes // 4, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)          # reads and writes exactly nbytes
    torch.cuda.synchronize()
    log(f"calibration copy: {nbytes} bytes read, {nbytes} bytes written")
    scene, cfg = synth.urban_ensemble()
    X = api.normalize_pixels(torch.from_numpy(scene.X).to(dev))
    api.ensemble(X, 6, cfg["seeds"], cfg["gammas"], T=T, K1=cfg["K1"], K2=cfg["K2"])
    torch.cuda.synchronize()
    log(f"profile run done (T={T})")


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


def bench_ragged(n_images, T):
    """Ragged batch: single runs (gamma 1, seed = image index) on n_images
    images of different (L, N, p), batched (one launch per kernel and group of
    equal p, replayed from a HIP graph) against per-image fits (each replayed
    from its own graph).  Returns image-iterations/s of both."""
    import numpy as np
    import torch
    from paper_2209_11002_amd import api, synth
    scenes, _ = synth.ragged_images(n_images)
    dev = torch.device("cuda:0")
    X = [api.normalize_pixels(torch.from_numpy(sc.X).to(dev)) for sc in scenes]
    ps = [sc.M.shape[1] for sc in scenes]
    seeds = list(range(n_images))
    gammas = [1.0] * n_images
    api.fit_ragged(X, ps, seeds, gammas, T=T, graph=True)            # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = api.fit_ragged(X, ps, seeds, gammas, T=T, graph=True)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    for k in range(n_images):                                         # capture
        api.fit(X[k], ps[k], T=T, gamma=1.0, seed=k, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [api.fit(X[k], ps[k], T=T, gamma=1.0, seed=k, graph=True) for k in range(n_images)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    same = all(np.array_equal(a["loss"], b["loss"]) for a, b in zip(rb, rs))
    pixels = sum(sc.X.shape[1] for sc in scenes)
    return dict(unit="image-iterations/s", images=n_images, T=T, pixels=pixels,
                batched=round(n_images * T / tb, 2), per_image=round(n_images * T / ts, 2),
                speedup=round(ts / tb, 3), identical_to_per_image=bool(same))


def bench_bf16_large(T):
    """BF16 X on the large smooth scene (L=224, N=512x614, p=12, M=20): the
    batched ensemble with X stored in bf16, against the same ensemble with
    float32 X (run-iterations/s of both, and the largest relative difference
    of the final objective between them)."""
    import numpy as np
    import torch
    from paper_2209_11002_amd import api, synth
    scene, cfg = synth.large_smooth()
    dev = torch.device("cuda:0")
    Xraw = torch.from_numpy(scene.X).to(dev)
    X32 = api.normalize_pixels(Xraw)
    X16 = api.normalize_pixels(Xraw, out_dtype=torch.bfloat16)
    del Xraw
    seeds, gammas = cfg["seeds"], cfg["gammas"]
    M, p = len(seeds), 12
    res = {}
    for name, X in (("bf16", X16), ("f32", X32)):
        api.ensemble(X, p, seeds, gammas, T=T, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.ensemble(X, p, seeds, gammas, T=T, graph=True)
        torch.cuda.synchronize()
        res[name] = (M * T / (time.perf_counter() - t0), r["loss"][:, -1].copy())
    rel = float(np.max(np.abs(res["bf16"][1] - res["f32"][1]) / res["f32"][1]))
    L, N = X32.shape
    return dict(unit="run-iterations/s", L=L, N=N, p=p, M=M, T=T, bf16=round(res["bf16"][0], 2),
                f32=round(res["f32"][0], 2), final_loss_max_rel_diff_bf16_vs_f32=rel)


def cpu_baseline(Xraw, p, seed, gamma, T_sample):
    """The float64 oracle as it stands, on the same scene, for T_sample outer
    iterations of one run; returns run-iterations/s and the threads used."""
    import numpy as np
    from oracle import edaa as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    X, _ = O.normalize_pixels(Xraw.astype(np.float64))
    t0 = time.perf_counter()
    O.edaa_fit(X, p, T=T_sample, gamma=gamma, seed=seed)
    dt = time.perf_counter() - t0
    return T_sample / dt, threads, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-runs", type=int, default=5, help="single runs timed for the plain path (0: skip)")
    ap.add_argument("--cpu-sample-T", type=int, default=40, help="oracle outer iterations timed (0: skip)")
    ap.add_argument("--n-seeds", type=int, default=10)
    ap.add_argument("--ragged-images", type=int, default=64, help="images of the ragged batch (0: skip)")
    ap.add_argument("--bf16-T", type=int, default=100, help="outer iterations of the BF16 large-scene runs (0: skip)")
    ap.add_argument("--profile-run", type=int, default=0, metavar="T",
                    help="run the counter-profiling workload with T outer iterations and exit")
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
        profile_run(args.profile_run)
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
    log(f"scene L={L} N={N} p={p} M={M} T={T}")
    Xraw = torch.from_numpy(scene.X).to(dev)
    out = dict(A=torch.empty((M, p, N), device=dev), B=torch.empty((M, N, p), device=dev),
               E=torch.empty((M, L, p), device=dev))

    def step(graph=False, time_passes=False):
        Xn = api.normalize_pixels(Xraw)
        return api.ensemble(Xn, p, seeds, gammas, T=T, K1=K1, K2=K2, graph=graph, out=out,
                            time_passes=time_passes)

    for w in range(args.warmup):
        step(time_passes=True)
        step(graph=True)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    # Timed region: eager launches, with HIP events recorded around every pass
    # launch on the library's stream (events inside a replayed graph carry no
    # timestamps on this runtime).

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
    ms_per_step = 1e3 * dt / args.steps
    value = M * T * args.steps / dt

    # the same steps replayed from the captured HIP graph (no events)
    t0 = time.perf_counter()
    for k in range(args.steps):
        rg = step(graph=True)
    torch.cuda.synchronize()
    gdt = time.perf_counter() - t0
    value_graph = M * T * args.steps / gdt
    assert np.array_equal(rg["loss"], r["loss"]), "graph replay differs from eager launches"
    log(f"graph replay: {value_graph:.1f} run-it/s")

    # algorithmic bytes and flops (float32 state, X read once per pass)
    Q = M * p
    xb = L * N * 4
    bpass_bytes = xb + 2 * Q * N * 4
    bpass_flops = 4.0 * L * N * Q
    apass_bytes = xb + 2 * Q * N * 4
    step_bytes = (2 * xb                       # normalisation
                  + xb + 2 * Q * N * 4         # A0 fill + init pass (writes B)
                  + T * (apass_bytes + K2 * bpass_bytes)
                  + xb + Q * N * 4             # closing pass
                  + 2 * Q * N * 4)             # B output
    b_avg_s = b_ms / max(b_n, 1) / 1e3
    a_avg_s = a_ms / max(a_n, 1) / 1e3
    achieved = bpass_flops / b_avg_s / 1e12
    roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=FP32_MFMA_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / FP32_MFMA_TFLOPS, 4), traffic=stored_traffic(),
                    kernel="k_bpass (B-pass)", avg_launch_us=round(b_avg_s * 1e6, 2),
                    algorithmic_bytes_per_launch=bpass_bytes, flops_per_launch=bpass_flops,
                    achieved_gbs=round(bpass_bytes / b_avg_s / 1e9, 1),
                    apass_avg_launch_us=round(a_avg_s * 1e6, 2))
    final_loss_batched = r["loss"][:, -1].copy()
    log(f"batched: {value:.1f} run-it/s, {ms_per_step:.1f} ms/step, B-pass {b_avg_s * 1e6:.1f} us")

    plain = None
    if args.plain_runs > 0:
        Xn = api.normalize_pixels(Xraw)
        api.fit(Xn, p, T=T, gamma=gammas[0], seed=seeds[0], graph=True)   # capture
        torch.cuda.synchronize()
        losses = []
        t0 = time.perf_counter()
        for m in range(args.plain_runs):
            rr = api.fit(Xn, p, T=T, K1=K1, K2=K2, gamma=gammas[m], seed=seeds[m], graph=True)
            losses.append(rr["loss"][-1])
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        pval = args.plain_runs * T / pdt
        rel = float(np.max(np.abs(np.array(losses) - final_loss_batched[:args.plain_runs])
                           / final_loss_batched[:args.plain_runs]))
        plain = dict(value=round(pval, 2), unit="run-iterations/s", runs=args.plain_runs,
                     batched_speedup=round(value / pval, 2), final_loss_max_rel_diff=rel)
        log(f"plain: {pval:.1f} run-it/s (speedup {value / pval:.2f}x, final-loss rel diff {rel:.2e})")

    ragged = None
    if args.ragged_images > 0:
        log(f"ragged batch: {args.ragged_images} images")
        ragged = bench_ragged(args.ragged_images, T)
        log(f"ragged: batched {ragged['batched']} vs per-image {ragged['per_image']} image-it/s")
    bf16 = None
    if args.bf16_T > 0:
        log("bf16 X, large smooth scene")
        bf16 = bench_bf16_large(args.bf16_T)
        log(f"bf16: {bf16['bf16']} run-it/s (f32 {bf16['f32']}), final-loss rel diff {bf16['final_loss_max_rel_diff_bf16_vs_f32']:.2e}")

    cpu = None
    if args.cpu_sample_T > 0:
        log("timing the float64 oracle on the host")
        v, threads, cdt = cpu_baseline(scene.X, p, seeds[0], gammas[0], args.cpu_sample_T)
        cpu = dict(value=round(v, 4), unit="run-iterations/s", cores=threads, kind="oracle",
                   sample=f"1 run x {args.cpu_sample_T} outer iterations (K1=K2=5) of the float64 oracle "
                          f"on the full {L}x{N} scene, {cdt:.1f} s")
        log(f"oracle: {v:.4f} run-it/s on {threads} threads")

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
                   "L": L, "N": N, "p": p, "M": M, "T": T, "K1": K1, "K2": K2},
        "hbm_gbs": round(step_bytes / (ms_per_step / 1e3) / 1e9, 1),
        "value_graph_replay": round(value_graph, 2),
        "roofline": roofline,
        "plain": plain,
        "ragged": ragged,
        "bf16_large": bf16,
        "cpu_baseline": cpu,
        "selected_run": int(r["selected"]),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
