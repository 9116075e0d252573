"""Benchmark: tomogram voxels per second for a full TTM pass on one MI355X.

A step is one full pass over the tomogram: prefilter + local normalisation,
the K FFT correlations on overlapping tiles (512^3 for the 512 x 928 x 928
tomogram: 4 tiles), per-voxel score and orientation (SS-HOPM) on every valid
voxel, and Find Peaks.  The tomogram and
the template spectra are resident on the GPU before timing starts; the
one-time tensor template and its spectra are built beforehand and are not
timed (the paper excludes template generation too).

Prints one JSON line (see the field list at the end of main()).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (synth config, FFT tile edge, peaks P)
    "c3_512x928x928_n6": ("c3_512x928x928_n6", 512, 2000),
    "c2_256cube_n6": ("c2_256cube_n6", 256, 200),
    "c1_64cube_n4": ("c1_64cube_n4", 64, 5),
    # 64 subtomograms, edges in {96,128,160,192}, 3 templates, one graph launch per batch
    "c5_batch64_n6": ("c5_batch64_n6", 0, 60),
}

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # published MI355X FP32 vector peak (dual-issue / packed)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def clean(o):
    """Strict JSON: non-finite floats become None."""
    if isinstance(o, float):
        return o if math.isfinite(o) else None
    if isinstance(o, dict):
        return {k: clean(v) for k, v in o.items()}
    if isinstance(o, (list, tuple)):
        return [clean(v) for v in o]
    return o


def extract_flops(n: int, n_starts: int = 16, shift_steps: int = 12) -> dict:
    """FP32 operations (an FMA counts 2) of the extraction kernels' pieces, d' = 3, degree n.

    Counted from the kernels' arithmetic: contract = C u^{n-1} (powers,
    monomials with their multinomial, 3 FMAs per monomial); step = one SS-HOPM
    update; newton = one Newton step (tangent basis, C u^{n-2}, 2 x 2 solve,
    retraction, new gradient); shift = Gershgorin interval of the unfolding
    block plus `shift_steps` Cholesky bisection tests; run = start
    normalisation and its first gradient, plus the gradient the reduction
    recomputes at the run's answer; score = ||C||_F; learned = features and
    the first gradient of the learned start (its BF16 MLP runs on the matrix
    cores and is counted apart); screen = <C, s^n> for every fixed start.
    """
    K = (n + 1) * (n + 2) // 2
    Kb = n * (n + 1) // 2
    K2 = (n - 1) * n // 2
    M = (n // 2 + 1) * (n // 2 + 2) // 2
    contract = 3 * (n - 1) + 9 * Kb
    contract2 = 3 * (n - 2) + 15 * K2
    chol = M * (M + 1) // 2 + sum(2 * j + 3 for j in range(M)) + sum((M - 1 - j) * (2 * j + 1) for j in range(M))
    return dict(score=2 * K + 1, step=contract + 23, newton=contract2 + contract + 106,
                shift=2 * M * M + shift_steps * chol, run=2 * contract + 10,
                learned=2 * K + contract, screen=n_starts * 2 * K,
                mlp_mfma=2 * (32 * 64 + 64 * 64 + 64 * 16))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_512x928x928_n6", choices=sorted(WORKLOADS))
    ap.add_argument("--fft", type=int, default=0, help="FFT tile edge (0: the workload's default)")
    ap.add_argument("--nq-base", type=int, default=1000, help="super-Fibonacci points per cube rotation")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=400, help="voxels in the oracle timing sample")
    ap.add_argument("--field-dtype", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--start", default="both", choices=["plain", "learned", "both"],
                    help="both = plain, learned (screened fallback) and learned without screening")
    ap.add_argument("--train-steps", type=int, default=120000)
    ap.add_argument("--net-cache", default="",
                    help="file for the trained learned-start network: loaded if present, else "
                         "written after training")
    ap.add_argument("--template-cache", default="",
                    help="file for the tensor template (Alg. 1): loaded if its key (template, "
                         "degree, form, rotations, mask) matches, else built and written")
    ap.add_argument("--train-volumes", type=int, default=10)
    ap.add_argument("--also-fft", type=int, default=256,
                    help="also time the learned pass on this FFT tile edge (0: no)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the tile correlations on the same stream as the extractions")
    ap.add_argument("--precision-report", action="store_true",
                    help="FP32 vs BF16 field storage: throughput and error against the FP64 oracle")
    ap.add_argument("--noise-sweep", action="store_true",
                    help="rotation and position error against the planted copies over SNR levels "
                         "(quaternion form, TTM and TTM-ref)")
    ap.add_argument("--snr", type=str, default="10,3,1,0.3,0.1", help="SNR levels of the noise sweep")
    ap.add_argument("--wedge", action="store_true",
                    help="noise sweep with a +-60 degree missing wedge and the wedge-aware template")
    ap.add_argument("--dense-snr", type=float, default=1.0,
                    help="noise sweep: SNR of the dense orientation pass, plain vs learned start "
                         "(0: none)")
    ap.add_argument("--tile-call", action="store_true",
                    help="time one full 512^3 tile's normalisation-and-correlation call alone "
                         "(degree 6, L = 40), for kernel profiling")
    ap.add_argument("--max-wrong", type=float, default=0.05,
                    help="fallback calibration: accepted learned voxels off by > 1 deg at most this often")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import synth
    from paper_2408_02398_amd import ttm

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(2)
    if args.noise_sweep:
        print(json.dumps(clean(noise_sweep(args))), flush=True)
        return
    if args.tile_call:
        print(json.dumps(clean(tile_call(args))), flush=True)
        return
    cfg_name, fft_n, top_p = WORKLOADS[args.workload]
    if args.fft:
        fft_n = args.fft
    if cfg_name == "c5_batch64_n6":
        print(json.dumps(clean(bench_batch(args, top_p))), flush=True)
        return
    p = synth.CONFIGS[cfg_name]
    n, L, r = p["degree"], p["L"], p["mask_radius"]

    if args.precision_report:
        print(json.dumps(clean(precision_report(args, cfg_name, fft_n, top_p))), flush=True)
        return
    t0 = time.time()
    log(f"[bench] generating {cfg_name} ...")
    wl = synth.make_config(cfg_name)
    log(f"[bench] generated in {time.time() - t0:.1f}s; {len(wl.centres)} copies")
    dev = torch.device("cuda:0")
    ctx = ttm.Context(0)
    d = ttm.make_desc(n, L, r)
    vol = torch.from_numpy(wl.volume).to(dev)
    Q = torch.from_numpy(synth.rotation_samples(args.nq_base)).float().to(dev)
    p = synth.CONFIGS[cfg_name]
    t1 = time.time()
    Tg = tensor_template_cached(args.template_cache, ctx, d, wl.template, Q, ttm, torch)
    spec = ttm.template_spectra(ctx, d, Tg, fft_n)
    torch.cuda.synchronize()
    log(f"[bench] tensor template ({Q.shape[0]} rotations) + spectra in {time.time() - t1:.2f}s")
    T_host = Tg.cpu().numpy() if not args.no_cpu_baseline else None
    starts = torch.from_numpy(synth.start_vectors()).to(dev)
    field_dtype = torch.bfloat16 if args.field_dtype == "bf16" else torch.float32
    lo, hi = ttm.valid_bounds(vol.shape, L)
    nvox = int(np.prod(vol.shape))
    nvalid = int(np.prod([h - l + 1 for l, h in zip(lo, hi)]))

    learn_info = None
    net, kappa = None, 0.0
    # the trained network depends on the workload's recipe and the training
    # settings: a cached one is used only under the same key
    import hashlib
    hk = hashlib.sha256()
    hk.update(np.ascontiguousarray(wl.template, dtype=np.float32).tobytes())
    hk.update(json.dumps([cfg_name, n, L, r, p["snr"], p["wedge"], p["n_blobs"], p["min_sep"],
                          args.train_steps, args.train_volumes, args.max_wrong, args.nq_base]).encode())
    net_key = hk.hexdigest()
    cache = None
    if args.start in ("learned", "both") and args.net_cache and os.path.exists(args.net_cache):
        cache = np.load(args.net_cache, allow_pickle=False)
        if "key" not in cache.files or str(cache["key"]) != net_key:
            log(f"[bench] {args.net_cache} holds a network for other settings: training anew")
            cache = None
    if cache is not None:
        # a network this script trained and saved earlier under the same key
        net = ttm.MLP(ctx, d, torch.from_numpy(cache["params"]).to(dev))
        kappa = float(cache["kappa"])
        learn_info = {"loaded_from": args.net_cache, "kappa": kappa}
        log(f"[bench] learned start loaded from {args.net_cache}")
    elif args.start in ("learned", "both"):
        from paper_2408_02398_amd import learn
        t2 = time.time()
        tr = [synth.make_tomogram(f"train{i}", (256, 256, 256), L=L, n_blobs=p["n_blobs"],
                                  n_copies=100, min_sep=p["min_sep"], mask_radius=r, degree=n,
                                  seed=1000 + i, snr=p["snr"], wedge=p["wedge"],
                                  template_seed=p["seed"]) for i in range(args.train_volumes + 1)]
        assert all(np.array_equal(t.template, wl.template) for t in tr)
        vols = [torch.from_numpy(t.volume).to(dev) for t in tr]
        spec_tr = spec if fft_n == 256 else ttm.template_spectra(ctx, d, Tg, 256)
        log(f"[bench] training tomograms generated in {time.time() - t2:.1f}s")
        net, kappa, learn_info = learn.build_learned_start(
            ctx, d, spec_tr, 256, vols, starts, steps=args.train_steps, max_wrong=args.max_wrong,
            log=log)
        del vols
        if args.net_cache:
            np.savez(args.net_cache, params=net.params.cpu().numpy(), kappa=np.float64(kappa),
                     key=np.array(net_key))

    # per-stage timing with events on the stream the library launches on
    stream = torch.cuda.current_stream()
    counters = torch.zeros(5, dtype=torch.int64, device=dev)   # extraction work (timed steps)

    def run_mode(mode: str):
        eng = ttm.Engine(ctx, d, spec, fft_n, vol.shape, starts, field_dtype=field_dtype,
                         mlp=net if mode.startswith("learned") else None, kappa=kappa,
                         screen=(mode == "learned"))

        def one_pass(timed: bool, count: bool = False):
            tm = {} if timed else None
            res = eng.run(vol, top_p=top_p, timing=tm, overlap=not args.no_overlap,
                          counters=counters if count else None)
            return tm, res.peaks

        for i in range(args.warmup):
            log(f"[bench] {mode}: warmup {i + 1}/{args.warmup}")
            one_pass(False)
        torch.cuda.synchronize()
        counters.zero_()
        eng.fallbacks.zero_()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stage = {"normalize": 0.0, "correlate": 0.0, "extract": 0.0, "peaks": 0.0}
        ext_launch_ms, corr_launch_ms = [], []
        torch.cuda.synchronize()
        start.record(stream)
        wall0 = time.time()
        for i in range(args.steps):
            tm, pk = one_pass(True)
            torch.cuda.synchronize()
            log(f"[bench] {mode}: step {i + 1}/{args.steps} done")
            stage["normalize"] += sum(a.elapsed_time(b) for a, b in tm["normalize"])
            stage["peaks"] += sum(a.elapsed_time(b) for a, b in tm["peaks"])
            for a, b, size in tm["correlate"]:
                t = a.elapsed_time(b)
                stage["correlate"] += t
                corr_launch_ms.append(t)
            for a, b, size in tm["extract"]:
                t = a.elapsed_time(b)
                stage["extract"] += t
                ext_launch_ms.append((t, int(np.prod(size))))
        stop.record(stream)
        torch.cuda.synchronize()
        fallbacks = int(eng.fallbacks.item()) // max(args.steps, 1)
        wall = time.time() - wall0
        # work counts (SS-HOPM updates, Newton steps, ...) come from one more,
        # untimed pass: their per-wavefront atomics would slow the timed ones.
        # It runs the correlations on the caller's stream, so its per-launch
        # event times are each stage's own (in the overlapped passes a side-stream
        # launch also spans the time it waits for CUs the extraction holds).
        counters.zero_()
        tm_s = {}
        eng.run(vol, top_p=top_p, timing=tm_s, overlap=False, counters=counters)
        torch.cuda.synchronize()
        serial = {"correlate": [(a.elapsed_time(b), size) for a, b, size in tm_s["correlate"]],
                  "extract": [a.elapsed_time(b) for a, b, _ in tm_s["extract"]]}
        serial_stages = {"normalize": sum(a.elapsed_time(b) for a, b in tm_s["normalize"]),
                         "correlate": sum(t for t, _ in serial["correlate"]),
                         "extract": sum(serial["extract"]),
                         "peaks": sum(a.elapsed_time(b) for a, b in tm_s["peaks"])}
        per_pass = [int(v) for v in counters.cpu().tolist()]
        eng.release()             # keep the maps for the accuracy gate, free the workspaces
        torch.cuda.empty_cache()
        res = dict(eng=eng, pk=pk, stage=stage, ext=ext_launch_ms, corr=corr_launch_ms, serial=serial,
                   serial_stages=serial_stages,
                   ms_step=start.elapsed_time(stop) / args.steps, wall=wall,
                   counters=[v * args.steps for v in per_pass], fallbacks=fallbacks)
        return res

    modes = ["plain", "learned", "learned_unscreened"] if args.start == "both" else [args.start]
    results = {m: run_mode(m) for m in modes}
    main_mode = "learned" if "learned" in results else "plain"
    R = results[main_mode]
    ms_step = R["ms_step"]
    value = nvox / (ms_step / 1e3)
    n_peaks = int(R["pk"].shape[0])
    n_tiles = len(R["eng"].boxes)

    # accuracy gate: learned vs plain (plain is the reference) on the voxels that matter
    gate = None
    if "learned" in results and "plain" in results:
        gate = accuracy_gate(results["plain"], results["learned"], lo, hi, top_p, ttm, torch)
        if "learned_unscreened" in results:
            gate["unscreened"] = accuracy_gate(results["plain"], results["learned_unscreened"], lo,
                                               hi, top_p, ttm, torch)

    # roofline of the dominant kernel
    K = ttm.n_components(n, 3)
    step_ = fft_n - L + 1
    stage = R["stage"]
    corr_launch_ms, ext_launch_ms = R["corr"], R["ext"]
    corr_avg = float(np.mean(corr_launch_ms))
    ext_avg = float(np.mean([t for t, _ in ext_launch_ms]))
    # per-tile launch (ttm_normalize_correlate on a full interior tile):
    # compulsory bytes = read the g tile, the K x/y-transformed template planes
    # and the mask's, write the w crop and read it back for the product, write
    # the K cropped field planes
    tse = ttm.template_spectrum_elems(fft_n, L)
    corr_bytes = 4 * fft_n ** 3 + (K + 1) * tse * 8 + 2 * 4 * step_ ** 3 + 4 * K * step_ ** 3
    corr_full = [t for t, (blo, size) in zip(corr_launch_ms, R["eng"].boxes * args.steps)
                 if size == (step_, step_, step_)]
    corr_full_avg = float(np.mean(corr_full)) if corr_full else corr_avg
    ser = R["serial"]
    ser_corr_full = [t for t, size in ser["correlate"] if size == (step_, step_, step_)]
    ser_corr = float(np.mean(ser_corr_full)) if ser_corr_full else float(np.mean([t for t, _ in ser["correlate"]]))
    ser_ext = float(np.mean(ser["extract"]))
    # the dominant stage by its own kernel time (the untimed serial pass)
    dominant = ("extract" if sum(ser["extract"]) >= sum(t for t, _ in ser["correlate"])
                else "correlate")
    f = extract_flops(n)
    steps_, newton_, oriented, shifts, runs = R["counters"]
    voxels = sum(nv for _, nv in ext_launch_ms)
    learned = main_mode.startswith("learned")
    flops = (voxels * f["score"] + shifts * f["shift"] + runs * f["run"] + steps_ * f["step"]
             + newton_ * f["newton"])
    if learned:
        flops += oriented * (f["learned"] + (f["screen"] if main_mode == "learned" else 0))
    mfma = oriented * f["mlp_mfma"] if learned else 0
    ach = flops / (stage["extract"] / 1e3) / 1e12
    # the survey's algorithmic model of the useful work per valid voxel (FP32):
    # learned start ~1 start x 15 SS-HOPM steps x 200 flop; plain 16 starts x
    # 45 steps x 200 flop (the BF16 network, 14 kflop per voxel, is counted apart)
    alg_per_voxel = 3.0e3 if learned else 16 * 45 * 200.0
    alg_ach = voxels * alg_per_voxel / (stage["extract"] / 1e3) / 1e12
    roofline = {"bound": "alu",
                "kernel": f"ttm_extract call ({'k_learned + ' if learned else ''}k_prepare, "
                          f"k_runs, k_reduce), degree {n}, {main_mode} start",
                "achieved": alg_ach, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": alg_ach / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                "achieved_is": "algorithmic FP32 flops per launch (the per-voxel model of the "
                               "useful work times the launch's valid voxels) / the launch's "
                               "average duration",
                "algorithmic_flops_per_voxel": alg_per_voxel,
                "achieved_executed": ach,
                "frac_executed": ach / FP32_VECTOR_PEAK_TFLOPS,
                "achieved_executed_is": "executed FP32 flops (op-count model of the kernels times "
                                        "the work counters; hardware FP32 counts agree, "
                                        "profiles/pmc_extract_c3_512x928x928_n6.md)",
                "avg_launch_ms": ext_avg,
                "isolated_avg_launch_ms": ser_ext,
                "flops_per_launch": flops / len(ext_launch_ms),
                "mlp_mfma_flops_per_launch": mfma / len(ext_launch_ms),
                "sshopm_updates_per_oriented_voxel": steps_ / max(oriented, 1),
                "newton_steps_per_oriented_voxel": newton_ / max(oriented, 1),
                "shift_bounds_per_oriented_voxel": shifts / max(oriented, 1),
                "runs_per_oriented_voxel": runs / max(oriented, 1)}
    corr_roof = {"bound": "hbm",
                 "kernel": f"ttm_normalize_correlate (local normalisation and the K correlations "
                           f"of one tile), full {fft_n}^3 tile",
                 "achieved": corr_bytes / (corr_full_avg / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "avg_launch_ms": corr_full_avg, "bytes_per_launch": corr_bytes,
                 "traffic": measured_traffic(fft_n, K),
                 "isolated_avg_launch_ms": ser_corr,
                 "achieved_isolated": corr_bytes / (ser_corr / 1e3) / 1e9,
                 "avg_launch_ms_note": "the timed passes overlap the correlations with the "
                                       "extraction, so a launch's event span includes time spent "
                                       "waiting for CUs; isolated_avg_launch_ms is its own time"}
    corr_roof["frac"] = corr_roof["achieved"] / HBM_PEAK_GBS
    corr_roof["frac_isolated"] = corr_roof["achieved_isolated"] / HBM_PEAK_GBS
    # the stage with the larger event-timed total is reported as "roofline"
    ext_roof = roofline
    if dominant == "correlate":
        roofline, corr_roof = corr_roof, ext_roof
    wall = R["wall"]

    # ground truth at the planted copies (reported, not gated): recall and
    # precision of the copies among the top-P peaks (a peak within r of a
    # centre), position error, and the axis error against R_true a (a = z)
    gt = ground_truth(wl, R["pk"], R["eng"].dir, r)
    tile256 = None
    if args.also_fft and args.also_fft != fft_n and main_mode.startswith("learned"):
        spec2 = ttm.template_spectra(ctx, d, Tg, args.also_fft)
        eng2 = ttm.Engine(ctx, d, spec2, args.also_fft, vol.shape, starts, field_dtype=field_dtype,
                          mlp=net, kappa=kappa)
        eng2.run(vol, top_p=top_p)
        torch.cuda.synchronize()
        a2, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a2.record(stream)
        for i in range(args.steps):
            r2 = eng2.run(vol, top_p=top_p)
        b2.record(stream)
        torch.cuda.synchronize()
        ms2 = a2.elapsed_time(b2) / args.steps
        tile256 = {"fft_tile": args.also_fft, "tiles": len(eng2.boxes), "ms_per_step": ms2,
                   "voxels_per_s": nvox / (ms2 / 1e3),
                   "peaks_identical": bool(torch.equal(r2.peaks, R["pk"]))}
        log(f"[bench] learned pass on {args.also_fft}^3 tiles: {ms2:.1f} ms")
        del eng2, spec2, r2
        torch.cuda.empty_cache()

    cpu = cpu_fft = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, Q.cpu().numpy().astype(np.float64), n, L, r, args.cpu_sample)
        log("[bench] CPU FFT pipeline baseline ...")
        cpu_fft = cpu_fft_baseline(wl, T_host, n, L, r, nvalid)
        log(f"[bench] CPU FFT pipeline: {cpu_fft['value']:.3g} voxels/s")

    out = {
        "metric": "tomogram voxels/sec scored (TTM full pass), learned vs plain start at <=1 deg error",
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32" if field_dtype == torch.float32 else "f32-fft/bf16-field")
                 + ("+bf16-mlp" if main_mode == "learned" else ""),
        "data": "synthetic",
        "config": {"workload": cfg_name, "shape": list(vol.shape), "degree": n, "K": K,
                   "template_edge": L, "mask_radius": r, "fft_tile": fft_n, "tiles": n_tiles,
                   "valid_voxels": nvalid, "top_p": top_p,
                   "start": "learned (MLP + multistart fallback)" if main_mode == "learned" else "plain 16-start",
                   "rotations": int(Q.shape[0])},
        "start_mode": {m: {"voxels_per_s": nvox / (results[m]["ms_step"] / 1e3),
                           "ms_per_step": results[m]["ms_step"],
                           "stages_ms_per_step": {k: v / args.steps for k, v in results[m]["stage"].items()},
                           "stages_isolated_ms_per_pass": results[m]["serial_stages"],
                           "fallback_voxels_per_step": results[m]["fallbacks"] if m != "plain" else None}
                       for m in results},
        "accuracy_gate": gate,
        "learned_start_training": learn_info,
        "stages_ms_per_step": {k: v / args.steps for k, v in stage.items()},
        "stages_isolated_ms_per_pass": R["serial_stages"],
        "stages_note": ("stages_ms_per_step are HIP-event spans of the timed passes: with the "
                        "correlations on a side stream under the extractions, a span includes time "
                        "spent waiting for CUs the other stream holds, so the spans add up to more "
                        "than ms_per_step; stages_isolated_ms_per_pass are each stage's own times "
                        "from one untimed pass with every stage on the caller's stream"),
        "valid_voxels_per_s": nvalid / (ms_step / 1e3),
        "peaks_found": n_peaks,
        "roofline": roofline,
        "dominant_stage": dominant,
        ("roofline_extract" if dominant == "correlate" else "roofline_correlate"): corr_roof,
        "cpu_baseline": cpu,
        "cpu_fft_baseline": cpu_fft,
        "ground_truth": gt,
        "other_tile": tile256,
        "wall_s": wall,
    }
    print(json.dumps(clean(out)), flush=True)


def ground_truth(wl, peaks, direction, r):
    """Detected copies among the peaks (a peak within r of a planted centre),
    position errors, and the axis error arccos|u . R_true a| (a = z axis) at
    the detected copies' peaks (Sec. 4.1 metrics; reported, not gated).  The
    axis form recovers R a only for a template symmetric about a: for any
    other template the field integrates each direction over all spins about
    it, and its maximiser need not be R a (the blob templates here have no
    such symmetry, so the axis error is context only; the quaternion form's
    rotation errors are measured by the noise sweep)."""
    pk = peaks.cpu().numpy().astype(np.float64)
    cen = wl.centres.astype(np.float64)
    if len(pk) == 0 or len(cen) == 0:
        return None
    found, used, pos_err, ang = 0, set(), [], []
    dmap = direction
    for j, c in enumerate(cen):
        dist = np.linalg.norm(pk - c, axis=1)
        i = int(np.argmin(dist))
        if dist[i] > r:
            continue
        found += 1
        used.add(i)
        pos_err.append(float(dist[i]))
        z, y, x = (int(v) for v in pk[i])
        u = dmap[z, y, x].cpu().numpy().astype(np.float64)
        a = wl.rotations[j][:, 2]
        cosv = abs(float(u @ a)) / max(np.linalg.norm(u), 1e-30)
        ang.append(float(np.degrees(np.arccos(min(1.0, cosv)))))
    pe, an = np.array(pos_err), np.array(ang)
    return {"copies": int(len(cen)), "peaks": int(len(pk)), "recall": found / len(cen),
            "precision": len(used) / len(pk),
            "position_err_vox": {"mean": float(pe.mean()), "max": float(pe.max())} if found else None,
            "axis_err_deg": {"mean": float(an.mean()), "median": float(np.median(an)),
                             "max": float(an.max())} if found else None,
            "axis_err_note": "axis form on a template without axial symmetry: not an "
                             "estimate of the copy's rotation"}


def accuracy_gate(plain, learned, lo, hi, top_p, ttm, torch):
    """Median angle between learned and plain directions on the top 1% scores
    plus the r_s = 3 voxel spheres around the plain pass's peaks (Sec. 3.3)."""
    sp = plain["eng"].score
    sl = slice(lo[0], hi[0] + 1), slice(lo[1], hi[1] + 1), slice(lo[2], hi[2] + 1)
    sv = sp[sl]
    gen = torch.Generator(device=sv.device)
    gen.manual_seed(0)
    flat = sv.reshape(-1)
    sample = flat[torch.randint(0, flat.numel(), (min(flat.numel(), 8_000_000),), generator=gen,
                                device=sv.device)]
    thr = torch.quantile(sample, 0.99)
    mask = torch.zeros_like(sp, dtype=torch.bool)
    mask[sl] = sv >= thr
    pk = plain["pk"].long()
    rs = 3
    offs = torch.stack(torch.meshgrid(*[torch.arange(-rs, rs + 1, device=sv.device)] * 3,
                                      indexing="ij"), -1).reshape(-1, 3)
    offs = offs[(offs ** 2).sum(1) <= rs * rs]
    pts = (pk[:, None, :] + offs[None]).reshape(-1, 3)
    for a in range(3):
        pts[:, a] = pts[:, a].clamp(lo[a], hi[a])
    mask[pts[:, 0], pts[:, 1], pts[:, 2]] = True
    ua, ub = plain["eng"].dir[mask], learned["eng"].dir[mask]
    c = torch.abs((ua * ub).sum(-1)) / (ua.norm(dim=-1) * ub.norm(dim=-1)).clamp_min(1e-30)
    ang = torch.rad2deg(torch.arccos(c.clamp(max=1.0)))
    # peaks: position agreement of the two passes
    pl, pn = plain["pk"], learned["pk"]
    same_peaks = bool(pl.shape == pn.shape and torch.equal(pl, pn))
    allv = (plain["eng"].dir[sl].reshape(-1, 3), learned["eng"].dir[sl].reshape(-1, 3))
    idx = torch.randint(0, allv[0].shape[0], (min(allv[0].shape[0], 4_000_000),), generator=gen,
                        device=sv.device)
    ca = torch.abs((allv[0][idx] * allv[1][idx]).sum(-1)).clamp(max=1.0)
    ang_all = torch.rad2deg(torch.arccos(ca))
    return {"voxels": int(mask.sum().item()), "median_deg": float(ang.median().item()),
            "p90_deg": float(torch.quantile(ang, 0.9).item()) if ang.numel() < 16_000_000 else None,
            "frac_within_1deg": float((ang <= 1.0).float().mean().item()),
            "pass": bool(ang.median().item() <= 1.0),
            "all_valid_sample_median_deg": float(ang_all.median().item()),
            "all_valid_sample_frac_within_1deg": float((ang_all <= 1.0).float().mean().item()),
            "peaks_identical": same_peaks}


def bench_batch(args, top_p):
    """64 uneven subtomograms with 3 templates, recorded into one HIP graph per batch:
    plain and learned starts, throughput = all subtomogram voxels / replay time."""
    import torch

    import synth
    from paper_2408_02398_amd import learn, ttm
    n = 6
    t0 = time.time()
    tmpls, items = synth.batch_items(seed=5, n_items=64)
    log(f"[bench] batch generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ctx = ttm.Context(0)
    Q = torch.from_numpy(synth.rotation_samples(args.nq_base)).float().to(dev)
    starts = torch.from_numpy(synth.start_vectors()).to(dev)
    templates = []
    for vol, r, tm in tmpls:
        d = ttm.make_desc(n, vol.shape[0], r)
        Tg, _ = ttm.build_tensor(ctx, d, torch.from_numpy(vol).to(dev), Q)
        templates.append((d, Tg))
    cost = ttm.autotune(ctx, templates[-1][0])
    log(f"[bench] FFT tile cost (ms): {cost}")
    shapes = [it["volume"].shape for it in items]
    owner = [it["template"] for it in items]
    nvox = int(sum(np.prod(s) for s in shapes))

    mlps, learn_info = None, []
    if args.start in ("learned", "both"):
        mlps = []
        for ti, (vol, r, tm) in enumerate(tmpls):
            d, Tg = templates[ti]
            spec = ttm.template_spectra(ctx, d, Tg, 256)
            trv = []
            for k in range(4):
                rng = np.random.default_rng(7000 + 10 * ti + k)
                cen = synth.place_centres(rng, (192, 192, 192), 40, r, margin=tm.L // 2 + 1)
                rot = synth.random_rotations(rng, len(cen))
                sig = synth.render_copies((192, 192, 192), tm, cen, rot)
                sd = float(np.sqrt(np.var(vol[synth.ball(tm.L, r)]) / 0.1))
                v = sig + (sd * rng.standard_normal((192, 192, 192), dtype=np.float32))
                trv.append(torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(dev))
            net, kap, info = learn.build_learned_start(ctx, d, spec, 256, trv, starts,
                                                       steps=args.train_steps // 2, log=log)
            mlps.append(net)
            learn_info.append(info)
    results = {}
    modes = ["plain", "learned"] if args.start == "both" else [args.start]
    for mode in modes:
        be = ttm.BatchEngine(ctx, templates, shapes, owner, starts, top_p,
                             mlps=mlps if mode == "learned" else None, kappa=-1e30, cost=cost)
        for i, it in enumerate(items):
            be.volumes[i].copy_(torch.from_numpy(it["volume"]).to(dev))
        be.capture()
        for _ in range(args.warmup):
            be.replay()
        torch.cuda.synchronize()
        be.fallbacks.zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.steps):
            be.replay()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        log(f"[bench] batch {mode}: {ms:.1f} ms per batch")
        results[mode] = dict(be=be, ms=ms, fallbacks=int(be.fallbacks.item()) // max(args.steps, 1))
    gate = None
    if "plain" in results and "learned" in results:
        angs = []
        for i in range(len(items)):
            bp, bl = results["plain"]["be"], results["learned"]["be"]
            d = templates[owner[i]][0]
            lo, hi = ttm.valid_bounds(shapes[i], d.L)
            sl = tuple(slice(x, y + 1) for x, y in zip(lo, hi))
            sc = bp.score[i][sl]
            thr = torch.quantile(sc.reshape(-1)[:: max(1, sc.numel() // 1_000_000)], 0.99)
            m = sc >= thr
            ua, ub = bp.direction[i][sl][m], bl.direction[i][sl][m]
            c = torch.abs((ua * ub).sum(-1)).clamp(max=1.0)
            angs.append(torch.rad2deg(torch.arccos(c)))
        ang = torch.cat(angs)
        gate = {"voxels": int(ang.numel()), "median_deg": float(ang.median()),
                "frac_within_1deg": float((ang <= 1.0).float().mean()),
                "pass": bool(ang.median() <= 1.0),
                "peaks_identical": all(torch.equal(results["plain"]["be"].peaks[i],
                                                   results["learned"]["be"].peaks[i])
                                       for i in range(len(items)))}
    main = "learned" if "learned" in results else "plain"
    ms = results[main]["ms"]
    return {"metric": "tomogram voxels/sec scored (TTM full pass), learned vs plain start at <=1 deg error",
            "value": nvox / (ms / 1e3), "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32" + ("+bf16-mlp" if main == "learned" else ""),
            "data": "synthetic",
            "config": {"workload": "c5_batch64_n6", "items": len(items), "degree": n, "K": 28,
                       "edges": sorted(set(int(s[0]) for s in shapes)), "templates": len(templates),
                       "fft_edges_chosen": {str(k): ttm.BatchEngine.__name__ and int(sum(1 for f in results[main]["be"].fft if f == k)) for k in sorted(set(results[main]["be"].fft))},
                       "voxels": nvox, "top_p_per_item": top_p,
                       "launch": "one HIP graph per batch",
                       "graph_branches": results[main]["be"].branches},
            "start_mode": {m: {"voxels_per_s": nvox / (results[m]["ms"] / 1e3), "ms_per_step": results[m]["ms"],
                               "fallback_voxels_per_step": results[m]["fallbacks"] if m != "plain" else None}
                           for m in results},
            "accuracy_gate": gate, "autotune_tile_ms": cost, "learned_start_training": learn_info}


def noise_sweep(args, grid=5, spacing=40, L=32, r=14.0, n=4, fft_n=256, rs=3.0):
    """The paper's robustness experiment (Sec. 4.1, the rotation-deviation-vs-SNR
    panel) on synthetic stand-ins: a 5 x 5 x 5 grid of randomly rotated copies of
    a 32^3 blob template in Gaussian noise at each SNR, the quaternion form
    (d' = 4) at degree 4 (K = 35).  Per SNR: a full pass (scores only), Find
    Peaks (125 peaks, 2r apart), then TTM-ref (Alg. 3, r_s = 3), whose output
    also holds each unrefined peak's own rotation (TTM).  Each planted copy is
    matched to the nearest peak within r; errors are the Euclidean position
    distance and the rotation distance 2 arccos|q1.q2| (Sec. 4.1).  With
    --wedge the tomograms lose the +-60 degree missing wedge and the tensor
    template is the wedge-aware one (ttm_build_tensor_wedge).  At --dense-snr the orientation of every
    valid voxel is computed too, with the multistart search and with the
    learned start (trained on four further tomograms of the same SNR), timed,
    with the fallback count and the learned answers' rotation distance to the
    multistart ones."""
    import torch

    import synth
    from paper_2408_02398_amd import ttm
    dev = torch.device("cuda:0")
    ctx = ttm.Context(0)
    d = ttm.make_desc(n, L, r, dprime=4)
    snrs = [float(v) for v in args.snr.split(",")]
    Q = torch.from_numpy(synth.rotation_samples(args.nq_base)).float().to(dev)
    starts = torch.from_numpy(synth.start_vectors(count=32, dim=4)).to(dev)
    T = spec = tn = eng = None
    rows = []
    for k, snr in enumerate(snrs):
        wl = synth.grid_tomogram(f"sweep_snr{snr:g}", grid, spacing, L, 4, r, n, seed=500 + k,
                                 snr=snr, template_seed=2, wedge=args.wedge)
        if T is None:
            T, tn = ttm.build_tensor(ctx, d, torch.from_numpy(wl.template).to(dev), Q,
                                     wedge=60.0 if args.wedge else None)
            spec = ttm.template_spectra(ctx, d, T, fft_n)
            eng = ttm.Engine(ctx, d, spec, fft_n, wl.volume.shape, None, orient=False)
        vol = torch.from_numpy(wl.volume).to(dev)
        P = grid ** 3
        res = eng.run(vol, top_p=P)
        ref = ttm.refine(ctx, d, res.g, res.w, T, tn, res.peaks.contiguous(), starts, r_s=rs)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(args.steps):
            res = eng.run(vol, top_p=P)
        e[1].record()
        for _ in range(args.steps):
            ref = ttm.refine(ctx, d, res.g, res.w, T, tn, res.peaks.contiguous(), starts, r_s=rs)
        e[2].record()
        torch.cuda.synchronize()
        pk = res.peaks.cpu().numpy().astype(np.float64)
        rp = ref["pos"].cpu().numpy().astype(np.float64)
        q_ttm, q_ref = ref["quat_peak"].cpu().numpy(), ref["quat"].cpu().numpy()
        pos_t, pos_r, rot_t, rot_r, used = [], [], [], [], set()
        for c, qt in zip(wl.centres.astype(np.float64), wl.quaternions):
            dist = np.linalg.norm(pk - c, axis=1)
            i = int(np.argmin(dist))
            if dist[i] > r:
                continue
            used.add(i)
            pos_t.append(dist[i])
            pos_r.append(float(np.linalg.norm(rp[i] - c)))
            for q, acc in ((q_ttm[i], rot_t), (q_ref[i], rot_r)):
                cq = abs(float(np.dot(q / np.linalg.norm(q), qt)))
                acc.append(float(np.degrees(2.0 * np.arccos(min(1.0, cq)))))

        def stats(v):
            v = np.asarray(v)
            return {"mean": float(v.mean()), "median": float(np.median(v)), "max": float(v.max())} \
                if len(v) else None
        row = {"snr": snr, "copies": int(len(wl.centres)), "peaks": int(len(pk)),
               "recall": len(pos_t) / len(wl.centres), "precision": len(used) / max(len(pk), 1),
               "ttm": {"position_err_vox": stats(pos_t), "rotation_err_deg": stats(rot_t)},
               "ttm_ref": {"position_err_vox": stats(pos_r), "rotation_err_deg": stats(rot_r),
                           "exact_positions": int(sum(1 for x in pos_r if x == 0.0))},
               "ms_pass": e[0].elapsed_time(e[1]) / args.steps,
               "ms_refine": e[1].elapsed_time(e[2]) / args.steps}
        log(f"[sweep] {row}")
        rows.append(row)
    dense = None
    if args.dense_snr > 0:
        dense = dense_quaternion_pass(args, ctx, d, spec, fft_n, starts, grid, spacing, L, r, n)
    return {"metric": "rotation and position error vs SNR, TTM and TTM-ref (quaternion form)",
            "unit": "deg / voxels", "data": "synthetic", "n_gpus": 1, "steps": args.steps,
            "config": {"workload": f"grid {grid}^3 copies, spacing {spacing}, template {L}^3 "
                                   f"(4 Gaussian blobs), r {r}, volume {2 * (L // 2 + 2) + (grid - 1) * spacing + 1}^3",
                       "degree": n, "dprime": 4, "K": 35, "fft_tile": fft_n, "r_s": rs,
                       "rotations": int(Q.shape[0]), "quaternion_starts": int(starts.shape[0]),
                       "missing_wedge": bool(args.wedge)},
            "sweep": rows, "dense_orientation": dense}


def dense_quaternion_pass(args, ctx, d, spec, fft_n, starts, grid, spacing, L, r, n):
    """Every valid voxel's rotation (quaternion form) on a grid tomogram at
    --dense-snr: the multistart pass and the learned-start pass (network trained
    on three further tomograms of the same SNR, kappa calibrated on a fourth),
    timed over --steps passes each."""
    import torch

    import synth
    from paper_2408_02398_amd import learn, ttm
    snr = args.dense_snr

    def tomo(seed):
        return synth.grid_tomogram(f"dense_{seed}", grid, spacing, L, 4, r, n, seed=seed, snr=snr,
                                   template_seed=2, wedge=args.wedge)

    vol = torch.from_numpy(tomo(700).volume).cuda()
    train = [torch.from_numpy(tomo(s).volume).cuda() for s in (701, 702, 703, 704)]
    t0 = time.time()
    net, kappa, info = learn.build_learned_start(ctx, d, spec, fft_n, train, starts, n_uniform=100000,
                                                 n_top=100000, steps=60000, batch=8192, lr=3e-3,
                                                 max_wrong=args.max_wrong, log=log)
    t_train = time.time() - t0
    out = {"snr": snr, "train_s": t_train, "kappa": kappa,
           "valid_voxels": int(np.prod([s - L + 1 for s in vol.shape])),
           "training": {k: info[k] for k in ("train_samples", "accepted_fraction",
                                             "wrong_without_fallback", "not_converged_fraction",
                                             "heldout_uniform_fallback", "heldout_uniform_within_1deg")}}
    maps = {}
    for mode in ("plain", "learned"):
        eng = ttm.Engine(ctx, d, spec, fft_n, vol.shape, starts, mlp=net if mode == "learned" else None,
                         kappa=kappa)
        eng.run(vol, top_p=grid ** 3)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        eng.fallbacks.zero_()
        e0.record()
        for _ in range(args.steps):
            eng.run(vol, top_p=grid ** 3)
        e1.record()
        torch.cuda.synchronize()
        out[mode] = {"ms_pass": e0.elapsed_time(e1) / args.steps,
                     "fallback_voxels": int(eng.fallbacks.item()) // args.steps if mode == "learned" else None}
        maps[mode] = eng.dir.clone()
        del eng
        torch.cuda.empty_cache()
    lo, hi = ttm.valid_bounds(vol.shape, L)
    sl = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
    qa, qb = maps["plain"][sl].reshape(-1, 4), maps["learned"][sl].reshape(-1, 4)
    cq = torch.abs((qa * qb).sum(-1)) / (qa.norm(dim=-1) * qb.norm(dim=-1)).clamp_min(1e-30)
    ang = torch.rad2deg(2.0 * torch.arccos(cq.clamp(max=1.0)))
    out["learned_vs_plain_rotation_deg"] = {"median": float(ang.median().item()),
                                            "frac_within_1deg": float((ang <= 1.0).float().mean().item())}
    out["speedup"] = out["plain"]["ms_pass"] / out["learned"]["ms_pass"]
    log(f"[sweep dense] {out}")
    return out


def precision_report(args, cfg_name, fft_n, top_p, n_sample=150):
    """Field stored in BF16 (FFTs and accumulation FP32, variance FP64) against FP32 storage:
    pass throughput (plain start), score / lambda / angle differences over all valid voxels, and
    both against the FP64 oracle at sampled voxels (oracle field by direct sums)."""
    import torch

    import synth
    from oracle import ttm as orc
    from paper_2408_02398_amd import ttm
    p = synth.CONFIGS[cfg_name]
    n, L, r = p["degree"], p["L"], p["mask_radius"]
    wl = synth.make_config(cfg_name)
    dev = torch.device("cuda:0")
    ctx = ttm.Context(0)
    d = ttm.make_desc(n, L, r)
    Qn = synth.rotation_samples(100)              # 2400 rotations: the oracle builds T too
    Tg, _ = ttm.build_tensor(ctx, d, torch.from_numpy(wl.template).to(dev),
                             torch.from_numpy(Qn).float().to(dev))
    spec = ttm.template_spectra(ctx, d, Tg, fft_n)
    starts = torch.from_numpy(synth.start_vectors()).to(dev)
    vol = torch.from_numpy(wl.volume).to(dev)
    lo, hi = ttm.valid_bounds(vol.shape, L)
    out = {"workload": cfg_name, "rotations": int(len(Qn))}
    maps = {}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        eng = ttm.Engine(ctx, d, spec, fft_n, vol.shape, starts, field_dtype=dt)
        eng.run(vol, top_p=top_p)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(args.steps):
            res = eng.run(vol, top_p=top_p)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / args.steps
        out[name] = {"ms_per_step": ms, "voxels_per_s": float(np.prod(vol.shape)) / (ms / 1e3)}
        maps[name] = (res.score.clone(), res.lam.clone(), res.direction.clone(), res.peaks.clone())
    sl = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
    s32, s16 = maps["f32"][0][sl], maps["bf16"][0][sl]
    floor = torch.maximum(s32, s32.median())
    u32, u16 = maps["f32"][2][sl].reshape(-1, 3), maps["bf16"][2][sl].reshape(-1, 3)
    ang = torch.rad2deg(torch.arccos(torch.abs((u32 * u16).sum(-1)).clamp(max=1.0)))
    out["bf16_vs_f32"] = {"score_max_rel": float(((s16 - s32).abs() / floor).max()),
                          "score_median_rel": float(((s16 - s32).abs() / floor).median()),
                          "angle_median_deg": float(ang.median()),
                          "angle_frac_within_1deg": float((ang <= 1).float().mean()),
                          "peaks_identical": bool(torch.equal(maps["f32"][3], maps["bf16"][3]))}
    # FP64 oracle at sampled voxels: the peaks of the FP32 pass plus random valid voxels
    rng = np.random.default_rng(5)
    pk = maps["f32"][3].cpu().numpy()[: n_sample // 3]
    rnd = np.stack([rng.integers(a, b + 1, n_sample - len(pk)) for a, b in zip(lo, hi)], 1)
    pts = np.concatenate([pk, rnd]).astype(np.int64)
    tn = orc.normalize_template(wl.template, r)
    T = orc.tensor_template(tn, Qn, n)
    g2 = orc.volume_g2_mean(orc.prefilter_volume(wl.volume))
    _, Co = orc.field_at(orc.patches_at(None, pts, L, f=wl.volume), orc.ball_mask(L, r), T, g2)
    so = orc.score(Co.T, n)
    st = synth.start_vectors().astype(np.float64)
    lam_o, u_o, ok = [], [], []
    for i in range(len(pts)):
        lmb, u, lams, us, _ = orc.orient_multistart(Co[i], n, st)
        lam_o.append(lmb)
        u_o.append(u)
        ok.append(orc.orientation_margin(lams, us, u) > 1e-4 * so[i])
    lam_o, u_o, ok = np.array(lam_o), np.array(u_o), np.array(ok)
    med = float(np.median(so))
    for name in ("f32", "bf16"):
        sc, lm, dr, _ = (m.cpu().numpy() for m in maps[name])
        sg = sc[pts[:, 0], pts[:, 1], pts[:, 2]]
        lg = lm[pts[:, 0], pts[:, 1], pts[:, 2]]
        ug = dr[pts[:, 0], pts[:, 1], pts[:, 2]]
        a = orc.angle_deg(ug, u_o)
        out[name]["vs_fp64_oracle"] = {
            "voxels": int(len(pts)),
            "score_max_rel": float(np.max(np.abs(sg - so) / np.maximum(so, med))),
            "lambda_max_rel": float(np.max(np.abs(lg - lam_o) / np.maximum(so, med))),
            "angle_median_deg": float(np.median(a[ok])) if ok.any() else None,
            "angle_max_deg_unambiguous": float(np.max(a[ok])) if ok.any() else None,
            "unambiguous": int(ok.sum())}
    return out


def tensor_template_cached(path, ctx, d, template, Q, ttm, torch):
    """The tensor template (Alg. 1, built once per template: the paper computes
    it once and reuses it), from ``path`` when the file's key matches this
    template, degree, form, rotation set and mask, else built on the GPU (and
    written to ``path`` if one is given)."""
    import hashlib
    h = hashlib.sha256()
    for a in (np.ascontiguousarray(template, dtype=np.float32), Q.cpu().numpy().astype(np.float32)):
        h.update(a.tobytes())
    h.update(np.array([d.degree, d.dprime, d.L], dtype=np.int64).tobytes())
    h.update(np.array([d.mask_radius, d.filter_a, *d.axis], dtype=np.float64).tobytes())
    key = h.hexdigest()
    if path and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        if str(z["key"]) == key:
            log(f"[bench] tensor template loaded from {path}")
            return torch.from_numpy(z["T"]).cuda()
    T, _ = ttm.build_tensor(ctx, d, torch.from_numpy(template).cuda(), Q)
    if path:
        np.savez(path, T=T.cpu().numpy(), key=np.array(key))
    return T


def tile_call(args, n=6, L=40, r=17.0, N=512):
    """One full-tile ttm_normalize_correlate call (random tomogram and tensor
    template of the c3 shapes), repeated: ms per call by HIP events."""
    import torch

    from paper_2408_02398_amd import ttm
    ctx = ttm.Context(0)
    d = ttm.make_desc(n, L, r)
    K = ttm.n_components(n)
    rng = np.random.default_rng(1)
    T = torch.from_numpy(rng.standard_normal((K, L ** 3)).astype(np.float32)).cuda()
    spec = ttm.template_spectra(ctx, d, T, N)
    vol = torch.from_numpy(rng.standard_normal((N, N, N), dtype=np.float32)).cuda()
    g, w, stats = ttm.prefilter(ctx, d, vol)
    c = L // 2
    crop = N - L + 1
    out = torch.empty((K, crop, crop, crop), dtype=torch.float32, device="cuda")
    ws = ttm._ws(d, ttm.L.TTM_OP_NORM_CORR, N, device="cuda")

    def call():
        ttm.normalize_correlate(ctx, d, g, stats, spec, N, (c, c, c), (crop,) * 3, w, out=out, ws=ws)
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        call()
    b.record()
    torch.cuda.synchronize()
    return {"mode": "tile_call", "call": "ttm_normalize_correlate", "fft_n": N, "K": K, "L": L,
            "steps": args.steps, "ms_per_call": a.elapsed_time(b) / args.steps}


def measured_traffic(fft_n, K):
    """HBM bytes of one full-tile ttm_normalize_correlate call from the rocprofv3
    FETCH_SIZE / WRITE_SIZE runs summarised in profiles/, or None when the
    kernel sources differ from the ones measured (or the tile edge, component
    count or call differs)."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        rec = json.load(open(os.path.join(root, "profiles", "traffic_correlate_512tile_c3.json")))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(root, f), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    if (h.hexdigest() != rec["sha256"] or rec["fft_n"] != fft_n or rec["K"] != K
            or rec.get("call") != "ttm_normalize_correlate"):
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(wl, Q, n, L, r, sample):
    """The FP64 oracle on a bounded sample: field, score and 16-start orientation per voxel."""
    from oracle import ttm as orc
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    import synth
    rng = np.random.default_rng(123)
    shape = wl.volume.shape
    c = L // 2
    pts = np.stack([rng.integers(c, s - L + c + 1, size=sample) for s in shape], axis=1)
    t0 = time.time()
    tn = orc.normalize_template(wl.template, r)
    T = orc.tensor_template(tn, Q[:: max(1, len(Q) // 2400)], n)   # template cost not counted
    t_tmpl = time.time() - t0
    g2 = float(np.mean(orc.prefilter_box(wl.volume, (0, 0, 0), (min(64, shape[0]),) + shape[1:]) ** 2))
    starts = synth.start_vectors().astype(np.float64)
    t0 = time.time()
    patches = orc.patches_at(None, pts, L, f=wl.volume)
    w, C = orc.field_at(patches, orc.ball_mask(L, r), T, g2)
    for i in range(len(pts)):
        orc.score(C[i], n)
        orc.orient_multistart(C[i], n, starts)
    dt = time.time() - t0
    return {"value": sample / dt, "unit": "voxels/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{sample} random valid voxels of the same tomogram: direct FP64 field "
                      f"(prefilter, local variance, K={C.shape[1]} correlations), score and "
                      f"16-start SS-HOPM per voxel; tensor template ({t_tmpl:.0f}s) excluded",
            "seconds": dt}


def cpu_fft_baseline(wl, T, n, L, r, nvalid, edge=256, sample=4000):
    """The paper's CPU pipeline as a like-for-like baseline (Sec. 4.3 runs TTM
    on a 10-core CPU): one edge^3 tile of the tomogram on every host core with
    scipy.fft -- prefilter, local normalisation by FFT correlations with the
    mask (Eq. norm_f), the K correlations with the tensor template (Alg. 2;
    the template and its spectra are built once and not timed, as on the GPU),
    the score, and 16-start SS-HOPM with the unfolding shift (Sec. 3.1; stop at
    |delta lambda| <= 1e-5 or 500 updates, no polish) on a random sample of the
    tile's valid voxels, vectorised over voxels and starts.  Throughput = the
    tile's valid voxels / (measured field time + sampled orientation time per
    voxel x valid voxels); the whole tomogram's time is extrapolated from it."""
    import scipy.fft as sfft
    import synth
    from oracle import sym
    from oracle import ttm as orc
    cores = len(os.sched_getaffinity(0))
    f = np.ascontiguousarray(wl.volume[:edge, :edge, :edge], dtype=np.float32)
    K = T.shape[0]
    V = edge - L + 1

    def conj_spec(ker):
        kp = np.zeros((edge, edge, edge), np.float32)
        kp[:L, :L, :L] = ker
        return np.conj(sfft.rfftn(kp, workers=cores))

    m = orc.ball_mask(L, r).astype(np.float32)
    M = float(m.sum())
    mspec = conj_spec(m)
    tspec = [conj_spec(T[a]) for a in range(K)]
    mu = np.asarray(sym.weights(n, 3), np.float64)
    t0 = time.perf_counter()
    g = orc.prefilter_volume(f).astype(np.float32)
    G = sfft.rfftn(g, workers=cores)
    s1 = sfft.irfftn(G * mspec, s=g.shape, workers=cores)[:V, :V, :V]
    s2 = sfft.irfftn(sfft.rfftn(g * g, workers=cores) * mspec, s=g.shape, workers=cores)[:V, :V, :V]
    var = s2 - s1 * s1 / M
    w = np.where(var > 1e-6 * M * float(np.mean(g.astype(np.float64) ** 2)),
                 1.0 / np.sqrt(np.maximum(var, 1e-30)), 0.0).astype(np.float32)
    C = np.empty((K, V, V, V), np.float32)
    for a in range(K):
        C[a] = sfft.irfftn(G * tspec[a], s=g.shape, workers=cores)[:V, :V, :V] * w
    score = np.sqrt(np.einsum("k,kzyx->zyx", mu.astype(np.float32), C * C))
    t_field = time.perf_counter() - t0
    # orientation on a sample of the tile's voxels
    rng = np.random.default_rng(7)
    idx = rng.choice(V ** 3, size=min(sample, V ** 3), replace=False)
    t0 = time.perf_counter()
    Cs = C.reshape(K, -1)[:, idx].T.astype(np.float64)
    cn = np.sqrt((Cs * Cs) @ mu)
    ok = cn > 0
    Cs[ok] /= cn[ok, None]
    alpha = np.array([max(0.0, -float(np.linalg.eigvalsh(sym.unfolding(c, n, 3)).min())) for c in Cs])
    mu1, tab = sym._raise_table(n, 3)
    ex = np.array(sym.multi_indices(n - 1, 3))               # exponents of the monomials
    st = synth.start_vectors().astype(np.float64)
    st /= np.linalg.norm(st, axis=1, keepdims=True)
    S, R = len(Cs), len(st)
    vox = np.repeat(np.arange(S), R)                         # run -> voxel
    U = np.tile(st, (S, 1))                                  # (S R, 3)
    Ct = (mu1[None, :, None] * Cs[:, tab])                   # (S, monomials, 3)

    def grad(U, v):
        P = U[:, :, None] ** np.arange(n)                    # (runs, 3, n) powers
        mono = P[:, 0, ex[:, 0]] * P[:, 1, ex[:, 1]] * P[:, 2, ex[:, 2]]
        return np.einsum("rk,rkd->rd", mono, Ct[v])

    Gd = grad(U, vox)
    lam = np.einsum("rd,rd->r", Gd, U)
    live = np.arange(S * R)
    for _ in range(500):
        u, gd, v = U[live], Gd[live], vox[live]
        Wv = gd + alpha[v, None] * u
        u = Wv / np.linalg.norm(Wv, axis=1, keepdims=True)
        gd = grad(u, v)
        ln = np.einsum("rd,rd->r", gd, u)
        go = np.abs(ln - lam[live]) > 1e-5
        U[live], Gd[live], lam[live] = u, gd, ln
        live = live[go]
        if live.size == 0:
            break
    best = np.argmax(lam.reshape(S, R), axis=1)
    u_best = U.reshape(S, R, 3)[np.arange(S), best]
    t_orient = (time.perf_counter() - t0) / len(idx)
    tile_s = t_field + t_orient * V ** 3
    del C, tspec
    return {"value": V ** 3 / tile_s, "unit": "voxels/s", "cores": int(cores), "kind": "cpu_fft_pipeline",
            "sample": f"one {edge}^3 tile ({V}^3 valid voxels) of the same tomogram: prefilter, FFT local "
                      f"normalisation and K={K} FFT correlations (scipy.fft, {cores} workers) timed whole "
                      f"({t_field:.1f} s); 16-start SS-HOPM timed on {len(idx)} random voxels of the tile "
                      f"({t_orient * 1e3:.2f} ms per voxel) and extrapolated",
            "tile_seconds": tile_s, "field_seconds": t_field, "orient_ms_per_voxel": t_orient * 1e3,
            "field_and_score_voxels_per_s": V ** 3 / t_field,
            "tomogram_seconds_estimate": nvalid * tile_s / V ** 3,
            "check_nonzero": bool(np.isfinite(score).all() and np.isfinite(u_best).all())}


if __name__ == "__main__":
    main()
