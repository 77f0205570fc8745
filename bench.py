"""Benchmark: SRP candidate-pair evaluations per second on one MI355X.

Workload (default): the room-scale configuration -- 16 microphones uniformly
random in a 1 x 1 x 0.5 m box (120 pairs), fs = 16 kHz, 1024-sample Hann
frames (513 bins), a 6 x 4 x 3 m room gridded at 5 cm (576,000 candidates),
500 frames of seeded free-field white-noise sources with 10 dB sensor noise,
N_aux = 2. Inputs are synthetic (workloads.make(2)) and already resident in
device memory when the timed region starts.

One step = one pass of the Nyquist hot path over the 500-frame batch:
srp_cross_spectra (windowed FFT + PHAT cross-spectra), srp_gcc_samples (GCC
samples at the critical lags), srp_map_nyquist (TDOA + sinc interpolation +
pair sum + per-frame argmax). `value` = F * J * P / step time. The
conventional map (srp_cross_spectra + srp_map_conventional) is timed beside
it on the same frames and reported under "conventional".

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 (matrix cores), published
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 / FP16 (matrix cores), published
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nyquist_f32_cfg2.json")


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2012_09499_amd", "csrc", "k_nyquist.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per launch from committed rocprofv3 PMC runs, if they were taken on
    this workload and the kernel source has not changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if t.get("workload") != workload:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(wl, n_cand: int, seed: int = 0):
    """The FP64 oracle on a bounded sample: all frames, a seeded candidate subset."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()
                            if i.get("user_api") == "blas"] or [1])
    except Exception:
        blas_threads = 1
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(wl.J, size=min(n_cand, wl.J), replace=False))
    cand = wl.candidates_at(idx)
    t0 = time.perf_counter()
    K = O.n_bins(wl.L, wl.fs)
    w = O.bin_weights(wl.L, K)
    win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, wl.n_aux)
    psi = O.phat_cross_spectra(O.spectra(wl.frames, O.window(wl.L), K))
    xi = O.gcc_samples(psi, wl.fs, wl.L, w, win)
    dt = O.tdoa(wl.mic_xyz, cand, wl.c)
    ref = O.srp_nyquist(xi, dt, win)
    O.peaks(ref)
    sec = time.perf_counter() - t0
    rate = wl.F * idx.size * wl.P / sec
    info = {"value": rate, "unit": "cand-pair evals/s", "cores": int(blas_threads),
            "kind": "oracle", "seconds": sec, "host_cpu_count": os.cpu_count(),
            "sample": (f"all {wl.F} frames, {idx.size} of {wl.J} candidates (seeded random); "
                       f"spectra + PHAT + GCC samples + Nyquist map + argmax in float64 NumPy; "
                       f"elementwise steps single-threaded, matrix products on "
                       f"{blas_threads} BLAS threads")}
    return info, idx, ref


def serving_run(seconds: float, rate_per_array: float = 31.25, seed: int = 4,
                dtype: str = "fp32"):
    """The serving workload: 64 arrays (M in {4, 8, 16, 32}, J log-uniform in
    [1e4, 2e6]), Poisson frame arrivals, continuous batching; maps in FP32
    (vector units) or BF16/FP16 (matrix cores)."""
    import torch
    import workloads as WL
    from paper_2012_09499_amd import serving as SV

    arrays = WL.serving_arrays(64, seed=seed)
    fs, L, c = 16000.0, 1024, 343.0
    rng = np.random.default_rng(seed)
    srv = SV.SrpServer(dtype=dtype)
    frames = {}
    t_setup = time.perf_counter()
    for a in arrays:
        srv.open_array(a["id"], a["mic_xyz"], a["grid"].points(), fs=fs, L=L, c=c, n_aux=2)
        r1, r2 = np.random.default_rng(rng.integers(1 << 31)), np.random.default_rng(
            rng.integers(1 << 31))
        fr = WL.synth_frames(a["mic_xyz"], a["source"], fs, L, 4, c, 10.0, r1, r2)
        frames[a["id"]] = fr
    t_setup = time.perf_counter() - t_setup
    # warm-up: one frame per array
    for a in arrays:
        srv.submit(a["id"], frames[a["id"]][0])
    srv.drain()
    srv.completed.clear()
    srv.batch_frames.clear()
    srv.batches = 0
    arrivals = []
    for a in arrays:
        t = 0.0
        while True:
            t += rng.exponential(1.0 / rate_per_array)
            if t >= seconds:
                break
            arrivals.append((t, a["id"]))
    arrivals.sort()
    t0 = time.perf_counter()
    k = 0
    while k < len(arrivals):
        now = time.perf_counter() - t0
        while k < len(arrivals) and arrivals[k][0] <= now:
            t, i = arrivals[k]
            srv.submit(i, frames[i][k % 4], t_arrival=t0 + t)
            k += 1
        srv.pump()
    srv.drain()
    span = time.perf_counter() - t0
    st = srv.stats(span)
    Js = [a["grid"].J for a in arrays]
    Ms = [len(a["mic_xyz"]) for a in arrays]
    st.update({"offered_frames_per_s": len(arrivals) / seconds, "seconds": seconds,
               "wall_seconds": span, "arrays": len(arrays),
               "J_range": [int(min(Js)), int(max(Js))], "mic_counts": sorted(set(Ms)),
               "setup_seconds": t_setup})
    return st


def paper_standin(n_sources: int = 48, frames: int = 16, seed: int = 2021):
    """Stand-in for the paper's Section 4 experiment on the GPU path.

    Far field, 6-mic circular array (r = 10 cm), the 8101-direction lower
    half-sphere grid, sqrt-Hann 2048-sample frames, c = 340 m/s, fs = 16 kHz
    (band limit 8 kHz), N_aux = 0..4, SNR in {-3, 0, 3, 6} dB. Source
    directions are seeded and uniform over the half sphere (off the grid);
    seeded white noise replaces speech. Two scenes:
      * "reverb_diffuse": late reverberation (T60 0.6 s, direct-to-reverberant
        ratio 0 dB) and a spherically isotropic noise field, standing in for
        the simulated room and diffuse babble;
      * "free_white": free field with independent white sensor noise.
    Per scene and N_aux: the complexity figures of Sections 2.4 / 3.3 from
    the library's own pair layout (with the paper's K = 1024), the median and
    quartiles of e_appr over all sources, SNRs and frames, and the median
    localisation error (degrees) of conventional and Nyquist SRP per SNR.
    """
    import torch
    import paper_2012_09499_amd as srp
    import workloads as WL

    fs, L, c, M, radius = 16000.0, 2048, 340.0, 6, 0.1
    mic = WL.uniform_circular_array(M, radius)
    dirs = WL.half_sphere_directions(2.0)
    J = dirs.shape[0]
    snrs = (-3.0, 0.0, 3.0, 6.0)
    rng = np.random.default_rng(seed)
    src = WL.hemisphere_direction(rng, n_sources)
    true_dir = np.repeat(src, frames, axis=0)
    scenes = {}
    for scene, kw in (("reverb_diffuse", dict(t60=0.6, drr_db=0.0, noise="diffuse")),
                      ("free_white", dict(t60=0.6, drr_db=200.0, n_refl=1, noise="white"))):
        t0 = time.time()
        per_snr = [[] for _ in snrs]
        for k in range(n_sources):
            r = np.random.default_rng([seed, k])
            for i, fr in enumerate(WL.synth_far_scene(mic, src[k], fs, L, frames, c, snrs, r,
                                                      **kw)):
                per_snr[i].append(fr)
        scenes[scene] = {snr: torch.from_numpy(np.concatenate(per_snr[i])).cuda()
                         for i, snr in enumerate(snrs)}
        print(f"[standin] scene {scene}: {n_sources} sources x {len(snrs)} SNRs synthesised in "
            f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    res = {"J": J, "M": M, "P": M * (M - 1) // 2, "sources": int(n_sources),
           "frames_per_source": frames, "snr_db": list(snrs), "complexity": [], "scenes": {}}
    for n_aux in range(5):
        g = srp.Geometry(mic, dirs, fs=fs, L=L, c=c, n_aux=n_aux, field="far",
                         window="sqrt_hann")
        N = g.W_total / g.P
        res["complexity"].append({"n_aux": n_aux, "N": N, "C_conv_K1024": J * g.P * 1024.0,
                                  "C_samp_K1024": N * g.P * 1024.0, "C_int": N * g.P * J,
                                  "R_samp": N / J, "R_int_K1024": N / 1024.0})
        for scene, data in scenes.items():
            eap, loc = [], {"conventional": {}, "nyquist": {}}
            for snr in snrs:
                fr = data[snr]
                pipe = srp.SrpPipeline(g, fr.shape[0], keep_map=True)
                # the pipeline reuses its map and peak buffers: copy each result out
                mc, pc = pipe.conventional(fr)
                mc, ic = mc.double(), srp.decode_peaks(pc)[0]
                mn, pn = pipe.nyquist(fr)
                mn, inn = mn.double(), srp.decode_peaks(pn)[0]
                e = 10.0 * torch.log10(((mc - mn) ** 2).sum(1) / (mc ** 2).sum(1))
                eap.append(e.cpu().numpy())
                for key, idx in (("conventional", ic), ("nyquist", inn)):
                    cosang = np.clip((dirs[idx] * true_dir).sum(1), -1.0, 1.0)
                    loc[key][snr] = float(np.median(np.degrees(np.arccos(cosang))))
            q1, q2, q3 = np.percentile(np.concatenate(eap), [25, 50, 75])
            res["scenes"].setdefault(scene, []).append(
                {"n_aux": n_aux, "e_appr_db": {"q1": float(q1), "median": float(q2),
                                               "q3": float(q3)},
                 "e_local_deg_median": loc})
        g.close()
    return res


def next_rows_leg(srp, torch, wl, g, frames, pipe, steps):
    """The band-limited map (f_max = fs/4: T = 2/fs, half the lags) and the
    refined peak search from the FP32 coarse peaks, on the timed workload."""
    dev = frames.device
    res = {}
    g2 = srp.Geometry(wl.mic_xyz, wl.candidates(), fs=wl.fs, L=wl.L, c=wl.c, n_aux=wl.n_aux,
                      f_max=wl.fs / 4.0)
    p2 = srp.SrpPipeline(g2, wl.F, device=dev, keep_map=False)
    band = {"f_max_hz": wl.fs / 4.0, "K": g2.K, "samples_per_frame_NP": g2.W_total}
    for dt in ("fp32", "bf16"):
        def step(ev=None):
            psi = srp.cross_spectra(g2, frames, out=p2.psi, workspace=p2.workspace)
            xi = srp.gcc_samples(g2, psi, out=p2.samples_buffer(dt), dtype=dt)
            if ev is not None:
                ev[0].record(torch.cuda.current_stream())
            srp.map_nyquist(g2, xi, dtype=dt, want_map=False, peaks_out=p2.peaks)
            if ev is not None:
                ev[1].record(torch.cuda.current_stream())
        step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            step(evs[k])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        t_map = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
        tf = 2.0 * g2.W_total * wl.J * wl.F / (t_map * 1e-3) / 1e12
        peak = PEAK_FP32_TFLOPS if dt == "fp32" else PEAK_BF16_TFLOPS
        band[dt] = {"ms_per_step": ms, "map_kernel_ms": t_map,
                    "value": wl.F * wl.J * wl.P / (ms * 1e-3), "unit": "cand-pair evals/s",
                    "achieved_tflops": tf, "frac": tf / peak}
    res["band_limited"] = band
    del p2, g2

    # refined search: two levels of a 3 x 3 x 3 lattice (spacing h/3, then h/9)
    # around each frame's coarse FP32 peak, from the same samples
    from paper_2012_09499_amd.refine import refine_peaks
    psi = srp.cross_spectra(g, frames, out=pipe.psi, workspace=pipe.workspace)
    xi = srp.gcc_samples(g, psi, out=pipe.samples_buffer("fp32"))
    srp.map_nyquist(g, xi, want_map=False, peaks_out=pipe.peaks)
    idx, _ = srp.decode_peaks(pipe.peaks)
    start = wl.candidates()[idx]
    h = wl.grid.h
    refine_peaks(g, xi, start, spacing=h, levels=2)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        pts, _ = refine_peaks(g, xi, start, spacing=h, levels=2)
    ms = (time.perf_counter() - t0) * 1e3 / reps
    npts = wl.F * 27 * 2

    def dist(q):
        return np.min(np.linalg.norm(q[:, None, :] - wl.sources[None, :, :], axis=-1), axis=1)
    res["refined_search"] = {
        "levels": 2, "lattice": "3x3x3", "points_per_frame": 54, "ms_per_call": ms,
        "points_per_s": npts / (ms * 1e-3), "cand_pair_evals_per_s": npts * wl.P / (ms * 1e-3),
        "median_dist_to_source_coarse_m": float(np.median(dist(start))),
        "median_dist_to_source_refined_m": float(np.median(dist(pts)))}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--conv-steps", type=int, default=3)
    ap.add_argument("--no-conventional", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--next-rows", action="store_true",
                    help="also measure the band-limited map (f_max = fs/4) and the refined "
                         "peak search (kept out of the default run: the band-limited map "
                         "launches the same kernel instances as the timed one, which would "
                         "mix two workloads in a kernel trace of the default command)")
    ap.add_argument("--cpu-candidates", type=int, default=120000,
                    help="candidates of the oracle's timed sample (about 10 s on 16 threads)")
    ap.add_argument("--serving-seconds", type=float, default=10.0,
                    help="length of the serving run (0 skips it)")
    ap.add_argument("--serving-leg", choices=("fp32", "bf16", "fp16"), default=None,
                    help="only run the serving workload in this precision (one JSON line)")
    ap.add_argument("--serving-rate", type=float, default=31.25,
                    help="frames/s per array of the serving workload")
    ap.add_argument("--paper-standin", action="store_true",
                    help="only run the stand-in for the paper's far-field experiment")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the SRP path "
              "shards over candidates with no exchange except a per-frame argmax reduction, "
              "and this build has no multi-GPU launcher.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2012_09499_amd as srp
    import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.serving_leg:
        print(json.dumps(serving_run(args.serving_seconds, rate_per_array=args.serving_rate,
                                     dtype=args.serving_leg)), flush=True)
        return
    if args.paper_standin:
        print(json.dumps({"paper_standin": paper_standin()}))
        return
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": src.numel() * 4,
                          "copy_calibration_bytes_written": dst.numel() * 4, "copies": 3}))
        return
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    wl = WL.make(args.config)
    print(f"[bench] workload {wl.name}: M={wl.M} P={wl.P} J={wl.J} F={wl.F} L={wl.L} "
          f"(generated in {time.perf_counter() - t_gen:.1f}s)", file=sys.stderr, flush=True)
    g = srp.Geometry(wl.mic_xyz, wl.candidates(), fs=wl.fs, L=wl.L, c=wl.c, n_aux=wl.n_aux)
    pipe = srp.SrpPipeline(g, wl.F, device=dev, keep_map=False)
    frames = torch.from_numpy(wl.frames).to(dev)
    stream = torch.cuda.current_stream()

    def nyquist_step(ev=None, dtype="fp32"):
        if ev is not None:
            ev[0].record(stream)
        psi = srp.cross_spectra(g, frames, out=pipe.psi, workspace=pipe.workspace)
        if ev is not None:
            ev[1].record(stream)
        xi = srp.gcc_samples(g, psi, out=pipe.samples_buffer(dtype), dtype=dtype)
        if ev is not None:
            ev[2].record(stream)
        srp.map_nyquist(g, xi, dtype=dtype, want_map=False, peaks_out=pipe.peaks)
        if ev is not None:
            ev[3].record(stream)

    for _ in range(args.warmup):
        nyquist_step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        nyquist_step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    t_spec = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    t_gcc = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    t_map = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    evals = float(wl.F) * wl.J * wl.P
    value = evals / (ms_step * 1e-3)
    print(f"[bench] nyquist fp32: {ms_step:.3f} ms/step (spectra {t_spec:.3f}, gcc {t_gcc:.3f}, "
          f"map {t_map:.3f} ms)", file=sys.stderr, flush=True)

    NP = g.W_total                               # N P samples per frame (Sec. 3.3)
    flops_map = 2.0 * NP * wl.J * wl.F           # 2 N P J per frame (Eq. SRPapproxcompR)
    flops_gcc = 4.0 * NP * g.K * wl.F            # N P K complex MACs, real part (Eq. SRPapproxcompC)
    achieved = flops_map / (t_map * 1e-3) / 1e12
    traffic = load_traffic(wl.name)
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                "kernel": "nyquist_f32_kernel (srp_map_nyquist, FP32 MFMA 32x32x2; one launch "
                          "of 8-tile frame blocks and, where they leave a partial round of the "
                          "CUs, one of shorter blocks; timed together per call)",
                "algorithmic_flops_per_launch": flops_map,
                "avg_launch_ms": t_map}

    out = {"metric": "SRP candidate-pair evals/s (Nyquist, FP32)", "value": value,
           "unit": "cand-pair evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded free-field white-noise sources, 10 dB sensor noise)",
           "config": {"workload": wl.name, "M": wl.M, "P": wl.P, "J": wl.J, "F": wl.F,
                      "L": wl.L, "K": g.K, "fs": wl.fs, "n_aux": wl.n_aux,
                      "samples_per_frame_NP": NP, "N_avg_samples_per_pair": NP / wl.P},
           "roofline": roofline,
           "kernels_ms": {"cross_spectra": t_spec, "gcc_samples": t_gcc, "map_nyquist": t_map},
           "gcc_samples_tflops": flops_gcc / (t_gcc * 1e-3) / 1e12}

    # low-precision Nyquist beside FP32 (same frames, same step structure)
    ref_pk = srp.decode_peaks(pipe.peaks)[0].copy()
    for dt in ("bf16", "fp16"):
        nyquist_step(dtype=dt)
        torch.cuda.synchronize()
        evl = [[torch.cuda.Event(enable_timing=True) for _ in range(4)]
               for _ in range(args.steps)]
        l0 = time.perf_counter()
        for k in range(args.steps):
            nyquist_step(evl[k], dtype=dt)
        torch.cuda.synchronize()
        ms_l = (time.perf_counter() - l0) * 1e3 / args.steps
        t_map_l = float(np.mean([e[2].elapsed_time(e[3]) for e in evl]))
        pk_l = srp.decode_peaks(pipe.peaks)[0]
        ach = flops_map / (t_map_l * 1e-3) / 1e12
        out[f"nyquist_{dt}"] = {
            "value": evals / (ms_l * 1e-3), "unit": "cand-pair evals/s", "ms_per_step": ms_l,
            "map_kernel_ms": t_map_l, "achieved_tflops": ach, "peak_tflops": PEAK_BF16_TFLOPS,
            "frac": ach / PEAK_BF16_TFLOPS, "speedup_vs_fp32": ms_step / ms_l,
            "argmax_agree_with_fp32": float(np.mean(pk_l == ref_pk))}
        print(f"[bench] nyquist {dt}: {ms_l:.3f} ms/step (map {t_map_l:.3f} ms, {ach:.0f} TFLOP/s)",
              file=sys.stderr, flush=True)

    # cached-weight BF16 Nyquist (weights built once per geometry in float64 and
    # rounded once; the map then reads them from HBM), if W fits in half the
    # free device memory
    w_bytes = srp.nyquist_weights_bytes(g, "bf16")
    free_b, _ = torch.cuda.mem_get_info(dev)
    if w_bytes <= 0.5 * free_b:
        torch.cuda.synchronize()
        b0 = time.perf_counter()
        W = srp.nyquist_weights(g, "bf16")
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - b0) * 1e3

        def cached_step(ev=None):
            if ev is not None:
                ev[0].record(stream)
            psi = srp.cross_spectra(g, frames, out=pipe.psi, workspace=pipe.workspace)
            xi = srp.gcc_samples(g, psi, out=pipe.samples_buffer("bf16"), dtype="bf16")
            if ev is not None:
                ev[1].record(stream)
            srp.map_nyquist_cached(g, W, xi, dtype="bf16", want_map=False, peaks_out=pipe.peaks)
            if ev is not None:
                ev[2].record(stream)

        cached_step()
        torch.cuda.synchronize()
        evc = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
               for _ in range(args.steps)]
        q0 = time.perf_counter()
        for k in range(args.steps):
            cached_step(evc[k])
        torch.cuda.synchronize()
        ms_c = (time.perf_counter() - q0) * 1e3 / args.steps
        t_map_c = float(np.mean([e[1].elapsed_time(e[2]) for e in evc]))
        pk_c = srp.decode_peaks(pipe.peaks)[0]
        ach = flops_map / (t_map_c * 1e-3) / 1e12
        out["nyquist_bf16_cached"] = {
            "value": evals / (ms_c * 1e-3), "unit": "cand-pair evals/s", "ms_per_step": ms_c,
            "map_kernel_ms": t_map_c, "achieved_tflops": ach, "peak_tflops": PEAK_BF16_TFLOPS,
            "frac": ach / PEAK_BF16_TFLOPS, "weights_bytes": w_bytes,
            "weights_hbm_GBps": w_bytes / (t_map_c * 1e-3) / 1e9,
            "weights_build_ms": build_ms, "speedup_vs_fp32": ms_step / ms_c,
            "argmax_agree_with_fp32": float(np.mean(pk_c == ref_pk))}
        print(f"[bench] nyquist bf16 cached: {ms_c:.3f} ms/step (map {t_map_c:.3f} ms, "
              f"{ach:.0f} TFLOP/s; W {w_bytes / 1e9:.1f} GB built in {build_ms:.0f} ms)",
              file=sys.stderr, flush=True)
        del W
    else:
        out["nyquist_bf16_cached"] = {"skipped": f"W needs {w_bytes / 1e9:.0f} GB"}

    if args.next_rows:
        nr = next_rows_leg(srp, torch, wl, g, frames, pipe, args.steps)
        out["next_rows"] = nr
        b = nr["band_limited"]
        print(f"[bench] band-limited (f_max {b['f_max_hz']:.0f} Hz): fp32 map "
              f"{b['fp32']['map_kernel_ms']:.2f} ms, bf16 map {b['bf16']['map_kernel_ms']:.2f} ms; "
              f"refined search {nr['refined_search']['ms_per_call']:.2f} ms per call, median "
              f"distance to a source {nr['refined_search']['median_dist_to_source_coarse_m']:.3f}"
              f" -> {nr['refined_search']['median_dist_to_source_refined_m']:.3f} m",
              file=sys.stderr, flush=True)

    if not args.no_conventional:
        def conv_step():
            psi = srp.cross_spectra(g, frames, out=pipe.psi, workspace=pipe.workspace)
            srp.map_conventional(g, psi, want_map=False, peaks_out=pipe.peaks)
        conv_step()
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for _ in range(args.conv_steps):
            conv_step()
        torch.cuda.synchronize()
        ms_conv = (time.perf_counter() - c0) * 1e3 / args.conv_steps
        flops_conv = 4.0 * g.K * wl.P * wl.J * wl.F   # J P K complex MACs, real part (Eq. SRPomp)
        out["conventional"] = {"value": evals / (ms_conv * 1e-3), "unit": "cand-pair evals/s",
                               "ms_per_step": ms_conv, "steps": args.conv_steps,
                               "algorithmic_tflops": flops_conv / (ms_conv * 1e-3) / 1e12,
                               "nyquist_speedup": ms_conv / ms_step,
                               "argmax_agree_with_nyquist_fp32":
                                   float(np.mean(srp.decode_peaks(pipe.peaks)[0] == ref_pk))}
        print(f"[bench] conventional fp32: {ms_conv:.1f} ms/step", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        cb, idx, ref = cpu_baseline(wl, args.cpu_candidates)
        out["cpu_baseline"] = cb
        # parity of the timed configuration on the sampled candidates (not timed)
        del pipe
        keep = srp.SrpPipeline(g, wl.F, device=dev, keep_map=True)
        sel = torch.from_numpy(idx).to(dev)
        out["parity_sampled"] = {"candidates": int(idx.size)}
        for dt in ("fp32", "bf16", "fp16"):
            m, _ = keep.nyquist(frames, dtype=dt)
            sub = m[:, sel].cpu().numpy().astype(np.float64)
            e = np.sqrt(((sub - ref) ** 2).sum(1) / (ref ** 2).sum(1))
            out["parity_sampled"][dt] = {"max_rel_err": float(e.max()),
                                         "median_rel_err": float(np.median(e))}
        err = np.asarray([out["parity_sampled"]["fp32"]["max_rel_err"]])
        print(f"[bench] cpu baseline {cb['value']:.3e} evals/s on {cb['cores']} BLAS threads "
              f"({cb['seconds']:.1f}s); sampled map rel err max {err.max():.2e}",
              file=sys.stderr, flush=True)

    if args.serving_seconds > 0:
        # the offered load (31.25 frames/s per array, 2,007 frames/s in all) in
        # FP32 and BF16, then 8x that load for a third of the time: the frames/s
        # completed there is the server's capacity in each precision
        legs = [("serving", "fp32", 31.25, args.serving_seconds),
                ("serving_bf16", "bf16", 31.25, args.serving_seconds),
                ("serving_capacity_fp32", "fp32", 250.0, args.serving_seconds / 3.0),
                ("serving_capacity_bf16", "bf16", 250.0, args.serving_seconds / 3.0)]
        for key, sdt, rate, secs in legs:
            # each serving configuration runs in a process of its own, as a
            # deployed server would (a child process, not an exec)
            cmd = [sys.executable, os.path.abspath(__file__), "--serving-leg", sdt,
                   "--serving-seconds", str(secs), "--serving-rate", str(rate)]
            r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
            if r.returncode != 0:
                raise RuntimeError(f"serving leg {key} failed:\n{r.stderr[-2000:]}")
            st = json.loads(r.stdout.strip().splitlines()[-1])
            out[key] = st
            print(f"[bench] {key}: {st['frames_per_s']:.0f} frames/s done of "
                  f"{st['offered_frames_per_s']:.0f} offered, p50 {st['latency_ms_p50']:.1f} ms, "
                  f"p99 {st['latency_ms_p99']:.1f} ms", file=sys.stderr, flush=True)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
