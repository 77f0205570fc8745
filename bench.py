"""Benchmark: SRP candidate-pair evaluations per second on one MI355X.

Workload (default): the room-scale configuration -- 16 microphones uniformly
random in a 1 x 1 x 0.5 m box (120 pairs), fs = 16 kHz, 1024-sample Hann
frames (513 bins), a 6 x 4 x 3 m room gridded at 5 cm (576,000 candidates),
500 frames of seeded free-field white-noise sources with 10 dB sensor noise,
N_aux = 2. Inputs are synthetic (workloads.make(2)) and already resident in
device memory when the timed region starts.

One step = one pass of the Nyquist hot path over the 500-frame batch:
srp_gcc_samples_frames (windowed FFT, PHAT phasors, cross-spectra formed on
chip, GCC samples at the critical lags), srp_map_nyquist (TDOA + sinc
interpolation + pair sum + per-frame argmax). `value` = F * J * P / step time. The
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
# Weight-generation bound of the BF16/FP16 map kernel: its non-matrix vector
# instructions per sinc weight and lane, (SQ_INSTS_VALU - SQ_INSTS_MFMA) x 64
# over J S ceil(F / 256) weights, from the SQ counters at the room scale
# ((9.751e8 - 1.298e8) x 64 / (576,000 x 6,544 x 2); the per-run TDOA split and
# staging included), issued at one wave64 instruction per 4 cycles per SIMD.
MX_VALU_PER_WEIGHT = 7.18
VALU_ISSUE_WAVE_INSTR_PER_S = 1024 * 2.4e9 / 4
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


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()
                    if i.get("user_api") == "blas"] or [1])
    except Exception:
        return 1


def _oracle_map(O, wl, xi, win, idx, workers, chunk=4096):
    """The oracle's Nyquist map at candidates idx, in candidate chunks spread over
    `workers` threads with one BLAS thread each (workers = 1: one thread)."""
    import concurrent.futures as cf
    from threadpoolctl import threadpool_limits
    out = np.empty((xi.shape[0], idx.size))

    def run(j0):
        j1 = min(idx.size, j0 + chunk)
        dt = O.tdoa(wl.mic_xyz, wl.candidates_at(idx[j0:j1]), wl.c)
        out[:, j0:j1] = O.srp_nyquist(xi, dt, win)

    with threadpool_limits(1):
        if workers == 1:
            for j0 in range(0, idx.size, chunk):
                run(j0)
        else:
            with cf.ThreadPoolExecutor(max_workers=workers) as ex:
                list(ex.map(run, range(0, idx.size, chunk)))
    return out


def cpu_baseline(wl, n_cand: int, n_cand_single: int, reps: int = 3, full_argmax: bool = True,
                 seed: int = 0):
    """The FP64 oracle timed on the host: spectra, PHAT, GCC samples and the
    Nyquist map of a seeded candidate sample over all frames, once on one
    thread and once on all cores (threads over candidate chunks, one BLAS
    thread each), the median of `reps` runs each; then (untimed for the rate)
    the oracle's map over ALL candidates, whose per-frame argmax the GPU paths
    are compared with. Returns (info, sample indices, sample map, full argmax)."""
    import oracle as O
    workers = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(wl.J, size=min(n_cand, wl.J), replace=False))
    idx1 = idx[:min(n_cand_single, idx.size)]
    K = O.n_bins(wl.L, wl.fs)
    w = O.bin_weights(wl.L, K)
    win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, wl.n_aux)

    def front():
        psi = O.phat_cross_spectra(O.spectra(wl.frames, O.window(wl.L), K))
        return O.gcc_samples(psi, wl.fs, wl.L, w, win)

    from threadpoolctl import threadpool_limits
    legs = {}
    ref = None
    for name, sel, nw in (("single_thread", idx1, 1), ("all_cores", idx, workers)):
        t_front, t_map = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            with threadpool_limits(1 if nw == 1 else None):
                xi = front()
            t1 = time.perf_counter()
            m = _oracle_map(O, wl, xi, win, sel, nw)
            O.peaks(m)
            t2 = time.perf_counter()
            t_front.append(t1 - t0)
            t_map.append(t2 - t1)
        tf, tm = float(np.median(t_front)), float(np.median(t_map))
        pairs = wl.F * sel.size * wl.P
        legs[name] = {"value": pairs / (tf + tm), "unit": "cand-pair evals/s",
                      "map_only_value": pairs / tm, "threads": nw,
                      "front_end_seconds_median": tf, "map_seconds_median": tm,
                      "front_end_seconds": t_front, "map_seconds": t_map,
                      "candidates": int(sel.size), "frames": wl.F}
        if name == "all_cores":
            ref = m
    full = None
    predicted = legs["all_cores"]["map_seconds_median"] * wl.J / idx.size
    if full_argmax and predicted > 180.0:
        full_argmax = False
        legs["full_map_skipped"] = f"predicted {predicted:.0f} s on {workers} threads"
    if full_argmax:
        t0 = time.perf_counter()
        xi = front()
        allidx = np.arange(wl.J)
        fm = _oracle_map(O, wl, xi, win, allidx, workers)
        full = {"argmax": np.argmax(fm, axis=1), "seconds": time.perf_counter() - t0}
        del fm
    info = {"value": legs["all_cores"]["value"], "unit": "cand-pair evals/s", "cores": workers,
            "kind": "oracle", "cpu_model": _cpu_model(), "host_cpu_count": os.cpu_count(),
            "blas_threads_default": _blas_threads(), "single_thread": legs["single_thread"],
            "all_cores": legs["all_cores"],
            "sample": (f"all {wl.F} frames; a seeded sample of {idx.size} of {wl.J} candidates "
                       f"on {workers} threads (candidate chunks, one BLAS thread each) and "
                       f"{idx1.size} of them on one thread; spectra + PHAT + GCC samples + "
                       f"Nyquist map + argmax in float64 NumPy; median of {reps} runs")}
    if full is not None:
        info["full_map_seconds_all_cores"] = full["seconds"]
    elif "full_map_skipped" in legs:
        info["full_map_skipped"] = legs["full_map_skipped"]
    return info, idx, ref, (None if full is None else full["argmax"])


def cpu_baseline_subset_parity(wl, idx, dtypes_maps, frames=None):
    """Sampled parity of larger configurations: the oracle's Nyquist map at the
    candidates idx (of `frames`, default all of the workload's) against each
    GPU map's columns there."""
    import oracle as O
    K = O.n_bins(wl.L, wl.fs)
    w = O.bin_weights(wl.L, K)
    win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, wl.n_aux)
    fr = wl.frames if frames is None else frames
    psi = O.phat_cross_spectra(O.spectra(fr, O.window(wl.L), K))
    xi = O.gcc_samples(psi, wl.fs, wl.L, w, win)
    ref = _oracle_map(O, wl, xi, win, idx, min(16, os.cpu_count() or 1))
    out = {}
    for dt, sub in dtypes_maps.items():
        e = np.sqrt(((sub - ref) ** 2).sum(1) / (ref ** 2).sum(1))
        out[dt] = {"max_rel_err": float(e.max()), "median_rel_err": float(np.median(e))}
    return out


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
    # deadline: one frame duration (L / fs = 64 ms), the real-time budget of a frame
    srv = SV.SrpServer(dtype=dtype, deadline_ms=1e3 * L / fs)
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
            xi = srp.gcc_samples_frames(g2, frames, out=p2.samples_buffer(dt), dtype=dt,
                                        workspace=p2.workspace)
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
    xi = srp.gcc_samples_frames(g, frames, out=pipe.samples_buffer("fp32"),
                                workspace=pipe.workspace)
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


def library_gemm_reference(torch, dev, n: int = 8192, reps: int = 10):
    """Rate of the vendor library's dense GEMM (torch.matmul -> hipBLASLt) on
    n x n x n operands per dtype, timed on the same device: the rate a plain
    matrix product reaches on this chip under its real clock and power limits,
    a practical ceiling to read the map kernels' utilisation against (the
    roofline itself keeps the published peak)."""
    res = {"n": n, "library": "torch.matmul (hipBLASLt)"}
    for name, dt in (("bf16", torch.bfloat16), ("fp16", torch.float16), ("fp32", torch.float32)):
        gen = torch.Generator(device=dev).manual_seed(0)
        a = torch.randn(n, n, device=dev, dtype=dt, generator=gen)
        b = torch.randn(n, n, device=dev, dtype=dt, generator=gen)
        for _ in range(3):
            c = a @ b
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"{name}_tflops"] = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
        del a, b, c
    torch.cuda.empty_cache()
    return res


def _timed(step, steps: int, n_marks: int):
    """Run `step(events)` `steps` times after one untimed call; return the wall
    ms per step and the mean ms between consecutive HIP-event marks."""
    import torch
    step(None)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(n_marks)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    gaps = [float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs]))
            for i in range(n_marks - 1)]
    return ms, gaps


def weight_bound(J: int, S: int, F: int, map_ms: float) -> dict:
    """Time the BF16/FP16 map's weight arithmetic alone would take: one set of
    sinc weights per (candidate, sample) and 256-frame block, at the measured
    vector instructions per weight and the SIMDs' issue rate (published clock)."""
    w = J * S * -(-F // 256)
    ms = w * MX_VALU_PER_WEIGHT / 64 / VALU_ISSUE_WAVE_INSTR_PER_S * 1e3
    return {"weights_per_call": w, "valu_lane_instr_per_weight": MX_VALU_PER_WEIGHT,
            "valu_issue_wave_instr_per_s": VALU_ISSUE_WAVE_INSTR_PER_S, "ms": ms,
            "frac_of_map_time": ms / map_ms,
            "per_weight_count_from": "SQ counters, room scale"}


def _dist_to_source(wl, idx):
    """Median over frames of the distance (m) from the picked candidate to the
    nearest true source."""
    q = wl.candidates_at(np.asarray(idx))
    d = np.linalg.norm(q[:, None, :] - wl.sources[None, :, :], axis=-1).min(axis=1)
    return float(np.median(d))


def other_geometry_leg(srp, torch, cfg: int, dtypes, steps: dict, F=None):
    """Nyquist map on the 32-mic (4M candidates, L = 2048) or the 64-mic
    (9M candidates, 48 kHz, L = 4096) geometry: per dtype, ms per step and the
    map kernel's TFLOP/s against the matrix-core peak. Returns the result, the
    workload, and a keep-map pipeline's maps for sampled parity."""
    import workloads as WL
    dev = torch.device("cuda:0")
    wl = WL.make(cfg, F=F)
    g = srp.Geometry(wl.mic_xyz, wl.candidates(), fs=wl.fs, L=wl.L, c=wl.c, n_aux=wl.n_aux)
    pipe = srp.SrpPipeline(g, wl.F, device=dev, keep_map=False)
    frames = torch.from_numpy(wl.frames).to(dev)
    stream = torch.cuda.current_stream()
    NP = g.W_total
    flops = 2.0 * NP * wl.J * wl.F
    res = {"workload": wl.name, "M": wl.M, "P": wl.P, "J": wl.J, "F": wl.F, "L": wl.L,
           "K": g.K, "fs": wl.fs, "samples_per_frame_NP": NP}
    peaks = {}
    for dt in dtypes:
        def step(ev, dt=dt):
            xi = srp.gcc_samples_frames(g, frames, out=pipe.samples_buffer(dt), dtype=dt,
                                        workspace=pipe.workspace)
            if ev is not None:
                ev[0].record(stream)
            srp.map_nyquist(g, xi, dtype=dt, want_map=False, peaks_out=pipe.peaks)
            if ev is not None:
                ev[1].record(stream)
        ms, (t_map,) = _timed(step, steps[dt], 2)
        idx = srp.decode_peaks(pipe.peaks)[0].copy()
        peaks[dt] = idx
        ach = flops / (t_map * 1e-3) / 1e12
        peak = PEAK_FP32_TFLOPS if dt == "fp32" else PEAK_BF16_TFLOPS
        # weight sets formed per second: one (candidate, pair) set of sinc
        # weights per frame block of up to 256 frames (both kernels)
        wp = wl.J * wl.P * (-(-wl.F // 256))
        res[dt] = {"steps": steps[dt], "ms_per_step": ms, "map_kernel_ms": t_map,
                   "value": wl.F * wl.J * wl.P / (ms * 1e-3), "unit": "cand-pair evals/s",
                   "achieved_tflops": ach, "peak_tflops": peak, "frac": ach / peak,
                   "weight_pairs_per_s": wp / (t_map * 1e-3),
                   "median_dist_to_source_m": _dist_to_source(wl, idx)}
        if dt != "fp32":
            res[dt]["weight_bound"] = weight_bound(wl.J, g.W_total, wl.F, t_map)
        print(f"[bench] {wl.name} nyquist {dt}: {ms:.1f} ms/step (map {t_map:.1f} ms, "
              f"{ach:.0f} TFLOP/s)", file=sys.stderr, flush=True)
    for a in dtypes:
        for b in dtypes:
            if a < b:
                res[f"argmax_agree_{a}_{b}"] = float(np.mean(peaks[a] == peaks[b]))
    del pipe
    return res, wl, g, frames, peaks


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--conv-steps", type=int, default=3)
    ap.add_argument("--no-conventional", action="store_true")
    ap.add_argument("--no-gemm-reference", action="store_true",
                    help="skip timing the library GEMM reference (practical matrix-core ceiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-geometries", action="store_true",
                    help="skip the 32-mic and 64-mic Nyquist legs")
    ap.add_argument("--next-rows", action="store_true",
                    help="also measure the band-limited map (f_max = fs/4) and the refined "
                         "peak search (kept out of the default run: the band-limited map "
                         "launches the same kernel instances as the timed one, which would "
                         "mix two workloads in a kernel trace of the default command)")
    ap.add_argument("--cpu-candidates", type=int, default=60000,
                    help="candidates of the oracle's all-core timed sample")
    ap.add_argument("--cpu-candidates-single", type=int, default=4000,
                    help="candidates of the oracle's single-thread timed sample")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-full-oracle-argmax", action="store_true",
                    help="skip the oracle's whole-map argmax of the timed workload")
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
    picks = {}   # per path: the per-frame argmax indices

    def nyquist_step(ev=None, dtype="fp32"):
        if ev is not None:
            ev[0].record(stream)
        xi = srp.gcc_samples_frames(g, frames, out=pipe.samples_buffer(dtype), dtype=dtype,
                                    workspace=pipe.workspace)
        if ev is not None:
            ev[1].record(stream)
        srp.map_nyquist(g, xi, dtype=dtype, want_map=False, peaks_out=pipe.peaks)
        if ev is not None:
            ev[2].record(stream)

    def two_call_front(ev=None):
        if ev is not None:
            ev[0].record(stream)
        psi = srp.cross_spectra(g, frames, out=pipe.psi, workspace=pipe.workspace)
        if ev is not None:
            ev[1].record(stream)
        srp.gcc_samples(g, psi, out=pipe.samples_buffer("fp32"))
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        nyquist_step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        nyquist_step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    t_front = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    t_map = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    evals = float(wl.F) * wl.J * wl.P
    value = evals / (ms_step * 1e-3)
    print(f"[bench] nyquist fp32: {ms_step:.3f} ms/step (front end {t_front:.3f}, "
          f"map {t_map:.3f} ms)", file=sys.stderr, flush=True)
    # the same front end as two calls (cross-spectra written, then read back)
    _, (t_spec, t_gcc) = _timed(two_call_front, args.steps, 3)
    print(f"[bench] two-call front end: cross_spectra {t_spec:.3f} + gcc_samples {t_gcc:.3f} ms",
          file=sys.stderr, flush=True)

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
           "kernels_ms": {"gcc_samples_frames": t_front, "map_nyquist": t_map},
           "front_end_gcc_tflops": flops_gcc / (t_front * 1e-3) / 1e12,
           "two_call_front_end_ms": {"cross_spectra": t_spec, "gcc_samples": t_gcc},
           "paper_complexity_no_hardware_stated": {
               "C_conv_per_frame_JPK": wl.J * wl.P * g.K, "C_samp_per_frame_NPK": NP * g.K,
               "C_int_per_frame_NPJ": NP * wl.J, "R_samp_N_over_J": NP / wl.P / wl.J,
               "R_int_N_over_K": NP / wl.P / g.K}}
    picks["nyquist_fp32"] = srp.decode_peaks(pipe.peaks)[0].copy()
    ref_pk = picks["nyquist_fp32"]

    # low-precision Nyquist beside FP32 (same frames, same step structure)
    for dt in ("bf16", "fp16"):
        ms_l, (t_front_l, t_map_l) = _timed(lambda ev, dt=dt: nyquist_step(ev, dtype=dt),
                                            args.steps, 3)
        pk_l = srp.decode_peaks(pipe.peaks)[0].copy()
        picks[f"nyquist_{dt}"] = pk_l
        ach = flops_map / (t_map_l * 1e-3) / 1e12
        out[f"nyquist_{dt}"] = {
            "value": evals / (ms_l * 1e-3), "unit": "cand-pair evals/s", "ms_per_step": ms_l,
            "map_kernel_ms": t_map_l, "front_end_ms": t_front_l, "achieved_tflops": ach,
            "peak_tflops": PEAK_BF16_TFLOPS,
            "frac": ach / PEAK_BF16_TFLOPS, "speedup_vs_fp32": ms_step / ms_l,
            "argmax_agree_with_fp32": float(np.mean(pk_l == ref_pk)),
            "weight_bound": weight_bound(wl.J, NP, wl.F, t_map_l)}
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
            xi = srp.gcc_samples_frames(g, frames, out=pipe.samples_buffer("bf16"), dtype="bf16",
                                        workspace=pipe.workspace)
            if ev is not None:
                ev[1].record(stream)
            srp.map_nyquist_cached(g, W, xi, dtype="bf16", want_map=False, peaks_out=pipe.peaks)
            if ev is not None:
                ev[2].record(stream)

        ms_c, (_, t_map_c) = _timed(cached_step, args.steps, 3)
        pk_c = srp.decode_peaks(pipe.peaks)[0].copy()
        picks["nyquist_bf16_cached"] = pk_c
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
        # conventional SRP (Eq. SRPomp) on the same frames: FP32 from the
        # complex spectra; BF16/FP16 from the weighted spectra rounded once
        flops_conv = 4.0 * g.K * wl.P * wl.J * wl.F   # J P K complex MACs, real part
        for dt in ("fp32", "bf16", "fp16"):
            low = dt != "fp32"
            spec = srp.spectra_lowp_buffer(g, wl.F, dt, dev) if low else None

            def conv_step(ev, dt=dt, low=low, spec=spec):
                psi = srp.cross_spectra(g, frames, out=pipe.psi, workspace=pipe.workspace)
                if low:
                    psi = srp.spectra_lowp(g, psi, dt, out=spec)
                if ev is not None:
                    ev[0].record(stream)
                srp.map_conventional(g, psi, dtype=dt, want_map=False, peaks_out=pipe.peaks)
                if ev is not None:
                    ev[1].record(stream)
            ms_conv, (t_cmap,) = _timed(conv_step, args.conv_steps, 2)
            pk = srp.decode_peaks(pipe.peaks)[0].copy()
            key = "conventional" if dt == "fp32" else f"conventional_{dt}"
            picks[key] = pk
            ach = flops_conv / (t_cmap * 1e-3) / 1e12
            peak = PEAK_FP32_TFLOPS if dt == "fp32" else PEAK_BF16_TFLOPS
            nyq = "nyquist_fp32" if dt == "fp32" else f"nyquist_{dt}"
            ms_nyq = ms_step if dt == "fp32" else out[nyq]["ms_per_step"]
            out[key] = {"value": evals / (ms_conv * 1e-3), "unit": "cand-pair evals/s",
                        "ms_per_step": ms_conv, "map_kernel_ms": t_cmap,
                        "steps": args.conv_steps, "algorithmic_tflops": ach,
                        "peak_tflops": peak, "frac": ach / peak,
                        "nyquist_speedup": ms_conv / ms_nyq,
                        "argmax_agree_with_nyquist_same_dtype": float(np.mean(pk == picks[nyq]))}
            del spec
            print(f"[bench] conventional {dt}: {ms_conv:.1f} ms/step (map {t_cmap:.1f} ms, "
                  f"{ach:.0f} TFLOP/s)", file=sys.stderr, flush=True)
        out["conventional_vs_nyquist_argmax"] = {
            dt: float(np.mean(picks["conventional" if dt == "fp32" else f"conventional_{dt}"]
                              == picks["conventional"]))
            for dt in ("fp32", "bf16", "fp16")}

    # localisation accuracy of every path: median distance from the pick to the
    # nearest true source (the same frames, the same sources)
    out["median_dist_to_source_m"] = {k: _dist_to_source(wl, v) for k, v in picks.items()}

    others = {}
    if not args.no_other_geometries:
        del pipe
        torch.cuda.empty_cache()
        r3, wl3, g3, fr3, pk3 = other_geometry_leg(
            srp, torch, 3, ("fp32", "bf16", "fp16"), {"fp32": 2, "bf16": 3, "fp16": 3})
        out["precision_32mic"] = r3
        others[3] = (wl3, g3, fr3, pk3)
        r5, wl5, g5, fr5, pk5 = other_geometry_leg(
            srp, torch, 5, ("bf16", "fp16"), {"bf16": 2, "fp16": 2})
        out["largest_64mic"] = r5
        others[5] = (wl5, g5, fr5, pk5)
        pipe = None

    if not args.no_cpu_baseline:
        cb, idx, ref, full_arg = cpu_baseline(wl, args.cpu_candidates, args.cpu_candidates_single,
                                              reps=args.cpu_reps,
                                              full_argmax=not args.no_full_oracle_argmax)
        gpu_rate = {"nyquist_fp32": value, "nyquist_bf16": out["nyquist_bf16"]["value"]}
        cb["gpu_over_oracle"] = {k: {"all_cores": v / cb["all_cores"]["value"],
                                     "single_thread": v / cb["single_thread"]["value"]}
                                 for k, v in gpu_rate.items()}
        out["cpu_baseline"] = cb
        if full_arg is not None:
            out["argmax_vs_oracle_full_map"] = {k: float(np.mean(v == full_arg))
                                                for k, v in picks.items()}
            out["median_dist_to_source_m"]["oracle_nyquist_fp64"] = _dist_to_source(wl, full_arg)
        # parity of the timed configuration on the sampled candidates (not timed)
        keep = srp.SrpPipeline(g, wl.F, device=dev, keep_map=True)
        sel = torch.from_numpy(idx).to(dev)
        maps = {}
        for dt in ("fp32", "bf16", "fp16"):
            m, _ = keep.nyquist(frames, dtype=dt)
            maps[dt] = m[:, sel].cpu().numpy().astype(np.float64)
        if "skipped" not in out.get("nyquist_bf16_cached", {"skipped": ""}):
            # the cached-weight map of the same frames (W built again)
            xi_c = srp.gcc_samples_frames(g, frames, dtype="bf16", workspace=keep.workspace)
            del keep
            torch.cuda.empty_cache()
            W = srp.nyquist_weights(g, "bf16")
            m, _ = srp.map_nyquist_cached(g, W, xi_c, dtype="bf16", want_peaks=False)
            maps["bf16_cached"] = m[:, sel].cpu().numpy().astype(np.float64)
            del W, m, xi_c
            torch.cuda.empty_cache()
        else:
            del keep
        e = {}
        for dt, sub in maps.items():
            r = np.sqrt(((sub - ref) ** 2).sum(1) / (ref ** 2).sum(1))
            e[dt] = {"max_rel_err": float(r.max()), "median_rel_err": float(np.median(r))}
        out["parity_sampled"] = {"candidates": int(idx.size), **e}
        print(f"[bench] cpu baseline {cb['value']:.3e} evals/s on {cb['cores']} threads, "
              f"{cb['single_thread']['value']:.3e} on one; sampled map rel err max "
              f"{e['fp32']['max_rel_err']:.2e} (fp32) {e['bf16']['max_rel_err']:.2e} (bf16)",
              file=sys.stderr, flush=True)
        # sampled parity of the other geometries: a seeded candidate sample and
        # the first frames (the oracle's GCC samples of all frames would take minutes)
        for cfg, key, n_c, n_f in ((3, "precision_32mic", 1000, 8), (5, "largest_64mic", 200, 2)):
            if cfg not in others:
                continue
            wlx, gx, frx, _ = others[cfg]
            rng = np.random.default_rng(cfg)
            idx_x = np.sort(rng.choice(wlx.J, size=n_c, replace=False))
            kp = srp.SrpPipeline(gx, n_f, device=dev, keep_map=True)
            selx = torch.from_numpy(idx_x).to(dev)
            subs = {}
            for dt in out[key]:
                if dt in ("fp32", "bf16", "fp16"):
                    m, _ = kp.nyquist(frx[:n_f], dtype=dt)
                    subs[dt] = m[:, selx].cpu().numpy().astype(np.float64)
            del kp
            out[key]["parity_sampled"] = {
                "candidates": n_c, "frames": n_f,
                **cpu_baseline_subset_parity(wlx, idx_x, subs, frames=wlx.frames[:n_f])}
            print(f"[bench] {key} sampled parity: " + ", ".join(
                f"{dt} {v['max_rel_err']:.2e}" for dt, v in out[key]["parity_sampled"].items()
                if isinstance(v, dict)), file=sys.stderr, flush=True)

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
                  f"p99 {st['latency_ms_p99']:.1f} ms, {100 * st['deadline_miss_rate']:.1f} % past "
                  f"the {st['deadline_ms']:.0f} ms deadline", file=sys.stderr, flush=True)

    if not args.no_gemm_reference:
        # the library GEMM's rate on this chip: each matrix-core leg's
        # algorithmic rate is also stated as a fraction of it
        ref = library_gemm_reference(torch, dev)
        out["library_gemm_reference"] = ref
        for key, leg in [("roofline", out["roofline"])] + [
                (k, v) for k, v in out.items()
                if k.startswith(("nyquist_", "conventional")) and isinstance(v, dict)]:
            ach = leg.get("achieved", leg.get("achieved_tflops", leg.get("algorithmic_tflops")))
            if ach is None:
                continue
            dt = "fp32" if key in ("roofline", "conventional") else (
                "fp16" if key.endswith("fp16") else "bf16")
            leg["frac_of_library_gemm"] = ach / ref[f"{dt}_tflops"]
        for key in ("precision_32mic", "largest_64mic"):
            for dt, leg in out.get(key, {}).items():
                if dt in ("fp32", "bf16", "fp16") and "achieved_tflops" in leg:
                    leg["frac_of_library_gemm"] = leg["achieved_tflops"] / ref[f"{dt}_tflops"]
        print(f"[bench] library GEMM {ref['n']}^3: bf16 {ref['bf16_tflops']:.0f}, fp16 "
              f"{ref['fp16_tflops']:.0f}, fp32 {ref['fp32_tflops']:.0f} TFLOP/s", file=sys.stderr,
              flush=True)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
