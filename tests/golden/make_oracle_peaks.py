"""Writes the float64 oracle's per-frame peaks of a whole Nyquist map.

Test data generator: it calls only `workloads` (seeded inputs) and `oracle`
(the method, float64), never the library. For one single-array workload it
evaluates the oracle's Nyquist map (Eq. SRPapprox summed over pairs as in
Eq. SRP_T_IFT) at every candidate and every frame, in candidate chunks spread
over threads, and keeps per frame the argmax (lowest index on ties, Section
2.2), the maximum and the L2 norm of the map over the candidates. The GPU
tests compare the library's argmax with these peaks where the map is too
large for the oracle to run inside a test.

    python tests/golden/make_oracle_peaks.py --config 3 --frames 200 --workers 8
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as WL  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, required=True)
    ap.add_argument("--frames", type=int, default=None)
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--chunk", type=int, default=4096)
    args = ap.parse_args()
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)  # one BLAS thread per worker thread
    except ImportError:
        pass
    t0 = time.perf_counter()
    wl = WL.make(args.config, F=args.frames)
    K = O.n_bins(wl.L, wl.fs)
    w = O.bin_weights(wl.L, K)
    win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, wl.n_aux)
    psi = O.phat_cross_spectra(O.spectra(wl.frames, O.window(wl.L), K))
    xi = O.gcc_samples(psi, wl.fs, wl.L, w, win)

    def chunk(j0):
        j1 = min(wl.J, j0 + args.chunk)
        dt = O.tdoa(wl.mic_xyz, wl.candidates(j0, j1), wl.c)
        m = O.srp_nyquist(xi, dt, win)  # [F][j1 - j0]
        loc = np.argmax(m, axis=1)
        return j0, loc + j0, m[np.arange(m.shape[0]), loc], (m * m).sum(axis=1)

    F = wl.F
    best_idx = np.zeros(F, dtype=np.int64)
    best_val = np.full(F, -np.inf)
    sumsq = np.zeros(F)
    starts = list(range(0, wl.J, args.chunk))
    done = 0
    with cf.ThreadPoolExecutor(max_workers=args.workers) as ex:
        results = {}
        for j0, idx, val, ss in ex.map(chunk, starts):
            results[j0] = (idx, val, ss)
            done += 1
            if done % 100 == 0:
                print(f"[oracle peaks] {done}/{len(starts)} chunks, "
                      f"{time.perf_counter() - t0:.0f} s", flush=True)
    for j0 in starts:  # ascending candidate order: strict '>' keeps the lowest index on ties
        idx, val, ss = results[j0]
        upd = val > best_val
        best_idx[upd] = idx[upd]
        best_val[upd] = val[upd]
        sumsq += ss
    sec = time.perf_counter() - t0
    out = {
        "workload": wl.name, "config": args.config, "F": F, "J": wl.J, "M": wl.M,
        "samples_per_frame": int(win["S"]),
        "what": "float64 oracle Nyquist map (srp_nyquist from gcc_samples of the frames): "
                "per frame argmax (lowest index on ties), maximum and L2 norm over all "
                "candidates",
        "command": f"python tests/golden/make_oracle_peaks.py --config {args.config} "
                   f"--frames {F} --workers {args.workers}",
        "seconds": round(sec, 1),
        "argmax": best_idx.tolist(),
        "max": best_val.tolist(),
        "l2": np.sqrt(sumsq).tolist(),
    }
    path = os.path.join(HERE, f"oracle_nyquist_peaks_{wl.name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} ({sec:.0f} s)")


if __name__ == "__main__":
    main()
