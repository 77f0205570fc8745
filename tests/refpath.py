"""Test helpers: run the oracle and the GPU path on the same seeded workload.

The oracle side calls only `oracle`; the GPU side calls only the C ABI through
paper_2012_09499_amd. Inputs come from `workloads`.
"""
from __future__ import annotations

import numpy as np

import oracle as O


def oracle_setup(wl, n_aux=None, window="hann"):
    f_max = wl.band_limit
    K = O.n_bins(wl.L, wl.fs, f_max)
    w = O.bin_weights(wl.L, K)
    win = O.pair_windows(wl.mic_xyz, wl.c, f_max, wl.n_aux if n_aux is None else n_aux)
    return K, w, win


def oracle_psi(wl, frames=None, window="hann"):
    K = O.n_bins(wl.L, wl.fs, wl.band_limit)
    fr = wl.frames if frames is None else frames
    return O.phat_cross_spectra(O.spectra(fr, O.window(wl.L, window), K))


def oracle_xi(wl, psi, n_aux=None):
    K, w, win = oracle_setup(wl, n_aux)
    return O.gcc_samples(psi, wl.fs, wl.L, w, win)


def oracle_nyquist(wl, xi, cand, n_aux=None):
    _, _, win = oracle_setup(wl, n_aux)
    dt = O.tdoa(wl.mic_xyz, cand, wl.c, field=wl.field)
    return O.srp_nyquist(xi, dt, win)


def oracle_conventional(wl, psi, cand):
    K, w, _ = oracle_setup(wl)
    dt = O.tdoa(wl.mic_xyz, cand, wl.c, field=wl.field)
    return O.srp_conventional(psi, dt, wl.fs, wl.L, w)


def check_argmax(gpu_idx, ref_map, rel_tol, frac=0.99):
    """Argmax agreement with the reference map.

    A frame whose argmax differs must be a near-tie that the map tolerance
    allows: if ||gpu - ref||_2 <= rel_tol ||ref||_2, the GPU's pick can trail
    the reference maximum by at most 2 rel_tol ||ref||_2. With >= 100 frames
    at least `frac` of them must be identical. Returns the identical count.
    """
    gpu_idx = np.asarray(gpu_idx)
    ref_idx = np.argmax(ref_map, axis=1)
    same = gpu_idx == ref_idx
    for f in np.nonzero(~same)[0]:
        bound = 2.0 * rel_tol * np.linalg.norm(ref_map[f])
        gap = ref_map[f, ref_idx[f]] - ref_map[f, gpu_idx[f]]
        assert gap <= bound, (f, gap, bound)
    if same.size >= 100:
        assert same.mean() >= frac, same.mean()
    return int(same.sum())
