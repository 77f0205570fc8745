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


# (label, identical frames, frames) of every argmax comparison of the session;
# tests/conftest.py writes them out at the end of a GPU run
ARGMAX_LOG = []


def check_argmax(gpu_idx, ref_map, rel_tol, frac=0.99, label="", gate_min_frames=1):
    """Argmax agreement with the reference map (Section 2.2: the estimate is the argmax).

    A frame whose argmax differs must be a near-tie that the map tolerance
    allows: if ||gpu - ref||_2 <= rel_tol ||ref||_2, the GPU's pick can trail
    the reference maximum by at most 2 rel_tol ||ref||_2. With at least
    `gate_min_frames` frames, at least `frac` of them must be identical (for
    fewer than 100 frames that means all of them). The fraction is recorded
    under `label` either way. Returns the identical fraction.
    """
    gpu_idx = np.asarray(gpu_idx)
    ref_idx = np.argmax(ref_map, axis=1)
    same = gpu_idx == ref_idx
    ARGMAX_LOG.append((label, int(same.sum()), int(same.size)))
    for f in np.nonzero(~same)[0]:
        bound = 2.0 * rel_tol * np.linalg.norm(ref_map[f])
        gap = ref_map[f, ref_idx[f]] - ref_map[f, gpu_idx[f]]
        assert gap <= bound, (label, f, gap, bound)
    if same.size >= gate_min_frames:
        assert same.sum() >= np.ceil(frac * same.size - 1e-9), (label, same.mean())
    return float(same.mean())


def sample_columns(g):
    """Columns of the library's sample layout that hold samples (window order)."""
    return np.concatenate([np.arange(int(o), int(o) + int(w))
                           for o, w in zip(g.offsets[:-1], g.W)])


def rounded(values, torch_dtype):
    """float64 values rounded once to a storage type and widened back (host)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(values)).to(torch_dtype).to(
        torch.float64).numpy()


def device_samples(g, xi_dense, torch_dtype, device="cuda"):
    """The oracle's GCC samples [F][sum_p W_p] (pair-major, no gaps) placed into the
    library's sample layout [F][S] (zeros in the alignment gaps), rounded once to
    the storage type and copied to the device. Returns (device tensor, the rounded
    dense values as float64), so that the oracle and the kernel read the very same
    numbers and the inputs of both come from the oracle."""
    import torch
    xr = rounded(xi_dense, torch_dtype)
    full = np.zeros((xr.shape[0], g.S))
    full[:, sample_columns(g)] = xr
    return torch.from_numpy(full).to(torch_dtype).to(device), xr


def device_psi(psi, device="cuda"):
    """The oracle's cross-spectra rounded once to complex64 and copied to the device.
    Returns (device tensor, the rounded values as complex128)."""
    import torch
    p64 = np.ascontiguousarray(psi).astype(np.complex64)
    return torch.from_numpy(p64).to(device), p64.astype(np.complex128)


def oracle_nyquist_parallel(wl, xi, idx=None, workers=None, chunk=4096):
    """The oracle's Nyquist map at candidates `idx` (all if None), [F][n] float64.

    The candidates are independent (Eq. SRPapprox per candidate), so the oracle
    runs on chunks of them in threads, each with one BLAS thread; the result is
    the oracle's own, column block by column block.
    """
    import concurrent.futures as cf
    import os
    n = wl.J if idx is None else len(idx)
    workers = workers or min(16, os.cpu_count() or 1)
    out = np.empty((xi.shape[0], n))

    def run(j0):
        j1 = min(n, j0 + chunk)
        cand = wl.candidates(j0, j1) if idx is None else wl.candidates_at(idx[j0:j1])
        out[:, j0:j1] = oracle_nyquist(wl, xi, cand)
        return j0

    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(1)
    except ImportError:
        limit = None
    try:
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(run, range(0, n, chunk)))
    finally:
        if limit is not None:
            limit.restore_original_limits()
    return out
