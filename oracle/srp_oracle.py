"""FP64 oracle: conventional SRP-PHAT and the Nyquist-Shannon SRP approximation.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain NumPy, float64.

Conventions (each one is the reading this oracle takes of the paper):
* microphones are 0-based; pair p = m(m-1)/2 + m' for m > m' (Section 2.1,
  the pair set with m > m');
* band limit f_max = omega_0 / 2 pi, critical period T = 1 / (2 f_max)
  (Section 3.1);
* frequency bins f_k = k fs / L for k = 0 .. K-1 with K = floor(f_max L / fs) + 1;
  bin weight w_k = 1 at k = 0 and at f_k = fs / 2, otherwise 2. This is the
  one-sided discrete form of the integral over [-omega_0, omega_0] for a
  conjugate-symmetric spectrum (Eq. SRP_T and the remark after Eq. SRP_T_IFT);
* discrete GCC xi_p(tau) = sum_k w_k Re[psi_p(k) exp(j 2 pi f_k tau)], with no
  1/(2 pi) or bin-width factor (Eq. GCC_IFT with the integral replaced by a
  sum, Section 2.4);
* SRP(i) = 2 sum_p xi_p(dt_p(i)) (Eq. SRP_T_IFT);
* the truncated interpolation runs over n = -(N_p + N_aux) .. N_p + N_aux, the
  symmetric window that gives the 2 N_p + 2 N_aux + 1 samples counted in
  Section 3.3 (the printed lower limit of Eq. SRPapprox is read as a typo);
* sinc(x) = sin(pi x) / (pi x) with sinc(0) = 1 (numpy.sinc), the normalised
  kernel that Whittaker-Shannon interpolation with period T requires;
* PHAT weight 1 / |y_m y_m'^*| with psi = 0 where that magnitude is zero;
* argmax ties go to the lowest candidate index.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

__all__ = [
    "pair_list", "critical_period", "n_bins", "bin_weights", "window", "pair_windows",
    "spectra", "phat_cross_spectra", "gcc_matrix", "tdoa", "gcc", "srp_conventional",
    "srp_beamformer", "gcc_samples", "srp_nyquist", "peaks", "rel_error", "e_appr_db",
    "complexity",
]


# ---------------------------------------------------------------- geometry

def pair_list(M: int):
    """Microphone pairs (m, m') with m > m', in pair-index order (Section 2.1).

    P = M(M-1)/2 pairs; pair p = m(m-1)/2 + m'.
    """
    return [(m, mp) for m in range(1, M) for mp in range(m)]


def critical_period(f_max: float) -> float:
    """T = pi / omega_0 with omega_0 = 2 pi f_max (Section 3.1)."""
    return 1.0 / (2.0 * f_max)


def n_bins(L: int, fs: float, f_max: Optional[float] = None) -> int:
    """Number of one-sided bins with f_k = k fs / L <= f_max."""
    f_max = fs / 2.0 if f_max is None else f_max
    return int(math.floor(f_max * L / fs)) + 1


def bin_weights(L: int, K: int) -> np.ndarray:
    """One-sided weights: 1 at DC and at the Nyquist bin 2k = L, else 2 (Eq. SRP_T)."""
    w = np.full(K, 2.0)
    w[0] = 1.0
    if 2 * (K - 1) == L:
        w[K - 1] = 1.0
    return w


def window(L: int, kind: str = "hann") -> np.ndarray:
    """Analysis window: periodic Hann, square-root periodic Hann, or rectangular."""
    t = np.arange(L, dtype=np.float64)
    hann = 0.5 - 0.5 * np.cos(2.0 * np.pi * t / L)
    if kind == "hann":
        return hann
    if kind == "sqrt_hann":
        return np.sqrt(hann)
    if kind == "rect":
        return np.ones(L)
    raise ValueError(kind)


def pair_windows(mic_xyz, c: float, f_max: float, n_aux: int):
    """Per-pair sample windows of the truncated interpolation (Section 3.2, 3.3).

    d_p = ||p_m - p_m'||, N_p = floor(dt_{p|0} / T) with dt_{p|0} = d_p / c,
    evaluated as floor(d_p / (c * T)); the window holds W_p = 2 N_p + 2 N_aux + 1
    lags n = -(N_p + N_aux) .. N_p + N_aux. `offsets` packs the windows
    pair-major (offsets[p] .. offsets[p+1]-1), S = offsets[P].
    """
    mic = np.asarray(mic_xyz, dtype=np.float64)
    T = critical_period(f_max)
    pairs = pair_list(mic.shape[0])
    def dist(a, b):
        # x, y, z summed in that order in float64, so floor() resolves an exact
        # tie the same way wherever this reading is implemented
        dx, dy, dz = float(a[0] - b[0]), float(a[1] - b[1]), float(a[2] - b[2])
        return math.sqrt(dx * dx + dy * dy + dz * dz)

    d = np.array([dist(mic[m], mic[mp]) for m, mp in pairs])
    N = np.array([int(math.floor(dp / (c * T))) for dp in d], dtype=np.int64)
    W = 2 * N + 2 * n_aux + 1
    offsets = np.zeros(len(pairs) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(W)
    return {"pairs": pairs, "d": d, "N": N, "W": W, "offsets": offsets,
            "S": int(offsets[-1]), "T": T, "n_aux": int(n_aux)}


# ---------------------------------------------------------------- spectra

def spectra(frames, win, K: int, literal: bool = False) -> np.ndarray:
    """Y[f][m][k] = sum_t win[t] y[f][m][t] exp(-j 2 pi k t / L), k < K (Section 2.1).

    `literal` evaluates the DFT as an explicit O(L^2) sum (tiny L only).
    """
    y = np.asarray(frames, dtype=np.float64) * np.asarray(win, dtype=np.float64)
    L = y.shape[-1]
    if literal:
        t = np.arange(L)
        k = np.arange(K)
        E = np.exp(-2j * np.pi * np.outer(t, k) / L)
        return y @ E
    return np.fft.rfft(y, axis=-1)[..., :K]


def phat_cross_spectra(Y) -> np.ndarray:
    """psi[f][p][k] = y_m y_m'^* / |y_m y_m'^*| (Eq. corrmatrix, PHAT weighting).

    Zero where |y_m y_m'^*| = 0.
    """
    Y = np.asarray(Y)
    M = Y.shape[1]
    out = np.empty((Y.shape[0], M * (M - 1) // 2, Y.shape[2]), dtype=np.complex128)
    for p, (m, mp) in enumerate(pair_list(M)):
        num = Y[:, m, :] * np.conj(Y[:, mp, :])
        den = np.abs(num)
        safe = np.where(den > 0.0, den, 1.0)
        out[:, p, :] = np.where(den > 0.0, num / safe, 0.0)
    return out


def gcc_matrix(Y) -> np.ndarray:
    """Full PHAT GCC matrix Psi[f][k][m][m'] of Eq. corrmatrix (all m, m')."""
    Y = np.asarray(Y)
    num = Y[:, :, None, :] * np.conj(Y[:, None, :, :])  # [F][M][M][K]
    den = np.abs(num)
    safe = np.where(den > 0.0, den, 1.0)
    psi = np.where(den > 0.0, num / safe, 0.0)
    return np.transpose(psi, (0, 3, 1, 2))


# ---------------------------------------------------------------- TDOA

def tdoa(mic_xyz, cand, c: float, field: str = "near") -> np.ndarray:
    """dt[i][p] in seconds for every candidate i and pair p.

    near: (||p_m - q_i|| - ||p_m' - q_i||) / c (Eq. Deltat_i);
    far:  (p_m - p_m')^T r_i / c, r_i a unit incident direction (Eq. Deltat_i_spher).
    """
    mic = np.asarray(mic_xyz, dtype=np.float64)
    q = np.asarray(cand, dtype=np.float64).reshape(-1, 3)
    pairs = pair_list(mic.shape[0])
    mi = np.array([a for a, _ in pairs], dtype=np.int64)
    mj = np.array([b for _, b in pairs], dtype=np.int64)
    if field == "near":
        r = np.sqrt(((q[:, None, :] - mic[None, :, :]) ** 2).sum(axis=2))  # [J][M]
        return (r[:, mi] - r[:, mj]) / c
    if field == "far":
        proj = q @ mic.T  # [J][M] = p_m . r_i
        return (proj[:, mi] - proj[:, mj]) / c
    raise ValueError(field)


# ---------------------------------------------------------------- GCC and SRP

def gcc(psi, tau, fs: float, L: int, w) -> np.ndarray:
    """Discrete GCC xi_p(tau) = sum_k w_k Re[psi_p(k) exp(j 2 pi f_k tau)] (Eq. GCC_IFT).

    psi: [F][P][K]; tau: [n][P] seconds (one lag per pair per row).
    Returns [F][n][P].
    """
    psi = np.asarray(psi)
    tau = np.asarray(tau, dtype=np.float64)
    F, P, K = psi.shape
    fk = np.arange(K) * (fs / L)
    out = np.empty((F, tau.shape[0], P))
    wpsi = psi * np.asarray(w)[None, None, :]
    for p in range(P):
        E = np.exp(2j * np.pi * np.outer(tau[:, p], fk))  # [n][K]
        out[:, :, p] = (E @ wpsi[:, p, :].T).real.T
    return out


def _chunk_rows(row_bytes: int, budget: int = 1 << 27) -> int:
    return max(1, budget // max(1, row_bytes))


def srp_conventional(psi, dt, fs: float, L: int, w) -> np.ndarray:
    """Conventional SRP map SRP(i) = 2 sum_p xi_p(dt_p(i)) (Eq. SRP_T_IFT, Section 2.4).

    One discrete IFT evaluation per candidate, pair and bin (J P K complex
    products). dt: [J][P] seconds. Returns [F][J].
    """
    psi = np.asarray(psi)
    dt = np.asarray(dt, dtype=np.float64)
    F, P, K = psi.shape
    J = dt.shape[0]
    out = np.zeros((F, J))
    step = _chunk_rows(16 * K * P)
    for j0 in range(0, J, step):
        j1 = min(J, j0 + step)
        out[:, j0:j1] = 2.0 * gcc(psi, dt[j0:j1], fs, L, w).sum(axis=2)
    return out


def srp_beamformer(Y, mic_xyz, cand, c: float, fs: float, L: int, w,
                   field: str = "near") -> np.ndarray:
    """SRP as delay-and-sum beamformer output power (Eq. h_steering, SRP_omegaT, SRP_T).

    SRP(i) = sum_k w_k (h^H Psi(k) h - tr Psi(k)) with
    h_m = exp(-j omega_k dt_{m,1}(i)) steered relative to the first microphone.
    Small inputs only (forms the full M x M matrix per bin).
    """
    Y = np.asarray(Y)
    F, M, K = Y.shape
    mic = np.asarray(mic_xyz, dtype=np.float64)
    q = np.asarray(cand, dtype=np.float64).reshape(-1, 3)
    if field == "near":
        r = np.sqrt(((q[:, None, :] - mic[None, :, :]) ** 2).sum(axis=2))
        dt_m1 = (r - r[:, :1]) / c  # [J][M]
    else:
        proj = q @ mic.T
        dt_m1 = (proj - proj[:, :1]) / c
    Psi = gcc_matrix(Y)  # [F][K][M][M]
    omega = 2.0 * np.pi * np.arange(K) * (fs / L)
    h = np.exp(-1j * omega[None, :, None] * dt_m1[:, None, :])  # [J][K][M]
    quad = np.einsum("jkm,fkmn,jkn->fjk", np.conj(h), Psi, h).real
    tr = np.einsum("fkmm->fk", Psi).real
    return ((quad - tr[:, None, :]) * np.asarray(w)[None, None, :]).sum(axis=2)


def gcc_samples(psi, fs: float, L: int, w, win: dict) -> np.ndarray:
    """GCC samples xi_p(nT) for n in each pair's window (Section 3.2, first step).

    Returns [F][S], pair-major, lags ascending, laid out by win["offsets"].
    """
    psi = np.asarray(psi)
    F, P, _ = psi.shape
    T = win["T"]
    out = np.empty((F, win["S"]))
    for p in range(P):
        h = int(win["N"][p]) + win["n_aux"]
        n = np.arange(-h, h + 1)
        o = int(win["offsets"][p])
        fk = np.arange(psi.shape[2]) * (fs / L)
        E = np.exp(2j * np.pi * np.outer(n * T, fk))  # [W_p][K]
        out[:, o:o + n.size] = (E @ (psi[:, p, :] * np.asarray(w)[None, :]).T).real.T
    return out


def srp_nyquist(xi, dt, win: dict, kernel=np.sinc) -> np.ndarray:
    """Nyquist-Shannon SRP approximation (Eq. SRPapprox summed with Eq. SRP_T_IFT).

    SRP_appr(i) = 2 sum_p sum_{|n| <= N_p + N_aux} xi_p(nT) sinc(dt_p(i)/T - n).
    The weights do not depend on the frame, so they are formed per block of
    candidates [J_b][S] and contracted with the samples [S][F] (Section 3.3
    notes they can be precomputed). `kernel` replaces sinc only in tests that
    check the sample and window bookkeeping against a kernel with a known
    exact result. Returns [F][J].
    """
    xi = np.asarray(xi, dtype=np.float64)
    dt = np.asarray(dt, dtype=np.float64)
    F, S = xi.shape
    J, P = dt.shape
    T = win["T"]
    x = dt / T  # [J][P]
    lag = np.empty(S)
    pair_of = np.empty(S, dtype=np.int64)
    for p in range(P):
        h = int(win["N"][p]) + win["n_aux"]
        o = int(win["offsets"][p])
        lag[o:o + 2 * h + 1] = np.arange(-h, h + 1)
        pair_of[o:o + 2 * h + 1] = p
    out = np.empty((F, J))
    step = _chunk_rows(8 * S)
    for j0 in range(0, J, step):
        j1 = min(J, j0 + step)
        W = kernel(x[j0:j1][:, pair_of] - lag[None, :])  # [J_b][S]
        out[:, j0:j1] = 2.0 * (W @ xi.T).T
    return out


def peaks(srp_map):
    """Per-frame argmax over candidates (Section 2.2), lowest index on ties."""
    m = np.asarray(srp_map)
    idx = np.argmax(m, axis=1)
    return idx, m[np.arange(m.shape[0]), idx]


def rel_error(a, b) -> np.ndarray:
    """Per-frame relative L2 error ||a - b|| / ||b|| over candidates."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.sqrt(((a - b) ** 2).sum(axis=-1))
    den = np.sqrt((b ** 2).sum(axis=-1))
    return num / np.where(den > 0, den, 1.0)


def e_appr_db(srp_appr, srp) -> np.ndarray:
    """Approximation error 10 log10(sum (SRP - SRP_appr)^2 / sum SRP^2) per frame (Section 4)."""
    a = np.asarray(srp_appr, dtype=np.float64)
    b = np.asarray(srp, dtype=np.float64)
    return 10.0 * np.log10(((b - a) ** 2).sum(axis=-1) / (b ** 2).sum(axis=-1))


def complexity(N_p, n_aux: int, J: int, K: int) -> dict:
    """Operation counts of Sections 2.4 and 3.3.

    N = (2/P) sum_p N_p + 2 N_aux + 1; C_conv = J P K; C_samp = N P K;
    C_int = N P J; R_samp = N / J; R_int = N / K; R = R_samp + R_int.
    """
    N_p = np.asarray(N_p, dtype=np.float64)
    P = N_p.size
    N = 2.0 / P * N_p.sum() + 2 * n_aux + 1
    c_conv = float(J) * P * K
    c_samp = N * P * K
    c_int = N * P * J
    return {"P": P, "N": N, "C_conv": c_conv, "C_samp": c_samp, "C_int": c_int,
            "R_samp": N / J, "R_int": N / K, "R": N / J + N / K}
