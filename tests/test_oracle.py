"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numbers the
paper prints for its worked example, closed forms, identities between two of
the paper's own forms, library routines for special cases, and literal brute
force on tiny inputs.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as WL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper_setup():
    with open(os.path.join(GOLDEN, "paper_worked_example.json")) as f:
        return json.load(f)


# ------------------------------------------------------------ geometry / counts

def test_worked_example_counts():
    """P = 15 and N = 14.2 + 2 N_aux for the paper's 6-mic UCA (Section 3.3, Section 4)."""
    g = _paper_setup()
    s = g["setup"]
    mic = WL.uniform_circular_array(s["M"], s["radius_m"])
    for n_aux in range(5):
        win = O.pair_windows(mic, s["c"], s["f_max_hz"], n_aux)
        cx = O.complexity(win["N"], n_aux, s["J"], s["K"])
        assert cx["P"] == g["printed"]["P"]["value"]
        assert abs(cx["N"] - 2 * n_aux - g["printed"]["N_minus_2_n_aux"]["value"]) \
            <= g["printed"]["N_minus_2_n_aux"]["abs_tol"]
        # the exact value implied by the hexagon distances r, r*sqrt(3), 2r
        assert sorted(win["N"].tolist()) == [4] * 6 + [8] * 6 + [9] * 3
        assert win["S"] == sum(2 * n + 2 * n_aux + 1 for n in win["N"])


def test_worked_example_complexity_printed():
    """C_conv, C_samp, C_int, R_samp, R_int as printed in Section 4 (N_aux = 2)."""
    g = _paper_setup()
    s = g["setup"]
    mic = WL.uniform_circular_array(s["M"], s["radius_m"])
    win = O.pair_windows(mic, s["c"], s["f_max_hz"], s["n_aux"])
    cx = O.complexity(win["N"], s["n_aux"], s["J"], s["K"])
    for key in ("C_conv", "C_samp", "C_int", "R_samp", "R_int"):
        pr = g["printed"][key]
        assert abs(cx[key] - pr["value"]) <= pr["abs_tol"], (key, cx[key], pr["value"])
    assert cx["C_conv"] == 124_431_360
    assert cx["R"] == pytest.approx(cx["R_samp"] + cx["R_int"])


def test_half_sphere_grid_size():
    """The 2-degree lower half-sphere grid has J = 8101 directions (Section 4)."""
    d = WL.half_sphere_directions(2.0)
    assert d.shape == (_paper_setup()["printed"]["J"]["value"], 3)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    assert np.all(d[:, 2] >= -1e-15)  # r = -(.., .., cos theta), theta in [90, 180]
    # no duplicate directions
    assert np.unique(np.round(d, 12), axis=0).shape[0] == d.shape[0]


def test_pair_order_and_count():
    for M in (2, 3, 6, 16):
        pl = O.pair_list(M)
        assert len(pl) == M * (M - 1) // 2
        for p, (m, mp) in enumerate(pl):
            assert m > mp and p == m * (m - 1) // 2 + mp


def test_tdoa_bounded_by_pair_distance():
    """|dt_p(i)| <= d_p / c for near and far field (Eq. Deltat_i_range)."""
    rng = np.random.default_rng(0)
    mic = rng.random((7, 3))
    cand = rng.random((500, 3)) * 5 - 2
    win = O.pair_windows(mic, 343.0, 8000.0, 0)
    dt = O.tdoa(mic, cand, 343.0)
    assert np.all(np.abs(dt) <= win["d"][None, :] / 343.0 + 1e-15)
    dirs = WL.half_sphere_directions(10.0)
    dtf = O.tdoa(mic, dirs, 343.0, field="far")
    assert np.all(np.abs(dtf) <= win["d"][None, :] / 343.0 + 1e-15)
    # the interval limits are reached on the line through both mics
    m, mp = O.pair_list(7)[4]
    q = mic[m] + 2.0 * (mic[m] - mic[mp])
    assert O.tdoa(mic, q[None], 343.0)[0, 4] == pytest.approx(-win["d"][4] / 343.0, rel=1e-12)


# ------------------------------------------------------------ spectra, PHAT, GCC

def test_spectra_rfft_equals_literal_dft():
    rng = np.random.default_rng(1)
    y = rng.standard_normal((2, 3, 64))
    win = O.window(64, "hann")
    K = O.n_bins(64, 16000.0)
    np.testing.assert_allclose(O.spectra(y, win, K), O.spectra(y, win, K, literal=True),
                               atol=1e-12)


def test_window_values():
    w = O.window(8, "hann")
    np.testing.assert_allclose(w, [0, 0.1464466094067262, 0.5, 0.8535533905932737, 1,
                                   0.8535533905932737, 0.5, 0.1464466094067262], atol=1e-15)
    np.testing.assert_allclose(O.window(8, "sqrt_hann") ** 2, w, atol=1e-15)


def test_bin_weights():
    np.testing.assert_array_equal(O.bin_weights(8, 5), [1, 2, 2, 2, 1])
    np.testing.assert_array_equal(O.bin_weights(9, 5), [1, 2, 2, 2, 2])   # odd L: no Nyquist bin
    np.testing.assert_array_equal(O.bin_weights(16, 5), [1, 2, 2, 2, 2])  # band-limited below fs/2
    assert O.n_bins(1024, 16000.0) == 513
    assert O.n_bins(2048, 16000.0, 4000.0) == 513


def _delayed_pair(L, D, seed=3):
    rng = np.random.default_rng(seed)
    y0 = rng.standard_normal(L)
    y1 = np.roll(y0, D)  # y1[t] = y0[t - D]: mic 1 hears the wave D samples later
    return np.stack([y0, y1])[None]  # [1][2][L]


@pytest.mark.parametrize("D", [0, 3, -5, 17])
def test_gcc_phat_peak_at_integer_delay(D):
    """Circular delay D with a rectangular window: psi = exp(-j2pi kD/L), xi(n) = L delta[n-D]."""
    L = 64
    y = _delayed_pair(L, D)
    K = O.n_bins(L, 16000.0)
    Y = O.spectra(y, O.window(L, "rect"), K)
    psi = O.phat_cross_spectra(Y)  # pair 0 = (m=1, m'=0)
    k = np.arange(K)
    np.testing.assert_allclose(psi[0, 0], np.exp(-2j * np.pi * k * D / L), atol=1e-12)
    w = O.bin_weights(L, K)
    lags = np.arange(-L // 2 + 1, L // 2 + 1)
    xi = O.gcc(psi, (lags / 16000.0)[:, None], 16000.0, L, w)[0, :, 0]
    expect = np.where((lags - D) % L == 0, float(L), 0.0)
    np.testing.assert_allclose(xi, expect, atol=1e-9)


def test_gcc_integer_lags_equal_scaled_irfft():
    """At f_max = fs/2 and tau = n/fs, xi_p(n) = L irfft(psi_p)[n mod L]."""
    rng = np.random.default_rng(2)
    L = 128
    y = rng.standard_normal((2, 4, L))
    K = O.n_bins(L, 16000.0)
    psi = O.phat_cross_spectra(O.spectra(y, O.window(L), K))
    w = O.bin_weights(L, K)
    n = np.arange(-10, 11)
    xi = O.gcc(psi, np.repeat((n / 16000.0)[:, None], psi.shape[1], 1), 16000.0, L, w)
    ref = L * np.fft.irfft(psi, L, axis=-1)[:, :, n % L]  # [F][P][n]
    np.testing.assert_allclose(xi, np.transpose(ref, (0, 2, 1)), atol=1e-9)


@pytest.mark.parametrize("u", [0.3, -7.25, 100.5, 1e-9])
def test_gcc_pure_delay_dirichlet_closed_form(u):
    """Pure delay D: xi(tau) = sin(pi u) cot(pi u / L), u = tau fs - D."""
    L, D, fs = 256, 9, 16000.0
    y = _delayed_pair(L, D)
    K = O.n_bins(L, fs)
    psi = O.phat_cross_spectra(O.spectra(y, O.window(L, "rect"), K))
    tau = (u + D) / fs
    xi = O.gcc(psi, np.array([[tau]]), fs, L, O.bin_weights(L, K))[0, 0, 0]
    assert xi == pytest.approx(math.sin(math.pi * u) / math.tan(math.pi * u / L), rel=1e-9,
                               abs=1e-9)


# ------------------------------------------------------------ SRP forms

def _tiny_scene(M=4, L=64, F=2, J_shape=(4, 3, 2), seed=5):
    wl = WL.make_custom(M=M, J_shape=J_shape, h=0.25, L=L, F=F, seed=seed, snr_db=10.0)
    K = O.n_bins(wl.L, wl.fs)
    Y = O.spectra(wl.frames, O.window(wl.L), K)
    psi = O.phat_cross_spectra(Y)
    return wl, K, Y, psi


@pytest.mark.parametrize("field", ["near", "far"])
def test_beamformer_form_equals_pairwise_form(field):
    """h^H Psi h - tr Psi summed over bins equals 2 sum_p xi_p(dt_p) (Eq. SRP_omegaT, SRP_T_IFT)."""
    wl, K, Y, psi = _tiny_scene()
    w = O.bin_weights(wl.L, K)
    cand = wl.candidates() if field == "near" else WL.half_sphere_directions(30.0)
    bf = O.srp_beamformer(Y, wl.mic_xyz, cand, wl.c, wl.fs, wl.L, w, field=field)
    dt = O.tdoa(wl.mic_xyz, cand, wl.c, field=field)
    pw = O.srp_conventional(psi, dt, wl.fs, wl.L, w)
    np.testing.assert_allclose(pw, bf, rtol=1e-12, atol=1e-10 * np.abs(bf).max())


def test_conventional_brute_force_loops():
    """Literal loops over candidates, pairs and bins (M = 3, L = 64)."""
    wl, K, Y, psi = _tiny_scene(M=3, L=64, F=2, J_shape=(5, 4, 2))
    w = O.bin_weights(wl.L, K)
    cand = wl.candidates()
    ref = np.zeros((wl.F, cand.shape[0]))
    for f in range(wl.F):
        for i in range(cand.shape[0]):
            acc = 0.0
            for m in range(1, 3):
                for mp in range(m):
                    p = m * (m - 1) // 2 + mp
                    dt = (math.dist(wl.mic_xyz[m], cand[i]) - math.dist(wl.mic_xyz[mp], cand[i])) / wl.c
                    for k in range(K):
                        ph = 2.0 * math.pi * (k * wl.fs / wl.L) * dt
                        z = psi[f, p, k]
                        acc += w[k] * (z.real * math.cos(ph) - z.imag * math.sin(ph))
            ref[f, i] = 2.0 * acc
    got = O.srp_conventional(psi, O.tdoa(wl.mic_xyz, cand, wl.c), wl.fs, wl.L, w)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-9)


def test_nyquist_brute_force_loops():
    """Literal loops with sinc = sin(pi x)/(pi x) over each pair's symmetric window."""
    wl, K, Y, psi = _tiny_scene(M=3, L=64, F=2, J_shape=(5, 4, 2))
    w = O.bin_weights(wl.L, K)
    n_aux = 2
    win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, n_aux)
    xi = O.gcc_samples(psi, wl.fs, wl.L, w, win)
    cand = wl.candidates()
    T = 1.0 / wl.fs
    ref = np.zeros((wl.F, cand.shape[0]))
    for f in range(wl.F):
        for i in range(cand.shape[0]):
            acc = 0.0
            for m in range(1, 3):
                for mp in range(m):
                    p = m * (m - 1) // 2 + mp
                    Np = math.floor(math.dist(wl.mic_xyz[m], wl.mic_xyz[mp]) / (wl.c * T))
                    x = (math.dist(wl.mic_xyz[m], cand[i]) - math.dist(wl.mic_xyz[mp], cand[i])) / wl.c / T
                    for n in range(-(Np + n_aux), Np + n_aux + 1):
                        # sample xi_p(nT) straight from its definition
                        s = 0.0
                        for k in range(K):
                            ph = 2.0 * math.pi * (k * wl.fs / wl.L) * n * T
                            z = psi[f, p, k]
                            s += w[k] * (z.real * math.cos(ph) - z.imag * math.sin(ph))
                        a = x - n
                        sinc = 1.0 if a == 0.0 else math.sin(math.pi * a) / (math.pi * a)
                        acc += s * sinc
            ref[f, i] = 2.0 * acc
    got = O.srp_nyquist(xi, O.tdoa(wl.mic_xyz, cand, wl.c), win)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-8)


def test_nyquist_with_dirichlet_kernel_reproduces_conventional():
    """Bookkeeping check: all L lags + the periodic (Dirichlet) kernel = conventional exactly.

    For odd L and f_max = fs/2, xi is a trigonometric polynomial of degree
    (L-1)/2 that L equispaced samples determine, interpolated exactly by
    D(u) = sin(pi u) / (L sin(pi u / L)). The symmetric window of every pair
    is widened to all L lags. Any slip in sample offsets, lag order, the
    dt/T scaling or the factor 2 breaks the equality.
    """
    L = 63
    wl = WL.make_custom(M=4, J_shape=(4, 3, 2), h=0.25, L=L, F=2, seed=8)
    K = O.n_bins(L, wl.fs)
    assert K == 32
    psi = O.phat_cross_spectra(O.spectra(wl.frames, O.window(L), K))
    w = O.bin_weights(L, K)
    win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, 0)
    h = (L - 1) // 2
    win["N"] = np.full_like(win["N"], h)
    win["W"] = 2 * win["N"] + 1
    win["offsets"] = np.concatenate([[0], np.cumsum(win["W"])])
    win["S"] = int(win["offsets"][-1])

    def dirichlet(u):
        s = np.sin(np.pi * u / L)
        safe = np.where(np.abs(s) < 1e-300, 1.0, s)
        return np.where(np.abs(s) < 1e-300, 1.0, np.sin(np.pi * u) / (L * safe))

    xi = O.gcc_samples(psi, wl.fs, L, w, win)
    dt = O.tdoa(wl.mic_xyz, wl.candidates(), wl.c)
    ny = O.srp_nyquist(xi, dt, win, kernel=dirichlet)
    conv = O.srp_conventional(psi, dt, wl.fs, L, w)
    np.testing.assert_allclose(ny, conv, rtol=1e-10, atol=1e-9 * np.abs(conv).max())


def test_nyquist_exact_at_integer_tdoa():
    """sinc(x - n) = delta at integer x: SRP_appr = SRP where every x_p(i) is an integer.

    Two mics 10 samples apart on the x axis; candidates on that axis beyond
    the pair give x = +/-10 and between them give integer x for cells at
    half-integer sample spacing.
    """
    fs, c, L = 16000.0, 343.0, 128
    d = 10 * c / fs
    mic = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    # x_p = (|q - p1| - |q - p0|) / (c T); for q = (a, 0, 0) between mics: x = (d - 2a) fs / c
    a = np.array([-1.0, 2.0 * d, 0.5 * d - 3 * c / (2 * fs), 0.5 * d + 4 * c / (2 * fs)])
    cand = np.stack([a, np.zeros_like(a), np.zeros_like(a)], axis=1)
    rng = np.random.default_rng(4)
    y = rng.standard_normal((3, 2, L))
    K = O.n_bins(L, fs)
    psi = O.phat_cross_spectra(O.spectra(y, O.window(L), K))
    w = O.bin_weights(L, K)
    dt = O.tdoa(mic, cand, c)
    x = dt * fs
    np.testing.assert_allclose(x[:, 0], np.round(x[:, 0]), atol=1e-9)
    for n_aux in (0, 1, 2):
        win = O.pair_windows(mic, c, fs / 2, n_aux)
        ny = O.srp_nyquist(O.gcc_samples(psi, fs, L, w, win), dt, win)
        conv = O.srp_conventional(psi, dt, fs, L, w)
        inside = np.abs(np.round(x[:, 0])) <= win["N"][0] + n_aux
        np.testing.assert_allclose(ny[:, inside], conv[:, inside], rtol=1e-7, atol=1e-6)


def test_nyquist_pure_delay_closed_form():
    """Pure delay D inside the window: xi_appr(tau) = L sinc(tau fs - D)."""
    fs, c, L, D = 16000.0, 343.0, 256, 4
    d = 12 * c / fs  # N_p = 12 (floor may give 11 at a rounding tie; D stays inside)
    mic = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    y = _delayed_pair(L, D)
    K = O.n_bins(L, fs)
    psi = O.phat_cross_spectra(O.spectra(y, O.window(L, "rect"), K))
    w = O.bin_weights(L, K)
    win = O.pair_windows(mic, c, fs / 2, 2)
    xi = O.gcc_samples(psi, fs, L, w, win)
    rng = np.random.default_rng(9)
    cand = np.column_stack([rng.uniform(-0.3, 0.6, 40), rng.uniform(-0.5, 0.5, 40),
                            rng.uniform(-0.5, 0.5, 40)])
    dt = O.tdoa(mic, cand, c)
    ny = O.srp_nyquist(xi, dt, win)
    expect = 2.0 * L * np.sinc(dt[:, 0] * fs - D)
    np.testing.assert_allclose(ny[0], expect, rtol=1e-9, atol=1e-9)


def test_approximation_error_shrinks_with_n_aux_and_peaks_agree():
    """e_appr on the 4-mic scene falls from N_aux = 0 to 2 (sanity band, Section 4)."""
    wl = WL.make(1, F=4)
    K = O.n_bins(wl.L, wl.fs)
    psi = O.phat_cross_spectra(O.spectra(wl.frames, O.window(wl.L), K))
    w = O.bin_weights(wl.L, K)
    cand = wl.candidates()
    dt = O.tdoa(wl.mic_xyz, cand, wl.c)
    conv = O.srp_conventional(psi, dt, wl.fs, wl.L, w)
    errs = []
    for n_aux in (0, 2, 4):
        win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, n_aux)
        ny = O.srp_nyquist(O.gcc_samples(psi, wl.fs, wl.L, w, win), dt, win)
        errs.append(np.median(O.e_appr_db(ny, conv)))
    assert errs[0] < -10.0
    assert errs[1] <= errs[0] + 0.5
    assert errs[2] <= errs[1] + 0.5
    # at N_aux = 2 the argmax matches conventional SRP and sits next to the source
    idx_c, _ = O.peaks(conv)
    idx_n, _ = O.peaks(ny)
    src_cell = wl.grid.index_of(wl.sources[0])
    pts = wl.candidates()
    for f in range(wl.F):
        assert np.linalg.norm(pts[idx_c[f]] - wl.sources[0]) <= 1.5 * wl.grid.h * math.sqrt(2)
        assert np.linalg.norm(pts[idx_n[f]] - pts[src_cell]) <= 1.5 * wl.grid.h * math.sqrt(2)


def test_all_zero_frames_give_zero_map():
    wl = WL.make_custom(M=3, J_shape=(3, 3, 2), L=64, F=2)
    y = np.zeros_like(wl.frames)
    K = O.n_bins(64, wl.fs)
    psi = O.phat_cross_spectra(O.spectra(y, O.window(64), K))
    assert np.all(psi == 0)
    w = O.bin_weights(64, K)
    win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, 2)
    dt = O.tdoa(wl.mic_xyz, wl.candidates(), wl.c)
    ny = O.srp_nyquist(O.gcc_samples(psi, wl.fs, 64, w, win), dt, win)
    assert np.all(ny == 0)
    idx, val = O.peaks(ny)
    assert np.all(idx == 0) and np.all(val == 0)


def test_peaks_lowest_index_on_ties_and_brute_force():
    m = np.array([[1.0, 3.0, 3.0, 2.0], [5.0, 5.0, 5.0, 5.0], [-1.0, -3.0, -0.5, -0.5]])
    idx, val = O.peaks(m)
    assert idx.tolist() == [1, 0, 2] and val.tolist() == [3.0, 5.0, -0.5]
    rng = np.random.default_rng(0)
    r = rng.standard_normal((5, 100))
    for f in range(5):
        best = 0
        for i in range(100):
            if r[f, i] > r[f, best]:
                best = i
        assert O.peaks(r)[0][f] == best


def test_error_metrics():
    b = np.array([[3.0, 4.0]])
    a = np.array([[3.0, 4.0 + 5e-3]])
    assert O.rel_error(a, b)[0] == pytest.approx(1e-3)
    assert O.e_appr_db(a, b)[0] == pytest.approx(-60.0)


def test_far_field_source_found():
    """Far-field stand-in for Section 4: the peak direction is the source direction."""
    wl = WL.make_far_field(F=2, L=512, snr_db=20.0, step_deg=10.0)
    K = O.n_bins(wl.L, wl.fs)
    psi = O.phat_cross_spectra(O.spectra(wl.frames, O.window(wl.L, "sqrt_hann"), K))
    w = O.bin_weights(wl.L, K)
    dt = O.tdoa(wl.mic_xyz, wl.directions, wl.c, field="far")
    conv = O.srp_conventional(psi, dt, wl.fs, wl.L, w)
    win = O.pair_windows(wl.mic_xyz, wl.c, wl.fs / 2, 2)
    ny = O.srp_nyquist(O.gcc_samples(psi, wl.fs, wl.L, w, win), dt, win)
    for mp in (conv, ny):
        idx, _ = O.peaks(mp)
        ang = np.degrees(np.arccos(np.clip(wl.directions[idx] @ wl.sources[0], -1, 1)))
        assert np.all(ang <= 10.0 + 1e-9)
