"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (written here, derived in the design doc):
* FP32 maps: relative L2 error per frame <= 1e-5; argmax identical in >= 99 %
  of frames, any other frame a near-tie within the map tolerance.
* BF16 / FP16 maps (weights and samples in that type, float32 accumulation):
  relative L2 error per frame <= 1e-2 against the FP64 oracle run from the
  frames; argmax as above with that tolerance.
* BF16 / FP16 GCC samples: exactly the float32 samples rounded to that type.
* FP64 map instances from the same float32 samples: <= 1e-12.
* PHAT cross-spectra: relative L2 error per frame <= 1e-5 (float32 FFT).
* GCC samples from the same psi: relative L2 error per frame <= 1e-5 (a
  float32 sum over 2K terms: about u sqrt(2K), ~3e-6 at K = 2049) and
  elementwise absolute error <= 1e-5 L.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests import refpath as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2012_09499_amd as srp  # noqa: E402

MAP_TOL = 1e-5
LOWP_TOL = 1e-2
PSI_TOL = 1e-5
XI_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    srp.lib()
    yield
    torch.cuda.synchronize()


def _frames(wl):
    return torch.from_numpy(wl.frames).cuda()


def _geom(wl, window="hann", n_aux=None, cand=None):
    cand = wl.candidates() if cand is None else cand
    return srp.Geometry(wl.mic_xyz, cand, fs=wl.fs, L=wl.L, c=wl.c, f_max=wl.band_limit,
                        n_aux=wl.n_aux if n_aux is None else n_aux, field=wl.field,
                        window=window)


def _rel(a, b):
    return O.rel_error(a, b)


def _c128(psi_t):
    return psi_t.cpu().numpy().astype(np.complex128)


CASES = {
    # name: (builder) -- several candidate tiles, a ragged frame tail, odd J
    "m4_L256_F3": lambda: WL.make_custom(M=4, J_shape=(9, 7, 5), L=256, F=3, seed=1),
    "m7_L1024_F70": lambda: WL.make_custom(M=7, J_shape=(13, 11, 7), h=0.09, L=1024, F=70, seed=2),
    "m2_L64_F1": lambda: WL.make_custom(M=2, J_shape=(1, 1, 1), L=64, F=1, seed=3),
    "m12_L512_F9_naux0": lambda: WL.make_custom(M=12, J_shape=(17, 5, 3), L=512, F=9, seed=4,
                                                n_aux=0),
    "m5_L4096_48k_F2": lambda: WL.make_custom(M=5, J_shape=(6, 5, 4), h=0.2, fs=48000.0,
                                              L=4096, F=2, seed=5, box=(1.2, 1.0, 0.6)),
    "m6_L1024_fmax4k_F4": lambda: WL.make_custom(M=6, J_shape=(7, 6, 5), L=1024, F=4, seed=6,
                                                 f_max=4000.0),
    # S ~ 48k samples (one-level FP32 sum near its limit), 2KP ~ 283k terms
    # (two-level conventional sum)
    "m24_L1024_48k_F3": lambda: WL.make_custom(M=24, J_shape=(9, 7, 5), h=0.15, fs=48000.0,
                                               L=1024, F=3, seed=9, box=(1.0, 1.0, 0.6)),
    # S ~ 85k samples: the two-level-sum Nyquist kernel variant
    "m32_L1024_48k_F3": lambda: WL.make_custom(M=32, J_shape=(9, 7, 5), h=0.15, fs=48000.0,
                                               L=1024, F=3, seed=9, box=(1.0, 1.0, 0.6)),
}


@pytest.fixture(scope="module")
def cases():
    return {k: v() for k, v in CASES.items()}


@pytest.mark.parametrize("name", list(CASES))
def test_cross_spectra(cases, name):
    wl = cases[name]
    g = _geom(wl)
    psi = srp.cross_spectra(g, _frames(wl))
    torch.cuda.synchronize()
    ref = R.oracle_psi(wl)
    got = _c128(psi)
    err = np.sqrt((np.abs(got - ref) ** 2).sum(axis=(1, 2)) / (np.abs(ref) ** 2).sum(axis=(1, 2)))
    assert err.max() <= PSI_TOL, err
    np.testing.assert_allclose(np.abs(got), 1.0, atol=1e-6)


@pytest.mark.parametrize("name", list(CASES))
def test_gcc_samples(cases, name):
    """GCC samples from the oracle's cross-spectra (rounded once to complex64 and
    given to the kernel) against the oracle's samples from the same values."""
    wl = cases[name]
    g = _geom(wl)
    psi_dev, psi_in = R.device_psi(R.oracle_psi(wl))
    xi = srp.gcc_samples(g, psi_dev)
    torch.cuda.synchronize()
    ref = R.oracle_xi(wl, psi_in)
    got = srp.unpack_samples(g, xi)
    # the layout's alignment gaps after each window are zeros
    full = xi.cpu().numpy()
    gaps = np.ones(g.S, dtype=bool)
    for o, w in zip(g.offsets[:-1], g.W):
        gaps[o:o + w] = False
    assert np.all(full[:, gaps] == 0.0) and np.all(g.offsets % 8 == 0)
    assert _rel(got, ref).max() <= XI_TOL
    # elementwise: a float32 sum of 2K terms whose magnitudes add up to at most
    # sum_k w_k <= L; the worst-case rounding bound 2K u L (u = 2^-24) exceeds
    # 1e-5 L, which typical error growth (sqrt(2K) u L) stays well below
    assert np.abs(got - ref).max() <= 1e-5 * wl.L


def _gaps_are_zero(g, xi):
    full = xi.float().cpu().numpy()
    gaps = np.ones(g.S, dtype=bool)
    for o, w in zip(g.offsets[:-1], g.W):
        gaps[o:o + w] = False
    return bool(np.all(full[:, gaps] == 0.0))


@pytest.mark.parametrize("name", list(CASES))
def test_gcc_samples_frames(cases, name):
    """Frames -> GCC samples in one call (FFT, PHAT phasors, cross-spectra formed
    on chip) against the oracle's samples from the frames in float64, and against
    the two-call path (srp_cross_spectra, srp_gcc_samples)."""
    wl = cases[name]
    g = _geom(wl)
    fr = _frames(wl)
    xi = srp.gcc_samples_frames(g, fr)
    two = srp.gcc_samples(g, srp.cross_spectra(g, fr))
    torch.cuda.synchronize()
    ref = R.oracle_xi(wl, R.oracle_psi(wl))
    got = srp.unpack_samples(g, xi)
    assert _gaps_are_zero(g, xi)
    assert _rel(got, ref).max() <= XI_TOL
    assert np.abs(got - ref).max() <= 1e-5 * wl.L
    assert _rel(got, srp.unpack_samples(g, two)).max() <= XI_TOL


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_gcc_samples_frames_lowp_rounded(cases, name, dtype):
    """BF16/FP16 samples of the fused call are its float32 samples rounded once."""
    wl = cases[name]
    g = _geom(wl)
    fr = _frames(wl)
    x32 = srp.gcc_samples_frames(g, fr)
    xlo = srp.gcc_samples_frames(g, fr, dtype=dtype)
    torch.cuda.synchronize()
    assert xlo.dtype == srp.sample_torch_dtype(dtype)
    assert torch.equal(x32.to(xlo.dtype), xlo)


def test_silent_microphones_give_zero_phasors():
    """A microphone whose frame is all zeros has Y = 0, so every pair with it has
    psi = 0 (PHAT of a zero product) and zero GCC samples, also when it shares a
    complex transform with a live microphone (mic 2 with mic 3) or is the odd
    one out (mic 6 of 7)."""
    wl = WL.make_custom(M=7, J_shape=(5, 4, 3), L=512, F=5, seed=21)
    fr = wl.frames.copy()
    fr[:, 2, :] = 0.0
    fr[1:3, 6, :] = 0.0
    wl.frames = fr
    g = _geom(wl)
    fr_d = _frames(wl)
    psi = srp.cross_spectra(g, fr_d)
    xi = srp.gcc_samples_frames(g, fr_d)
    torch.cuda.synchronize()
    psi_ref = R.oracle_psi(wl)
    got = _c128(psi)
    assert np.all(got[psi_ref == 0] == 0) and np.all(np.abs(got[psi_ref != 0]) > 0.99)
    err = np.sqrt((np.abs(got - psi_ref) ** 2).sum(axis=(1, 2)) /
                  (np.abs(psi_ref) ** 2).sum(axis=(1, 2)))
    assert err.max() <= PSI_TOL
    ref = R.oracle_xi(wl, psi_ref)
    gx = srp.unpack_samples(g, xi)
    assert np.all(gx[ref == 0] == 0)
    assert _rel(gx, ref).max() <= XI_TOL


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_nyquist_map_from_same_samples(cases, name, dtype):
    """The map kernel alone: the oracle's GCC samples, rounded once to float32, go
    to the kernel and to the oracle's map."""
    wl = cases[name]
    g = _geom(wl)
    xi, xin = R.device_samples(g, R.oracle_xi(wl, R.oracle_psi(wl)), torch.float32)
    m, pk = srp.map_nyquist(g, xi, dtype=dtype)
    torch.cuda.synchronize()
    ref = R.oracle_nyquist(wl, xin, wl.candidates())
    got = m.cpu().numpy().astype(np.float64)
    tol = MAP_TOL if dtype == "fp32" else 1e-12
    # the fp64 kernel writes a float32 map: compare at float32 resolution
    if dtype == "fp64":
        ref32 = ref.astype(np.float32).astype(np.float64)
        assert np.abs(got - ref32).max() <= 2 ** -23 * np.abs(ref).max() + 1e-30
    else:
        assert _rel(got, ref).max() <= tol
    idx, val = srp.decode_peaks(pk)
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    np.testing.assert_array_equal(val, got.max(axis=1).astype(np.float32))
    R.check_argmax(idx, ref, MAP_TOL, label=f"nyquist-same-samples/{name}/{dtype}")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_conventional_map(cases, name, dtype):
    """The conventional kernel alone, from the oracle's cross-spectra rounded once
    to complex64 (the same values feed the oracle's map)."""
    wl = cases[name]
    g = _geom(wl)
    psi, psi_in = R.device_psi(R.oracle_psi(wl))
    m, pk = srp.map_conventional(g, psi, dtype=dtype)
    torch.cuda.synchronize()
    ref = R.oracle_conventional(wl, psi_in, wl.candidates())
    got = m.cpu().numpy().astype(np.float64)
    if dtype == "fp64":
        ref32 = ref.astype(np.float32).astype(np.float64)
        assert np.abs(got - ref32).max() <= 2 ** -23 * np.abs(ref).max() * 1.01 + 1e-30
    else:
        assert _rel(got, ref).max() <= MAP_TOL
    idx, _ = srp.decode_peaks(pk)
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    R.check_argmax(idx, ref, MAP_TOL, label=f"conventional/{name}/{dtype}")


@pytest.mark.parametrize("name", list(CASES))
def test_pipeline_from_frames(cases, name):
    """Frames -> peaks, both methods, against the oracle run from the frames in FP64."""
    wl = cases[name]
    g = _geom(wl)
    pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
    fr = _frames(wl)
    psi_ref = R.oracle_psi(wl)
    cand = wl.candidates()
    m, pk = pipe.nyquist(fr)
    torch.cuda.synchronize()
    ref = R.oracle_nyquist(wl, R.oracle_xi(wl, psi_ref), cand)
    assert _rel(m.cpu().numpy(), ref).max() <= MAP_TOL
    R.check_argmax(srp.decode_peaks(pk)[0], ref, MAP_TOL, label=f"pipeline-nyquist/{name}/fp32")
    m, pk = pipe.conventional(fr)
    torch.cuda.synchronize()
    refc = R.oracle_conventional(wl, psi_ref, cand)
    assert _rel(m.cpu().numpy(), refc).max() <= MAP_TOL
    R.check_argmax(srp.decode_peaks(pk)[0], refc, MAP_TOL,
                   label=f"pipeline-conventional/{name}/fp32")


def test_peaks_only_equals_map_argmax(cases):
    wl = cases["m7_L1024_F70"]
    g = _geom(wl)
    pipe = srp.SrpPipeline(g, wl.F, keep_map=False)
    fr = _frames(wl)
    _, pk1 = pipe.nyquist(fr)
    xi = srp.gcc_samples_frames(g, fr)  # the samples the pipeline's Nyquist path uses
    m, _ = srp.map_nyquist(g, xi, want_peaks=False)
    pk2 = srp.argmax(m)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(pk1.cpu().numpy(), pk2.cpu().numpy())


def test_argmax_kernel_random_and_ties():
    rng = np.random.default_rng(0)
    for F, J in [(1, 1), (3, 1000), (5, 2049 * 3 + 17), (2, 70000)]:
        a = rng.standard_normal((F, J)).astype(np.float32)
        a[0, J // 2] = a[0].max() + 1.0
        if J > 10:
            a[-1, 7] = a[-1, J - 3] = a[-1].max() + 2.0  # tie: lowest index wins
        pk = srp.argmax(torch.from_numpy(a).cuda())
        idx, val = srp.decode_peaks(pk)
        np.testing.assert_array_equal(idx, np.argmax(a, axis=1))
        np.testing.assert_array_equal(val, a.max(axis=1))
    neg = -np.abs(rng.standard_normal((2, 300))).astype(np.float32) - 1.0
    idx, val = srp.decode_peaks(srp.argmax(torch.from_numpy(neg).cuda()))
    np.testing.assert_array_equal(idx, np.argmax(neg, axis=1))


def test_zero_frames_give_zero_map_and_index_zero():
    wl = WL.make_custom(M=4, J_shape=(9, 7, 5), L=256, F=3, seed=1)
    g = _geom(wl)
    z = torch.zeros((3, 4, 256), dtype=torch.float32, device="cuda")
    pipe = srp.SrpPipeline(g, 3, keep_map=True)
    for run in (pipe.nyquist, pipe.conventional):
        m, pk = run(z)
        torch.cuda.synchronize()
        assert torch.count_nonzero(m).item() == 0
        idx, val = srp.decode_peaks(pk)
        assert np.all(idx == 0) and np.all(val == 0)


def test_far_field_pipeline():
    wl = WL.make_far_field(F=3, L=1024, step_deg=4.0)
    g = _geom(wl, window="sqrt_hann")
    pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
    fr = _frames(wl)
    psi_ref = R.oracle_psi(wl, window="sqrt_hann")
    m, pk = pipe.nyquist(fr)
    torch.cuda.synchronize()
    ref = R.oracle_nyquist(wl, R.oracle_xi(wl, psi_ref), wl.directions)
    assert _rel(m.cpu().numpy(), ref).max() <= MAP_TOL
    R.check_argmax(srp.decode_peaks(pk)[0], ref, MAP_TOL, label="far-field/nyquist/fp32")
    m, pk = pipe.conventional(fr)
    torch.cuda.synchronize()
    refc = R.oracle_conventional(wl, psi_ref, wl.directions)
    assert _rel(m.cpu().numpy(), refc).max() <= MAP_TOL


def test_integer_tdoa_candidates_exact_weight():
    """Candidates whose x_p is an exact integer hit the sinc(0) = 1 case."""
    fs, c, L = 16000.0, 343.0, 256
    d = 10 * c / fs
    mic = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    cand = np.array([[-1.0, 0.0, 0.0], [2.0 * d, 0.0, 0.0], [0.5 * d, 0.0, 0.0],
                     [0.5 * d, 1.0, 0.0]])
    rng = np.random.default_rng(3)
    y = rng.standard_normal((4, 2, L)).astype(np.float32)
    g = srp.Geometry(mic, cand, fs=fs, L=L, c=c, n_aux=2)
    pipe = srp.SrpPipeline(g, 4, keep_map=True)
    m, _ = pipe.nyquist(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    wl = WL.Workload(name="int", mic_xyz=mic, grid=None, fs=fs, L=L, F=4, c=c, n_aux=2, frames=y)
    psi = R.oracle_psi(wl)
    ref = R.oracle_nyquist(wl, R.oracle_xi(wl, psi), cand)
    assert _rel(m.cpu().numpy(), ref).max() <= MAP_TOL
    conv = R.oracle_conventional(wl, psi, cand)
    # exact interpolation at the integer-TDOA candidates (sinc(x - n) = delta)
    np.testing.assert_allclose(m.cpu().numpy()[:, :3], conv[:, :3], rtol=2e-5,
                               atol=2e-5 * np.abs(conv).max())


def test_repeat_runs_bitwise_identical(cases):
    wl = cases["m7_L1024_F70"]
    g = _geom(wl)
    pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
    fr = _frames(wl)
    m1 = pipe.nyquist(fr)[0].clone()
    m2 = pipe.nyquist(fr)[0].clone()
    c1 = pipe.conventional(fr)[0].clone()
    c2 = pipe.conventional(fr)[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(c1, c2)


def test_config1_full():
    """4-mic 2-D scene, 2500 candidates, 10 frames, both methods, N_aux 0..4."""
    for n_aux in range(5):
        wl = WL.make(1, n_aux=n_aux)
        g = _geom(wl)
        pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
        fr = _frames(wl)
        psi_ref = R.oracle_psi(wl)
        m, pk = pipe.nyquist(fr)
        torch.cuda.synchronize()
        ref = R.oracle_nyquist(wl, R.oracle_xi(wl, psi_ref), wl.candidates())
        assert _rel(m.cpu().numpy(), ref).max() <= MAP_TOL
        R.check_argmax(srp.decode_peaks(pk)[0], ref, MAP_TOL,
                       label=f"config1/nyquist/naux{n_aux}/fp32")
    m, pk = pipe.conventional(fr)
    torch.cuda.synchronize()
    refc = R.oracle_conventional(wl, psi_ref, wl.candidates())
    assert _rel(m.cpu().numpy(), refc).max() <= MAP_TOL
    R.check_argmax(srp.decode_peaks(pk)[0], refc, MAP_TOL, label="config1/conventional/fp32")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_lowp_samples_are_rounded_fp32_samples(cases, name, dtype):
    wl = cases[name]
    g = _geom(wl)
    psi = srp.cross_spectra(g, _frames(wl))
    x32 = srp.gcc_samples(g, psi)
    xlo = srp.gcc_samples(g, psi, dtype=dtype)
    torch.cuda.synchronize()
    assert xlo.dtype == srp.sample_torch_dtype(dtype)
    assert torch.equal(x32.to(xlo.dtype), xlo)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_nyquist_lowp_pipeline(cases, name, dtype):
    """Frames -> BF16/FP16 Nyquist map against the FP64 oracle run from the frames."""
    wl = cases[name]
    g = _geom(wl)
    pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
    m, pk = pipe.nyquist(_frames(wl), dtype=dtype)
    torch.cuda.synchronize()
    psi_ref = R.oracle_psi(wl)
    ref = R.oracle_nyquist(wl, R.oracle_xi(wl, psi_ref), wl.candidates())
    got = m.cpu().numpy().astype(np.float64)
    err = _rel(got, ref)
    assert err.max() <= LOWP_TOL, err
    idx = srp.decode_peaks(pk)[0]
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    R.check_argmax(idx, ref, LOWP_TOL, label=f"pipeline-nyquist/{name}/{dtype}")


@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_lowp_map_with_far_origin(dtype):
    """The BF16/FP16 map of an array and grid placed 1 km from the origin.

    Those kernels take TDOAs in float32 from positions relative to the
    microphone centroid, so the shift must change nothing beyond rounding:
    within the low-precision tolerance of the float64 oracle of the shifted
    geometry, and close to the map of the unshifted one.
    """
    wl = WL.make_custom(M=6, J_shape=(9, 7, 5), L=512, F=6, seed=31)
    shift = np.array([1000.0, -700.0, 300.0])
    far = WL.Workload(name="far-origin", mic_xyz=wl.mic_xyz + shift, grid=None, fs=wl.fs, L=wl.L,
                      F=wl.F, c=wl.c, n_aux=wl.n_aux, frames=wl.frames)
    cand = wl.candidates() + shift
    maps = []
    for mic, cq in ((wl.mic_xyz, wl.candidates()), (far.mic_xyz, cand)):
        g = srp.Geometry(mic, cq, fs=wl.fs, L=wl.L, c=wl.c, n_aux=wl.n_aux)
        pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
        m, _ = pipe.nyquist(_frames(wl), dtype=dtype)
        torch.cuda.synchronize()
        maps.append(m.cpu().numpy().astype(np.float64))
        g.close()
    ref = R.oracle_nyquist(far, R.oracle_xi(far, R.oracle_psi(far)), cand)
    assert _rel(maps[1], ref).max() <= LOWP_TOL
    # the two maps differ by the float64 rounding of the shifted coordinates
    # (and the weight roundings it flips), far below the tolerance
    assert np.abs(maps[1] - maps[0]).max() <= 2e-3 * np.abs(maps[0]).max()


@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_lowp_long_windows_both_run_lists(dtype):
    """BF16/FP16 Nyquist map with pair windows of 85 .. 447 lags over 260 frames.

    One 256-frame block runs with 8 frame tiles on lag runs of at most 128
    lags (each window in 1 to 4 runs), the 4-frame tail with one frame tile on
    runs of at most 256 lags (1 or 2 runs): both run lists of the kernel,
    against the float64 oracle.
    """
    wl = WL.make_custom(M=6, J_shape=(6, 5, 4), h=0.25, fs=48000.0, L=1024, F=260, seed=41,
                        box=(1.6, 1.4, 0.8))
    g = _geom(wl)
    pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
    m, pk = pipe.nyquist(_frames(wl), dtype=dtype)
    torch.cuda.synchronize()
    ref = R.oracle_nyquist(wl, R.oracle_xi(wl, R.oracle_psi(wl)), wl.candidates())
    got = m.cpu().numpy().astype(np.float64)
    assert _rel(got, ref).max() <= LOWP_TOL
    idx = srp.decode_peaks(pk)[0]
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    R.check_argmax(idx, ref, LOWP_TOL, label=f"long-windows/{dtype}")
    g.close()


@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp16"])
def test_near_integer_tdoa_stays_finite(dtype):
    """TDOAs within 1e-10 .. 1e-7 samples of an integer (|x - rint(x)| tiny but not 0).

    Regression: a weight denominator formed as base + (xf - j) lost xf and hit
    exactly 0 there, giving NaN maps.
    """
    fs, c, L = 16000.0, 343.0, 256
    d = 10 * c / fs
    mic = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    xs = [k + e for k in (-7, -3, 0, 1, 3, 7) for e in (1e-10, -1e-10, 3e-8, -1e-7)]
    a = (d - np.asarray(xs) * c / fs) / 2.0  # on the axis between the mics: x = (d - 2a) fs / c
    cand = np.stack([a, np.zeros_like(a), np.zeros_like(a)], axis=1)
    rng = np.random.default_rng(5)
    y = rng.standard_normal((3, 2, L)).astype(np.float32)
    g = srp.Geometry(mic, cand, fs=fs, L=L, c=c, n_aux=2)
    pipe = srp.SrpPipeline(g, 3, keep_map=True)
    m, _ = pipe.nyquist(torch.from_numpy(y).cuda(), dtype=dtype)
    torch.cuda.synchronize()
    got = m.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(got))
    wl = WL.Workload(name="nearint", mic_xyz=mic, grid=None, fs=fs, L=L, F=3, c=c, n_aux=2,
                     frames=y)
    ref = R.oracle_nyquist(wl, R.oracle_xi(wl, R.oracle_psi(wl)), cand)
    assert _rel(got, ref).max() <= (MAP_TOL if dtype == "fp32" else LOWP_TOL)


@pytest.fixture(scope="module")
def many_frames():
    # 520 frames: two full 256-frame blocks and a tail of 8
    wl = WL.make_custom(M=5, J_shape=(10, 6, 5), L=256, F=520, seed=11)
    return wl, R.oracle_xi(wl, R.oracle_psi(wl))


def _tdt(dtype):
    return srp.sample_torch_dtype(dtype)


@pytest.mark.parametrize("F", [256, 257, 288, 500, 520])
@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp16"])
def test_nyquist_frame_block_boundaries(many_frames, F, dtype):
    """Frame counts around the interpolation kernels' frame blocks (256 frames
    per block, tail blocks of 1-7 32-frame tiles, a last block with fewer rows
    than its tiles). The oracle's samples, rounded once to the storage type, feed
    both the kernel and the oracle's map."""
    wl, xi_ref = many_frames
    g = _geom(wl)
    xi, xin = R.device_samples(g, xi_ref[:F], _tdt(dtype))
    m, pk = srp.map_nyquist(g, xi, dtype=dtype)
    torch.cuda.synchronize()
    ref = R.oracle_nyquist(wl, xin, wl.candidates())
    got = m.cpu().numpy().astype(np.float64)
    assert got.shape == (F, wl.J) and np.all(np.isfinite(got))
    tol = MAP_TOL if dtype == "fp32" else LOWP_TOL
    assert _rel(got, ref).max() <= tol
    idx, _ = srp.decode_peaks(pk)
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    R.check_argmax(idx, ref, tol, label=f"frame-blocks/F{F}/{dtype}")


@pytest.mark.parametrize("F", [127, 128, 129, 520])
def test_gcc_samples_frames_frame_blocks(many_frames, F):
    """Frame counts around the fused GCC kernel's 128-frame workgroups."""
    wl, xi_ref = many_frames
    g = _geom(wl)
    xi = srp.gcc_samples_frames(g, _frames(wl)[:F])
    torch.cuda.synchronize()
    assert xi.shape == (F, g.S) and _gaps_are_zero(g, xi)
    assert _rel(srp.unpack_samples(g, xi), xi_ref[:F]).max() <= XI_TOL


@pytest.fixture(scope="module")
def wide_grid():
    # 76,800 candidates (300 blocks of 256) x 300 frames: 600 workgroups of
    # 256 candidates x 256 frames, which on a 256-CU device fill two whole
    # rounds (one workgroup per CU, in every precision) and leave 44
    # candidate blocks, so the map call runs as two launches split at candidate
    # 65,536 (the rest with 64-frame blocks, the last of them 44 frames)
    wl = WL.make_custom(M=8, J_shape=(80, 40, 24), L=256, F=300, seed=12)
    xi_ref = R.oracle_xi(wl, R.oracle_psi(wl))
    return wl, xi_ref, R.oracle_nyquist(wl, xi_ref, wl.candidates())


@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp16"])
def test_nyquist_launch_split_boundary(wide_grid, dtype):
    """The whole map across the two-launch split: the oracle's samples rounded to
    the storage type feed the kernel and the oracle's map; then the whole path
    from the frames against the float64 oracle map of the frames."""
    wl, xi_ref, map_ref = wide_grid
    g = _geom(wl)
    xi, xin = R.device_samples(g, xi_ref, _tdt(dtype))
    m, pk = srp.map_nyquist(g, xi, dtype=dtype)
    torch.cuda.synchronize()
    ref = R.oracle_nyquist(wl, xin, wl.candidates())
    got = m.cpu().numpy().astype(np.float64)
    assert got.shape == (wl.F, wl.J) and np.all(np.isfinite(got))
    tol = MAP_TOL if dtype == "fp32" else LOWP_TOL
    assert _rel(got, ref).max() <= tol
    # the candidate blocks next to the split, alone
    cut = 256 * 256
    near = slice(cut - 512, cut + 512)
    assert _rel(got[:, near], ref[:, near]).max() <= tol
    idx, _ = srp.decode_peaks(pk)
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    # the whole path from the frames against the float64 oracle of the frames.
    # A 0.4 m array over an 8 m grid leaves long ridges of nearly equal map
    # values along the range direction: in 214 of the 300 frames the oracle's
    # two largest values differ by less than 1e-3 of the maximum, in 20 by less
    # than 1e-4. Rounding samples and weights to a 16-bit type moves the argmax
    # along such ridges in some of those frames (the recorded fractions); every
    # differing frame must be a near-tie within the map tolerance, and among the
    # frames whose two largest oracle values differ by more than the storage
    # type's unit roundoff (2^-8 for BF16, 2^-11 for FP16) the argmax must agree
    # in at least 99 % of them. FP32 must agree in 99 % of all frames.
    pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
    m2, pk2 = pipe.nyquist(_frames(wl), dtype=dtype)
    torch.cuda.synchronize()
    got2 = m2.cpu().numpy().astype(np.float64)
    assert _rel(got2, map_ref).max() <= tol
    idx2 = srp.decode_peaks(pk2)[0]
    if dtype == "fp32":
        R.check_argmax(idx2, map_ref, tol, label="launch-split-from-frames/fp32")
    else:
        R.check_argmax(idx2, map_ref, tol, label=f"launch-split-from-frames/{dtype}",
                       gate_min_frames=10 ** 9)
        top2 = np.sort(map_ref, axis=1)[:, -2:]
        gap = (top2[:, 1] - top2[:, 0]) / np.abs(top2[:, 1])
        u = 2.0 ** -8 if dtype == "bf16" else 2.0 ** -11
        resolved = gap > u
        same = idx2 == np.argmax(map_ref, axis=1)
        R.ARGMAX_LOG.append((f"launch-split-from-frames-gap-above-unit-roundoff/{dtype}",
                             int(same[resolved].sum()), int(resolved.sum())))
        # (FP16: 162 such frames; BF16: 1)
        assert resolved.any() and same[resolved].mean() >= 0.99, (
            resolved.sum(), same[resolved].mean())


def test_conventional_unsupported_dtype_writes_nothing(cases):
    """A dtype without a conventional kernel is refused before anything is enqueued:
    the caller's map and peaks keep their contents."""
    wl = cases["m4_L256_F3"]
    g = _geom(wl)
    psi = srp.cross_spectra(g, _frames(wl))
    pk = torch.full((wl.F, 2), -12345, dtype=torch.int64, device="cuda")
    m = torch.full((wl.F, g.J), 7.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    for dt in [d for d in ("bf16", "fp16") if not srp.conventional_supports(d)]:
        with pytest.raises(srp.SrpError) as e:
            srp.map_conventional(g, psi, dtype=dt, map_out=m, peaks_out=pk)
        assert e.value.status == srp.SRP_ERR_UNSUPPORTED
    # an unknown dtype code is an invalid argument, also before anything runs
    lib = srp.lib()
    st = lib.srp_map_conventional(g.handle, psi.data_ptr(), wl.F, 9, m.data_ptr(),
                                  pk.data_ptr(), None)
    assert st == srp.SRP_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((pk == -12345).all()) and bool((m == 7.0).all())


def _weighted_lowp(wl, g, psi, tdt):
    """The oracle's cross-spectra weighted by the bin weights and rounded once to
    the storage type, in the [F][P][Kp][2] layout of the BF16/FP16 conventional
    map; returns (device tensor, the values as psi again (rounded w psi / w))."""
    K, w, _ = R.oracle_setup(wl)
    F, P, _ = psi.shape
    Kp = (K + 7) // 8 * 8
    z = np.zeros((F, P, Kp, 2))
    z[:, :, :K, 0] = (psi * w).real
    z[:, :, :K, 1] = (psi * w).imag
    zr = R.rounded(z, tdt)
    back = (zr[:, :, :K, 0] + 1j * zr[:, :, :K, 1]) / w  # w in {1, 2}: exact
    return torch.from_numpy(z).to(tdt).cuda(), back


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_spectra_lowp_is_rounded_weighted_psi(cases, name, dtype):
    """srp_spectra_lowp from the oracle's cross-spectra (rounded to complex64)
    equals w_k psi rounded once to the storage type, bit for bit, zeros past K."""
    wl = cases[name]
    g = _geom(wl)
    psi_dev, psi_in = R.device_psi(R.oracle_psi(wl))
    got = srp.spectra_lowp(g, psi_dev, dtype)
    torch.cuda.synchronize()
    K, w, _ = R.oracle_setup(wl)
    ref = torch.zeros(got.shape, dtype=torch.float32)
    p32 = torch.from_numpy(psi_in.astype(np.complex64))
    w32 = torch.from_numpy(w.astype(np.float32))
    ref[:, :, :K, 0] = p32.real * w32
    ref[:, :, :K, 1] = p32.imag * w32
    assert torch.equal(got.cpu(), ref.to(got.dtype))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_conventional_lowp_map_kernel(cases, name, dtype):
    """The BF16/FP16 conventional kernel alone: the oracle's weighted spectra
    rounded to the storage type feed the kernel and the oracle's map."""
    wl = cases[name]
    g = _geom(wl)
    spec, psi_in = _weighted_lowp(wl, g, R.oracle_psi(wl), srp.sample_torch_dtype(dtype))
    m, pk = srp.map_conventional(g, spec, dtype=dtype)
    torch.cuda.synchronize()
    ref = R.oracle_conventional(wl, psi_in, wl.candidates())
    got = m.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(got))
    assert _rel(got, ref).max() <= LOWP_TOL
    idx = srp.decode_peaks(pk)[0]
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    R.check_argmax(idx, ref, LOWP_TOL, label=f"conventional-kernel/{name}/{dtype}")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_conventional_lowp_pipeline(cases, name, dtype):
    """Frames -> BF16/FP16 conventional map against the FP64 oracle of the frames."""
    wl = cases[name]
    g = _geom(wl)
    pipe = srp.SrpPipeline(g, wl.F, keep_map=True)
    m, pk = pipe.conventional(_frames(wl), dtype=dtype)
    torch.cuda.synchronize()
    ref = R.oracle_conventional(wl, R.oracle_psi(wl), wl.candidates())
    got = m.cpu().numpy().astype(np.float64)
    assert _rel(got, ref).max() <= LOWP_TOL
    idx = srp.decode_peaks(pk)[0]
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    R.check_argmax(idx, ref, LOWP_TOL, label=f"pipeline-conventional/{name}/{dtype}")
