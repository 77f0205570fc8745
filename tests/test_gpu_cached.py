"""Cached-weight Nyquist maps (srp_nyquist_weights + srp_map_nyquist_cached), GPU.

* The weight matrix W [J][Sw] equals the oracle's float64 sinc weights
  sinc(dt_p(i)/T - n) (numpy.sinc) rounded once to bfloat16 / half, in the
  packed column layout (window of pair p at its padded offset, zeros in the
  gap columns and past S): at least 99.9 % of the entries bit-equal, the
  others one unit in the last place apart (a float64 value within a rounding
  of a tie may round either way) or within 1e-9 of each other (an exact
  integer TDOA seen as integer + 1e-17 by one side).
* The map equals 2 xi W^T evaluated in float64 from the very bf16/fp16
  arrays the kernel read (float32 accumulation: 1e-5 relative), and the
  oracle's float64 Nyquist map within the BF16/FP16 tolerance 1e-2, with the
  argmax checked as for every other map.
* Argument errors. (The room-scale workload, 16 mics / 576,000 candidates /
  500 frames, is checked over its whole map in test_gpu_fullsize.py.)
"""
import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests import refpath as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2012_09499_amd as srp  # noqa: E402

TOL = 1e-2
CASES = {
    "m4_L256_F3": lambda: WL.make_custom(M=4, J_shape=(9, 7, 5), L=256, F=3, seed=1),
    "m7_L1024_F70": lambda: WL.make_custom(M=7, J_shape=(13, 11, 7), h=0.09, L=1024, F=70,
                                           seed=2),
    "m5_L4096_48k_F2": lambda: WL.make_custom(M=5, J_shape=(6, 5, 4), h=0.2, fs=48000.0,
                                              L=4096, F=2, seed=5, box=(1.2, 1.0, 0.6)),
    "m6_L1024_fmax4k_F4": lambda: WL.make_custom(M=6, J_shape=(7, 6, 5), L=1024, F=4, seed=6,
                                                 f_max=4000.0),
    "farfield_uca6_F300": lambda: WL.make_far_field(F=300, L=1024, step_deg=6.0),
}


def _geom(wl):
    return srp.Geometry(wl.mic_xyz, wl.candidates(), fs=wl.fs, L=wl.L, c=wl.c, n_aux=wl.n_aux,
                        field=wl.field, f_max=wl.f_max)


def _ref_weights(wl, cand, cols):
    """Oracle sinc weights in the library's packed column layout (float64)."""
    _, _, win = R.oracle_setup(wl)
    dt = O.tdoa(wl.mic_xyz, cand, wl.c, field=wl.field)          # [n][P]
    x = dt / win["T"]
    _, off, S = srp.pair_layout(wl.mic_xyz, wl.c, wl.band_limit, wl.n_aux)
    Wm = np.zeros((cand.shape[0], cols))
    for p in range(len(win["pairs"])):
        h = (win["W"][p] - 1) // 2
        n = np.arange(-h, h + 1)
        Wm[:, off[p]:off[p] + win["W"][p]] = np.sinc(x[:, p:p + 1] - n[None, :])
    return Wm


def _round(v, dtype):
    t = torch.from_numpy(v).to(torch.bfloat16 if dtype == "bf16" else torch.float16)
    return t.to(torch.float64).numpy()


def _ulp_apart(a, b, dtype):
    ta = torch.from_numpy(a).to(torch.bfloat16 if dtype == "bf16" else torch.float16)
    tb = torch.from_numpy(b).to(torch.bfloat16 if dtype == "bf16" else torch.float16)
    ia = ta.view(torch.int16).to(torch.int32).numpy()
    ib = tb.view(torch.int16).to(torch.int32).numpy()
    return np.abs(ia - ib)


@pytest.fixture(scope="module")
def cases():
    return {k: v() for k, v in CASES.items()}


@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
@pytest.mark.parametrize("name", list(CASES))
def test_weights_are_rounded_float64_sinc(cases, name, dtype):
    wl = cases[name]
    g = _geom(wl)
    W = srp.nyquist_weights(g, dtype)
    torch.cuda.synchronize()
    assert W.shape[1] % 128 == 0 and W.shape[1] >= g.S
    got = W.to(torch.float64).cpu().numpy()
    ref = _round(_ref_weights(wl, wl.candidates(), W.shape[1]), dtype)
    d = _ulp_apart(got, ref, dtype)
    # bit-equal almost everywhere; one unit apart where the float64 value sits
    # within a rounding of a tie; and where dt_p(i)/T is an exact integer (the
    # circular array's symmetric directions) one side may see a fraction of
    # 1e-17 instead of 0, turning an exact 0 weight into ~1e-17
    tiny = np.abs(got - ref) <= 1e-9
    assert np.all((d <= 1) | tiny)
    assert ((d == 0) | tiny).mean() >= 0.999, ((d != 0) & ~tiny).sum()
    # gap columns and the columns past S are exactly zero
    _, off, S = srp.pair_layout(wl.mic_xyz, wl.c, wl.band_limit, wl.n_aux)
    _, _, win = R.oracle_setup(wl)
    mask = np.ones(W.shape[1], dtype=bool)
    for p in range(len(off) - 1):
        mask[off[p]:off[p] + win["W"][p]] = False
    assert np.all(got[:, mask] == 0.0)
    g.close()


@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
@pytest.mark.parametrize("name", list(CASES))
def test_cached_map_is_the_product_and_matches_oracle(cases, name, dtype):
    wl = cases[name]
    g = _geom(wl)
    tdt = srp.sample_torch_dtype(dtype)
    xi_ref = R.oracle_xi(wl, R.oracle_psi(wl))
    # the product kernel alone: the oracle's weights and samples, each rounded
    # once to the storage type, feed the kernel; their product in float64 is the
    # expected map (float32 accumulation: 1e-5 relative)
    cols = srp.nyquist_weights_bytes(g, dtype) // (2 * g.J)
    Wr = _round(_ref_weights(wl, wl.candidates(), cols), dtype)
    W_in = torch.from_numpy(Wr).to(tdt).cuda()
    xi_in, xr = R.device_samples(g, xi_ref, tdt)
    m, pk = srp.map_nyquist_cached(g, W_in, xi_in, dtype=dtype)
    torch.cuda.synchronize()
    got = m.cpu().numpy().astype(np.float64)
    full = np.zeros((wl.F, g.S))
    full[:, R.sample_columns(g)] = xr
    prod = 2.0 * full @ Wr[:, :g.S].T
    assert O.rel_error(got, prod).max() <= 1e-5
    np.testing.assert_array_equal(srp.decode_peaks(pk)[0], np.argmax(got, axis=1))
    del W_in
    # the whole cached path (library weights, samples from the frames) against
    # the float64 oracle map of the frames, within the BF16/FP16 tolerance
    W = srp.nyquist_weights(g, dtype)
    fr = torch.from_numpy(wl.frames).cuda()
    xi = srp.gcc_samples(g, srp.cross_spectra(g, fr), dtype=dtype)
    m, pk = srp.map_nyquist_cached(g, W, xi, dtype=dtype)
    torch.cuda.synchronize()
    got = m.cpu().numpy().astype(np.float64)
    ref = R.oracle_nyquist(wl, xi_ref, wl.candidates())
    assert O.rel_error(got, ref).max() <= TOL
    idx = srp.decode_peaks(pk)[0]
    np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
    R.check_argmax(idx, ref, TOL, label=f"cached/{name}/{dtype}")
    g.close()


def test_cached_argument_errors():
    wl = CASES["m4_L256_F3"]()
    g = _geom(wl)
    with pytest.raises(srp.SrpError, match="BF16 or FP16"):
        srp.nyquist_weights_bytes(g, "fp32")
    W = srp.nyquist_weights(g, "bf16")
    fr = torch.from_numpy(wl.frames).cuda()
    xi = srp.gcc_samples(g, srp.cross_spectra(g, fr), dtype="bf16")
    with pytest.raises(TypeError):
        srp.map_nyquist_cached(g, W, xi, dtype="fp16")
    with pytest.raises(ValueError):
        srp.map_nyquist_cached(g, W[:5], xi, dtype="bf16")
    small = torch.empty(16, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(srp.SrpError, match="too small"):
        srp.lib()  # noqa: B018 (loaded)
        S = srp._lib
        S._check(S.lib().srp_nyquist_weights(g.handle, S.DTYPES["bf16"], small.data_ptr(), 32,
                                             None))
    g.close()
