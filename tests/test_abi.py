"""C-ABI boundary tests that need no GPU.

The library must load, export every function include/srp.h declares, agree
with the oracle on the host-side pair layout, and reject invalid arguments
with SRP_ERR_INVALID_ARG before touching a device.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as WL
from paper_2012_09499_amd import _lib as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "srp.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(srp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = S.lib()
    names = _declared()
    assert "srp_map_nyquist" in names and "srp_geometry" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(S.EXPORTS)
    assert "gfx950" in S.version()


@pytest.mark.parametrize("seed", range(5))
def test_pair_layout_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    M = int(rng.integers(2, 40))
    mic = rng.random((M, 3)) * rng.uniform(0.05, 2.0)
    fs = float(rng.choice([16000.0, 48000.0]))
    f_max = fs / 2 if seed % 2 == 0 else fs / 4
    n_aux = int(rng.integers(0, 4))
    N_p, off, Sx = S.pair_layout(mic, 343.0, f_max, n_aux)
    win = O.pair_windows(mic, 343.0, f_max, n_aux)
    np.testing.assert_array_equal(N_p, win["N"])
    # library layout: each window starts at a multiple of 8 samples
    padded = (win["W"] + 7) // 8 * 8
    np.testing.assert_array_equal(off, np.concatenate([[0], np.cumsum(padded)]))
    assert np.all(off % 8 == 0) and np.all(np.diff(off) >= win["W"])
    assert Sx == off[-1]


def test_pair_layout_paper_array():
    mic = WL.uniform_circular_array(6, 0.1)
    N_p, off, Sx = S.pair_layout(mic, 340.0, 8000.0, 2)
    assert sorted(N_p.tolist()) == [4] * 6 + [8] * 6 + [9] * 3
    # windows of 13, 21 and 23 samples, each padded to a multiple of 8
    assert Sx == 6 * 16 + 6 * 24 + 3 * 24


def _geometry_status(**kw):
    lib = S.lib()
    args = dict(mic=np.zeros((4, 3)) + np.arange(4)[:, None] * 0.1, M=4,
                cand=np.ones((10, 3)), J=10, field=0, c=343.0, fs=16000.0, L=1024,
                f_max=8000.0, n_aux=2, window=0)
    args.update(kw)
    h = C.c_void_p()
    mic = np.ascontiguousarray(args["mic"], dtype=np.float64)
    cand = np.ascontiguousarray(args["cand"], dtype=np.float64)
    st = lib.srp_geometry(mic.ctypes.data if args["mic"] is not None else None, args["M"],
                          cand.ctypes.data if args["cand"] is not None else None, args["J"],
                          args["field"], args["c"], args["fs"], args["L"], args["f_max"],
                          args["n_aux"], args["window"], None, C.byref(h))
    return st, h.value


@pytest.mark.parametrize("bad", [
    dict(M=1), dict(J=0), dict(L=1000), dict(L=8), dict(L=16384), dict(f_max=8001.0),
    dict(f_max=0.0), dict(n_aux=-1), dict(c=0.0), dict(field=7), dict(window=9),
    dict(fs=-1.0), dict(cand=np.ones((10, 3)), field=1),  # far-field directions must be unit
    dict(mic=np.array([[0, 0, 0], [5.0, 0, 0], [0, 0, 0.1], [0, 0.1, 0]]), L=64),  # window > L
])
def test_geometry_rejects_invalid_arguments(bad):
    st, h = _geometry_status(**bad)
    assert st == S.SRP_ERR_INVALID_ARG and not h
    assert S.lib().srp_last_error().decode()


def test_calls_reject_null_and_bad_sizes_without_device():
    lib = S.lib()
    assert lib.srp_cross_spectra(None, None, 1, 0, None, 0, None, None) == S.SRP_ERR_INVALID_ARG
    assert lib.srp_gcc_samples(None, None, 1, 0, None, None) == S.SRP_ERR_INVALID_ARG
    assert lib.srp_map_nyquist(None, None, 1, 0, None, None, None) == S.SRP_ERR_INVALID_ARG
    assert lib.srp_map_conventional(None, None, 1, 0, None, None, None) == S.SRP_ERR_INVALID_ARG
    assert lib.srp_argmax(None, 1, 1, None, None) == S.SRP_ERR_INVALID_ARG
    buf = C.create_string_buffer(64)
    assert lib.srp_argmax(buf, 0, 4, buf, None) == S.SRP_ERR_INVALID_ARG
    assert lib.srp_argmax(buf, 2, 0, buf, None) == S.SRP_ERR_INVALID_ARG
    n = C.c_size_t(0)
    assert lib.srp_cross_spectra_workspace(None, 1, C.byref(n)) == S.SRP_ERR_INVALID_ARG
    lib.srp_geometry_destroy(None)  # no-op


def test_pair_layout_rejects_invalid():
    with pytest.raises(S.SrpError):
        S.pair_layout(np.zeros((1, 3)), 343.0, 8000.0, 2)
    with pytest.raises(S.SrpError):
        S.pair_layout(np.zeros((3, 3)), 343.0, 8000.0, -1)
    with pytest.raises(S.SrpError):
        S.pair_layout(np.full((3, 3), np.nan), 343.0, 8000.0, 0)


def test_batched_rejects_empty_arena_without_device():
    lib = S.lib()
    items = (S.BatchItem * 1)()
    buf = C.create_string_buffer(256)
    # a NULL item geometry and an empty arena are refused before any device work
    assert lib.srp_map_nyquist_batched(items, 1, buf, 0, 0, buf, 256, None) == \
        S.SRP_ERR_INVALID_ARG
    assert "xi_elems" in lib.srp_last_error().decode()
    assert lib.srp_map_nyquist_batched(items, 1, buf, 64, 0, buf, 256, None) == \
        S.SRP_ERR_INVALID_ARG
    assert "geometry" in lib.srp_last_error().decode()
