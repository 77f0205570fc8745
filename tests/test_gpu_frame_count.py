"""Non-positive frame counts are refused by every per-frame call of the C ABI, GPU.

Each call gets F = 0 and F = -1 with a valid geometry and valid device buffers.
It must return SRP_ERR_INVALID_ARG (the header's rule: arguments are validated
before anything is enqueued) and leave every output buffer as it was: they are
filled with a sentinel beforehand and compared after a device synchronisation.
"""
import pytest

import workloads as WL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2012_09499_amd as srp  # noqa: E402
from paper_2012_09499_amd import _lib as S  # noqa: E402


def test_calls_refuse_non_positive_frame_counts():
    wl = WL.make_custom(M=4, J_shape=(9, 7, 5), L=256, F=3, seed=1)
    g = srp.Geometry(wl.mic_xyz, wl.candidates(), fs=wl.fs, L=wl.L, c=wl.c, n_aux=wl.n_aux)
    lib = S.lib()
    F = wl.F
    frames = torch.from_numpy(wl.frames).cuda()
    ws = torch.empty(g.workspace_bytes(F), dtype=torch.uint8, device="cuda")
    # valid inputs for the calls that take spectra or samples
    psi = srp.cross_spectra(g, frames, workspace=ws)
    xi = srp.gcc_samples(g, psi)
    xi_b = srp.gcc_samples(g, psi, dtype="bf16")
    weights = srp.nyquist_weights(g, "bf16")
    lowp = srp.spectra_lowp_buffer(g, F, "bf16")
    torch.cuda.synchronize()

    sentinel = 7.0
    psi_out = torch.full_like(psi, sentinel)
    xi_out = torch.full_like(xi, sentinel)
    lowp_out = torch.full_like(lowp, sentinel)
    map_out = torch.full((F, g.J), sentinel, dtype=torch.float32, device="cuda")
    peaks_out = torch.full((F, 2), 7, dtype=torch.int64, device="cuda")
    points = torch.zeros((F, 2, 3), dtype=torch.float64, device="cuda")
    values_out = torch.full((F, 2), sentinel, dtype=torch.float32, device="cuda")
    h = g.handle
    fp32, bf16 = S.DTYPES["fp32"], S.DTYPES["bf16"]
    for bad in (0, -1):
        calls = {
            "srp_cross_spectra": lambda: lib.srp_cross_spectra(
                h, frames.data_ptr(), bad, 0, ws.data_ptr(), ws.numel(), psi_out.data_ptr(), None),
            "srp_cross_spectra_noalloc": lambda: lib.srp_cross_spectra_noalloc(
                h, frames.data_ptr(), bad, 0, psi_out.data_ptr(), None),
            "srp_gcc_samples": lambda: lib.srp_gcc_samples(
                h, psi.data_ptr(), bad, fp32, xi_out.data_ptr(), None),
            "srp_gcc_samples_frames": lambda: lib.srp_gcc_samples_frames(
                h, frames.data_ptr(), bad, 0, fp32, ws.data_ptr(), ws.numel(), xi_out.data_ptr(),
                None),
            "srp_spectra_lowp": lambda: lib.srp_spectra_lowp(
                h, psi.data_ptr(), bad, bf16, lowp_out.data_ptr(),
                lowp_out.numel() * lowp_out.element_size(), None),
            "srp_map_nyquist": lambda: lib.srp_map_nyquist(
                h, xi.data_ptr(), bad, fp32, map_out.data_ptr(), peaks_out.data_ptr(), None),
            "srp_map_conventional": lambda: lib.srp_map_conventional(
                h, psi.data_ptr(), bad, fp32, map_out.data_ptr(), peaks_out.data_ptr(), None),
            "srp_map_nyquist_cached": lambda: lib.srp_map_nyquist_cached(
                h, weights.data_ptr(), xi_b.data_ptr(), bad, bf16, map_out.data_ptr(),
                peaks_out.data_ptr(), None),
            "srp_map_nyquist_points": lambda: lib.srp_map_nyquist_points(
                h, xi.data_ptr(), bad, points.data_ptr(), 2, values_out.data_ptr(), None),
        }
        for name, call in calls.items():
            st = call()
            assert st == S.SRP_ERR_INVALID_ARG, (name, bad, st)
    torch.cuda.synchronize()
    for t in (psi_out, xi_out, lowp_out, map_out, values_out):
        assert bool((t == sentinel).all())
    assert bool((peaks_out == 7).all())
    g.close()
