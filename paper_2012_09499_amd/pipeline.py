"""Frame-batch pipeline over the C ABI with preallocated device buffers.

Nyquist path: srp_gcc_samples_frames (FFT, PHAT phasors and GCC samples,
the cross-spectra formed on chip) -> srp_map_nyquist.
Conventional path: srp_cross_spectra -> srp_map_conventional (BF16/FP16:
srp_cross_spectra -> srp_spectra_lowp -> srp_map_conventional).
Every step is a libsrp kernel; buffers are torch tensors allocated once.
The map and peaks returned by `nyquist` and `conventional` are views of the
pipeline's own buffers: the next call overwrites them, so copy a result out
before running the other path on the same pipeline.
"""
from __future__ import annotations

from . import _lib as S


class SrpPipeline:
    def __init__(self, geom: S.Geometry, F: int, device="cuda", keep_map: bool = False):
        import torch
        self.g = geom
        self.F = int(F)
        self.workspace = torch.empty(geom.workspace_bytes(F), dtype=torch.uint8, device=device)
        self.psi = torch.empty((F, geom.P, geom.K), dtype=torch.complex64, device=device)
        self.device = device
        self.xi = torch.empty((F, geom.S), dtype=torch.float32, device=device)
        self._xi_lowp = {}
        self._spec_lowp = {}
        self.peaks = torch.empty((F, 2), dtype=torch.int64, device=device)
        self.map = (torch.empty((F, geom.J), dtype=torch.float32, device=device)
                    if keep_map else None)

    def spectra(self, frames):
        return S.cross_spectra(self.g, frames, out=self.psi[:frames.shape[0]],
                               workspace=self.workspace)

    def samples_buffer(self, dtype: str):
        import torch
        if S.sample_torch_dtype(dtype) == torch.float32:
            return self.xi
        if dtype not in self._xi_lowp:
            self._xi_lowp[dtype] = torch.empty((self.F, self.g.S),
                                               dtype=S.sample_torch_dtype(dtype),
                                               device=self.device)
        return self._xi_lowp[dtype]

    def nyquist(self, frames, dtype: str = "fp32", weights=None):
        """Nyquist map of a frame batch; with `weights` (from nyquist_weights for
        this geometry and dtype) the map reads the cached weights instead of
        forming them."""
        F = frames.shape[0]
        xi = S.gcc_samples_frames(self.g, frames, out=self.samples_buffer(dtype)[:F],
                                  dtype=dtype, workspace=self.workspace)
        if weights is not None:
            return S.map_nyquist_cached(self.g, weights, xi, dtype=dtype,
                                        want_map=self.map is not None,
                                        map_out=None if self.map is None else self.map[:F],
                                        peaks_out=self.peaks[:F])
        return S.map_nyquist(self.g, xi, dtype=dtype, want_map=self.map is not None,
                             map_out=None if self.map is None else self.map[:F],
                             peaks_out=self.peaks[:F])

    def conventional(self, frames, dtype: str = "fp32"):
        F = frames.shape[0]
        psi = self.spectra(frames)
        if dtype in ("bf16", "fp16"):
            if dtype not in self._spec_lowp:
                self._spec_lowp[dtype] = S.spectra_lowp_buffer(self.g, self.F, dtype,
                                                               self.device)
            psi = S.spectra_lowp(self.g, psi, dtype, out=self._spec_lowp[dtype][:F])
        return S.map_conventional(self.g, psi, dtype=dtype, want_map=self.map is not None,
                                  map_out=None if self.map is None else self.map[:F],
                                  peaks_out=self.peaks[:F])
