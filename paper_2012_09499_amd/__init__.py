"""MI355X-native steered response power (SRP) maps: conventional SRP-PHAT and the
Nyquist-Shannon approximation of Dietzen, De Sena and van Waterschoot (WASPAA 2021).

All computation runs in libsrp.so (hand-written HIP kernels for gfx950,
include/srp.h); this package is its thin Python binding plus a frame
pipeline helper.
"""
from ._lib import (DTYPES, EXPORTS, Geometry, SrpError, argmax, cross_spectra, decode_peaks,  # noqa: F401
                   SRP_OK, SRP_ERR_INVALID_ARG, SRP_ERR_OUT_OF_MEMORY, SRP_ERR_DEVICE,
                   SRP_ERR_UNSUPPORTED, conventional_supports, cross_spectra_noalloc,
                   batched_workspace_bytes, gcc_samples, gcc_samples_frames, lib, map_conventional, map_nyquist,
                   map_nyquist_batched, map_nyquist_cached, map_nyquist_points, nyquist_weights,
                   spectra_lowp, spectra_lowp_buffer,
                   nyquist_weights_bytes, pair_layout, sample_torch_dtype, unpack_samples,
                   version)
from .pipeline import SrpPipeline  # noqa: F401
from .refine import refine_peaks  # noqa: F401
