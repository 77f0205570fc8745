"""Refined spatial search from one set of GCC samples.

The Nyquist approximation defines SRP_appr as a continuous function of the
candidate position (Eq. SRPapprox evaluated at dt_p(q) for any q), so the peak
of a coarse map can be refined without new spectra or samples: around the
current best point of every frame, evaluate a small local lattice whose
spacing shrinks by `factor` per level (srp_map_nyquist_points), keep its
maximum (srp_argmax), repeat. The paper mentions such refined searches as a
possible combination beyond its scope (Section 1, Section 3.3); here they are
an option on top of srp_map_nyquist.

Near field: a (2 r + 1)^3 lattice of positions, spacing h / factor^level.
Far field: a (2 r + 1)^2 patch of directions in (polar, azimuth) angle,
spacing step / factor^level, mapped to unit vectors with the candidate grid's
convention r = -(sin t cos p, sin t sin p, cos t).
Every lattice contains its centre, so the value never decreases from one
level to the next.
"""
from __future__ import annotations

import math

import numpy as np

from . import _lib as S


def _lattice(radius: int, dims: int) -> np.ndarray:
    r = np.arange(-radius, radius + 1, dtype=np.float64)
    grids = np.meshgrid(*([r] * dims), indexing="ij")
    return np.stack([gd.ravel() for gd in grids], axis=1)


def _angles(d: np.ndarray):
    # inverse of r = -(sin t cos p, sin t sin p, cos t)
    t = np.arccos(np.clip(-d[..., 2], -1.0, 1.0))
    p = np.arctan2(-d[..., 1], -d[..., 0])
    return t, p


def _direction(t, p):
    st = np.sin(t)
    return -np.stack([st * np.cos(p), st * np.sin(p), np.cos(t)], axis=-1)


def refine_peaks(g: S.Geometry, xi, start, *, spacing: float, levels: int = 2,
                 factor: int = 3, radius: int = 1, stream=None):
    """Refines per-frame peaks on successively finer local lattices.

    g: the geometry the samples belong to; xi: [F][S] float32 CUDA samples
    (srp_gcc_samples, fp32); start: [F][3] float64 starting points (e.g. the
    coarse map's argmax candidates); spacing: the coarse grid's spacing in
    metres (near field) or radians (far field).
    Returns (points [F][3] float64, values [F] float64), both numpy.
    """
    import torch
    cur = np.array(start, dtype=np.float64, copy=True).reshape(-1, 3)
    F = cur.shape[0]
    if xi.shape[0] != F:
        raise ValueError("start must hold one point per frame of xi")
    far = g.field == "far"
    offs = _lattice(radius, 2 if far else 3)
    Q = offs.shape[0]
    vals = np.full(F, -np.inf)
    peaks = torch.empty((F, 2), dtype=torch.int64, device=xi.device)
    for level in range(1, levels + 1):
        h = spacing / float(factor) ** level
        if far:
            t, p = _angles(cur)
            tt = t[:, None] + h * offs[None, :, 0]
            pp = p[:, None] + h * offs[None, :, 1]
            pts = _direction(tt, pp)
        else:
            pts = cur[:, None, :] + h * offs[None, :, :]
        dev_pts = torch.from_numpy(np.ascontiguousarray(pts)).to(xi.device)
        v = S.map_nyquist_points(g, xi, dev_pts, stream=stream)
        S.argmax(v, peaks_out=peaks, stream=stream)
        idx, val = S.decode_peaks(peaks)
        cur = pts[np.arange(F), idx]
        vals = np.asarray(val, dtype=np.float64)
    return cur, vals


def grid_spacing_far(step_deg: float) -> float:
    return math.radians(step_deg)
