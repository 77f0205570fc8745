"""Seeded synthetic inputs for SRP mapping.

This module only *generates inputs*: microphone and candidate geometry and
multichannel microphone frames. It holds none of the SRP method's arithmetic
(no spectra, PHAT, GCC, TDOA tables, interpolation or maps), so both the CPU
oracle's tests and the GPU path may consume what it produces.

Signal model (free field, no reflections): every source emits seeded white
Gaussian noise; microphone m receives, for every source s, the source signal
delayed by r_sm / c and attenuated by 1 / r_sm, where r_sm is the
source-to-microphone distance. The fractional delay is applied as a phase
ramp exp(-j 2 pi f tau) on a zero-padded spectrum of the whole signal, which
is then trimmed, so no circular wrap reaches the kept samples. Independent
white sensor noise is added per microphone at a stated SNR (mean signal
power over microphones divided by noise power). Frames are consecutive,
non-overlapping L-sample blocks; windowing is part of the method, not of the
input.

These stand in for the paper's reverberant speech-and-babble scenes (its
Section 4), whose corpus, noise recordings and room simulator are not
available here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SPEED_OF_SOUND = 343.0


@dataclasses.dataclass
class Grid:
    """Cell-centred Cartesian grid: q = origin + (idx + 1/2) * h.

    Candidate index i = (iz * ny + iy) * nx + ix (x fastest).
    """
    origin: tuple
    h: float
    shape: tuple  # (nx, ny, nz)

    @property
    def J(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def points(self, start: int = 0, stop: Optional[int] = None) -> np.ndarray:
        """Candidate coordinates [n][3] float64 for indices start..stop-1."""
        stop = self.J if stop is None else stop
        idx = np.arange(start, stop, dtype=np.int64)
        return self.points_at(idx)

    def points_at(self, idx: np.ndarray) -> np.ndarray:
        nx, ny, _ = self.shape
        idx = np.asarray(idx, dtype=np.int64)
        ix = idx % nx
        iy = (idx // nx) % ny
        iz = idx // (nx * ny)
        o = np.asarray(self.origin, dtype=np.float64)
        pts = np.empty((idx.size, 3), dtype=np.float64)
        pts[:, 0] = o[0] + (ix + 0.5) * self.h
        pts[:, 1] = o[1] + (iy + 0.5) * self.h
        pts[:, 2] = o[2] + (iz + 0.5) * self.h
        return pts

    def index_of(self, xyz) -> int:
        """Index of the cell containing xyz (clipped to the grid)."""
        o = np.asarray(self.origin, dtype=np.float64)
        rel = (np.asarray(xyz, dtype=np.float64) - o) / self.h
        ijk = np.clip(np.floor(rel).astype(np.int64), 0, np.asarray(self.shape) - 1)
        nx, ny, _ = self.shape
        return int((ijk[2] * ny + ijk[1]) * nx + ijk[0])


def cell_grid(lo, hi, h) -> Grid:
    """Cell-centred grid covering the box [lo, hi] with cell size h.

    A dimension with lo == hi gives one layer at that coordinate.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    shape = []
    origin = []
    for d in range(3):
        ext = hi[d] - lo[d]
        if ext <= 0.0:
            shape.append(1)
            origin.append(lo[d] - 0.5 * h)
        else:
            shape.append(max(1, int(round(ext / h))))
            origin.append(lo[d])
    return Grid(origin=tuple(origin), h=float(h), shape=tuple(shape))


@dataclasses.dataclass
class Workload:
    """One synthetic SRP workload (geometry + frames + design parameters)."""
    name: str
    mic_xyz: np.ndarray          # [M][3] float64, metres
    grid: Optional[Grid]         # near-field candidate grid (None for far field)
    fs: float
    L: int
    F: int
    c: float
    n_aux: int
    field: str = "near"          # "near" | "far"
    directions: Optional[np.ndarray] = None  # [J][3] unit vectors (far field)
    sources: Optional[np.ndarray] = None     # [S][3] true source positions
    snr_db: float = 20.0
    seed: int = 0
    frames: Optional[np.ndarray] = None      # [F][M][L] float32
    f_max: Optional[float] = None            # band limit, default fs/2

    @property
    def M(self) -> int:
        return int(self.mic_xyz.shape[0])

    @property
    def P(self) -> int:
        return self.M * (self.M - 1) // 2

    @property
    def J(self) -> int:
        if self.field == "far":
            return int(self.directions.shape[0])
        return self.grid.J

    @property
    def band_limit(self) -> float:
        return self.fs / 2.0 if self.f_max is None else self.f_max

    def candidates(self, start: int = 0, stop: Optional[int] = None) -> np.ndarray:
        if self.field == "far":
            stop = self.J if stop is None else stop
            return np.ascontiguousarray(self.directions[start:stop])
        return self.grid.points(start, stop)

    def candidates_at(self, idx) -> np.ndarray:
        if self.field == "far":
            return np.ascontiguousarray(self.directions[np.asarray(idx)])
        return self.grid.points_at(np.asarray(idx))


def _streams(seed: int, n: int = 4):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def uniform_box(rng, n, centre, size) -> np.ndarray:
    centre = np.asarray(centre, dtype=np.float64)
    size = np.asarray(size, dtype=np.float64)
    return centre + (rng.random((n, 3)) - 0.5) * size


def uniform_circular_array(M: int, radius: float, centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """M microphones equally spaced on a horizontal circle (the paper's array shape)."""
    phi = 2.0 * np.pi * np.arange(M) / M
    c = np.asarray(centre, dtype=np.float64)
    return np.stack([c[0] + radius * np.cos(phi), c[1] + radius * np.sin(phi),
                     np.full(M, c[2])], axis=1)


def half_sphere_directions(step_deg: float = 2.0) -> np.ndarray:
    """Far-field candidate grid of the paper's Section 4 (lower half sphere).

    Polar angle theta from 90 to 180 degrees and azimuth phi from 0 to
    360 - step degrees, both in `step` increments, with
    r = -(sin t cos p, sin t sin p, cos t). All azimuths at the pole
    theta = 180 give the same direction and are kept once. With 2-degree
    steps this is 45 * 180 + 1 = 8101 directions.
    """
    n_theta = int(round(90.0 / step_deg)) + 1
    n_phi = int(round(360.0 / step_deg))
    dirs = []
    for it in range(n_theta):
        th = math.radians(90.0 + it * step_deg)
        if it == n_theta - 1:
            phis = [0.0]
        else:
            phis = [math.radians(ip * step_deg) for ip in range(n_phi)]
        for ph in phis:
            dirs.append((-math.sin(th) * math.cos(ph), -math.sin(th) * math.sin(ph),
                         -math.cos(th)))
    d = np.asarray(dirs, dtype=np.float64)
    # pole: cos(180 deg) is -1 and sin is ~1e-16; make it exactly (0, 0, 1)
    d[-1] = (0.0, 0.0, 1.0)
    return d


def place_sources(rng, n, room_lo, room_hi, array_centre, margin=0.5, min_dist=1.0,
                  plane_z: Optional[float] = None) -> np.ndarray:
    """Uniform source positions with a wall margin and a minimum array distance."""
    lo = np.asarray(room_lo, dtype=np.float64) + margin
    hi = np.asarray(room_hi, dtype=np.float64) - margin
    out = []
    while len(out) < n:
        q = lo + rng.random(3) * (hi - lo)
        if plane_z is not None:
            q[2] = plane_z
        if np.linalg.norm(q - np.asarray(array_centre)) >= min_dist:
            out.append(q)
    return np.asarray(out)


def synth_frames(mic_xyz, sources, fs, L, F, c, snr_db, rng_sig, rng_noise,
                 field="near") -> np.ndarray:
    """Free-field multichannel white-noise frames [F][M][L] float32.

    For field == "far", `sources` holds unit propagation directions r
    (pointing from the source towards the array) and the delay at mic m is
    p_m . r / c, with unit gain.
    """
    mic = np.asarray(mic_xyz, dtype=np.float64)
    M = mic.shape[0]
    n_keep = F * L
    if field == "far":
        delays = (mic @ np.asarray(sources, dtype=np.float64).T).T / c     # [S][M]
        gains = np.ones_like(delays)
    else:
        r = np.linalg.norm(mic[None, :, :] - np.asarray(sources)[:, None, :], axis=2)  # [S][M]
        delays = r / c
        gains = 1.0 / r
    dmin = float(np.floor(delays.min() * fs)) - 2.0
    dmax = float(np.ceil(delays.max() * fs)) + 2.0
    pad = int(max(64.0, dmax - dmin + 64.0))
    n_src = n_keep + 2 * pad
    n_fft = 1 << int(math.ceil(math.log2(n_src + pad)))
    freqs = np.fft.rfftfreq(n_fft, d=1.0 / fs)
    out = np.zeros((M, n_keep), dtype=np.float64)
    for s in range(delays.shape[0]):
        src = rng_sig.standard_normal(n_src)
        spec = np.fft.rfft(src, n_fft)
        for m in range(M):
            tau = delays[s, m] - dmin / fs  # >= 2 samples, < pad
            sh = np.fft.irfft(spec * np.exp(-2j * np.pi * freqs * tau), n_fft)
            out[m] += gains[s, m] * sh[pad:pad + n_keep]
    p_sig = float(np.mean(out ** 2))
    p_noise = p_sig / (10.0 ** (snr_db / 10.0))
    out += np.sqrt(p_noise) * rng_noise.standard_normal(out.shape)
    frames = out.reshape(M, F, L).transpose(1, 0, 2)
    return np.ascontiguousarray(frames, dtype=np.float32)



def hemisphere_direction(rng, n: int) -> np.ndarray:
    """n propagation directions uniform over the half sphere r_z >= 0 that the
    far-field candidate grid covers (uniform r_z and azimuth give a uniform
    density on the sphere), generally between grid points."""
    z = rng.random(n)
    ph = 2.0 * np.pi * rng.random(n)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)


def _sphere_directions(rng, n: int) -> np.ndarray:
    z = 2.0 * rng.random(n) - 1.0
    ph = 2.0 * np.pi * rng.random(n)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)


def synth_far_scene(mic_xyz, direction, fs, L, F, c, snr_db, rng, t60: float = 0.6,
                    drr_db: float = 0.0, n_refl: int = 64, noise: str = "diffuse"):
    """Far-field scene [F][M][L] float32 closer to a reverberant room with
    diffuse noise than `synth_frames`.

    * Direct path: seeded white noise arriving along the unit propagation
      direction `direction` (delay p_m . r / c, unit gain).
    * Late reverberation: `n_refl` copies of the same signal from directions
      uniform over the whole sphere, each with an extra delay uniform in
      [2 ms, T60 / 2] and a Gaussian amplitude under the exponential envelope
      exp(-3 ln(10) t / T60); their total energy is set so that
      direct / reverberant energy is `drr_db`.
    * Noise (`noise` = "diffuse"): a spherically isotropic field, made per
      frequency by mixing independent white spectra with a square-root factor
      of the coherence matrix sinc(2 f d_mm' / c) (normalised sinc), as in the
      usual method for generating sensor signals in isotropic noise fields;
      "white" gives independent sensor noise instead. Scaled to `snr_db`
      against the mean reverberant-signal power.

    With a sequence of SNRs the same signal and noise are mixed at each one
    and a list of frame arrays is returned.
    """
    mic = np.asarray(mic_xyz, dtype=np.float64)
    M = mic.shape[0]
    n_keep = F * L
    u0 = np.asarray(direction, dtype=np.float64).reshape(3)
    ext = rng.uniform(0.002, 0.5 * t60, n_refl)
    amp = rng.standard_normal(n_refl) * np.exp(-3.0 * math.log(10.0) * ext / t60)
    amp *= math.sqrt(10.0 ** (-drr_db / 10.0) / float(np.sum(amp * amp)))
    dirs = _sphere_directions(rng, n_refl)
    tau = np.concatenate([(mic @ u0)[None, :] / c, ext[:, None] + (dirs @ mic.T) / c])  # [1+R][M]
    gain = np.concatenate([[1.0], amp])
    tau = tau - tau.min() + 2.0 / fs
    pad = int(math.ceil(tau.max() * fs)) + 64
    n_src = n_keep + pad
    n_fft = 1 << int(math.ceil(math.log2(n_src + 64)))
    freqs = np.fft.rfftfreq(n_fft, d=1.0 / fs)
    spec = np.fft.rfft(rng.standard_normal(n_src), n_fft)
    out = np.empty((M, n_keep), dtype=np.float64)
    for m in range(M):
        h = gain @ np.exp(-2j * np.pi * tau[:, m:m + 1] * freqs[None, :])
        out[m] = np.fft.irfft(spec * h, n_fft)[pad:pad + n_keep]
    p_sig = float(np.mean(out ** 2))
    if noise == "diffuse":
        d = np.linalg.norm(mic[:, None, :] - mic[None, :, :], axis=2)
        gamma = np.sinc(2.0 * freqs[:, None, None] * d[None, :, :] / c)
        lam, vec = np.linalg.eigh(gamma)
        fac = vec * np.sqrt(np.clip(lam, 0.0, None))[:, None, :]
        white = rng.standard_normal((freqs.size, M)) + 1j * rng.standard_normal((freqs.size, M))
        nspec = np.einsum("fmk,fk->mf", fac, white)
        nz = np.fft.irfft(nspec, n_fft, axis=1)[:, :n_keep]
    elif noise == "white":
        nz = rng.standard_normal((M, n_keep))
    else:
        raise ValueError(f"unknown noise {noise!r}")
    nz *= 1.0 / math.sqrt(float(np.mean(nz ** 2)))

    def mix(snr):
        fr = (out + math.sqrt(p_sig / (10.0 ** (snr / 10.0))) * nz).reshape(M, F, L)
        return np.ascontiguousarray(fr.transpose(1, 0, 2), dtype=np.float32)

    if np.ndim(snr_db) == 0:
        return mix(float(snr_db))
    return [mix(float(snr)) for snr in snr_db]

CONFIG_NAMES = {
    1: "cfg1-plain-4mic-2500cand",
    2: "cfg2-room-16mic-576kcand-500fr",
    3: "cfg3-precision-32mic-4Mcand-200fr",
    4: "cfg4-serving-64arrays",
    5: "cfg5-largest-64mic-9Mcand-100fr",
}


def make(cfg: int, *, frames: bool = True, n_aux: int = 2, F: Optional[int] = None,
         seed: Optional[int] = None) -> Workload:
    """Build one of the single-array workloads (1, 2, 3 or 5).

    `F` overrides the frame count (e.g. a smaller test batch); `seed`
    overrides the default seed (= config number).
    """
    seed = cfg if seed is None else seed
    g_rng, s_rng, sig_rng, n_rng = _streams(seed)
    if cfg == 1:
        centre = np.array([1.5, 1.5, 1.5])
        half = 0.1
        mic = centre + np.array([[-half, -half, 0.0], [half, -half, 0.0],
                                 [half, half, 0.0], [-half, half, 0.0]])
        grid = cell_grid((0.0, 0.0, 1.5), (3.0, 3.0, 1.5), 0.06)
        srcs = place_sources(s_rng, 1, (0.0, 0.0, 1.5), (3.0, 3.0, 1.5), centre, plane_z=1.5)
        fs, L, Fd, snr = 16000.0, 1024, 10, 20.0
    elif cfg == 2:
        centre = np.array([3.0, 2.0, 1.5])
        mic = uniform_box(g_rng, 16, centre, (1.0, 1.0, 0.5))
        grid = cell_grid((0.0, 0.0, 0.0), (6.0, 4.0, 3.0), 0.05)
        n_s = int(s_rng.integers(1, 3))
        srcs = place_sources(s_rng, n_s, (0.0, 0.0, 0.0), (6.0, 4.0, 3.0), centre)
        fs, L, Fd, snr = 16000.0, 1024, 500, 10.0
    elif cfg == 3:
        centre = np.array([2.0, 2.0, 1.0])
        mic = uniform_box(g_rng, 32, centre, (1.0, 1.0, 0.5))
        grid = cell_grid((0.0, 0.0, 0.0), (4.0, 4.0, 2.0), 0.02)
        n_s = int(s_rng.integers(1, 3))
        srcs = place_sources(s_rng, n_s, (0.0, 0.0, 0.0), (4.0, 4.0, 2.0), centre)
        fs, L, Fd, snr = 16000.0, 2048, 200, 10.0
    elif cfg == 5:
        centre = np.array([3.0, 2.0, 1.5])
        mic = uniform_box(g_rng, 64, centre, (2.0, 2.0, 1.0))
        grid = cell_grid((0.0, 0.0, 0.0), (6.0, 4.0, 3.0), 0.02)
        srcs = place_sources(s_rng, 3, (0.0, 0.0, 0.0), (6.0, 4.0, 3.0), centre)
        fs, L, Fd, snr = 48000.0, 4096, 100, 5.0
    else:
        raise ValueError(f"single-array config must be 1, 2, 3 or 5, not {cfg}")
    Fn = Fd if F is None else int(F)
    wl = Workload(name=CONFIG_NAMES[cfg], mic_xyz=mic, grid=grid, fs=fs, L=L, F=Fn,
                  c=SPEED_OF_SOUND, n_aux=n_aux, sources=srcs, snr_db=snr, seed=seed)
    if frames:
        wl.frames = synth_frames(mic, srcs, fs, L, Fn, wl.c, snr, sig_rng, n_rng)
    return wl


def make_custom(M: int, J_shape=(8, 6, 5), h=0.1, fs=16000.0, L=256, F=4, n_aux=2,
                box=(0.4, 0.4, 0.2), snr_db=20.0, seed=0, n_src=1,
                f_max: Optional[float] = None) -> Workload:
    """A small random workload for tests: M mics in a box centred in a grid volume."""
    g_rng, s_rng, sig_rng, n_rng = _streams(seed)
    nx, ny, nz = J_shape
    size = np.array([nx * h, ny * h, nz * h])
    centre = size / 2.0
    mic = uniform_box(g_rng, M, centre, box)
    grid = Grid(origin=(0.0, 0.0, 0.0), h=h, shape=tuple(J_shape))
    srcs = centre + (s_rng.random((n_src, 3)) - 0.5) * size * 0.8
    wl = Workload(name=f"custom-M{M}-J{grid.J}-L{L}-F{F}", mic_xyz=mic, grid=grid, fs=fs,
                  L=L, F=F, c=SPEED_OF_SOUND, n_aux=n_aux, sources=srcs, snr_db=snr_db,
                  seed=seed, f_max=f_max)
    wl.frames = synth_frames(mic, srcs, fs, L, F, wl.c, snr_db, sig_rng, n_rng)
    return wl


def make_far_field(M: int = 6, radius: float = 0.1, L: int = 2048, F: int = 4, n_aux: int = 2,
                   c: float = 340.0, fs: float = 16000.0, snr_db: float = 10.0, seed: int = 11,
                   step_deg: float = 2.0) -> Workload:
    """Stand-in for the paper's Section 4 setup: UCA, far-field half-sphere grid.

    The array (radius 10 cm, 6 mics, horizontal) sits at the origin; the
    source is a seeded direction from the candidate set, with white noise
    instead of speech and white sensor noise instead of babble.
    """
    _, s_rng, sig_rng, n_rng = _streams(seed)
    mic = uniform_circular_array(M, radius)
    dirs = half_sphere_directions(step_deg)
    src_idx = int(s_rng.integers(0, dirs.shape[0]))
    srcs = dirs[src_idx:src_idx + 1]
    wl = Workload(name=f"farfield-uca{M}-J{dirs.shape[0]}", mic_xyz=mic, grid=None, fs=fs,
                  L=L, F=F, c=c, n_aux=n_aux, field="far", directions=dirs, sources=srcs,
                  snr_db=snr_db, seed=seed)
    wl.frames = synth_frames(mic, srcs, fs, L, F, c, snr_db, sig_rng, n_rng, field="far")
    return wl


def serving_arrays(n_arrays: int = 64, seed: int = 4, j_lo: float = 1e4, j_hi: float = 2e6,
                   mic_counts=(4, 8, 16, 32)):
    """Array descriptions of the serving workload (64 arrays of mixed size).

    Returns a list of dicts with mic_xyz, grid and a source position; J is
    drawn log-uniform in [j_lo, j_hi] and realised as a cell-centred grid in
    a 6 x 4 x 3 m room with h = (72 / J)^(1/3).
    """
    g_rng, s_rng, _, _ = _streams(seed)
    out = []
    for a in range(n_arrays):
        M = int(mic_counts[int(g_rng.integers(0, len(mic_counts)))])
        centre = np.array([3.0, 2.0, 1.5])
        mic = uniform_box(g_rng, M, centre, (1.0, 1.0, 0.5))
        J_target = math.exp(g_rng.uniform(math.log(j_lo), math.log(j_hi)))
        h = (72.0 / J_target) ** (1.0 / 3.0)
        grid = cell_grid((0.0, 0.0, 0.0), (6.0, 4.0, 3.0), h)
        src = place_sources(s_rng, 1, (0.0, 0.0, 0.0), (6.0, 4.0, 3.0), centre)
        out.append({"id": a, "mic_xyz": mic, "grid": grid, "source": src})
    return out
