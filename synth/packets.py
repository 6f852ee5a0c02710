"""Synthetic IQ packet generator (tissue + motion + vessels + noise).

Recipe (all draws from ``numpy.random.default_rng`` on PCG64):

* Speckle: i.i.d. CN(0, 1) scatterers smoothed by a separable 3x3 PSF built
  from [1, 2, 1] and scaled to unit energy (sum of squares 1), so every
  speckle field has unit mean power per pixel.
* Tissue: one speckle field on a depth-padded grid (16 px each side), scaled
  to ``tissue_db`` above blood, zero inside vessels. Axial motion
  d(t) = A sin(2 pi f t / PRF + phi), f = 2 Hz, PRF = 500 Hz (the phantom
  shaker and frame rate of the Experimental Studies section), applied per frame
  as a band-limited Fourier shift along depth on the padded grid, then cropped.
* Blood: horizontal vessels |y - y_c| <= r, each filled with its own speckle
  strip (0 dB) advected laterally by v px/frame with a Fourier shift along x on
  a strip long enough that wrapped content only enters from outside the view.
* Noise: i.i.d. CN(0, 10^(noise_db/10)) per pixel and frame (-10 dB re blood).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

_PAD = 16


@dataclass(frozen=True)
class PacketSpec:
    ny: int
    nx: int
    nt: int
    tissue_db: float
    motion_px: float
    tubes: tuple = field(default_factory=tuple)  # ((y_center, radius, v_px_per_frame), ...)
    noise_db: float = -10.0
    motion_hz: float = 2.0
    prf_hz: float = 500.0
    seed: int = 0


def _psf() -> np.ndarray:
    h1 = np.array([1.0, 2.0, 1.0])
    h = np.outer(h1, h1)
    return h / math.sqrt(float(np.sum(h * h)))


def _speckle(rng: np.random.Generator, shape) -> np.ndarray:
    """Unit-power complex speckle: CN(0,1) scatterers * 3x3 PSF (periodic)."""
    z = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)
    h = _psf()
    out = np.zeros(shape, dtype=np.complex128)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            out += h[dy + 1, dx + 1] * np.roll(np.roll(z, dy, axis=0), dx, axis=1)
    return out


def tube_mask(spec: PacketSpec) -> np.ndarray:
    y = np.arange(spec.ny)[:, None]
    m = np.zeros((spec.ny, spec.nx), dtype=bool)
    for (yc, r, _v) in spec.tubes:
        m |= np.broadcast_to(np.abs(y - yc) <= r, (spec.ny, spec.nx))
    return m


def make_packet(spec: PacketSpec):
    """Return (iq complex64 [nt][ny][nx], vessel mask bool [ny][nx])."""
    rng = np.random.default_rng(np.random.PCG64(spec.seed))
    ny, nx, nt = spec.ny, spec.nx, spec.nt
    t = np.arange(nt, dtype=np.float64)
    mask = tube_mask(spec)

    # Tissue with axial sub-pixel motion.
    ly = ny + 2 * _PAD
    tissue0 = _speckle(rng, (ly, nx)) * 10.0 ** (spec.tissue_db / 20.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    disp = spec.motion_px * np.sin(2.0 * math.pi * spec.motion_hz * t / spec.prf_hz + phi)
    ky = np.fft.fftfreq(ly)
    spec_t = np.fft.fft(tissue0, axis=0)
    frames = np.empty((nt, ny, nx), dtype=np.complex128)
    for i in range(nt):
        shifted = np.fft.ifft(spec_t * np.exp(-2j * math.pi * ky * disp[i])[:, None], axis=0)
        frames[i] = shifted[_PAD:_PAD + ny]
    frames *= ~mask

    # Vessels: laterally advected speckle strips.
    for (yc, r, v) in spec.tubes:
        y0, y1 = max(0, yc - r), min(ny - 1, yc + r)
        rows = y1 - y0 + 1
        if rows <= 0:
            continue
        lx = nx + _PAD + int(math.ceil(abs(v) * nt)) + _PAD
        strip = _speckle(rng, (rows + 2, lx))[1:-1]
        kx = np.fft.fftfreq(lx)
        sf = np.fft.fft(strip, axis=1)
        for i in range(nt):
            moved = np.fft.ifft(sf * np.exp(-2j * math.pi * kx * (v * t[i]))[None, :], axis=1)
            frames[i, y0:y1 + 1, :] += moved[:, _PAD:_PAD + nx]

    # White noise.
    sn = math.sqrt(10.0 ** (spec.noise_db / 10.0) / 2.0)
    frames += sn * (rng.standard_normal(frames.shape) + 1j * rng.standard_normal(frames.shape))
    return np.ascontiguousarray(frames.astype(np.complex64)), mask


def _draw_tubes(rng: np.random.Generator, ny: int, n: int, rmin: int, rmax: int,
                vmin: float, vmax: float):
    """n vessels with radii in [rmin, rmax], speeds in [vmin, vmax] and
    non-overlapping depth bands (3 px gap), kept 8 px away from the edges."""
    tubes = []
    for _ in range(1000):
        if len(tubes) == n:
            break
        r = int(rng.integers(rmin, rmax + 1))
        yc = int(rng.integers(8 + r, ny - 8 - r))
        if all(abs(yc - y2) > r + r2 + 3 for (y2, r2, _v) in tubes):
            tubes.append((yc, r, float(rng.uniform(vmin, vmax))))
    return tuple(sorted(tubes))


def spec_small(seed: int = 0) -> PacketSpec:
    """64 x 64 x 32, tissue 50 dB, 0.2 px motion, two r=4 vessels at 0.5 px/frame."""
    return PacketSpec(64, 64, 32, 50.0, 0.2, ((21, 4, 0.5), (42, 4, 0.5)), seed=seed)


def spec_clinical(p: int = 0, tissue_db: float = 50.0, seed_base: int = 1000,
                  ny: int = 256, nx: int = 192, nt: int = 128) -> PacketSpec:
    """256 x 192 x 128, motion U(0,1) px, six vessels r in 2..6, v in U(0.05, 1)."""
    seed = seed_base + p
    rng = np.random.default_rng(np.random.PCG64([seed, 1]))
    amp = float(rng.uniform(0.0, 1.0))
    tubes = _draw_tubes(rng, ny, 6, 2, 6, 0.05, 1.0)
    return PacketSpec(ny, nx, nt, tissue_db, amp, tubes, seed=seed)


def spec_precision(p: int = 0) -> PacketSpec:
    """The clinical shape with tissue 60 dB above blood."""
    return spec_clinical(p, tissue_db=60.0, seed_base=2000)


def spec_learned(seed: int) -> PacketSpec:
    """512 x 256 x 128, tissue U(40, 60) dB, motion U(0, 1) px, 6-12 vessels."""
    rng = np.random.default_rng(np.random.PCG64([seed, 1]))
    tdb = float(rng.uniform(40.0, 60.0))
    amp = float(rng.uniform(0.0, 1.0))
    n = int(rng.integers(6, 13))
    tubes = _draw_tubes(rng, 512, n, 2, 6, 0.05, 1.0)
    return PacketSpec(512, 256, 128, tdb, amp, tubes, seed=seed)


def batch_specs(list_seed: int = 3000, n: int = 64):
    """Uneven stream: Nt in {32, 64, 100, 200} (n/4 each, shuffled), Ny in
    U{128..400}, Nx in U{128..256}, square window grids g in U{2..10}.
    Returns a list of (PacketSpec, g)."""
    rng = np.random.default_rng(np.random.PCG64([list_seed, 2]))
    nts = np.repeat(np.array([32, 64, 100, 200]), max(1, n // 4))[:n]
    rng.shuffle(nts)
    out = []
    for p in range(n):
        ny = int(rng.integers(128, 401))
        nx = int(rng.integers(128, 257))
        g = int(rng.integers(2, 11))
        amp = float(rng.uniform(0.0, 1.0))
        tubes = _draw_tubes(rng, ny, 6, 2, 6, 0.05, 1.0)
        out.append((PacketSpec(ny, nx, int(nts[p]), 50.0, amp, tubes, seed=list_seed + p), g))
    return out

