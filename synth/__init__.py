"""Seeded synthetic hyperspectral cubes with mixed noise.

This module is the only code shared by the FP64 oracle and the GPU path:
it draws inputs and holds none of the denoiser's arithmetic.

Shapes follow the paper's m x n x p cube (height x width x bands); arrays are
returned band-major, ``(b, h, w)`` with ``w`` fastest, which is the layout the
GPU library consumes.

Clean cube: ``R`` Voronoi regions (sites uniform on the pixel plane, nearest
site by Euclidean distance, ties to the lowest index); each region carries a
spectrum that is a sum of three Gaussians in the band index, min-max
normalised to [0, 1].  The result is piecewise constant in space and smooth
along the spectrum, the structure the paper's regulariser models (sparse and
low-rank gradient maps, Sec. III-A).

Noise follows the simulated cases of the paper's Sec. IV-B: zero-mean
Gaussian noise whose stated level is the standard deviation (the paper's
noisy-PSNR column of Table I is 20.0 dB at level 0.1, which only a standard
deviation gives), vertical stripes (a constant offset on random columns of
some bands) and salt-and-pepper pixels (set to 0 or 1).  Order: Gaussian,
then stripes, then impulses (impulses overwrite).  Nothing is clipped.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class NoiseSpec:
    sigma_lo: float            # per-band Gaussian std drawn from U[lo, hi]
    sigma_hi: float
    impulse: float             # fraction of salt-and-pepper pixels per band
    stripe_band_frac: float    # fraction of bands carrying stripes
    stripe_amp: float = 0.25   # stripe offsets ~ U[-amp, amp]


@dataclasses.dataclass(frozen=True)
class CubeSpec:
    h: int
    w: int
    b: int
    regions: int
    noise: NoiseSpec
    seed: int


def voronoi_labels(h: int, w: int, regions: int, rng: np.random.Generator) -> np.ndarray:
    """Label every pixel with its nearest Voronoi site (ties -> lowest index)."""
    sites = rng.uniform(0.0, 1.0, size=(regions, 2)) * np.array([h, w], dtype=np.float64)
    ii, jj = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64),
                         indexing="ij")
    d2 = (ii[None] - sites[:, 0, None, None]) ** 2 + (jj[None] - sites[:, 1, None, None]) ** 2
    return np.argmin(d2, axis=0)  # argmin returns the first (lowest) index on ties


def gaussian_mixture_spectra(b: int, regions: int, rng: np.random.Generator) -> np.ndarray:
    """(regions, b) spectra: sum of 3 Gaussians in the band index, each min-max normalised."""
    j = np.arange(b, dtype=np.float64)
    out = np.empty((regions, b))
    for r in range(regions):
        c = rng.uniform(0.0, b, size=3)
        s = rng.uniform(b / 20.0, b / 4.0, size=3)
        a = rng.uniform(0.2, 1.0, size=3)
        spec = (a[:, None] * np.exp(-((j[None] - c[:, None]) ** 2) / (2.0 * s[:, None] ** 2))).sum(0)
        lo, hi = spec.min(), spec.max()
        out[r] = (spec - lo) / (hi - lo) if hi > lo else np.zeros(b)
    return out


def clean_cube(h: int, w: int, b: int, regions: int, rng: np.random.Generator) -> np.ndarray:
    labels = voronoi_labels(h, w, regions, rng)
    spectra = gaussian_mixture_spectra(b, regions, rng)
    return np.ascontiguousarray(spectra[labels].transpose(2, 0, 1))  # (b, h, w)


def add_noise(clean: np.ndarray, noise: NoiseSpec, rng: np.random.Generator) -> np.ndarray:
    b, h, w = clean.shape
    noisy = clean.copy()
    sig = rng.uniform(noise.sigma_lo, noise.sigma_hi, size=b)
    noisy += sig[:, None, None] * rng.standard_normal((b, h, w))
    if noise.stripe_band_frac > 0:
        nb = int(round(noise.stripe_band_frac * b))
        bands = rng.choice(b, size=nb, replace=False)
        lo, hi = math.ceil(0.1 * w), math.ceil(0.2 * w)
        for j in np.sort(bands):
            ncol = int(rng.integers(lo, hi + 1))
            cols = rng.choice(w, size=ncol, replace=False)
            noisy[j][:, cols] += rng.uniform(-noise.stripe_amp, noise.stripe_amp, size=ncol)[None, :]
    if noise.impulse > 0:
        mask = rng.uniform(size=(b, h, w)) < noise.impulse
        salt = rng.uniform(size=(b, h, w)) < 0.5
        noisy[mask] = salt[mask].astype(np.float64)
    return noisy


def make_cube(spec: CubeSpec) -> Tuple[np.ndarray, np.ndarray]:
    """Return (clean, noisy), both float64 of shape (b, h, w)."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    clean = clean_cube(spec.h, spec.w, spec.b, spec.regions, rng)
    noisy = add_noise(clean, spec.noise, rng)
    return clean, noisy


# --- the workloads -----------------------------------------------------------

NOISE_SMALL = NoiseSpec(0.05, 0.15, 0.10, 0.0)        # 32x32x16 case
NOISE_MIXED = NoiseSpec(0.10, 0.20, 0.15, 0.30)       # 200x200x160, 256x256x191, ragged batch
NOISE_DIFF = NoiseSpec(0.15, 0.15, 0.10, 0.0)         # 8 x 64x64x32 differentiation batch


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    cubes: Tuple[CubeSpec, ...]
    iters: int


def workload(name: str, seed: Optional[int] = None) -> Workload:
    """Named workloads (sizes, noise mixes and iteration counts)."""
    if name == "small":         # 32x32x16, 20 iterations
        s = 1 if seed is None else seed
        return Workload(name, (CubeSpec(32, 32, 16, 12, NOISE_SMALL, s),), 20)
    if name == "pavia":         # 200x200x160, 50 iterations
        s = 1 if seed is None else seed
        return Workload(name, (CubeSpec(200, 200, 160, 60, NOISE_MIXED, s),), 50)
    if name == "wdc":           # 256x256x191, 50 iterations
        s = 1 if seed is None else seed
        return Workload(name, (CubeSpec(256, 256, 191, 60, NOISE_MIXED, s),), 50)
    if name == "diff":          # 8 x 64x64x32, 10 unrolled iterations
        base = 100 if seed is None else seed
        return Workload(name, tuple(CubeSpec(64, 64, 32, 20, NOISE_DIFF, base + i)
                                    for i in range(8)), 10)
    if name == "ragged":        # 32 cubes, h,w ~ U[48,160], b ~ U[31,191], 30 iterations
        s = 5 if seed is None else seed
        rng = np.random.Generator(np.random.PCG64(s))
        hs = rng.integers(48, 161, size=32)
        ws = rng.integers(48, 161, size=32)
        bs = rng.integers(31, 192, size=32)
        return Workload(name, tuple(CubeSpec(int(hs[i]), int(ws[i]), int(bs[i]), 60, NOISE_MIXED,
                                             1000 * s + i) for i in range(32)), 30)
    raise KeyError(name)


def random_state(b: int, h: int, w: int, seed: int, scale: float = 1.0) -> dict:
    """A seeded, arbitrary ADMM state (for one-step parity tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    def cube():
        return scale * rng.standard_normal((b, h, w))
    def trip():
        return np.stack([cube() for _ in range(3)])
    return {"Z": cube(), "S": cube(), "G1": cube(), "G2": cube(),
            "F": trip(), "E": trip(), "G3": trip(), "G4": trip()}
