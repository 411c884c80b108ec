"""Seeded synthetic inputs for the FDAS hot path.

This module is shared by the tests, the benchmark and the oracle's checks. It
holds the input recipe only (noise, injected accelerated sinusoids, candidate
perturbations) and none of the search's own arithmetic.

Recipe (mirrors the SKA-like configuration of the paper's Results section:
600 s at 64 us sampling, DM trials at full and 2x/4x decimated resolution,
193 acceleration trials):

* Noise: float64 N(0, sd) from ``numpy.random.default_rng(SeedSequence([cfg_seed,
  series_index]))``.
* Injection: ``a * cos(2*pi*(r0*u + z*u**2/2) + phi)`` with ``u = n/N``, evaluated
  in float64 and added to the noise before the cast to float32.  ``r0`` is the
  start-of-observation frequency in Fourier bins and ``z = fdot*T**2`` the drift
  in bins, so the mean frequency of the injection is ``r0 + z/2``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

TSAMP = 64e-6  # s, the paper's SKA-like sampling time


@dataclasses.dataclass
class Injection:
    amp: float
    r0: float      # start frequency in bins
    z: float       # drift over the observation in bins
    phase: float

    @property
    def r_mean(self) -> float:
        return self.r0 + 0.5 * self.z


def rng_for(cfg_seed: int, series_index: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg_seed), int(series_index)]))


def chirp(n: int, inj: Injection) -> np.ndarray:
    """The injected accelerated sinusoid, float64."""
    u = np.arange(n, dtype=np.float64) / n
    return inj.amp * np.cos(2.0 * np.pi * (inj.r0 * u + 0.5 * inj.z * u * u) + inj.phase)


def make_series(n: int, injections: Sequence[Injection], cfg_seed: int, series_index: int,
                noise_sd: float = 1.0) -> np.ndarray:
    """Gaussian noise plus injections, cast to float32 after adding in float64."""
    x = np.zeros(n, dtype=np.float64)
    if noise_sd > 0:
        x += noise_sd * rng_for(cfg_seed, series_index).standard_normal(n)
    for inj in injections:
        x += chirp(n, inj)
    return x.astype(np.float32)


def make_series_device(n: int, injections: Sequence[Injection], cfg_seed: int, series_index: int,
                       noise_sd: float = 1.0, device: str = "cuda", chunk: int = 64):
    """Same recipe as make_series (same noise bits, FP64 sum, one cast), with
    the injections evaluated on a torch device; returns a float32 tensor there.
    For series carrying thousands of injections."""
    import torch
    x = torch.zeros(n, dtype=torch.float64, device=device)
    if noise_sd > 0:
        x += torch.from_numpy(noise_sd * rng_for(cfg_seed, series_index).standard_normal(n)).to(device)
    u = torch.arange(n, dtype=torch.float64, device=device) / n
    for i in range(0, len(injections), chunk):
        part = injections[i:i + chunk]
        a = torch.tensor([j.amp for j in part], dtype=torch.float64, device=device)
        r0 = torch.tensor([j.r0 for j in part], dtype=torch.float64, device=device)
        z = torch.tensor([j.z for j in part], dtype=torch.float64, device=device)
        ph = torch.tensor([j.phase for j in part], dtype=torch.float64, device=device)
        for k in range(len(part)):
            x += a[k] * torch.cos(2.0 * np.pi * (r0[k] * u + 0.5 * z[k] * u * u) + ph[k])
    return x.to(torch.float32)


# ---------------------------------------------------------------- configurations

def small_case(seed: int = 1, noise: bool = True):
    """N=2^17, 64 us sampling, one injection a=0.05 at r0=5000 with z=+20.

    Search grid: z in [-16, 16] step 2 (17 templates), segment 2048 bins, median
    normalisation, harmonic sums 1/2/4.
    """
    n = 1 << 17
    ph = float(rng_for(seed, 10_000).uniform(0, 2 * np.pi))
    inj = [Injection(0.05, 5000.0, 20.0, ph)]
    x = make_series(n, inj, seed, 0, noise_sd=1.0 if noise else 0.0)
    params = dict(n_samples=n, tsamp=TSAMP, z_min=-16.0, z_max=16.0, z_step=2.0,
                  n_harmonics=4, segment_len=2048, norm="median")
    return x, inj, params


def draw_injections(rng: np.random.Generator, k: int, n: int, amp=(0.01, 0.05),
                    r_lo=1e4, r_hi=4e6, z_abs=90.0, min_sep=300.0) -> List[Injection]:
    out: List[Injection] = []
    r_hi = min(r_hi, 0.45 * n)
    tries = 0
    while len(out) < k:
        tries += 1
        if tries > 10_000:
            raise RuntimeError("could not place injections")
        r0 = float(rng.uniform(r_lo, r_hi))
        if any(abs(r0 - o.r0) < min_sep for o in out):
            continue
        out.append(Injection(float(rng.uniform(*amp)), r0, float(rng.uniform(-z_abs, z_abs)),
                             float(rng.uniform(0, 2 * np.pi))))
    return out


def ska_single(seed: int = 2, n: int = 1 << 23, n_inj: int = 8):
    """One full-resolution SKA-like series: N=2^23 (536.9 s at 64 us), 8 injections
    with amplitude 0.01-0.05, r in [1e4, 4e6], z in [-90, 90]; 193 templates over
    z in [-96, 96] step 1, segment 8192 bins."""
    rng = rng_for(seed, 20_000)
    inj = draw_injections(rng, n_inj, n)
    x = make_series(n, inj, seed, 0)
    params = dict(n_samples=n, tsamp=TSAMP, z_min=-96.0, z_max=96.0, z_step=1.0,
                  n_harmonics=16, segment_len=8192, norm="median")
    return x, inj, params


def batch_layout(counts_by_len: Sequence[tuple]) -> List[int]:
    """Series lengths for a batch, longest first: [(n, count), ...]."""
    lens: List[int] = []
    for n, c in counts_by_len:
        lens += [int(n)] * int(c)
    return lens


def batch_series(lengths: Sequence[int], seed: int, inj_per_series=(0, 2),
                 amp=(0.01, 0.05), z_abs=90.0, scale_decimated=True):
    """Seeded uneven batch: each series is N(0,1) noise plus 0-2 injections.

    A series ``d`` times shorter than the longest stands for a ``d``-fold
    decimated DM trial; its injection amplitude is scaled by sqrt(d), which is
    what block-averaging by ``d`` does to a sinusoid's signal-to-noise ratio.
    """
    nmax = max(lengths)
    xs, truths = [], []
    for i, n in enumerate(lengths):
        rng = rng_for(seed, 30_000 + i)
        k = int(rng.integers(inj_per_series[0], inj_per_series[1] + 1))
        inj = draw_injections(rng, k, n, amp=amp, z_abs=z_abs) if k else []
        if scale_decimated:
            d = nmax // n
            for j in inj:
                j.amp *= math.sqrt(d)
        xs.append(make_series(n, inj, seed, i))
        truths.append(inj)
    return xs, truths


def batch_injections(lengths: Sequence[int], seed: int, inj_per_series=(0, 2), amp=(0.01, 0.05), z_abs=90.0,
                     scale_decimated=True) -> List[List[Injection]]:
    """The injections batch_series would draw, without generating the noise."""
    nmax = max(lengths)
    truths = []
    for i, n in enumerate(lengths):
        rng = rng_for(seed, 30_000 + i)
        k = int(rng.integers(inj_per_series[0], inj_per_series[1] + 1))
        inj = draw_injections(rng, k, n, amp=amp, z_abs=z_abs) if k else []
        if scale_decimated:
            d = nmax // n
            for j in inj:
                j.amp *= math.sqrt(d)
        truths.append(inj)
    return truths


def ska_full(seed: int = 5, n: int = 1 << 23, counts=(3050, 1500, 1375), frac: float = 0.01,
             amp=(0.01, 0.05), z_abs=96.0):
    """The full SKA-like run: 5925 DM trials (3050 at N, 1500 at N/2 and 1375
    at N/4 samples); a seeded 1 % of them (59) carry one injection each, with
    amplitude U[0.01, 0.05] scaled by sqrt(decimation) and z in U[-96, 96].
    Returns (lengths, injections per trial)."""
    lens = [n] * counts[0] + [n // 2] * counts[1] + [n // 4] * counts[2]
    rng = rng_for(seed, 50_000)
    chosen = rng.choice(len(lens), int(round(frac * len(lens))), replace=False)
    truths: List[List[Injection]] = [[] for _ in lens]
    for i in sorted(int(c) for c in chosen):
        inj = draw_injections(rng_for(seed, 50_001 + i), 1, lens[i], amp=amp, z_abs=z_abs)
        for j in inj:
            j.amp *= math.sqrt(n // lens[i])
        truths[i] = inj
    return lens, truths


def fill_series_device(out, injections: Sequence[Injection], cfg_seed: int, series_index: int):
    """Large-batch variant of make_series for benchmarks: the N(0,1) noise comes
    from torch's device generator seeded with (cfg_seed, series_index) instead
    of numpy's, the injections are added in float64, and the sum is cast into
    the float32 device tensor ``out``."""
    import torch
    n = out.numel()
    g = torch.Generator(device=out.device)
    g.manual_seed(int(np.random.SeedSequence([cfg_seed, series_index]).generate_state(1, np.uint64)[0]) & ((1 << 63) - 1))
    x = torch.randn(n, dtype=torch.float64, device=out.device, generator=g)
    u = torch.arange(n, dtype=torch.float64, device=out.device) / n
    for j in injections:
        x += j.amp * torch.cos(2.0 * np.pi * (j.r0 * u + 0.5 * j.z * u * u) + j.phase)
    out.copy_(x.to(torch.float32))


def concat(xs: Sequence[np.ndarray]):
    lengths = np.array([len(x) for x in xs], dtype=np.int64)
    offsets = np.zeros(len(xs), dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)[:-1]
    return np.concatenate(xs).astype(np.float32), offsets, lengths


def refine_candidates(seed: int, n_cand: int, r_first=1e4, r_gap=500.0, z_abs=90.0,
                      amp=(0.02, 0.05), dr=0.5, dz=1.0):
    """Truths at r_mean = r_first + r_gap*i + U(0,1), z ~ U[-z_abs, z_abs], and
    starting points perturbed by U(-dr, dr) bins and U(-dz, dz) in z."""
    rng = rng_for(seed, 40_000)
    truths, starts = [], []
    for i in range(n_cand):
        rm = r_first + r_gap * i + float(rng.uniform(0, 1))
        z = float(rng.uniform(-z_abs, z_abs))
        a = float(rng.uniform(*amp))
        ph = float(rng.uniform(0, 2 * np.pi))
        truths.append(Injection(a, rm - 0.5 * z, z, ph))
        starts.append((rm + float(rng.uniform(-dr, dr)), z + float(rng.uniform(-dz, dz))))
    return truths, np.array(starts, dtype=np.float64)
