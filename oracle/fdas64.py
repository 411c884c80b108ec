"""Plain FP64 CPU reference for the FDAS hot path.

TEST INFRASTRUCTURE ONLY.  This module exists to check the HIP library; it is
imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the CPU-baseline
leg of ``bench.py`` and by nothing else.  It shares no code, tables or
constants with ``paper_2211_13517_amd`` and never imports it.  It is written
for obviousness, not speed: every step is the definition of the quantity,
evaluated in float64 with numpy/scipy primitives (FFT, Fresnel integrals,
incomplete gamma) and no blocking or reordering beyond what the definition
states.

What the paper fixes and what is read into it
----------------------------------------------
The paper (section 2.1, "FDAS") describes the Fourier Domain Acceleration
Search as a matched filter against templates of constant acceleration, whose
cost grows linearly with the number of acceleration trials; section 2.2
("Mixed-Precision") says the search convolves in the frequency domain with
FFTs and that the convolution stage is the costly part; section 3 ("Results")
gives the SKA-like workload (600 s at 64 us, 5925 DM trials, 193 acceleration
trials).  It prints no formulas.  The formulas below are derived from first
principles for that statement of the method; each place where a choice had to
be made is marked READING and is listed with its justification in the design
notes of the repository.

Notation
--------
``N`` samples, ``T = N*tsamp``.  Fourier bin ``r`` (frequency r/T), drift
``z = fdot*T^2`` (bins over the observation).  ``A_r`` the spectrum,
``B_r = N/2`` bins.  ``rho(q, z)`` the response of bin ``rbar+q`` to a signal
whose mean frequency is ``rbar`` and whose drift is ``z``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.special as sps

LN2 = math.log(2.0)

# --------------------------------------------------------------------- spectrum


def spectrum(x: np.ndarray) -> np.ndarray:
    """Complex spectrum of a real series, bins 0..N/2-1 (section 2.2: the search
    works on the Fourier transform of the time series).

    A_r = sum_n x_n exp(-2 pi i r n / N), r < N/2.  The Nyquist bin is dropped so
    that a series of N samples gives N/2 bins, and A_0 is set to zero because it
    carries only the mean of the series (READING: DC zeroed).
    """
    x = np.asarray(x)
    n = x.shape[-1]
    if n % 2:
        raise ValueError("series length must be even")
    a = np.fft.rfft(x.astype(np.float64))[..., : n // 2].copy()
    a[..., 0] = 0.0
    return a


# ---------------------------------------------------------------- normalisation


def block_lower_median(p: np.ndarray, block: int) -> np.ndarray:
    """Lower median (0-based rank (B-1)//2 after sorting) of each block of B
    consecutive values."""
    if p.shape[-1] % block:
        raise ValueError("block must divide the number of bins")
    pb = p.reshape(-1, block)
    k = (block - 1) // 2
    return np.partition(pb, k, axis=1)[:, k]


def normalise(a: np.ndarray, mode: str, block: int = 2048, noise_var: float = 1.0,
              n_samples: Optional[int] = None, return_medians: bool = False):
    """Spectrum normalisation so that pure noise has unit mean power.

    * ``none``: unchanged.
    * ``variance``: A / sqrt(N sigma^2); white noise of variance sigma^2 then has
      E|A'|^2 = 1 (used for closed-form checks).
    * ``median`` (READING of "power normalised by the local median"): blocks of B
      bins; m_b is the lower median of |A|^2 in the block; A' = A sqrt(ln2/m_b).
      The median of an Exp(1) variable is ln 2, so noise powers become Exp(1).
      A block whose median is zero is scaled by zero.
    * ``rednoise`` (READING: whitening of a red-noise continuum ahead of the
      search, which the paper leaves implicit): as ``median``, but the block
      of B bins starting at bin s = b B is cut into equal sub-blocks of
      width rednoise_width(b, B) = clamp(largest power of two <= s/8, 32, B),
      each scaled by its own lower median.  A block is then at most an
      eighth of its frequency wide, so a power law f^-2 varies by at most
      (9/8)^2 across it; from bin 8 B on the blocks are whole.
    """
    a = np.asarray(a, dtype=np.complex128)
    if mode == "none":
        return (a, None) if return_medians else a
    if mode == "variance":
        n = n_samples if n_samples is not None else 2 * a.shape[-1]
        out = a / math.sqrt(n * noise_var)
        return (out, None) if return_medians else out
    if mode not in ("median", "rednoise"):
        raise ValueError(mode)
    p = a.real ** 2 + a.imag ** 2
    if mode == "median":
        med = block_lower_median(p, block)
        scale = np.where(med > 0, np.sqrt(LN2 / np.where(med > 0, med, 1.0)), 0.0)
        out = (a.reshape(-1, block) * scale[:, None]).reshape(a.shape)
        return (out, med) if return_medians else out
    out = np.empty_like(a)
    meds = []
    for b in range(a.shape[-1] // block):
        w = rednoise_width(b, block)
        seg = slice(b * block, (b + 1) * block)
        med = block_lower_median(p[seg], w)
        scale = np.where(med > 0, np.sqrt(LN2 / np.where(med > 0, med, 1.0)), 0.0)
        out[seg] = (a[seg].reshape(-1, w) * scale[:, None]).reshape(-1)
        meds.append(med)
    return (out, meds) if return_medians else out


def rednoise_width(b: int, block: int) -> int:
    """Sub-block width inside block b of the rednoise normalisation: the
    largest power of two <= b*block/8, kept within [32, block]."""
    s8 = b * block // 8
    w = 1 << (s8.bit_length() - 1) if s8 > 0 else 1
    return int(min(max(w, 32), block))


# ------------------------------------------------------------------- z grid


def z_grid(z_min: float, z_max: float, z_step: float) -> np.ndarray:
    """Acceleration trials z_j = z_min + j*dz, j = 0..Z-1 (section 2.1: one
    template per acceleration value)."""
    nz = int(round((z_max - z_min) / z_step)) + 1
    return z_min + z_step * np.arange(nz, dtype=np.float64)


def half_width(z, margin: int = 16):
    """Template half-width h(z) = ceil(|z|/2) + m in bins (READING).

    A signal drifting by z bins sweeps |z|/2 bins either side of its mean
    frequency; the margin m keeps the sinc-like skirts of the response."""
    return np.ceil(np.abs(np.asarray(z, dtype=np.float64)) / 2.0).astype(np.int64) + int(margin)


# ------------------------------------------------------------ Fresnel response

_Z_QUAD = 1e-2  # below this |z| the response is integrated numerically
# Below this |z| the derivatives are integrated numerically: the closed forms
# divide by z twice, which magnifies the ~1e-13 error of the Fresnel integrals
# at large argument by (q/z)^2 (5e-8 at z = 0.04, q = 15; 4e-13 at z = 2).
_Z_DQUAD = 2.0


def _gauss_legendre_01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _quad_nodes(q, z) -> int:
    cyc = float(np.max(np.abs(q))) + 0.5 * float(np.max(np.abs(z))) + 1.0
    return int(4 * math.ceil(cyc)) + 96


def response_quadrature(q, z, weight: str = "1") -> np.ndarray:
    """Gauss-Legendre quadrature of the defining integral

        rho(q, z) = int_0^1 exp(-2 pi i q u + i pi z (u - 1/2)^2) du

    optionally with an extra factor (u - 1/2) ("v") or (u - 1/2)^2 ("v2") or u ("u").
    Node count grows with the number of oscillations so the rule is converged
    to rounding."""
    q, z = np.broadcast_arrays(np.asarray(q, dtype=np.float64), np.asarray(z, dtype=np.float64))
    if q.size == 0:
        return np.zeros(q.shape, np.complex128)
    u, w = _gauss_legendre_01(_quad_nodes(q, z))
    qf, zf = q.reshape(-1, 1), z.reshape(-1, 1)
    ph = -2.0 * np.pi * qf * u + np.pi * zf * (u - 0.5) ** 2
    f = np.exp(1j * ph)
    if weight == "v":
        f = f * (u - 0.5)
    elif weight == "v2":
        f = f * (u - 0.5) ** 2
    elif weight == "u":
        f = f * u
    return (f @ w).reshape(q.shape)


def _fresnel_F(x):
    s, c = sps.fresnel(x)
    return c + 1j * s


def response(q, z) -> np.ndarray:
    """rho(q, z), the normalised DFT response of an accelerated sinusoid.

    Derivation (READING, first principles for the matched filter of section
    2.1): a sinusoid a cos(2 pi (r0 u + z u^2/2) + phi), u = t/T, has
    instantaneous frequency r0 + z u bins and mean frequency rbar = r0 + z/2.
    Its DFT at bin rbar + q is (N a / 2) e^{i theta} rho(q, z) with

        rho(q, z) = int_0^1 exp(-2 pi i q u + i pi z (u - 1/2)^2) du
                  = e^{-i pi q} R(q, z),
        R(q, z)   = int_{-1/2}^{1/2} exp(-2 pi i q v + i pi z v^2) dv.

    Completing the square for z > 0 with F(x) = C(x) + i S(x) (Fresnel
    integrals, int_0^x exp(i pi t^2 / 2) dt):

        R = exp(-i pi q^2 / z) / sqrt(2 z) [F(y+) - F(y-)],
        y+- = sqrt(2/z) (+-z/2 - q),

    R(q, -z) = conj R(-q, z) for z < 0, and for |z| below 1e-2 the integral is
    evaluated by quadrature (which at z = 0 gives sinc q).
    """
    q, z = np.broadcast_arrays(np.asarray(q, dtype=np.float64), np.asarray(z, dtype=np.float64))
    out = np.empty(q.shape, dtype=np.complex128)
    small = np.abs(z) < _Z_QUAD
    if np.any(small):
        out[small] = response_quadrature(q[small], z[small])
    big = ~small
    if np.any(big):
        qb, zb = q[big], z[big]
        neg = zb < 0
        qq = np.where(neg, -qb, qb)
        za = np.abs(zb)
        s = np.sqrt(2.0 / za)
        yp = s * (0.5 * za - qq)
        ym = s * (-0.5 * za - qq)
        r = np.exp(-1j * np.pi * qq * qq / za) / np.sqrt(2.0 * za) * (_fresnel_F(yp) - _fresnel_F(ym))
        r = np.where(neg, np.conj(r), r)
        out[big] = np.exp(-1j * np.pi * qb) * r
    return out


def response_derivatives(q, z) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """rho and its partial derivatives d rho/dq and d rho/dz.

    With phi(u) = -2 pi q u + pi z (u - 1/2)^2, integration by parts of
    phi'(u) e^{i phi} gives, for z != 0,

        I1 = int (u - 1/2) e^{i phi} du = (q rho + (e1 - e0)/(2 pi i)) / z
        I2 = int (u - 1/2)^2 e^{i phi} du = (q I1 + ((e1 + e0)/2 - rho)/(2 pi i)) / z

    with e0 = e^{i phi(0)}, e1 = e^{i phi(1)}; then d rho/dq = -2 pi i (I1 + rho/2)
    and d rho/dz = i pi I2.  |z| < 2 uses quadrature of the defining integrals
    (d rho/dq = -2 pi i int u e^{i phi}, d rho/dz = i pi int (u-1/2)^2 e^{i phi}).
    """
    q, z = np.broadcast_arrays(np.asarray(q, dtype=np.float64), np.asarray(z, dtype=np.float64))
    rho = response(q, z)
    dq = np.empty_like(rho)
    dz = np.empty_like(rho)
    small = np.abs(z) < _Z_DQUAD
    if np.any(small):
        qs, zs = q[small], z[small]
        dq[small] = -2j * np.pi * response_quadrature(qs, zs, "u")
        dz[small] = 1j * np.pi * response_quadrature(qs, zs, "v2")
    big = ~small
    if np.any(big):
        qb, zb, rb = q[big], z[big], rho[big]
        e0 = np.exp(1j * np.pi * zb / 4.0)
        e1 = np.exp(1j * (-2.0 * np.pi * qb + np.pi * zb / 4.0))
        i1 = (qb * rb + (e1 - e0) / (2j * np.pi)) / zb
        i2 = (qb * i1 + (0.5 * (e1 + e0) - rb) / (2j * np.pi)) / zb
        dq[big] = -2j * np.pi * (i1 + 0.5 * rb)
        dz[big] = 1j * np.pi * i2
    return rho, dq, dz


# -------------------------------------------------------------------- templates


def template_taps(zs: Sequence[float], margin: int = 16) -> Tuple[np.ndarray, int]:
    """Matched-filter taps for every acceleration trial (section 2.1).

    t_q(z) = conj(rho(q, z)) / sqrt(E(z)) for |q| <= h(z), else 0, with
    E(z) = sum_{|q|<=h(z)} |rho(q, z)|^2 (READING: unit-energy templates keep
    the noise power at mean 1 on every z row).  Returned as [Z][2 h_max + 1],
    column q + h_max, with h_max = h(max |z|).
    """
    zs = np.asarray(zs, dtype=np.float64)
    hz = half_width(zs, margin)
    hmax = int(hz.max())
    q = np.arange(-hmax, hmax + 1, dtype=np.float64)
    rho = response(q[None, :], zs[:, None])
    mask = np.abs(q)[None, :] <= hz[:, None]
    rho = np.where(mask, rho, 0.0)
    energy = np.sum(np.abs(rho) ** 2, axis=1)
    taps = np.conj(rho) / np.sqrt(energy)[:, None]
    return taps, hmax


def template_energy(zs, margin: int = 16) -> np.ndarray:
    zs = np.asarray(zs, dtype=np.float64)
    hz = half_width(zs, margin)
    out = np.empty(zs.shape)
    for i, (z, h) in enumerate(zip(zs.ravel(), hz.ravel())):
        q = np.arange(-h, h + 1, dtype=np.float64)
        out.flat[i] = np.sum(np.abs(response(q, z)) ** 2)
    return out


# ------------------------------------------------------------------ correlation


def correlate_direct(a: np.ndarray, taps_row: np.ndarray, r: np.ndarray) -> np.ndarray:
    """y(r) = sum_{q=-h}^{h} A_{r+q} t_q with A_k = 0 outside [0, len(A)), evaluated
    term by term at the bins ``r`` (the definition of the matched-filter output)."""
    h = (len(taps_row) - 1) // 2
    r = np.asarray(r, dtype=np.int64)
    k = r[:, None] + np.arange(-h, h + 1)[None, :]
    valid = (k >= 0) & (k < len(a))
    ak = np.where(valid, a[np.clip(k, 0, len(a) - 1)], 0.0)
    return ak @ taps_row


def correlate(a: np.ndarray, taps_row: np.ndarray) -> np.ndarray:
    """Same correlation for every bin, computed as one zero-padded full-length FFT
    product (section 2.2: convolution in the frequency domain).  Deliberately no
    overlap-save segmentation: the GPU segments, the oracle does not."""
    a = np.asarray(a, dtype=np.complex128)
    h = (len(taps_row) - 1) // 2
    n = len(a)
    nfft = 1 << int(math.ceil(math.log2(n + 2 * h + 1)))
    rev = taps_row[::-1]
    full = np.fft.ifft(np.fft.fft(a, nfft) * np.fft.fft(rev, nfft))
    return full[h: h + n]


def correlate_cyclic(a: np.ndarray, taps_full: np.ndarray) -> np.ndarray:
    """Cyclic correlation y_r = sum_q A_{(r+q) mod n} c_q over all n offsets q
    (``taps_full[q mod n] = c_q``).  With c' the reversed taps, y = A (*) c' and
    FFT(c') = conj(FFT(conj c))."""
    a = np.asarray(a, dtype=np.complex128)
    return np.fft.ifft(np.fft.fft(a) * np.conj(np.fft.fft(np.conj(taps_full))))


def power_plane(a_norm: np.ndarray, zs: Sequence[float], margin: int = 16,
                rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """P[j][r] = |y_j(r)|^2 for every acceleration trial z_j and bin r: the
    z-major power plane of the matched filter (section 2.1)."""
    taps, _ = template_taps(zs, margin)
    rows = range(len(zs)) if rows is None else rows
    out = np.empty((len(rows), len(a_norm)), dtype=np.float64)
    for i, j in enumerate(rows):
        y = correlate(a_norm, taps[j])
        out[i] = y.real ** 2 + y.imag ** 2
    return out


def interbin_plane(a_norm: np.ndarray, zs: Sequence[float], margin: int = 16,
                   rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """The power plane at half-bin resolution (interbinning; READING, the paper
    is silent): column 2r holds P[j][r] = |y_j(r)|^2 and column 2r + 1 the
    half-bin power |y_j(r) - y_j(r + 1)|^2 / 2, with y_j(N/2) taken from the
    spectrum extended by zeros like every other out-of-range bin.

    Why this value: the template autocorrelation sum_q rho(q + d, z) conj rho(q, z)
    is, by Parseval over u in [0, 1), the integral of exp(-2 pi i d u), i.e.
    exp(-i pi d) sinc(d) for every z.  So after the matched filter a signal at
    rbar leaves y(r) proportional to exp(-i pi (r - rbar)) sinc(r - rbar), and
    for rbar midway between r and r + 1 the two neighbours are (2/pi) of its
    amplitude with opposite signs: (pi/4)(y_r - y_{r+1}) recovers it.  The same
    autocorrelation vanishes at integer lags (sinc(1) = 0), so noise outputs of
    neighbouring bins are uncorrelated and E|y_r - y_{r+1}|^2 = 2; the factor
    8/pi^2 that brings noise back to unit mean turns (pi/4)^2 into 1/2.  A tone
    midway between bins then keeps 8/pi^2 = 0.81 of its power instead of
    sinc(1/2)^2 = 0.405."""
    taps, _ = template_taps(zs, margin)
    rows = range(len(zs)) if rows is None else rows
    a_ext = np.concatenate([np.asarray(a_norm, dtype=np.complex128), [0.0]])
    nb = len(a_norm)
    out = np.empty((len(rows), 2 * nb), dtype=np.float64)
    for i, j in enumerate(rows):
        y = correlate(a_ext, taps[j])        # bins 0 .. N/2
        d = y[:-1] - y[1:]
        out[i, 0::2] = y[:-1].real ** 2 + y[:-1].imag ** 2
        out[i, 1::2] = 0.5 * (d.real ** 2 + d.imag ** 2)
    return out


def power_cells(a_norm: np.ndarray, taps: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """P at individual cells (row j, bin r) by the direct sum, for sampled checks."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    out = np.empty(len(rows))
    for j in np.unique(rows):
        sel = rows == j
        y = correlate_direct(a_norm, taps[j], cols[sel])
        out[sel] = y.real ** 2 + y.imag ** 2
    return out


def interbin_cells(a_norm: np.ndarray, taps: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Columns of the half-bin plane (interbin_plane) at individual cells by the
    direct sum: column c = 2r is |y(r)|^2, c = 2r + 1 is |y(r) - y(r + 1)|^2 / 2."""
    rows = np.asarray(rows)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.empty(len(rows))
    for j in np.unique(rows):
        sel = rows == j
        r = cols[sel] // 2
        y0 = correlate_direct(a_norm, taps[j], r)
        y1 = correlate_direct(a_norm, taps[j], r + 1)
        d = y0 - y1
        out[sel] = np.where(cols[sel] % 2 == 0, y0.real ** 2 + y0.imag ** 2, 0.5 * (d.real ** 2 + d.imag ** 2))
    return out


# --------------------------------------------------------------- harmonic sum


def harmonic_terms(n_rows: int, n_bins: int, j0: int, n_harm: int):
    """Index maps of the nested, highest-harmonic-indexed harmonic sum (READING).

    A cell (R, j), with m = j - j0 the signed z index, holds the sum for a pulsar
    whose H-th harmonic sits at bin R and drift z_j: harmonic k of H lies at
    r_k = round_half_up(k R / H) and m_k = sgn(m) round_half_up(k |m| / H).
    Returns (rk, jk) for k = 1..n_harm against the top stage H = n_harm; the
    lower stages H' use the sub-terms k' = k H / H' (they coincide exactly)."""
    R = np.arange(n_bins, dtype=np.int64)
    m = np.arange(n_rows, dtype=np.int64) - j0
    H = n_harm
    ks = np.arange(1, H + 1, dtype=np.int64)
    rk = (2 * ks[:, None] * R[None, :] + H) // (2 * H)           # [k][R]
    mk = np.sign(m)[None, :] * ((2 * ks[:, None] * np.abs(m)[None, :] + H) // (2 * H))
    jk = j0 + mk                                                 # [k][j]
    return rk, jk


def harmonic_sums(plane: np.ndarray, j0: int, n_harm: int) -> Dict[int, np.ndarray]:
    """S_H(R, j) = sum_{k=1}^{H} P[j0 + m_k][r_k] for H = 1, 2, 4, ..., n_harm
    (incoherent harmonic summing; the paper cites GPU harmonic summing in its
    introduction)."""
    nz, nb = plane.shape
    rk, jk = harmonic_terms(nz, nb, j0, n_harm)
    terms = np.stack([plane[jk[k][:, None], rk[k][None, :]] for k in range(n_harm)])  # [k][j][R]
    out = {}
    H = 1
    while H <= n_harm:
        step = n_harm // H
        out[H] = terms[step - 1::step].sum(axis=0)
        H *= 2
    return out


def harmonic_sum_cells(plane: np.ndarray, j0: int, n_harm: int, rows: np.ndarray, cols: np.ndarray
                       ) -> Dict[int, np.ndarray]:
    """S_H at the cells (rows[i], cols[i]) only, for H = 1, 2, ..., n_harm: the
    same terms as harmonic_sums (harmonic k of the top stage at bin
    round_half_up(k R / n_harm) and trial j0 + sgn(m) round_half_up(k |m| / n_harm)),
    for planes too large to sum whole."""
    R = np.asarray(cols, dtype=np.int64)
    m = np.asarray(rows, dtype=np.int64) - j0
    H = n_harm
    terms = []
    for k in range(1, H + 1):
        rk = (2 * k * R + H) // (2 * H)
        mk = np.sign(m) * ((2 * k * np.abs(m) + H) // (2 * H))
        terms.append(plane[j0 + mk, rk].astype(np.float64))
    terms = np.stack(terms)                                      # [k][cell]
    out = {}
    h = 1
    while h <= H:
        step = H // h
        out[h] = terms[step - 1::step].sum(axis=0)
        h *= 2
    return out


def stages(n_harm: int) -> List[int]:
    return [1 << i for i in range(int(math.log2(n_harm)) + 1)]


# ------------------------------------------------------------- significance


def gauss_tail(sigma: float) -> float:
    """P(X > sigma) for X ~ N(0, 1)."""
    return 0.5 * math.erfc(sigma / math.sqrt(2.0))


def threshold(n_harm_stage: int, sigma: float = 6.0) -> float:
    """tau_H with P(Gamma(H, 1) > tau_H) = P(N(0,1) > sigma) (READING of "threshold at
    6 sigma": noise S_H is a sum of H unit-mean exponentials)."""
    return float(sps.gammainccinv(n_harm_stage, gauss_tail(sigma)))


def log_tail_gamma(s, h: int):
    """ln P(Gamma(h, 1) > s) = -s + ln sum_{k<h} s^k / k! (integer shape)."""
    s = np.asarray(s, dtype=np.float64)
    k = np.arange(h, dtype=np.float64)
    with np.errstate(divide="ignore"):
        terms = k[None, :] * np.log(np.maximum(s.reshape(-1, 1), 1e-300)) - sps.gammaln(k + 1.0)[None, :]
    return (-s.reshape(-1) + sps.logsumexp(terms, axis=1)).reshape(s.shape)


def gaussian_sigma(s, h: int):
    """Gaussian-equivalent significance of a harmonic sum S_H under noise."""
    return -sps.ndtri_exp(log_tail_gamma(s, h))


@dataclass
class Candidate:
    series: int
    harm: int
    R: int
    j: int
    r: float
    z: float
    power: float
    sigma: float


def best_stage(sums: Dict[int, np.ndarray], R: np.ndarray, n_bins: int, r_lo: int, h_max: int,
               sigma: float = 6.0):
    """The stage a cell reports: among the stages H searched at bin R
    (R >= H r_lo and R < n_bins - h_max) whose sum passes (S_H >= tau_H), the one
    with the smallest noise tail probability.  Works elementwise on arrays of
    sums (whole planes or lists of cells); returns (H or 0, ln tail)."""
    shape = next(iter(sums.values())).shape
    best_lq = np.full(shape, np.inf)
    best_h = np.zeros(shape, dtype=np.int64)
    for H, S in sums.items():
        tau = threshold(H, sigma)
        ok = (S >= tau) & (R >= H * r_lo) & (R < n_bins - h_max)
        if not np.any(ok):
            continue
        lq = np.full(shape, np.inf)
        lq[ok] = log_tail_gamma(S[ok], H)
        better = lq < best_lq
        best_lq = np.where(better, lq, best_lq)
        best_h = np.where(better, H, best_h)
    return best_h, best_lq


def search(plane: np.ndarray, zs: np.ndarray, n_harm: int, r_lo: int, h_max: int,
           sigma: float = 6.0, series: int = 0, res: int = 1) -> List[Candidate]:
    """Threshold the harmonic sums and emit at most one candidate per cell.

    Cell (R, j) is searched at stage H when R >= H r_lo and R < B_r - h_max;
    it passes when S_H >= tau_H.  Among passing stages the one with the smallest
    noise tail probability (largest Gaussian significance) is reported, with
    fundamental r = R/H and z = z_j/H.  With res = 2 the plane is the
    half-bin one (interbin_plane): R counts half bins, the limits are
    2 H r_lo and 2 (B_r - h_max), and r = R / (2 H) bins."""
    nz, nb = plane.shape
    j0 = int(np.argmin(np.abs(zs)))
    sums = harmonic_sums(plane, j0, n_harm)
    best_h, best_lq = best_stage(sums, np.arange(nb)[None, :], nb, res * r_lo, res * h_max, sigma)
    out = []
    jj, rr = np.nonzero(best_h)
    for j, R_ in zip(jj, rr):
        H = int(best_h[j, R_])
        S = float(sums[H][j, R_])
        out.append(Candidate(series, H, int(R_), int(j), R_ / (res * H), float(zs[j]) / H, S,
                             float(-sps.ndtri_exp(best_lq[j, R_]))))
    return out


def local_maxima(series: np.ndarray, R: np.ndarray, j: np.ndarray, sigma: np.ndarray,
                 radius_r: int = 2, radius_j: int = 2) -> np.ndarray:
    """Keep flags of candidate clustering (READING: the paper's pipeline ends
    at candidates; a standard sift keeps local maxima): record i survives when
    no record of its series with |R' - R| <= radius_r and |j' - j| <= radius_j
    has a larger sigma, equal sigmas going to the smaller (j, R).  Sorted
    lookups over the 8- or 24-cell neighbourhood (R < 2^23 holds half-bin
    cells too)."""
    series = np.asarray(series, np.int64)
    key = (series << 35) | (np.asarray(j, np.int64) << 23) | np.asarray(R, np.int64)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    ss = np.asarray(sigma)[order]
    keep = np.ones(len(ks), bool)
    Rs, js, sers = np.asarray(R, np.int64)[order], np.asarray(j, np.int64)[order], series[order]
    for dj in range(-radius_j, radius_j + 1):
        for dr in range(-radius_r, radius_r + 1):
            if dj == 0 and dr == 0:
                continue
            ok = (js + dj >= 0) & (Rs + dr >= 0) & (js + dj < (1 << 12)) & (Rs + dr < (1 << 23))
            nk = (sers << 35) | ((js + dj) << 23) | (Rs + dr)
            pos = np.minimum(np.searchsorted(ks, nk), len(ks) - 1)
            hit = ok & (ks[pos] == nk)
            beats = (ss[pos] > ss) | ((ss[pos] == ss) & (nk < ks))
            keep &= ~(hit & beats)
    out = np.zeros(len(ks), bool)
    out[order] = keep
    return out


# ---------------------------------------------------------------- refinement


def rz_window(r: float, z: float, margin: int = 16):
    """Bins used to interpolate the response at (r, z): k0 = floor(r),
    w = margin + ceil(|z|/2), k = k0-w+1 .. k0+w (READING: 32 bins at z = 0,
    widened so the drift span is always covered)."""
    k0 = int(math.floor(r))
    w = int(margin + math.ceil(abs(z) / 2.0))
    return np.arange(k0 - w + 1, k0 + w + 1, dtype=np.int64)


def _window_values(a, ks):
    valid = (ks >= 0) & (ks < len(a))
    return np.where(valid, a[np.clip(ks, 0, len(a) - 1)], 0.0)


def rz_amplitude(a: np.ndarray, r: float, z: float, margin: int = 16) -> complex:
    """Fourier-interpolated matched-filter output at off-grid (r, z):
    y(r, z) = sum_k A_k conj(rho(k - r, z)) over the window (no renormalisation)."""
    ks = rz_window(r, z, margin)
    ak = _window_values(a, ks)
    return complex(np.sum(ak * np.conj(response(ks - r, z))))


def rz_power(a, r, z, margin: int = 16) -> float:
    y = rz_amplitude(a, r, z, margin)
    return y.real ** 2 + y.imag ** 2


def rz_power_grad(a: np.ndarray, r: float, z: float, margin: int = 16):
    """P = |y|^2 with dP/dr, dP/dz and dP/dA_k (as d/dRe + i d/dIm) on the window.

    dy/dr = -sum A_k conj(d rho/dq), dy/dz = sum A_k conj(d rho/dz),
    dP/dx = 2 Re(conj(y) dy/dx), dP/dA_k = 2 y rho(k - r, z)."""
    ks = rz_window(r, z, margin)
    ak = _window_values(a, ks)
    rho, dq, dz = response_derivatives(ks - r, z)
    y = np.sum(ak * np.conj(rho))
    dydr = -np.sum(ak * np.conj(dq))
    dydz = np.sum(ak * np.conj(dz))
    p = float(abs(y) ** 2)
    gr = float(2.0 * np.real(np.conj(y) * dydr))
    gz = float(2.0 * np.real(np.conj(y) * dydz))
    ga = 2.0 * y * rho
    valid = (ks >= 0) & (ks < len(a))
    return p, gr, gz, ks[valid], ga[valid]


def refine_optimum(a: np.ndarray, r0: float, z0: float, margin: int = 16,
                   dr: float = 0.6, dz: float = 1.2, step_r: float = 0.01, step_z: float = 0.02,
                   polish: int = 8, max_moves: int = 8):
    """Oracle local maximum of P(r, z) near (r0, z0): dense grid search over a
    window that is re-centred on its best point until that point lies inside
    it, then Newton steps on the FP64 gradient with a finite-difference
    Hessian."""
    rc, zc = r0, z0
    for _ in range(max_moves):
        rs = rc + np.arange(-dr, dr + 1e-12, step_r)
        zs = zc + np.arange(-dz, dz + 1e-12, step_z)
        best = (-1.0, rc, zc)
        edge = False
        for iz, z in enumerate(zs):
            for ir, r in enumerate(rs):
                p = rz_power(a, r, z, margin)
                if p > best[0]:
                    best = (p, r, z)
                    edge = ir in (0, len(rs) - 1) or iz in (0, len(zs) - 1)
        if not edge:
            break
        rc, zc = best[1], best[2]
    p, r, z = best
    for _ in range(polish):
        _, gr, gz, _, _ = rz_power_grad(a, r, z, margin)
        e = 1e-4
        g_rp = rz_power_grad(a, r + e, z, margin)
        g_rm = rz_power_grad(a, r - e, z, margin)
        g_zp = rz_power_grad(a, r, z + e, margin)
        g_zm = rz_power_grad(a, r, z - e, margin)
        hrr = (g_rp[1] - g_rm[1]) / (2 * e)
        hzz = (g_zp[2] - g_zm[2]) / (2 * e)
        hrz = 0.5 * ((g_rp[2] - g_rm[2]) / (2 * e) + (g_zp[1] - g_zm[1]) / (2 * e))
        det = hrr * hzz - hrz * hrz
        if not (hrr < 0 and det > 0):
            break
        sr = -(hzz * gr - hrz * gz) / det
        sz = -(-hrz * gr + hrr * gz) / det
        if abs(sr) > 0.05 or abs(sz) > 0.1:
            break
        pn = rz_power(a, r + sr, z + sz, margin)
        if pn < p:
            break
        r, z, p = r + sr, z + sz, pn
        if abs(sr) < 1e-9 and abs(sz) < 1e-9:
            break
    return r, z, p


def rz_power_harmonics(a: np.ndarray, r: float, z: float, n_harm: int, margin: int = 16) -> float:
    """S(r, z) = sum_{k=1}^{n_harm} P(k r, k z): the incoherent sum over the
    harmonics of a fundamental at (r, z).  Harmonic k of a signal whose
    frequency drifts by z bins over the observation lies at k times its
    frequency and drifts by k z (READING: refinement of a harmonic-sum
    candidate maximises the same sum off the grid)."""
    return float(sum(rz_power(a, k * r, k * z, margin) for k in range(1, n_harm + 1)))


def rz_power_harmonics_grad(a: np.ndarray, r: float, z: float, n_harm: int, margin: int = 16):
    """S with dS/dr = sum_k k dP/dr(k r, k z) and dS/dz = sum_k k dP/dz(k r, k z)."""
    S = gr = gz = 0.0
    for k in range(1, n_harm + 1):
        p, dr, dz, _, _ = rz_power_grad(a, k * r, k * z, margin)
        S += p
        gr += k * dr
        gz += k * dz
    return S, gr, gz


def refine_harmonic_optimum(a: np.ndarray, r0: float, z0: float, n_harm: int, margin: int = 16,
                            polish: int = 8, max_moves: int = 8):
    """Oracle local maximum of S(r, z) near the fundamental (r0, z0): the grid
    search of refine_optimum with window and steps divided by n_harm (the
    top harmonic moves n_harm times as fast; steps 0.02/n_harm bin and
    0.04/n_harm z), re-centred until its best point is interior, then Newton
    steps on the FP64 gradient with a finite-difference Hessian."""
    H = n_harm
    dr, dz, step_r, step_z = 0.6 / H, 1.2 / H, 0.02 / H, 0.04 / H
    rc, zc = r0, z0
    for _ in range(max_moves):
        rs = rc + np.arange(-dr, dr + 1e-12, step_r)
        zs = zc + np.arange(-dz, dz + 1e-12, step_z)
        best = (-1.0, rc, zc)
        edge = False
        for iz, z in enumerate(zs):
            for ir, r in enumerate(rs):
                p = rz_power_harmonics(a, r, z, H, margin)
                if p > best[0]:
                    best = (p, r, z)
                    edge = ir in (0, len(rs) - 1) or iz in (0, len(zs) - 1)
        if not edge:
            break
        rc, zc = best[1], best[2]
    p, r, z = best
    for _ in range(polish):
        _, gr, gz = rz_power_harmonics_grad(a, r, z, H, margin)
        e = 1e-4 / H
        g_rp = rz_power_harmonics_grad(a, r + e, z, H, margin)
        g_rm = rz_power_harmonics_grad(a, r - e, z, H, margin)
        g_zp = rz_power_harmonics_grad(a, r, z + e, H, margin)
        g_zm = rz_power_harmonics_grad(a, r, z - e, H, margin)
        hrr = (g_rp[1] - g_rm[1]) / (2 * e)
        hzz = (g_zp[2] - g_zm[2]) / (2 * e)
        hrz = 0.5 * ((g_rp[2] - g_rm[2]) / (2 * e) + (g_zp[1] - g_zm[1]) / (2 * e))
        det = hrr * hzz - hrz * hrz
        if not (hrr < 0 and det > 0):
            break
        sr = -(hzz * gr - hrz * gz) / det
        sz = -(-hrz * gr + hrr * gz) / det
        if abs(sr) > 0.05 / H or abs(sz) > 0.1 / H:
            break
        pn = rz_power_harmonics(a, r + sr, z + sz, H, margin)
        if pn < p:
            break
        r, z, p = r + sr, z + sz, pn
        if abs(sr) < 1e-9 and abs(sz) < 1e-9:
            break
    return r, z, p


# ---------------------------------------------------------------- error metrics


def power_errors(p_test: np.ndarray, p_ref: np.ndarray, tau1: float,
                 extra_mask: Optional[np.ndarray] = None) -> Dict[str, float]:
    """Relative power error on detections (section 2.2 quotes the error in the
    magnitude of detection strength; READING: relative error of power).

    Detection set: cells with P_ref >= tau_1, plus any extra (injected) cells.
    Also the median over P_ref >= 1 and the largest absolute error anywhere."""
    p_test = np.asarray(p_test, dtype=np.float64)
    p_ref = np.asarray(p_ref, dtype=np.float64)
    det = p_ref >= tau1
    if extra_mask is not None:
        det = det | extra_mask
    rel = np.abs(p_test - p_ref) / np.maximum(p_ref, 1e-300)
    out = {
        "n_det": int(det.sum()),
        "max_rel_det": float(rel[det].max()) if det.any() else 0.0,
        "median_rel_det": float(np.median(rel[det])) if det.any() else 0.0,
        "median_rel_ge1": float(np.median(rel[p_ref >= 1.0])) if (p_ref >= 1.0).any() else 0.0,
        "max_abs": float(np.max(np.abs(p_test - p_ref))) if p_ref.size else 0.0,
    }
    return out
