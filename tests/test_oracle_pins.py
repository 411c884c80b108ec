"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: closed forms,
brute force on tiny inputs, an independent quadrature of a defining integral,
invariants, or a hand-worked fixture.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.special as sps

import synth
from oracle import fdas64 as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- spectrum

def test_spectrum_brute_force_dft_tiny():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(64).astype(np.float32)
    n = len(x)
    want = np.array([sum(float(x[t]) * np.exp(-2j * np.pi * r * t / n) for t in range(n))
                     for r in range(n // 2)])
    want[0] = 0
    np.testing.assert_allclose(o.spectrum(x), want, rtol=0, atol=1e-12)


def test_spectrum_parseval():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(1 << 14)
    a = o.spectrum(x)
    n = len(x)
    dc = math.fsum(x)                                    # X_0 by direct sum
    nyq = math.fsum(x * (-1.0) ** np.arange(n))          # X_{N/2} by direct sum
    lhs = math.fsum(x * x)
    rhs = (dc * dc + 2.0 * math.fsum(np.abs(a[1:]) ** 2) + nyq * nyq) / n
    assert abs(lhs - rhs) <= 1e-12 * lhs


def test_spectrum_integer_bin_sinusoid_closed_form():
    n, a, r, ph = 1 << 17, 0.05, 5000, 0.7
    x = a * np.cos(2 * np.pi * r * np.arange(n) / n + ph)
    s = o.normalise(o.spectrum(x), "variance", n_samples=n)
    p = np.abs(s) ** 2
    assert abs(p[r] - n * a * a / 4) < 1e-9 * (n * a * a / 4)   # 81.92
    assert abs(p[r] - 81.92) < 1e-9
    assert abs(np.angle(s[r]) - ph) < 1e-9
    p[r] = 0
    assert p.max() < 1e-18


# ----------------------------------------------------------- normalisation

def test_median_normalisation_constructed_blocks():
    b = 2048
    rng = np.random.default_rng(2)
    blocks = []
    for i in range(4):
        vals = rng.permutation(np.arange(1, b + 1, dtype=np.float64)) * (i + 1)
        ph = rng.uniform(0, 2 * np.pi, b)
        blocks.append(np.sqrt(vals) * np.exp(1j * ph))
    a = np.concatenate(blocks)
    out, med = o.normalise(a, "median", block=b, return_medians=True)
    # lower median of {1..2048} * (i+1) is 1024 * (i+1)
    np.testing.assert_allclose(med, [1024.0 * (i + 1) for i in range(4)], rtol=1e-15)
    for i in range(4):
        seg = out[i * b:(i + 1) * b]
        np.testing.assert_allclose(seg, a[i * b:(i + 1) * b] * math.sqrt(math.log(2) / (1024.0 * (i + 1))),
                                   rtol=1e-15)
        # the median power of every block becomes ln 2 exactly (up to rounding)
        assert abs(np.sort(np.abs(seg) ** 2)[(b - 1) // 2] - math.log(2)) < 1e-14


def test_rednoise_widths_follow_the_rule():
    # sub-block width: largest power of two <= (block start)/8, within [32, B]
    assert [o.rednoise_width(b, 2048) for b in range(10)] == [32, 256, 512, 512, 1024, 1024, 1024, 1024, 2048, 2048]
    assert [o.rednoise_width(b, 256) for b in range(9)] == [32, 32, 64, 64, 128, 128, 128, 128, 256]


def test_rednoise_normalisation_constructed_sub_blocks():
    # every sub-block of width w holds a permutation of {1..w} times its own
    # factor, so its lower median is (w // 2) times that factor exactly
    B, nblk = 256, 10
    rng = np.random.default_rng(3)
    parts, want = [], []
    f = 1.0
    for b in range(nblk):
        w = o.rednoise_width(b, B)
        for _ in range(B // w):
            f *= 1.37
            vals = rng.permutation(np.arange(1, w + 1, dtype=np.float64)) * f
            parts.append(np.sqrt(vals) * np.exp(1j * rng.uniform(0, 2 * np.pi, w)))
            want.append((w, (w // 2) * f))
    a = np.concatenate(parts)
    out, meds = o.normalise(a, "rednoise", block=B, return_medians=True)
    np.testing.assert_allclose(np.concatenate(meds), [m for _, m in want], rtol=1e-15)
    pos = 0
    for w, m in want:
        np.testing.assert_allclose(out[pos:pos + w], a[pos:pos + w] * math.sqrt(math.log(2) / m), rtol=1e-15)
        pos += w


def test_rednoise_normalisation_whitens_a_steep_continuum():
    # white noise plus a random walk (power ~ 1/f^2, 1e4 times the white level
    # at bin 100): per-block medians leave the lowest bins far from unit mean,
    # frequency-scaled sub-blocks bring them back within the median's scatter
    n = 1 << 18
    rng = np.random.default_rng(12)
    x = rng.standard_normal(n) + 0.6 * np.cumsum(rng.standard_normal(n)) / math.sqrt(n) * 40
    x = (x - x.mean()).astype(np.float32)
    a = o.spectrum(x)
    for mode, bound in (("rednoise", 0.25), ("median", None)):
        p = np.abs(o.normalise(a, mode)) ** 2
        means = [p[lo:lo + 64].mean() for lo in range(64, 2048, 64)]
        if bound is None:
            assert max(means) > 5.0       # the block median cannot follow the slope
        else:
            assert max(abs(np.log(means))) < math.log(1 + 4 * bound), means
    p = np.abs(o.normalise(a, "rednoise")) ** 2
    assert abs(p[16384:].mean() - 1.0) < 0.01   # whole blocks higher up


def test_median_normalisation_noise_unit_mean():
    x = synth.make_series(1 << 20, [], cfg_seed=9, series_index=0)
    a = o.normalise(o.spectrum(x), "median")
    p = np.abs(a[1:]) ** 2
    assert abs(p.mean() - 1.0) < 0.01
    v = o.normalise(o.spectrum(x), "variance", n_samples=len(x))
    assert abs(np.mean(np.abs(v[1:]) ** 2) - 1.0) < 0.01


def test_zero_median_block_scales_to_zero():
    a = np.zeros(4096, complex)
    a[5] = 3.0
    out = o.normalise(a, "median")
    assert np.all(out == 0)


# ------------------------------------------------------- Fresnel response

RESP_POINTS = [(0.0, 20.0), (3.0, 20.0), (-7.0, 20.0), (0.37, 5.5), (12.0, -33.0), (-64.0, 96.0),
               (64.0, -96.0), (1.5, 0.02), (-2.25, -1.0), (40.0, 0.5), (0.0, 96.0), (10.0, 3e-3)]


def _mp_rho(q, z):
    f = lambda u: mpmath.expj(-2 * mpmath.pi * q * u + mpmath.pi * z * (u - 0.5) ** 2)
    pts = mpmath.linspace(0, 1, 2 + int(abs(q) + abs(z)))
    return complex(mpmath.quad(f, pts))


@pytest.mark.parametrize("q,z", RESP_POINTS)
def test_response_matches_mpmath_quadrature(q, z):
    mpmath.mp.dps = 30
    assert abs(complex(o.response(q, z)) - _mp_rho(q, z)) < 1e-12


def test_response_matches_fine_simpson_grid():
    rng = np.random.default_rng(3)
    q = rng.uniform(-70, 70, 200)
    z = rng.uniform(-100, 100, 200)
    u = np.linspace(0, 1, 200001)
    w = np.ones_like(u)
    w[1:-1:2], w[2:-1:2] = 4, 2
    w /= 3 * (len(u) - 1)
    f = np.exp(1j * (-2 * np.pi * q[:, None] * u + np.pi * z[:, None] * (u - 0.5) ** 2))
    np.testing.assert_allclose(o.response(q, z), f @ w, rtol=0, atol=1e-9)


def test_response_integer_q_at_zero_drift_is_delta():
    q = np.arange(-20, 21, dtype=float)
    r = o.response(q, 0.0)
    want = (q == 0).astype(float)
    np.testing.assert_allclose(r, want, atol=1e-13)


def test_response_parseval_over_all_q():
    # sum over integer q of |rho(q,z)|^2 = int_0^1 |e^{i phi}|^2 du = 1
    q = np.arange(-20000, 20001, dtype=float)
    for z in (5.0, 37.0, -96.0):
        s = np.sum(np.abs(o.response(q, z)) ** 2)
        assert abs(s - 1.0) < 5e-5


def test_response_symmetries():
    rng = np.random.default_rng(4)
    q = rng.uniform(-50, 50, 50)
    z = rng.uniform(1, 90, 50)
    R = lambda q, z: np.exp(1j * np.pi * q) * o.response(q, z)
    np.testing.assert_allclose(R(q, z), R(-q, z), atol=1e-12)           # even in q
    np.testing.assert_allclose(R(q, -z), np.conj(R(q, z)), atol=1e-12)  # conjugate under z -> -z


@pytest.mark.parametrize("z", [20.0, -35.0])
def test_chirp_spectrum_follows_response(z):
    """DFT of a synthesised chirp: A_{rbar+q} = (N a/2) e^{i theta} rho(q, z)."""
    n, a = 1 << 17, 0.05
    r0 = 5000.0 - z / 2          # mean frequency rbar = 5000 exactly
    inj = synth.Injection(a, r0, z, 0.3)
    x = synth.chirp(n, inj)
    A = o.spectrum(x)
    rbar = 5000
    q = np.arange(-30, 31)
    ratio = A[rbar + q] / (n * a / 2 * o.response(q.astype(float), z))
    assert np.max(np.abs(np.abs(ratio) - 1)) < 1e-4
    ph = np.angle(ratio / ratio[30])
    assert np.max(np.abs(ph)) < 1e-4


def test_response_derivatives_match_finite_differences_and_mpmath():
    mpmath.mp.dps = 30
    for q, z in [(0.3, 17.0), (-12.7, -44.0), (5.5, 0.004), (30.0, 90.0)]:
        rho, dq, dz = o.response_derivatives(q, z)
        e = 1e-5
        fq = (o.response(q + e, z) - o.response(q - e, z)) / (2 * e)
        fz = (o.response(q, z + e) - o.response(q, z - e)) / (2 * e)
        assert abs(complex(dq) - complex(fq)) < 1e-7 * max(1, abs(complex(dq)))
        assert abs(complex(dz) - complex(fz)) < 1e-7 * max(1, abs(complex(dz)))
        g = lambda u: (-2j * mpmath.pi * u) * mpmath.expj(-2 * mpmath.pi * q * u + mpmath.pi * z * (u - 0.5) ** 2)
        h = lambda u: (1j * mpmath.pi * (u - 0.5) ** 2) * mpmath.expj(-2 * mpmath.pi * q * u + mpmath.pi * z * (u - 0.5) ** 2)
        pts = mpmath.linspace(0, 1, 2 + int(abs(q) + abs(z)))
        assert abs(complex(dq) - complex(mpmath.quad(g, pts))) < 1e-11
        assert abs(complex(dz) - complex(mpmath.quad(h, pts))) < 1e-11


# -------------------------------------------------------------- templates

def test_template_zero_drift_is_delta_and_unit_energy():
    zs = o.z_grid(-16, 16, 2)
    taps, hmax = o.template_taps(zs)
    assert hmax == 24
    j0 = int(np.argmin(np.abs(zs)))
    want = np.zeros(2 * hmax + 1)
    want[hmax] = 1
    np.testing.assert_allclose(taps[j0], want, atol=1e-13)
    np.testing.assert_allclose(np.sum(np.abs(taps) ** 2, axis=1), 1.0, rtol=1e-13)
    # support is |q| <= ceil(|z|/2) + 16
    for z, row in zip(zs, taps):
        h = int(math.ceil(abs(z) / 2)) + 16
        q = np.arange(-hmax, hmax + 1)
        assert np.all(row[np.abs(q) > h] == 0)
        assert np.all(np.abs(row[np.abs(q) <= h]) > 0) or z == 0


def _fresnel_coefficients_by_fft(z, qmax, m=1 << 20):
    """rho(q, z) for |q| <= qmax as Fourier coefficients of
    g(u) = exp(i pi z (u - 1/2)^2) on [0, 1): midpoint sums of M and 2M points
    by FFT, Richardson-combined (g(0) = g(1), so the midpoint error is
    c/M^2 + O(1/M^4)).  Independent of the oracle's Fresnel evaluation."""
    def mid(mm):
        u = (np.arange(mm) + 0.5) / mm
        c = np.fft.fft(np.exp(1j * np.pi * z * (u - 0.5) ** 2)) / mm
        q = np.arange(-qmax, qmax + 1)
        return c[q % mm] * np.exp(-1j * np.pi * q / mm)
    return (4.0 * mid(2 * m) - mid(m)) / 3.0


@pytest.mark.parametrize("z", [16.0, 20.0, 48.0, 96.0, -35.0, 3.5])
def test_template_energy_and_taps_match_fine_fourier_series(z):
    """E(z) = sum_{|q| <= h(z)} |rho(q, z)|^2, and the taps conj(rho)/sqrt(E),
    against the Fourier coefficients of the unit-modulus chirp computed by
    FFT: the energy the templates leave out is the chirp's spectrum beyond
    +-h(z), so 0.99 < E < 1, falling with |z|."""
    h = int(o.half_width(np.array([z]))[0])
    rho = _fresnel_coefficients_by_fft(z, h)
    e_ref = float(np.sum(np.abs(rho) ** 2))
    e = float(o.template_energy(np.array([z]))[0])
    assert abs(e - e_ref) < 1e-10, (z, e, e_ref)
    assert 0.99 < e < 1.0
    taps, hmax = o.template_taps(np.array([z]))
    col = np.arange(-h, h + 1) + hmax
    np.testing.assert_allclose(taps[0, col], np.conj(rho) / math.sqrt(e_ref), rtol=0, atol=1e-10)


def test_template_energy_falls_with_drift():
    e = o.template_energy(np.array([16.0, 20.0, 48.0, 96.0]))
    assert np.all(np.diff(e) < 0)


def test_ska_grid_has_193_trials():
    g = json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))
    zs = o.z_grid(-96, 96, 1)
    assert len(zs) == g["ska_like"]["acceleration_trials"]
    assert int(o.half_width(zs).max()) == 64


# ------------------------------------------------------------ correlation

def test_fft_correlation_matches_direct_sum():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(3000) + 1j * rng.standard_normal(3000)
    taps = rng.standard_normal(41) + 1j * rng.standard_normal(41)
    y = o.correlate(a, taps)
    r = np.arange(3000)
    np.testing.assert_allclose(y, o.correlate_direct(a, taps, r), atol=1e-11)
    # and the direct sum itself against a plain loop at a few bins (edges zero-padded)
    for rr in (0, 7, 1500, 2999):
        s = sum(a[rr + q] * taps[q + 20] for q in range(-20, 21) if 0 <= rr + q < 3000)
        assert abs(y[rr] - s) < 1e-11


def test_correlation_equals_time_domain_dechirp():
    """With the discrete, untruncated template c_q = DFT_N(g)/N of the chirp
    g_n = exp(i pi z (n/N - 1/2)^2), correlating the full spectrum with conj(c)
    equals the DFT of the dechirped series x * conj(g)."""
    n, z = 4096, 7.3
    rng = np.random.default_rng(6)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    t = np.arange(n) / n
    g = np.exp(1j * np.pi * z * (t - 0.5) ** 2)
    X = np.fft.fft(x)
    c = np.fft.fft(g) / n
    y = o.correlate_cyclic(X, np.conj(c))
    np.testing.assert_allclose(y, np.fft.fft(x * np.conj(g)), atol=1e-9 * n)
    # non-cyclic form on a band-limited spectrum, taps |q| <= n/4, output bin n/2
    Xb = np.zeros(n, complex)
    Xb[n // 4: 3 * n // 4] = X[n // 4: 3 * n // 4]
    xb = np.fft.ifft(Xb)
    q = np.arange(-n // 4, n // 4 + 1)
    taps = np.conj(c[q % n])
    yb = o.correlate_direct(Xb, taps, np.array([n // 2]))[0]
    assert abs(yb - np.fft.fft(xb * np.conj(g))[n // 2]) < 1e-9 * n
    # and the continuous response approximates the discrete template
    assert np.max(np.abs(o.response(q.astype(float), z) - c[q % n])) < 5e-3


def test_injected_chirp_recovered_with_fresnel_energy():
    """Noise-free accelerated sinusoid: the plane peaks at (rbar, z) with
    P = (N a^2/4) E(z)."""
    n, a = 1 << 17, 0.05
    for z, r0 in ((20.0, 5000.0), (-20.0, 5020.0)):
        x = synth.chirp(n, synth.Injection(a, r0, z, 1.1))
        s = o.normalise(o.spectrum(x), "variance", n_samples=n)
        zs = o.z_grid(-24, 24, 2)
        P = o.power_plane(s, zs)
        j, r = np.unravel_index(np.argmax(P), P.shape)
        assert zs[j] == z and r == int(r0 + z / 2)
        want = n * a * a / 4 * o.template_energy(np.array([z]))[0]
        assert abs(P[j, r] - want) < 2e-3 * want


def test_small_case_edge_detection_and_scalloping_closed_forms():
    n, a = 1 << 17, 0.05
    x = synth.chirp(n, synth.Injection(a, 5000.0, 20.0, 0.2))
    s = o.normalise(o.spectrum(x), "variance", n_samples=n)
    zs = o.z_grid(-16, 16, 2)
    P = o.power_plane(s, zs)
    j, r = np.unravel_index(np.argmax(P), P.shape)
    assert (zs[j], r) == (16.0, 5010)
    # z mismatch dz = 4: |int_{-1/2}^{1/2} e^{i pi dz v^2} dv|^2 = (2/dz)(C^2+S^2)(sqrt(dz/2))
    S, C = sps.fresnel(math.sqrt(2.0))
    mism = (2 / 4.0) * (C * C + S * S)
    assert abs(P[j, r] - 81.92 * mism) < 0.01 * 81.92 * mism
    # half-bin scalloping at z = 0: |A|^2 = 81.92 * (2/pi)^2 (to O(1/N))
    xh = a * np.cos(2 * np.pi * 5000.5 * np.arange(n) / n)
    sh = o.normalise(o.spectrum(xh), "variance", n_samples=n)
    assert abs(np.max(np.abs(sh) ** 2) - 81.92 * 4 / np.pi ** 2) < 2e-4 * 33.2
    # exact: DFT of a sampled cosine is a sum of two Dirichlet kernels
    D = lambda d: np.exp(-1j * np.pi * d * (n - 1) / n) * np.sin(np.pi * d) / np.sin(np.pi * d / n)
    k = 5000
    want = (a / 2) * (D(k - 5000.5) + D(k + 5000.5)) / math.sqrt(n)
    assert abs(sh[k] - want) < 1e-10


def test_noise_rows_have_unit_mean_power():
    x = synth.make_series(1 << 18, [], 11, 0)
    s = o.normalise(o.spectrum(x), "median")
    zs = np.array([-96.0, -41.0, 0.0, 17.0, 96.0])
    P = o.power_plane(s, zs)
    m = P[:, 200:-200].mean(axis=1)
    assert np.all(np.abs(m - 1) < 0.02)
    # exponential marginal: P(P > 3) = e^-3
    frac = (P[:, 200:-200] > 3).mean(axis=1)
    assert np.all(np.abs(frac - math.exp(-3)) < 0.005)


# ------------------------------------------------------------ interbinning

def test_interbin_midway_tone_keeps_8_over_pi2():
    # a z = 0 tone midway between bins 5000 and 5001: each neighbour holds
    # (2/pi)^2 of the peak, the half-bin column (8/pi^2) of it (sinc response
    # of the DFT, up to the O(1/N) image term)
    n, a = 1 << 17, 0.05
    x = a * np.cos(2 * np.pi * 5000.5 * np.arange(n) / n + 0.3)
    s = o.normalise(o.spectrum(x), "variance", n_samples=n)
    P2 = o.interbin_plane(s, [0.0])
    assert abs(P2[0, 2 * 5000 + 1] - 81.92 * 8 / np.pi ** 2) < 1e-6 * 66.4
    for c in (2 * 5000, 2 * 5001):
        assert abs(P2[0, c] - 81.92 * 4 / np.pi ** 2) < 2e-4 * 33.2


def test_interbin_integer_tone_halves_into_both_neighbours():
    # a tone on bin 5000 has A_k = 0 at every other bin, so both half-bin
    # columns next to it hold exactly |A_5000|^2 / 2
    n, a = 1 << 17, 0.05
    x = a * np.cos(2 * np.pi * 5000 * np.arange(n) / n + 0.7)
    s = o.normalise(o.spectrum(x), "variance", n_samples=n)
    P2 = o.interbin_plane(s, [0.0])
    assert abs(P2[0, 2 * 5000] - 81.92) < 1e-9
    assert abs(P2[0, 2 * 5000 - 1] - 40.96) < 1e-9 and abs(P2[0, 2 * 5000 + 1] - 40.96) < 1e-9
    # the even columns are the plain plane
    assert np.array_equal(P2[0, 0::2], o.power_plane(s, [0.0])[0])
    P2[0, 2 * 5000 - 1: 2 * 5000 + 2] = 0
    assert P2.max() < 1e-18


@pytest.mark.parametrize("z", [20.0, -60.0, 96.0])
def test_interbin_accelerated_midway_chirp(z):
    # the template autocorrelation is exp(-i pi d) sinc(d) at every z, so a chirp
    # whose mean frequency is midway between bins gives (8/pi^2) E(z) of the
    # peak in its half-bin column, to the truncation of the templates
    n, a = 1 << 17, 0.05
    x = synth.chirp(n, synth.Injection(a, 5000.5 - z / 2, z, 0.2))
    s = o.normalise(o.spectrum(x), "variance", n_samples=n)
    E = o.template_energy([z])[0]
    P2 = o.interbin_plane(s, [z])
    assert abs(P2[0, 2 * 5000 + 1] / (81.92 * 8 / np.pi ** 2 * E) - 1) < 5e-3


def test_interbin_noise_has_unit_mean_exponential_power():
    x = synth.make_series(1 << 18, [], 11, 0)
    s = o.normalise(o.spectrum(x), "variance", n_samples=1 << 18)
    P2 = o.interbin_plane(s, np.array([-96.0, -41.0, 0.0, 17.0, 96.0]))
    half = P2[:, 401:-400:2]
    assert np.all(np.abs(half.mean(axis=1) - 1) < 0.015)
    assert np.all(np.abs((half > 3).mean(axis=1) - math.exp(-3)) < 0.003)


def test_interbin_cells_direct_sum_agrees_with_whole_plane():
    rng = np.random.default_rng(12)
    n = 1 << 12
    a = rng.standard_normal(n // 2) + 1j * rng.standard_normal(n // 2)
    zs = o.z_grid(-16, 16, 2)
    taps, _ = o.template_taps(zs)
    whole = o.interbin_plane(a, zs)
    rows = rng.integers(0, len(zs), 400)
    cols = rng.integers(0, n, 400)
    cols[:4] = [0, 1, n - 2, n - 1]            # both ends of the spectrum
    np.testing.assert_allclose(o.interbin_cells(a, taps, rows, cols), whole[rows, cols], rtol=1e-10, atol=1e-10)


def test_interbin_search_finds_a_midway_tone_the_bin_search_misses():
    # peak power 40: midway between bins each bin keeps 0.405 x 40 = 16.2 and
    # the half-bin 0.81 x 40 = 32.4, against tau_1 = 20.74 (noise-free)
    n = 1 << 17
    a = math.sqrt(4 * 40.0 / n)
    x = a * np.cos(2 * np.pi * 7000.5 * np.arange(n) / n + 1.1)
    s = o.normalise(o.spectrum(x), "variance", n_samples=n)
    zs = np.array([0.0])
    assert o.search(o.power_plane(s, zs), zs, 2, r_lo=24, h_max=24) == []
    c = o.search(o.interbin_plane(s, zs), zs, 2, r_lo=24, h_max=24, res=2)
    best = max(c, key=lambda k: k.sigma)
    assert (best.harm, best.R, best.r) == (1, 14001, 7000.5)
    assert abs(best.power - 40 * 8 / np.pi ** 2) < 1e-3
    # every record lies on the tone or on the cells whose harmonics reach it
    assert all(k.harm == 1 and k.R == 14001 or k.harm == 2 and abs(k.R - 28002) <= 1 for k in c)


# ---------------------------------------------------------- harmonic sums

def _plane_from_formula(nz, nb):
    j = np.arange(nz)[:, None]
    r = np.arange(nb)[None, :]
    return (100 * j + r).astype(float)


def test_harmonic_sum_worked_fixture():
    g = json.load(open(os.path.join(GOLDEN, "harmonic_sum_worked.json")))
    P = _plane_from_formula(5, 12)
    sums = o.harmonic_sums(P, g["j0"], g["n_harm"])
    rows = np.array([c["j"] for c in g["cells"]])
    cols = np.array([c["R"] for c in g["cells"]])
    at = o.harmonic_sum_cells(P, g["j0"], g["n_harm"], rows, cols)
    for i, cell in enumerate(g["cells"]):
        for H, v in cell["S"].items():
            assert sums[int(H)][cell["j"], cell["R"]] == v, (cell, H)
            assert at[int(H)][i] == v, (cell, H)


def test_harmonic_sum_cells_agree_with_whole_plane_sums():
    rng = np.random.default_rng(8)
    P = rng.exponential(size=(41, 700))
    for j0, nh in ((20, 16), (20, 8), (3, 4), (20, 1)):
        sums = o.harmonic_sums(P, j0, nh)
        rows = rng.integers(0, 41, 500)
        cols = rng.integers(0, 700, 500)
        at = o.harmonic_sum_cells(P, j0, nh, rows, cols)
        for H in at:
            np.testing.assert_array_equal(at[H], sums[H][rows, cols])


def test_harmonic_sum_invariants():
    rng = np.random.default_rng(7)
    P = rng.exponential(size=(33, 400))
    j0 = 16
    sums = o.harmonic_sums(P, j0, 16)
    np.testing.assert_array_equal(sums[1], P)
    c = np.full((33, 400), 2.5)
    sc = o.harmonic_sums(c, j0, 16)
    for H in (1, 2, 4, 8, 16):
        np.testing.assert_allclose(sc[H], 2.5 * H)
    # mirror symmetry in z
    sm = o.harmonic_sums(P[::-1].copy(), j0, 16)
    for H in (2, 4, 8, 16):
        np.testing.assert_array_equal(sm[H], sums[H][::-1])
    # stages nest: each stage contains the previous one plus non-negative terms
    for H in (2, 4, 8, 16):
        assert np.all(sums[H] >= sums[H // 2])


def test_harmonic_sum_collects_a_pulsar_harmonic_comb():
    """Harmonics h = 1..16 of a fundamental (r_f, m_f) at (h r_f, h m_f): the cell of
    the H-th harmonic sums exactly the first H of them."""
    nz, nb, j0 = 193, 4000, 96
    for rf, mf in ((97, 3), (211, -5), (50, 0)):
        P = np.zeros((nz, nb))
        for h in range(1, 17):
            P[j0 + h * mf, h * rf] += 1.0 + 0.01 * h
        sums = o.harmonic_sums(P, j0, 16)
        for H in (1, 2, 4, 8, 16):
            want = sum(1.0 + 0.01 * h for h in range(1, H + 1))
            assert abs(sums[H][j0 + H * mf, H * rf] - want) < 1e-12
            at = o.harmonic_sum_cells(P, j0, 16, np.array([j0 + 16 * mf]), np.array([16 * rf]))
            want16 = sum(1.0 + 0.01 * h for h in range(1, 17))
            assert abs(at[16][0] - want16) < 1e-12


# ------------------------------------------------------------ thresholds

def test_thresholds_closed_forms():
    tail = 0.5 * math.erfc(6 / math.sqrt(2))
    assert abs(o.threshold(1) - (-math.log(tail))) < 1e-9
    for H in (1, 2, 4, 8, 16):
        t = o.threshold(H)
        q = math.exp(-t) * math.fsum(t ** k / math.factorial(k) for k in range(H))
        assert abs(q / tail - 1) < 1e-9
        assert abs(float(o.gaussian_sigma(t, H)) - 6.0) < 1e-8
    assert all(o.threshold(2 * H) > o.threshold(H) for H in (1, 2, 4, 8))


def test_gaussian_sigma_large_power_no_underflow():
    s = o.gaussian_sigma(np.array([2000.0, 5000.0]), 16)
    assert np.all(np.isfinite(s)) and s[1] > s[0] > 50


def test_best_stage_hand_worked():
    """ln P(Gamma(1) > 25) = -25 and ln P(Gamma(2) > 30) = -30 + ln 31 = -26.57:
    stage 2 is the more significant; stage 4 (S = 20 < 29.17) fails.  With
    R below 2 r_lo, stage 2 is not searched and stage 1 is reported; at the
    upper edge (R >= n_bins - h_max) nothing is."""
    sums = {1: np.array([25.0, 25.0, 25.0]), 2: np.array([30.0, 30.0, 30.0]), 4: np.array([20.0, 20.0, 20.0])}
    R = np.array([500, 150, 990])
    h, lq = o.best_stage(sums, R, n_bins=1000, r_lo=100, h_max=16)
    assert h.tolist() == [2, 1, 0]
    assert abs(lq[0] - (-30.0 + math.log(31.0))) < 1e-12 and abs(lq[1] + 25.0) < 1e-12


def test_local_maxima_against_brute_force():
    rng = np.random.default_rng(11)
    for trial in range(15):
        n = 150
        cells = set()
        while len(cells) < n:
            cells.add((int(rng.integers(0, 3)), int(rng.integers(0, 30)), int(rng.integers(0, 9))))
        ser, R, j = (np.array(v) for v in zip(*cells))
        sig = rng.integers(0, 6, n).astype(np.float32)   # many ties
        got = o.local_maxima(ser, R, j, sig)
        key = ser * 2 ** 34 + j * 2 ** 22 + R
        for a in range(n):
            beaten = any(ser[b] == ser[a] and abs(R[b] - R[a]) <= 2 and abs(j[b] - j[a]) <= 2 and
                         (sig[b] > sig[a] or (sig[b] == sig[a] and key[b] < key[a])) for b in range(n) if b != a)
            assert got[a] == (not beaten), (trial, a)


def test_local_maxima_hand_worked():
    # a 3x3 patch around (R, j) = (100, 10) peaking at its centre, a lone record
    # 3 bins away (outside the radius) and a record of another series
    R = np.array([99, 100, 101, 99, 100, 101, 99, 100, 101, 103, 100])
    j = np.array([9, 9, 9, 10, 10, 10, 11, 11, 11, 10, 10])
    s = np.array([0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1])
    sig = np.array([6.1, 6.5, 6.2, 7.0, 9.0, 7.5, 6.0, 6.4, 6.3, 8.0, 6.0], np.float32)
    assert o.local_maxima(s, R, j, sig).tolist() == [False] * 4 + [True] + [False] * 4 + [True, True]


def test_search_finds_injection_and_reports_fundamental():
    n = 1 << 17
    x = synth.make_series(n, [synth.Injection(0.05, 5000.0, 12.0, 0.5)], 3, 0)
    s = o.normalise(o.spectrum(x), "median")
    zs = o.z_grid(-16, 16, 2)
    P = o.power_plane(s, zs)
    c = o.search(P, zs, 4, r_lo=24, h_max=24)
    best = max(c, key=lambda k: k.sigma)
    assert best.harm == 1 and abs(best.r - 5006) <= 1 and abs(best.z - 12) <= 2
    # noise-only: no candidate at 6 sigma expected in 1.1e6 cells x 3 stages
    y = synth.make_series(n, [], 4, 0)
    P0 = o.power_plane(o.normalise(o.spectrum(y), "median"), zs)
    assert len(o.search(P0, zs, 4, r_lo=24, h_max=24)) <= 2


# ------------------------------------------------------------ refinement

def test_rz_power_reduces_to_bin_power():
    rng = np.random.default_rng(8)
    a = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    for r in (50, 123, 300):
        assert abs(o.rz_power(a, float(r), 0.0) - abs(a[r]) ** 2) < 1e-12


def test_rz_power_half_bin_window_energy():
    n, a = 1 << 17, 0.05
    x = synth.chirp(n, synth.Injection(a, 5000.5, 0.0, 0.4))
    s = o.normalise(o.spectrum(x), "variance", n_samples=n)
    k = np.arange(-15, 17) - 0.5
    ew = np.sum(np.sinc(k) ** 2)
    # y = sqrt(81.92) sum_k sinc(k - r)^2 over the window, so P = 81.92 * ew^2
    assert abs(o.rz_power(s, 5000.5, 0.0) - 81.92 * ew * ew) < 2e-3 * 81.92


def test_rz_gradients_match_central_differences():
    n = 1 << 16
    x = synth.make_series(n, [synth.Injection(0.08, 3000.0, 31.0, 0.4)], 5, 0)
    s = o.normalise(o.spectrum(x), "median")
    for r, z in ((3015.3, 30.2), (3016.1, 31.7), (2000.4, -12.3)):
        p, gr, gz, ks, ga = o.rz_power_grad(s, r, z)
        h = 1e-3
        fr = (o.rz_power(s, r + h, z) - o.rz_power(s, r - h, z)) / (2 * h)
        fz = (o.rz_power(s, r, z + h) - o.rz_power(s, r, z - h)) / (2 * h)
        assert abs(gr - fr) < 1e-4 * max(1, abs(fr)) + 1e-5 * p
        assert abs(gz - fz) < 1e-4 * max(1, abs(fz)) + 1e-5 * p
        # dP/dA_k as d/dRe + i d/dIm, by finite differences on two bins
        for idx in (3, len(ks) // 2):
            k = ks[idx]
            e = 1e-6
            sp_ = s.copy(); sp_[k] += e
            sm_ = s.copy(); sm_[k] -= e
            dre = (o.rz_power(sp_, r, z) - o.rz_power(sm_, r, z)) / (2 * e)
            sp_ = s.copy(); sp_[k] += 1j * e
            sm_ = s.copy(); sm_[k] -= 1j * e
            dim = (o.rz_power(sp_, r, z) - o.rz_power(sm_, r, z)) / (2 * e)
            assert abs(ga[idx] - (dre + 1j * dim)) < 1e-5 * max(1, abs(ga[idx]))


def _harmonic_train(n, rbar, z, amps, phase=0.4):
    """Noise-free signal whose harmonic k sits at k rbar (mean) and drifts by k z."""
    u = np.arange(n) / n
    x = np.zeros(n)
    for k, a in enumerate(amps, 1):
        x += a * np.cos(2 * np.pi * (k * (rbar - z / 2) * u + 0.5 * k * z * u * u) + phase * k)
    return x


def test_rz_power_harmonics_of_a_noise_free_harmonic_train():
    # S at the true fundamental: each harmonic contributes (N a_k^2 / 4) W_k^2,
    # W_k the response energy inside its window (the matched sum of the
    # signal's own response), harmonics far apart do not interact
    n = 1 << 17
    rbar, z, amps = 1003.2, 6.4, [0.03, 0.02, 0.015, 0.01]
    s = o.normalise(o.spectrum(_harmonic_train(n, rbar, z, amps)), "variance", n_samples=n)
    want = 0.0
    for k, a in enumerate(amps, 1):
        ks = o.rz_window(k * rbar, k * z)
        W = np.sum(np.abs(o.response(ks - k * rbar, k * z)) ** 2)
        want += n * a * a / 4 * W * W
    assert abs(o.rz_power_harmonics(s, rbar, z, 4) / want - 1) < 5e-4
    # one harmonic is the single-harmonic power
    assert o.rz_power_harmonics(s, rbar, z, 1) == o.rz_power(s, rbar, z)


def test_rz_power_harmonics_gradient_matches_central_differences():
    n = 1 << 17
    s = o.normalise(o.spectrum(_harmonic_train(n, 1003.2, 6.4, [0.03, 0.02, 0.015, 0.01])), "variance",
                    n_samples=n)
    for r, z in [(1003.23, 6.37), (1003.11, 6.52), (1002.95, 6.3)]:
        S, gr, gz = o.rz_power_harmonics_grad(s, r, z, 4)
        h = 1e-5
        fr = (o.rz_power_harmonics(s, r + h, z, 4) - o.rz_power_harmonics(s, r - h, z, 4)) / (2 * h)
        fz = (o.rz_power_harmonics(s, r, z + h, 4) - o.rz_power_harmonics(s, r, z - h, 4)) / (2 * h)
        assert abs(gr - fr) < 1e-5 * max(1.0, S) and abs(gz - fz) < 1e-5 * max(1.0, S)


def test_refine_harmonic_optimum_finds_the_noise_free_fundamental():
    # k rbar and k z stay clear of the window steps (integer k r, even k z)
    n = 1 << 17
    rbar, z = 1003.2, 6.4
    s = o.normalise(o.spectrum(_harmonic_train(n, rbar, z, [0.03, 0.02, 0.015, 0.01])), "variance",
                    n_samples=n)
    r, zz, p = o.refine_harmonic_optimum(s, rbar + 0.02, z - 0.04, 4)
    assert abs(r - rbar) < 1e-3 and abs(zz - z) < 1e-2
    assert p >= o.rz_power_harmonics(s, rbar, z, 4) * (1 - 1e-6)


def test_refine_optimum_on_noise_free_signal():
    n = 1 << 17
    inj = synth.Injection(0.05, 4000.3, 14.6, 0.9)
    x = synth.chirp(n, inj)
    s = o.normalise(o.spectrum(x), "variance", n_samples=n)
    r, z, p = o.refine_optimum(s, inj.r_mean + 0.3, inj.z - 0.5)
    assert abs(r - inj.r_mean) < 0.01 and abs(z - inj.z) < 0.05
    assert p > 0.95 * 81.92


# ------------------------------------------------------------ error metric

def test_power_errors_metric():
    ref = np.array([0.5, 30.0, 100.0, 2.0])
    test = ref * np.array([1.5, 1.01, 0.98, 1.0])
    e = o.power_errors(test, ref, tau1=20.0)
    assert e["n_det"] == 2
    assert abs(e["max_rel_det"] - 0.02) < 1e-12
    assert abs(e["max_abs"] - 2.0) < 1e-12
