"""GPU: the 1024-point convolution of a 16-bit plane, whose inverse FFTs run
their two 16-point DFT stages in FP16 on the matrix cores (FP16 products with
the templates, FP32 sums, operands scaled per segment by a power of two),
against the oracle's FP64 plane, every cell.

Tolerance, from that arithmetic.  Each FP16 rounding of an operand x_n
(half an ulp, 2^-11 relative at most) adds to an output y_k = sum_n x_n w^nk
an error whose size is set by sum_n |x_n|^2 = mean_k |y_k|^2 (Parseval), so
the error of every output of a segment is a small multiple of 2^-11 A, with
A^2 the mean power over the segment's L outputs: about 2^-10.5 A rms for the
five roundings on the path (segment spectrum, template, product, stage-1
result, DFT weights).  With D = 2^-7 A (twice a five-sigma tail) and the
16-bit storage of the power (2^-9 relative; 2^-7 allowed),
    |P_gpu - P| <= 2^-7 max(P, 1) + 2 sqrt(P) D + D^2.
A 16-bit spectrum (store dtype) adds its own rounding, |dA| <= u |A| with
u = 2^-9 (BF16) or 2^-11 (FP16): by Cauchy-Schwarz over the unit-energy taps
the output moves by at most u sqrt(E_r), E_r = sum_{|q| <= h_max} |A_{r+q}|^2,
which joins D.  A weak cell in a segment that holds a very strong signal
therefore carries an error set by that signal, not by its own power;
detections keep the 3 % bound of the 16-bit path.
"""
import numpy as np
import pytest

import synth
from oracle import fdas64 as o

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def window_energy(a, h):
    """E_r = sum_{|q| <= h} |a_{r+q}|^2 (zero outside the spectrum)."""
    c = np.concatenate([[0.0], np.cumsum(np.abs(a) ** 2)])
    r = np.arange(len(a))
    return c[np.minimum(r + h + 1, len(a))] - c[np.maximum(r - h, 0)]


def segment_rms(ref, L, U, h):
    """sqrt of the mean power over each segment's L outputs, per cell."""
    Z, nb = ref.shape
    A = np.empty_like(ref)
    for s in range((nb + U - 1) // U):
        a0, a1 = max(s * U - h, 0), min(s * U - h + L, nb)
        A[:, s * U:min((s + 1) * U, nb)] = np.sqrt(ref[:, a0:a1].mean(axis=1))[:, None]
    return A


def check_detections(err, ref, bound, strong, res=1):
    """Cells at or above the single-harmonic threshold: within 3 %.  Next to
    a very strong tone a weak cell's error is set by the tone (the bound),
    which can exceed 3 % of the cell's own power whatever the arithmetic (the
    16-bit spectrum's rounding alone does), so there the 3 % is checked
    where the bound allows it, and at the strong tones' peak rows and columns
    at 1 %."""
    det = ref >= o.threshold(1)
    assert det.any()
    rel = err / np.maximum(ref, 1e-30)
    if not strong:
        assert float(rel[det].max()) < 3e-2
        return
    tight = det & (bound <= 3e-2 * ref)
    assert tight.any() and float(rel[tight].max()) < 3e-2
    for c in (21003, 39995):  # the strong tones' mean bins (res columns per bin)
        cols = slice(res * (c - 8), res * (c + 9))
        j, r = np.unravel_index(np.argmax(ref[:, cols]), ref[:, cols].shape)
        assert rel[:, cols][j, r] < 1e-2, (c, float(rel[:, cols][j, r]))


@pytest.mark.parametrize("store,plane,strong", [("bf16", "bf16", False), ("f16", "f16", False),
                                                ("bf16", "bf16", True), ("f32", "bf16", True)])
def test_fp16_matrix_core_plane_matches_oracle(lib, store, plane, strong):
    """N = 2^17, 17 templates, L = 1024: the small case (one injection of
    peak power ~ 80), and the same series with two more tones of peak power
    ~ 4e4 and ~ 8e3 (strong).  Every cell within the bound above; cells at
    or above the single-harmonic threshold within 3 %; without strong tones
    also every cell within the 16-bit path's flat 5e-2 max(P, 1)."""
    import torch
    x, inj, _ = synth.small_case(seed=1)
    n = len(x)
    if strong:
        extra = [synth.Injection(2.0, 21000.5, 6.0, 0.3), synth.Injection(0.5, 40000.0, -10.0, 1.1)]
        x = (x.astype(np.float64) + sum(synth.chirp(n, i) for i in extra)).astype(np.float32)
    say("FP16 matrix-core convolution", store, plane, "strong tones" if strong else "small case")
    pl = lib.Plan(store=store, plane=plane, n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, n_harmonics=4,
                  segment_len=1024)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
    zs = o.z_grid(-16, 16, 2)
    a = o.normalise(o.spectrum(x), "median")
    ref = o.power_plane(a, zs)
    got = P.float().cpu().numpy().astype(np.float64).reshape(pl.Z, -1)
    err = np.abs(got - ref)
    A = segment_rms(ref, pl.L, pl.U, pl.seg_margin)
    u = {"f32": 0.0, "bf16": 2.0 ** -9, "f16": 2.0 ** -11}[store]
    D = 2.0 ** -7 * A + u * np.sqrt(window_energy(a, pl.hmax))[None, :]
    bound = 2.0 ** -7 * np.maximum(ref, 1.0) + 2.0 * np.sqrt(ref) * D + D * D
    bad = err > bound
    assert not bad.any(), (np.argwhere(bad)[:5], float((err / bound).max()))
    check_detections(err, ref, bound, strong)
    if strong:
        assert ref.max() > 3e4  # a tone ~1000 times the single-harmonic threshold
    else:
        assert np.all(err < 5e-2 * np.maximum(ref, 1.0)), float((err / np.maximum(ref, 1.0)).max())


@pytest.mark.parametrize("strong", [False, True])
def test_fp16_matrix_core_half_bin_plane_matches_oracle(lib, strong):
    """The same on the half-bin plane (BF16): each output's successor y[k+1]
    comes from the next lane (DPP), from lane 0 of the row in the next
    register, or across rows (a shuffle).  Bin columns within the bound
    above; half-bin columns h = |y_k - y_{k+1}|^2 / 2, whose difference errs
    by at most 2 D, within 2^-7 max(h, 1) + 2 sqrt(2 h) D + 2 D^2, D taken
    at the larger spectrum window of the two bins."""
    import torch
    x, inj, _ = synth.small_case(seed=1)
    n = len(x)
    if strong:
        extra = [synth.Injection(2.0, 21000.5, 6.0, 0.3), synth.Injection(0.5, 40000.0, -10.0, 1.1)]
        x = (x.astype(np.float64) + sum(synth.chirp(n, i) for i in extra)).astype(np.float32)
    say("FP16 matrix-core convolution, half-bin plane", "strong tones" if strong else "small case")
    pl = lib.Plan(store="bf16", plane="bf16", n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, n_harmonics=4,
                  segment_len=1024, interbin=1)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
    zs = o.z_grid(-16, 16, 2)
    a = o.normalise(o.spectrum(x), "median")
    ref = o.interbin_plane(a, zs)
    got = P.float().cpu().numpy().astype(np.float64).reshape(pl.Z, -1)
    err = np.abs(got - ref)
    pb, ph = ref[:, 0::2], ref[:, 1::2]
    A = segment_rms(pb, pl.L, pl.U, pl.seg_margin)
    w = np.sqrt(window_energy(a, pl.hmax))
    w = np.maximum(w, np.concatenate([w[1:], [0.0]]))
    D = 2.0 ** -7 * A + 2.0 ** -9 * w[None, :]
    bb = 2.0 ** -7 * np.maximum(pb, 1.0) + 2.0 * np.sqrt(pb) * D + D * D
    bh = 2.0 ** -7 * np.maximum(ph, 1.0) + 2.0 * np.sqrt(2.0 * ph) * D + 2.0 * D * D
    for e_, b_, what in ((err[:, 0::2], bb, "bins"), (err[:, 1::2], bh, "half bins")):
        bad = e_ > b_
        assert not bad.any(), (what, np.argwhere(bad)[:5], float((e_ / b_).max()))
    bound = np.empty_like(ref)
    bound[:, 0::2], bound[:, 1::2] = bb, bh
    check_detections(err, ref, bound, strong, res=2)


@pytest.mark.parametrize("store,plane,interbin", [("bf16", "bf16", 0), ("bf16", "bf16", 1), ("f32", "f32", 0)])
def test_plane_does_not_depend_on_template_grouping(lib, store, plane, interbin):
    """The templates a wavefront runs per loaded segment (automatic, all 17,
    5, 1) change which wavefront computes an output, never its arithmetic:
    the planes and their column maxima are bit-identical."""
    import torch
    x, inj, _ = synth.small_case(seed=1)
    n = len(x)
    xt = torch.from_numpy(x).to("cuda")
    say("template grouping invariance", store, plane, interbin)
    ref = None
    for tpt in (0, 17, 5, 1):
        pl = lib.Plan(store=store, plane=plane, n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, n_harmonics=4,
                      segment_len=1024, interbin=interbin, templates_per_tile=tpt)
        P = pl.convolve(xt, [0], [n])
        got = (P.view(torch.int16 if P.element_size() == 2 else torch.int32).cpu().numpy().copy(),
               pl.maxima(P).view(torch.int16 if P.element_size() == 2 else torch.int32).cpu().numpy().copy())
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), tpt
