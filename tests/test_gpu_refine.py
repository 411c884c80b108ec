"""GPU parity of the off-grid power P(r, z), its adjoint and refinement,
through the C ABI, against the FP64 oracle evaluated on the same spectrum."""
import math

import numpy as np
import pytest

import synth
from oracle import fdas64 as o

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def setup(lib, n, n_truth, seed, store="f32", small_z_first=False):
    truths, starts = synth.refine_candidates(seed, n_truth, r_gap=400.0)
    if small_z_first:
        t = truths[0]
        truths[0] = synth.Injection(t.amp, t.r_mean - 0.005, 0.01, t.phase)
    xt = synth.make_series_device(n, truths, seed, 0)
    pl = lib.Plan(store=store, n_samples=n, z_min=-96.0, z_max=96.0, z_step=1.0, make_templates=False)
    spec = pl.spectrum(xt, [0], [n])
    a = spec.float().cpu().numpy().astype(np.float64)
    a = a[:, 0] + 1j * a[:, 1]
    return pl, spec, a, truths, starts


def smooth_in_z(z, h):
    """True where z - h, z and z + h share the window half-width ceil(|z|/2)."""
    c = np.ceil(np.abs(z) / 2)
    return (np.ceil(np.abs(z + h) / 2) == c) & (np.ceil(np.abs(z - h) / 2) == c)


def test_rz_power_and_y_match_oracle(lib):
    import torch
    n = 1 << 18
    say("fdas_rz_power", n)
    pl, spec, a, truths, starts = setup(lib, n, 64, 41)
    st = starts.copy()
    st[:4, 1] = [0.0, 1e-3, -0.02, 0.3]   # small-|z| branch and z = 0
    st[4:8, 0] = np.floor(st[4:8, 0])     # integer r
    nb = n // 2                           # windows cut by the spectrum's ends
    st[8:14, 0] = [0.3, 5.5, 17.9, nb - 3.2, nb - 0.5, nb - 20.25]
    st[8:14, 1] = [0.0, 30.0, -60.0, 12.0, -0.01, 90.0]
    r = torch.tensor(st[:, 0], dtype=torch.float64, device="cuda")
    z = torch.tensor(st[:, 1], dtype=torch.float64, device="cuda")
    p, y = pl.rz_power(spec, r, z)
    p = p.cpu().numpy()
    y = y.cpu().numpy()
    rf, zf = r.cpu().numpy(), z.cpu().numpy()
    for i in range(len(st)):
        yo = o.rz_amplitude(a, rf[i], zf[i])
        assert abs(y[i] - yo) <= 1e-9 * max(1.0, abs(yo)), (i, y[i], yo)
        assert abs(p[i] - abs(yo) ** 2) <= 1e-9 * max(1.0, abs(yo) ** 2)


def test_rz_gradients_match_oracle_and_differences(lib):
    import torch
    n = 1 << 18
    say("fdas_rz_power_grad", n)
    pl, spec, a, truths, starts = setup(lib, n, 48, 42)
    st = starts.copy()
    st[:3, 1] = [0.0, 2e-3, -0.04]
    r = torch.tensor(st[:, 0], dtype=torch.float64, device="cuda")
    z = torch.tensor(st[:, 1], dtype=torch.float64, device="cuda")
    gp = torch.linspace(0.5, 2.0, len(st), device="cuda", dtype=torch.float64)
    p, y = pl.rz_power(spec, r, z)
    gr, gz, gs = pl.rz_power_grad(spec, r, z, gp, y=y)
    gr2, gz2, gs2 = pl.rz_power_grad(spec, r, z, gp, y=y)
    assert torch.equal(gs, gs2) and torch.equal(gr, gr2)   # deterministic accumulation
    gr, gz, gs = gr.cpu().numpy(), gz.cpu().numpy(), gs.cpu().numpy().astype(np.complex128)
    rf, zf = r.cpu().numpy(), z.cpu().numpy()
    g = gp.cpu().numpy()
    want_gs = np.zeros(len(a), complex)
    for i in range(len(st)):
        P, dr, dz, ks, ga = o.rz_power_grad(a, rf[i], zf[i])
        assert abs(gr[i] - g[i] * dr) <= 1e-8 * max(1.0, abs(g[i] * dr)), (i, gr[i], g[i] * dr)
        assert abs(gz[i] - g[i] * dz) <= 1e-8 * max(1.0, abs(g[i] * dz)), (i, gz[i], g[i] * dz)
        want_gs[ks] += g[i] * ga
    np.testing.assert_allclose(gs, want_gs, rtol=0, atol=1e-5 * np.abs(want_gs).max())
    # central differences of the GPU's own forward, h = 1e-3
    h = 1e-3
    rr, zz = rf[:16], zf[:16]
    def P(rv, zv):
        pp, _ = pl.rz_power(spec, torch.tensor(rv, dtype=torch.float64, device="cuda"),
                            torch.tensor(zv, dtype=torch.float64, device="cuda"), keep_y=False)
        return pp.cpu().numpy().astype(np.float64)
    fr = (P(rr + h, zz) - P(rr - h, zz)) / (2 * h)
    fz = (P(rr, zz + h) - P(rr, zz - h)) / (2 * h)
    scale = np.maximum(1.0, P(rr, zz))
    # P is piecewise smooth (window steps at integer r and even z): a central
    # difference is taken only where both points lie in the same piece
    okr = np.floor(rr + h) == np.floor(rr - h)
    assert np.all((np.abs(gr[:16] / g[:16] - fr) <= 1e-4 * scale)[okr])
    ok = smooth_in_z(zz, h)
    assert ok.sum() >= 14 and okr.sum() >= 14
    assert np.all((np.abs(gz[:16] / g[:16] - fz) <= 1e-4 * scale)[ok])


def test_autograd_function(lib):
    import torch
    n = 1 << 17
    say("RZPower autograd", n)
    truths, starts = synth.refine_candidates(43, 8, r_gap=400.0)
    x = synth.make_series(n, truths, 43, 0)
    pl = lib.Plan(n_samples=n, z_min=-96.0, z_max=96.0, z_step=1.0, make_templates=False)
    spec = pl.spectrum(torch.from_numpy(x).to("cuda"), [0], [n])
    sc = torch.view_as_complex(spec.clone()).requires_grad_(True)
    r = torch.tensor(starts[:, 0], dtype=torch.float64, device="cuda", requires_grad=True)
    z = torch.tensor(starts[:, 1], dtype=torch.float64, device="cuda", requires_grad=True)
    p = lib.rz_power(sc, r, z, pl)
    (p * torch.arange(1, 9, device="cuda")).sum().backward()
    gr, gz, gs = pl.rz_power_grad(spec, r.detach(), z.detach(), torch.arange(1, 9, device="cuda").double())
    assert torch.allclose(r.grad, gr) and torch.allclose(z.grad, gz)
    assert torch.equal(sc.grad, gs)


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_refine_reaches_oracle_optimum(lib, store):
    import torch
    n = 1 << 18
    say("fdas_refine", n, store)
    pl, spec, a, truths, starts = setup(lib, n, 12, 44, store=store, small_z_first=True)
    st = starts.copy()
    st[0] = (truths[0].r_mean + 0.3, 0.02)           # near-zero drift start (truth z = 0.01)
    r = torch.tensor(st[:, 0], dtype=torch.float64, device="cuda")
    z = torch.tensor(st[:, 1], dtype=torch.float64, device="cuda")
    rr, zz, pf = pl.refine(spec, r, z, n_iter=40)
    rr, zz, pf = rr.cpu().numpy(), zz.cpu().numpy(), pf.cpu().numpy()
    for i in range(len(st)):
        ro, zo, po = o.refine_optimum(a, st[i, 0], st[i, 1])
        # the FP64 final power is the oracle's P at the returned position
        assert abs(pf[i] - o.rz_power(a, rr[i], zz[i])) <= 1e-9 * po
        assert abs(pf[i] - po) <= 1e-3 * po, (i, pf[i], po)
        assert abs(rr[i] - ro) <= 0.02 and abs(zz[i] - zo) <= 0.1, (i, rr[i], ro, zz[i], zo)


def test_refine_full_size_sampled(lib):
    """N = 2^22 with 4096 candidates perturbed by up to 0.5 bin and 1 z;
    64 are checked against the oracle's gradient and optimum."""
    import torch
    n = 1 << 22
    say("fdas_refine full size", n)
    pl, spec, a, truths, starts = setup(lib, n, 4096, 4)
    r = torch.tensor(starts[:, 0], dtype=torch.float64, device="cuda")
    z = torch.tensor(starts[:, 1], dtype=torch.float64, device="cuda")
    gp = torch.ones(4096, device="cuda", dtype=torch.float64)
    p, y = pl.rz_power(spec, r, z)
    gr, gz, _ = pl.rz_power_grad(spec, r, z, gp, y=y, want_spectrum=False)
    rr, zz, pf = pl.refine(spec, r, z, n_iter=40)
    sel = np.random.default_rng(0).choice(4096, 64, replace=False)
    rf, zf = r.cpu().numpy(), z.cpu().numpy()
    gr, gz = gr.cpu().numpy(), gz.cpu().numpy()
    rr, zz, pf = rr.cpu().numpy(), zz.cpu().numpy(), pf.cpu().numpy()
    for i in sel[:64]:
        P, dr, dz, _, _ = o.rz_power_grad(a, rf[i], zf[i])
        assert abs(gr[i] - dr) <= 1e-8 * max(1.0, abs(dr)) and abs(gz[i] - dz) <= 1e-8 * max(1.0, abs(dz))
        # central differences, h = 1e-3, of the GPU's own forward
        h = 1e-3
        rp = torch.tensor([rf[i] + h, rf[i] - h, rf[i], rf[i]], dtype=torch.float64, device="cuda")
        zp = torch.tensor([zf[i], zf[i], zf[i] + h, zf[i] - h], dtype=torch.float64, device="cuda")
        pp, _ = pl.rz_power(spec, rp, zp, keep_y=False)
        pp = pp.cpu().numpy()
        if np.floor(rf[i] + h) == np.floor(rf[i] - h):
            assert abs((pp[0] - pp[1]) / (2 * h) - gr[i]) <= 1e-4 * max(1.0, P)
        if smooth_in_z(zf[i], h):
            assert abs((pp[2] - pp[3]) / (2 * h) - gz[i]) <= 1e-4 * max(1.0, P)
    for i in sel[:16]:
        ro, zo, po = o.refine_optimum(a, rf[i], zf[i])
        assert abs(pf[i] - po) <= 1e-3 * po and abs(rr[i] - ro) <= 0.02, i
        # The window half-width m + ceil(|z|/2) steps at even z, so P is
        # piecewise smooth: ascent may stop at the maximum of the piece next
        # to the oracle's (grid search sees across the step).  Then the two
        # agree in P (above) but z may differ by up to the step's reach.
        same_piece = np.ceil(abs(zz[i]) / 2) == np.ceil(abs(zo) / 2)
        assert abs(zz[i] - zo) <= (0.1 if same_piece else 0.5), (i, zz[i], zo)
    # every truth's refined position lies within a bin and 1 z of it
    tr = np.array([t.r_mean for t in truths])
    tz = np.array([t.z for t in truths])
    assert np.mean((np.abs(rr - tr) < 1.0) & (np.abs(zz - tz) < 1.5)) > 0.99


# ------------------------------------------------------- harmonic refinement

def harmonic_trains(seed, n_train, H, n):
    """Fundamentals drawn in [3000, (N/2 - 400)/H] so that no harmonic of one
    train comes within 300 bins of a harmonic of another, z in [-20, 20],
    amplitudes falling as 1/k; each train is H injections (harmonic k at
    k rbar drifting by k z)."""
    rng = np.random.default_rng(seed)
    inj, truth = [], []
    taken = []
    for i in range(n_train):
        while True:
            rbar = rng.uniform(3000.0, (n // 2 - 400) / H)
            pos = rbar * np.arange(1, H + 1)
            if all(np.min(np.abs(pos - p)) > 300 for p in taken):
                break
        taken.extend(pos)
        z = rng.uniform(-20, 20)
        a0 = rng.uniform(0.04, 0.06)
        for k in range(1, H + 1):
            inj.append(synth.Injection(a0 / k, k * (rbar - z / 2), k * z, rng.uniform(0, 2 * np.pi)))
        truth.append((rbar, z))
    return inj, np.array(truth)


def test_refine_harmonics_with_one_harmonic_is_refine(lib):
    import torch
    n = 1 << 18
    say("fdas_refine_harmonics H = 1 vs fdas_refine", n)
    pl, spec, a, truths, starts = setup(lib, n, 24, 45)
    r = torch.tensor(starts[:, 0], dtype=torch.float64, device="cuda")
    z = torch.tensor(starts[:, 1], dtype=torch.float64, device="cuda")
    r1, z1, p1 = pl.refine(spec, r, z, n_iter=40)
    r2, z2, p2 = pl.refine_harmonics(spec, r, z, 1, n_iter=40)
    assert torch.equal(r1, r2) and torch.equal(z1, z2) and torch.equal(p1, p2)


def test_refine_harmonics_objective_matches_oracle(lib):
    """n_iter = 0: S(r, z) for mixed harmonic counts, including positions whose
    upper harmonics leave the spectrum (zeros there) and invalid counts."""
    import torch
    n = 1 << 18
    say("fdas_refine_harmonics objective", n)
    inj, truth = harmonic_trains(46, 8, 4, n)
    x = synth.make_series(n, inj, 46, 0)
    pl = lib.Plan(n_samples=n, z_min=-96.0, z_max=96.0, z_step=1.0, make_templates=False)
    spec = pl.spectrum(torch.from_numpy(x).to("cuda"), [0], [n])
    a = spec.float().cpu().numpy().astype(np.float64)
    a = a[:, 0] + 1j * a[:, 1]
    rng = np.random.default_rng(7)
    hs = np.array([1, 2, 3, 4, 8, 16, 5, 32] * 4, dtype=np.int32)
    rr = np.concatenate([truth[:, 0], rng.uniform(100, 20000, 16), [n // 2 / 3 - 1.5, n // 2 / 5 + 0.25,
                                                                    n // 2 - 10.7, 40.2, 7.9, 60000.5, 1000.0,
                                                                    2345.6]])
    zz = np.concatenate([truth[:, 1], rng.uniform(-6, 6, 16), [0.0, 3.0, -5.5, 1e-3, 2.0, -1.0, 0.0, 5.9]])
    hs = hs[: len(rr)]
    hs[-2:] = [0, 33]                       # invalid counts
    r = torch.tensor(rr, dtype=torch.float64, device="cuda")
    z = torch.tensor(zz, dtype=torch.float64, device="cuda")
    ro, zo, S = pl.refine_harmonics(spec, r, z, torch.tensor(hs), n_iter=0)
    S = S.cpu().numpy()
    assert torch.equal(ro, r) and torch.equal(zo, z)
    for i in range(len(rr) - 2):
        want = o.rz_power_harmonics(a, rr[i], zz[i], int(hs[i]))
        assert abs(S[i] - want) <= 1e-9 * max(1.0, want), (i, hs[i], S[i], want)
    assert np.isnan(S[-2:]).all()


@pytest.mark.parametrize("store,H", [("f32", 4), ("bf16", 4), ("f32", 8), ("bf16", 16), ("f32", 3), ("f32", 2)])
def test_refine_harmonics_reaches_oracle_optimum(lib, store, H):
    """Harmonic trains in noise, starts off by up to 0.3/H bin and 0.6/H z at
    the fundamental: the GPU ascent of S reaches the oracle's optimum (S to
    1e-3; position to 0.02 bin, z to 0.1, or 0.5 where a window step lies in
    between), and its final S is the oracle's S at the returned position."""
    import torch
    n = 1 << 18
    say("fdas_refine_harmonics", store, H)
    # H = 16: all four lane groups busy; H = 2, 3: groups idle in every step
    n_train = {4: 6, 16: 2}.get(H, 3)
    inj, truth = harmonic_trains(47 + H, n_train, H, n)
    x = synth.make_series(n, inj, 47, H)
    pl = lib.Plan(store=store, n_samples=n, z_min=-96.0, z_max=96.0, z_step=1.0, make_templates=False)
    spec = pl.spectrum(torch.from_numpy(x).to("cuda"), [0], [n])
    a = spec.float().cpu().numpy().astype(np.float64)
    a = a[:, 0] + 1j * a[:, 1]
    rng = np.random.default_rng(48)
    st = truth + np.stack([rng.uniform(-0.3, 0.3, n_train), rng.uniform(-0.6, 0.6, n_train)], axis=1) / H
    r = torch.tensor(st[:, 0], dtype=torch.float64, device="cuda")
    z = torch.tensor(st[:, 1], dtype=torch.float64, device="cuda")
    rr, zz, S = pl.refine_harmonics(spec, r, z, H, n_iter=60)
    rr, zz, S = rr.cpu().numpy(), zz.cpu().numpy(), S.cpu().numpy()
    for i in range(n_train):
        assert abs(S[i] - o.rz_power_harmonics(a, rr[i], zz[i], H)) <= 1e-9 * S[i]
        ro, zo, So = o.refine_harmonic_optimum(a, st[i, 0], st[i, 1], H)
        assert abs(S[i] - So) <= 1e-3 * So, (i, S[i], So)
        assert abs(rr[i] - ro) <= 0.02, (i, rr[i], ro)
        same_piece = all(np.ceil(abs(k * zz[i]) / 2) == np.ceil(abs(k * zo) / 2) for k in range(1, H + 1))
        assert abs(zz[i] - zo) <= (0.1 if same_piece else 0.5), (i, zz[i], zo)
        # the refined fundamental is the train's, within a bin and 1.5 z at its top harmonic up
        # to H = 8; with amplitudes falling as 1/k every harmonic adds the same z curvature at
        # the fundamental, so the noise error there shrinks only as 1/sqrt(H) while the top
        # harmonic multiplies it by H: the z bound grows as sqrt(H / 8) above H = 8
        zb = 1.5 * max(1.0, math.sqrt(H / 8.0))
        assert abs(rr[i] - truth[i, 0]) * H < 1.0 and abs(zz[i] - truth[i, 1]) * H < zb


def test_invalid_positions_give_nan(lib):
    """Non-finite r or z, |z| > 2^17 or |r| >= 2^52 evaluate to NaN without
    touching the spectrum; refinement leaves such candidates where they are
    (the values used here are harmless even without the check: a NaN window
    converts to zero width, z just past 2^17 to a finite window, and r = 2^53
    reads only bins past the spectrum)."""
    import torch
    n = 1 << 17
    say("invalid refinement positions", n)
    pl = lib.Plan(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, make_templates=False)
    spec = pl.spectrum(torch.from_numpy(synth.make_series(n, [], 5, 0)).to("cuda"), [0], [n])
    r = torch.tensor([float("nan"), 1000.0, 2.0 ** 53, 1000.3], dtype=torch.float64, device="cuda")
    z = torch.tensor([0.0, 131074.0, 0.0, 2.0], dtype=torch.float64, device="cuda")
    p, y = pl.rz_power(spec, r, z)
    p = p.cpu().numpy()
    assert np.isnan(p[:3]).all() and np.isfinite(p[3])
    gr, gz, gs = pl.rz_power_grad(spec, r, z, torch.ones(4, dtype=torch.float64, device="cuda"))
    assert np.isnan(gr.cpu().numpy()[:3]).all() and torch.isfinite(gs).all()
    rr, zz, pf = pl.refine(spec, r, z, n_iter=5)
    assert torch.equal(zz[:3], z[:3]) and torch.equal(rr[1:3], r[1:3]) and np.isnan(pf.cpu().numpy()[:3]).all()
    r2, z2, S = pl.refine_harmonics(spec, torch.tensor([500.0], dtype=torch.float64, device="cuda"),
                                    torch.tensor([70000.0], dtype=torch.float64, device="cuda"), 16, n_iter=3)
    assert np.isnan(S.cpu().numpy()).all()   # harmonic 2 already lies at z = 140000


def test_spectrum_gradient_of_large_terms_does_not_overflow(lib):
    """Terms far beyond 2^23 (spectrum scaled by 10^4, grad_p up to 10^3:
    sums ~ 4e7): the fixed-point unit shrinks so that no sum
    overflows, and grad_spectrum matches the oracle's gradient to 1e-5 of
    its largest value, bit for bit the same in a second call; a NaN grad_p
    leaves its terms out and is reported, the other candidates' terms stay."""
    import torch
    n = 1 << 18
    say("fdas_rz_power_grad large terms", n)
    pl, spec, a, truths, starts = setup(lib, n, 24, 44)
    spec_big = spec * 1.0e4
    a_big = spec_big.cpu().numpy().astype(np.float64)
    a_big = a_big[:, 0] + 1j * a_big[:, 1]
    r = torch.tensor(starts[:, 0], dtype=torch.float64, device="cuda")
    z = torch.tensor(starts[:, 1], dtype=torch.float64, device="cuda")
    gp = torch.linspace(1.0, 1000.0, len(starts), device="cuda", dtype=torch.float64)
    p, y = pl.rz_power(spec_big, r, z)
    gr, gz, gs = pl.rz_power_grad(spec_big, r, z, gp, y=y)
    _, _, gs2 = pl.rz_power_grad(spec_big, r, z, gp)   # y recomputed
    pl.check()
    assert torch.equal(gs, gs2)
    gs = gs.cpu().numpy().astype(np.complex128)
    rf, zf, g = r.cpu().numpy(), z.cpu().numpy(), gp.cpu().numpy()
    want = np.zeros(len(a_big), complex)
    for i in range(len(starts)):
        _, _, _, ks, ga = o.rz_power_grad(a_big, rf[i], zf[i])
        want[ks] += g[i] * ga
    big = np.abs(want).max()
    assert big > 2.0 ** 23          # a fixed 2^-40 unit would have overflowed
    np.testing.assert_allclose(gs, want, rtol=0, atol=1e-5 * big)
    # a NaN upstream gradient: reported, its terms left out
    gp_nan = gp.clone()
    gp_nan[0] = float("nan")
    _, _, gs3 = pl.rz_power_grad(spec_big, r, z, gp_nan, y=y)
    with pytest.raises(lib.FdasError, match="not finite"):
        pl.check()
    pl.check()
    _, _, _, ks0, ga0 = o.rz_power_grad(a_big, rf[0], zf[0])
    want3 = want.copy()
    want3[ks0] -= g[0] * ga0
    np.testing.assert_allclose(gs3.cpu().numpy().astype(np.complex128), want3, rtol=0, atol=1e-5 * big)
