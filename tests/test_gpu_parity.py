"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Every case prints the entry point, shape and seed it runs before it runs.
Tolerances: FP32 storage 1e-4 relative power error (|dP| <= 1e-4 max(P, 1));
BF16/FP16 storage 3e-2 relative on detections (the 3 % sensitivity bound the
paper quotes for a bfloat16 convolution stage) and 5e-2 max(P,1) elsewhere.
"""
import math

import numpy as np
import pytest

import synth
from oracle import fdas64 as o

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def to_np_complex(spec_t):
    a = spec_t.float().cpu().numpy().astype(np.float64)
    return a[:, 0] + 1j * a[:, 1]


def plane_np(plane_t, Z, nbins):
    return plane_t.float().cpu().numpy().astype(np.float64).reshape(Z, nbins)


# ---------------------------------------------------------------- FFT engine

@pytest.mark.parametrize("L", [256, 512, 1024, 2048, 4096, 8192])
def test_fft_engine_matches_fp64_fft(lib, L):
    import torch
    say("fdas_test_fft", L)
    plan = lib.Plan(n_samples=1 << 17, z_min=-16.0, z_max=16.0, z_step=2.0, segment_len=1024, make_templates=False)
    rng = np.random.default_rng(L)
    batch = 37
    x = (rng.standard_normal((batch, L)) + 1j * rng.standard_normal((batch, L))).astype(np.complex64)
    xt = torch.from_numpy(x).to(plan.device)
    for d in (-1, 1):
        y = plan.test_fft(xt, d).cpu().numpy().astype(np.complex128)
        ref = np.fft.fft(x.astype(np.complex128), axis=1) if d < 0 else np.fft.ifft(x.astype(np.complex128), axis=1) * L
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        assert err < 1e-6 * math.log2(L), (L, d, err)


# ---------------------------------------------------------------- templates

@pytest.mark.parametrize("grid,L", [((-16.0, 16.0, 2.0), 1024), ((-96.0, 96.0, 1.0), 8192), ((-96.0, 96.0, 1.0), 1024)])
def test_templates_match_oracle(lib, grid, L):
    say("fdas_make_templates", grid, L)
    zmin, zmax, dz = grid
    plan = lib.Plan(n_samples=1 << 17, z_min=zmin, z_max=zmax, z_step=dz, segment_len=L)
    taps_t, spec_t = plan.templates()
    taps = taps_t.cpu().numpy()
    zs = o.z_grid(zmin, zmax, dz)
    ref, hmax = o.template_taps(zs)
    assert hmax == plan.hmax
    np.testing.assert_allclose(taps, ref, rtol=0, atol=1e-12)
    # spectra: T[k] = (1/L) sum_q t_q exp(2 pi i k q / L), from the oracle's taps
    K = 2 * hmax + 1
    arr = np.zeros((len(zs), L), complex)
    for i in range(K):
        arr[:, (L - (i - hmax)) % L] = ref[:, i]
    want = np.fft.fft(arr, axis=1) / L
    got = spec_t.float().cpu().numpy().astype(np.float64)
    got = got[..., 0] + 1j * got[..., 1]
    scale = np.abs(want).max()
    assert np.max(np.abs(got - want)) < 2e-7 * scale


# ---------------------------------------------------------------- spectrum

@pytest.mark.parametrize("n", [1 << 17, 1 << 18, 1 << 21, 1 << 23])
def test_spectrum_matches_oracle(lib, n):
    import torch
    say("fdas_spectrum", n)
    x = synth.make_series(n, [synth.Injection(0.05, 5000.0, 12.0, 0.3)], 21, n)
    xt = torch.from_numpy(x).to("cuda")
    for norm in ("none", "median", "variance", "rednoise"):
        plan = lib.Plan(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, segment_len=1024, norm=norm,
                        make_templates=False)
        s = to_np_complex(plan.spectrum(xt, [0], [n]))
        ref = o.normalise(o.spectrum(x), norm, n_samples=n)
        # per bin: |dA_r| <= 1e-5 max(|A_r|, rms |A|) (the rms is ~1 after
        # normalisation, sqrt(N) without it)
        rms = math.sqrt(np.mean(np.abs(ref) ** 2))
        worst = np.max(np.abs(s - ref) / np.maximum(np.abs(ref), rms))
        say(f"  {norm}: worst per-bin error {worst:.2e} of max(|A|, rms)")
        assert worst <= 1e-5, (norm, worst)
        assert s[0] == 0


def test_median_block_selection_is_exact(lib):
    """Lower median per block: with every |A|^2 distinct in FP32 the GPU's scale
    must be sqrt(ln2 / m_b) of the FP32 values' exact rank-(B-1)/2 element."""
    import torch
    n = 1 << 17
    say("fdas_spectrum median exact", n)
    x = synth.make_series(n, [], 22, 0)
    xt = torch.from_numpy(x).to("cuda")
    raw = lib.Plan(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, norm="none", make_templates=False)
    med = lib.Plan(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, norm="median", make_templates=False)
    a = raw.spectrum(xt, [0], [n]).cpu().numpy().astype(np.float32)
    b = med.spectrum(xt, [0], [n]).cpu().numpy().astype(np.float64)
    p32 = a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1]
    blocks = p32.reshape(-1, 2048)
    m = np.sort(blocks, axis=1)[:, 1023].astype(np.float64)
    scale = np.sqrt(np.log(2.0) / m)
    got_scale = np.abs(b[:, 0] + 1j * b[:, 1]).reshape(-1, 2048)[:, 5:] / np.abs(
        a[:, 0].astype(np.float64) + 1j * a[:, 1]).reshape(-1, 2048)[:, 5:]
    np.testing.assert_allclose(np.median(got_scale, axis=1), scale, rtol=2e-6)


@pytest.mark.parametrize("B", [256, 2048, 4096])
def test_rednoise_sub_block_selection_is_exact(lib, B):
    """Rednoise normalisation: in every sub-block (width 32 ... B by the
    frequency rule) the GPU's scale is sqrt(ln2 / m) of the exact rank-(w-1)/2
    element of the FP32 powers, on a series with a steep red continuum."""
    import torch
    n = 1 << 18
    say("fdas_spectrum rednoise exact", n, B)
    rng = np.random.default_rng(23)
    x = rng.standard_normal(n) + 24.0 * np.cumsum(rng.standard_normal(n)) / math.sqrt(n)
    x = (x - x.mean()).astype(np.float32)
    xt = torch.from_numpy(x).to("cuda")
    kw = dict(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, norm_block=B, make_templates=False)
    raw = lib.Plan(norm="none", **kw)
    red = lib.Plan(norm="rednoise", **kw)
    a = raw.spectrum(xt, [0], [n]).cpu().numpy().astype(np.float32)
    b = red.spectrum(xt, [0], [n]).cpu().numpy().astype(np.float64)
    p32 = a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1]
    mag_a = np.abs(a[:, 0].astype(np.float64) + 1j * a[:, 1])
    mag_b = np.abs(b[:, 0] + 1j * b[:, 1])
    checked = 0
    for blk in range(min(n // 2 // B, 12)):
        w = o.rednoise_width(blk, B)
        for j in range(B // w):
            lo = blk * B + j * w
            m = np.sort(p32[lo: lo + w])[(w - 1) // 2].astype(np.float64)
            ok = mag_a[lo: lo + w] > 0
            got = np.median(mag_b[lo: lo + w][ok] / mag_a[lo: lo + w][ok])
            assert abs(got / math.sqrt(math.log(2.0) / m) - 1) < 2e-6, (blk, j, w)
            checked += 1
    assert checked >= 12


# ---------------------------------------------------------------- power plane

def gpu_plane(lib, x, params, store="f32", plane="f32", norm="median"):
    import torch
    n = len(x)
    pl = lib.Plan(store=store, plane=plane, norm=norm, **params)
    xt = torch.from_numpy(x).to("cuda")
    spec = pl.new_spectrum(n // 2)
    P = pl.convolve(xt, [0], [n], spectrum=spec)
    return pl, P, spec


def small_params(L=2048):
    return dict(n_samples=1 << 17, z_min=-16.0, z_max=16.0, z_step=2.0, n_harmonics=4, segment_len=L)


@pytest.mark.parametrize("L", [1024, 2048, 4096, 8192])
def test_plane_fp32_small_case_full_parity(lib, L):
    x, inj, _ = synth.small_case(seed=1)
    say("fdas_convolve f32 small case", L)
    pl, P, _ = gpu_plane(lib, x, small_params(L))
    zs = o.z_grid(-16, 16, 2)
    ref = o.power_plane(o.normalise(o.spectrum(x), "median"), zs)
    got = plane_np(P, pl.Z, len(x) // 2)
    bad = np.abs(got - ref) > 1e-4 * np.maximum(ref, 1.0)
    assert not bad.any(), (np.argwhere(bad)[:5], np.abs(got - ref).max())
    # the noisy peak sits where the oracle's does, next to the injection
    assert np.argmax(got) == np.argmax(ref)
    j, r = np.unravel_index(np.argmax(got), got.shape)
    assert abs(r - 5010) <= 2 and zs[j] >= 12


@pytest.mark.parametrize("radix,interbin", [(8, 0), (4, 0), (8, 1), (4, 1)])
def test_plane_radix_plans_match_oracle(lib, radix, interbin):
    """The 1024-point convolution FFT built with passes of radix 8 (8 8 8 2)
    and 4 (five passes), the autotuner's other radix plans: every cell of the
    small case's FP32 plane (bin or half-bin) within 1e-4 max(P, 1) of the
    oracle's."""
    x, inj, _ = synth.small_case(seed=1)
    say("fdas_convolve radix plan", radix, "interbin" if interbin else "bins")
    n = len(x)
    pl = lib.Plan(store="f32", plane="f32", n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, n_harmonics=4,
                  segment_len=1024, fft_radix=radix, interbin=interbin)
    import torch
    P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
    zs = o.z_grid(-16, 16, 2)
    a = o.normalise(o.spectrum(x), "median")
    ref = o.interbin_plane(a, zs) if interbin else o.power_plane(a, zs)
    got = P.cpu().numpy().astype(np.float64).reshape(pl.Z, -1)
    bad = np.abs(got - ref) > 1e-4 * np.maximum(ref, 1.0)
    assert not bad.any(), (np.argwhere(bad)[:5], np.abs(got - ref).max())


@pytest.mark.parametrize("store,plane", [("bf16", "bf16"), ("bf16", "f32"), ("f16", "f16")])
def test_plane_reduced_precision_small_case(lib, store, plane):
    x, inj, _ = synth.small_case(seed=1)
    say("fdas_convolve", store, plane, "small case")
    pl, P, _ = gpu_plane(lib, x, small_params(2048), store=store, plane=plane)
    zs = o.z_grid(-16, 16, 2)
    ref = o.power_plane(o.normalise(o.spectrum(x), "median"), zs)
    got = plane_np(P, pl.Z, len(x) // 2)
    e = o.power_errors(got, ref, tau1=o.threshold(1))
    assert e["max_rel_det"] < 3e-2, e
    assert np.all(np.abs(got - ref) < 5e-2 * np.maximum(ref, 1.0))


def test_plane_ragged_batch_parity(lib):
    """Uneven batch (full-length, 2x- and 4x-decimated series) in one call,
    checked series by series against the oracle; includes a tail segment."""
    import torch
    n = 1 << 19
    lens = [n, n // 2, n // 4, n, n // 4, n // 2]
    xs, truths = synth.batch_series(lens, seed=31, amp=(0.05, 0.08))
    flat, offs, lens_a = synth.concat(xs)
    say("fdas_convolve ragged batch", lens)
    pl = lib.Plan(n_samples=n, max_batch_samples=int(lens_a.sum()), z_min=-16.0, z_max=16.0, z_step=2.0,
                  n_harmonics=4, segment_len=1024)
    P = pl.convolve(torch.from_numpy(flat).to("cuda"), offs, lens_a)
    got = P.cpu().numpy().astype(np.float64)
    zs = o.z_grid(-16, 16, 2)
    pos = 0
    for x in xs:
        nb = len(x) // 2
        ref = o.power_plane(o.normalise(o.spectrum(x), "median"), zs)
        g = got[pos: pos + pl.Z * nb].reshape(pl.Z, nb)
        assert np.all(np.abs(g - ref) <= 1e-4 * np.maximum(ref, 1.0))
        pos += pl.Z * nb


@pytest.mark.parametrize("L,store,plane", [(8192, "f32", "f32"), (8192, "bf16", "bf16"), (1024, "bf16", "bf16")])
def test_plane_ska_full_size_sampled(lib, L, store, plane):
    """N = 2^23, 193 templates: GPU plane at sampled cells and at every injected
    peak against the oracle's direct sums."""
    x, inj, params = synth.ska_single(seed=2)
    params = dict(params)
    params["segment_len"] = L
    params.pop("norm")
    say("fdas_convolve SKA single", L, store, plane)
    pl, P, _ = gpu_plane(lib, x, params, store=store, plane=plane)
    nb = len(x) // 2
    got = P.view(pl.Z, nb)
    zs = o.z_grid(-96, 96, 1)
    taps, _ = o.template_taps(zs)
    a = o.normalise(o.spectrum(x), "median")
    rng = np.random.default_rng(5)
    rows = rng.integers(0, pl.Z, 3000)
    cols = rng.integers(0, nb, 3000)
    cols[:50] = np.arange(50)                 # spectrum start
    cols[50:100] = nb - 1 - np.arange(50)     # spectrum end (tail segment)
    # injected peaks: nearest grid cell to (rbar, z)
    pk_r = np.array([int(round(i.r_mean)) for i in inj])
    pk_j = np.array([int(round(i.z - zs[0])) for i in inj])
    rows = np.concatenate([rows, pk_j])
    cols = np.concatenate([cols, pk_r])
    ref = o.power_cells(a, taps, rows, cols)
    g = got[rows, cols].float().cpu().numpy().astype(np.float64)
    tol = 1e-4 if store == "f32" else 3e-2
    assert np.all(np.abs(g - ref) <= tol * np.maximum(ref, 1.0)), np.max(np.abs(g - ref) / np.maximum(ref, 1))
    # every injection is far above threshold at its peak cell
    assert np.all(g[-len(inj):] > o.threshold(1))


@pytest.mark.parametrize("store,tol", [("bf16", 3e-2), ("f32", 1e-4)])
def test_power_error_and_recall_against_oracle_ska_single(lib, store, tol):
    """The precision statement at full size, in the bench's configuration
    (N = 2^23, 193 templates, L = 1024, 8 injections): relative power error
    against the FP64 oracle at every cell within +-3 bins and +-4 z of each
    injection's peak whose oracle power is at least tau_1, and recall of the
    injections by the GPU's harmonic-sum candidates (within 1 bin and 1 z)."""
    import torch
    x, inj, params = synth.ska_single(seed=2)
    params = dict(params)
    params["segment_len"] = 1024
    params.pop("norm")
    say("precision vs oracle, SKA single", store)
    pl, P, _ = gpu_plane(lib, x, params, store=store, plane=store)
    n = len(x)
    nb = n // 2
    zs = o.z_grid(-96, 96, 1)
    taps, _ = o.template_taps(zs)
    a = o.normalise(o.spectrum(x), "median")
    rows, cols = [], []
    for i in inj:
        rc, jc = int(round(i.r_mean)), int(round(i.z + 96))
        for dj in range(-4, 5):
            for dr in range(-3, 4):
                if 0 <= jc + dj < pl.Z:
                    rows.append(jc + dj)
                    cols.append(rc + dr)
    rows, cols = np.array(rows), np.array(cols)
    ref = o.power_cells(a, taps, rows, cols)
    got = P.view(pl.Z, nb)[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].float().cpu().numpy()
    det = ref >= o.threshold(1)
    rel = np.abs(got.astype(np.float64) - ref)[det] / ref[det]
    cap = 1 << 20
    cands, count = pl.harmonic_sum(P, [n], capacity=cap)
    pl.check(count, cap)
    c = lib.candidates_to_numpy(cands, int(count.item()))
    found = sum(bool(np.any((np.abs(c["r"] - i.r_mean) <= 1.0) & (np.abs(c["z"] - i.z) <= 1.0))) for i in inj)
    say(f"{store}: {det.sum()} detection cells, max rel {rel.max():.3e}, median rel {np.median(rel):.3e}, "
        f"recall {found}/{len(inj)}")
    assert det.sum() >= 100
    assert rel.max() < tol
    assert found == len(inj)


# ---------------------------------------------------------------- harmonic sum

def run_search(lib, x, params, store="f32", plane="f32", capacity=1 << 16):
    pl, P, _ = gpu_plane(lib, x, params, store=store, plane=plane)
    n = len(x)
    cands, count = pl.harmonic_sum(P, [n], capacity=capacity)
    pl.check(count, capacity)
    c = lib.candidates_to_numpy(cands, int(count.item()))
    return pl, P, c


def test_harmonic_sum_candidates_match_oracle(lib):
    n = 1 << 17
    inj = [synth.Injection(0.05, 3000.0, 8.0, 0.1), synth.Injection(0.03, 11000.0, -12.0, 0.7)]
    x = synth.make_series(n, inj, 7, 0)
    params = small_params(1024)
    say("fdas_harmonic_sum small case")
    pl, P, c = run_search(lib, x, params)
    zs = o.z_grid(-16, 16, 2)
    got_plane = plane_np(P, pl.Z, n // 2)
    # oracle search on the oracle's own plane
    ref_plane = o.power_plane(o.normalise(o.spectrum(x), "median"), zs)
    ref = o.search(ref_plane, zs, 4, r_lo=pl.hmax, h_max=pl.hmax)
    tau = {H: o.threshold(H) for H in (1, 2, 4)}
    sums = o.harmonic_sums(ref_plane, int(np.argmin(np.abs(zs))), 4)

    def borderline(R, j):
        return any(abs(sums[H][j, R] - tau[H]) <= 1e-4 * tau[H] for H in (1, 2, 4))

    got = {(int(k["R"]), int(k["j"])): int(k["harm"]) for k in c}
    want = {(k.R, k.j): k.harm for k in ref}
    assert len(got) == len(c)  # one record per cell
    for cell in set(got) ^ set(want):
        assert borderline(*cell), cell
    for cell in set(got) & set(want):
        if got[cell] != want[cell]:
            assert borderline(*cell), cell
    assert len(want) >= 5
    # the GPU's reported power is the sum of its own plane's terms
    sums_gpu = o.harmonic_sums(got_plane, int(np.argmin(np.abs(zs))), 4)
    for k in c[:200]:
        assert abs(k["power"] - sums_gpu[int(k["harm"])][k["j"], k["R"]]) <= 1e-4 * k["power"]
        assert abs(k["sigma"] - o.gaussian_sigma(float(k["power"]), int(k["harm"]))) < 1e-3 * k["sigma"]


@pytest.mark.parametrize("plane_dt,nh", [("bf16", 16), ("f16", 16), ("f32", 16), ("bf16", 8), ("f32", 2), ("bf16", 1)])
def test_harmonic_sum_ragged_batch_matches_oracle(lib, plane_dt, nh):
    """Harmonic sums to nh over a ragged batch (2^19, 2^18 and 2^17 samples:
    the three length classes of one launch, 97 trials: bands on both sides of
    z = 0 and a one-trial edge band), against the oracle's sums of the GPU's
    own plane: the candidate cells, their stage and their power agree except
    where a sum lies within 1e-5 of a threshold (FP32 against FP64
    accumulation); every record's fundamental r = R/H and z = z_j/H is the
    oracle's."""
    import torch
    n = 1 << 19
    lens = [n, n // 2, n // 4, n // 4]
    xs, truths = synth.batch_series(lens, seed=61, inj_per_series=(1, 2), amp=(0.04, 0.07), z_abs=44.0)
    x, offs, _ = synth.concat(xs)
    say("fdas_harmonic_sum ragged batch", plane_dt, nh)
    pl = lib.Plan(store=plane_dt, plane=plane_dt, n_samples=n, max_batch_samples=sum(lens), z_min=-48.0,
                  z_max=48.0, z_step=1.0, n_harmonics=nh, segment_len=1024)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), offs, lens)
    cap = 1 << 22
    cands, count = pl.harmonic_sum(P, lens, capacity=cap)
    pl.check(count, cap)
    c = lib.candidates_to_numpy(cands, int(count.item()))
    zs = o.z_grid(-48, 48, 1)
    j0 = int(np.argmin(np.abs(zs)))
    tau = {H: o.threshold(H) for H in o.stages(nh)}
    Pall = P.float().cpu().numpy().astype(np.float64)
    off = 0
    n_cells = 0
    for s_, L_ in enumerate(lens):
        nb = L_ // 2
        plane = Pall[off: off + pl.Z * nb].reshape(pl.Z, nb)
        off += pl.Z * nb
        sums = o.harmonic_sums(plane, j0, nh)
        want = {(k.R, k.j): k for k in o.search(plane, zs, nh, r_lo=pl.hmax, h_max=pl.hmax)}
        mine = c[c["series"] == s_]
        got = {(int(k["R"]), int(k["j"])): k for k in mine}
        assert len(got) == len(mine)  # one record per cell

        def borderline(R, j):
            return any(abs(sums[H][j, R] - tau[H]) <= 1e-5 * tau[H] for H in tau)

        for cell in set(got) ^ set(want):
            assert borderline(*cell), (s_, cell)
        for cell in set(got) & set(want):
            g, w = got[cell], want[cell]
            if int(g["harm"]) != w.harm:
                assert borderline(*cell), (s_, cell, int(g["harm"]), w.harm)
                continue
            assert abs(float(g["power"]) - w.power) <= 1e-5 * w.power, (s_, cell)
            assert g["r"] == np.float32(w.r) and g["z"] == np.float32(w.z), (s_, cell, g["r"], w.r, g["z"], w.z)
        assert len(want) >= 20, (s_, len(want))
        n_cells += len(want)
    assert n_cells == len(c) or abs(n_cells - len(c)) <= 0.001 * n_cells


def test_cluster_matches_oracle_local_maxima(lib):
    """fdas_cluster on the records of a ragged batch search equals the
    oracle's local maxima of the same records, for three neighbourhoods, and
    when the record count exceeds the buffer."""
    import torch
    n = 1 << 18
    lens = [n, n // 2, n, n // 2]
    xs, truths = synth.batch_series(lens, seed=62, inj_per_series=(1, 2), amp=(0.04, 0.07), z_abs=44.0)
    x, offs, _ = synth.concat(xs)
    say("fdas_cluster")
    pl = lib.Plan(store="bf16", plane="bf16", n_samples=n, max_batch_samples=sum(lens), z_min=-48.0, z_max=48.0,
                  z_step=1.0, n_harmonics=16, segment_len=1024)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), offs, lens)
    cap = 1 << 22
    cands, count = pl.harmonic_sum(P, lens, capacity=cap)
    pl.check(count, cap)
    n_rec = int(count.item())
    c = lib.candidates_to_numpy(cands, n_rec)
    for rr, rj in ((2, 2), (0, 3), (5, 1)):
        keep = pl.cluster(cands, count, rr, rj)[:n_rec].cpu().numpy().astype(bool)
        want = o.local_maxima(c["series"], c["R"], c["j"], c["sigma"], rr, rj)
        assert np.array_equal(keep, want), (rr, rj, np.nonzero(keep != want)[0][:5])
        assert 0 < keep.sum() < n_rec
    # more records than the buffer holds: the first 500 are clustered
    small = cands[:500].clone()
    keep = pl.cluster(small, count, 2, 2).cpu().numpy().astype(bool)
    c5 = c[:500]
    assert np.array_equal(keep, o.local_maxima(c5["series"], c5["R"], c5["j"], c5["sigma"], 2, 2))


@pytest.mark.parametrize("z_max", [0, 1, 7, 15, 16, 17])
def test_harmonic_sum_small_z_grids(lib, z_max):
    """Z = 2 z_max + 1 trials = 1, 3, 15, 31, 33, 35: a single trial, bands
    cut by both plane edges, and grids one trial either side of a multiple of
    the 16-trial band.  A noise series with a strong injection; the GPU's
    candidates against the oracle's search of the GPU's own plane."""
    import torch
    n = 1 << 17
    inj = [synth.Injection(0.06, 12000.0, min(z_max, 5.0), 0.3)]
    x = synth.make_series(n, inj, 70 + z_max, 0)
    say("fdas_harmonic_sum small z grid", z_max)
    pl = lib.Plan(store="bf16", plane="bf16", n_samples=n, z_min=-float(z_max), z_max=float(z_max), z_step=1.0,
                  n_harmonics=16, segment_len=1024)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
    cap = 1 << 20
    cands, count = pl.harmonic_sum(P, [n], capacity=cap)
    pl.check(count, cap)
    c = lib.candidates_to_numpy(cands, int(count.item()))
    plane = plane_np(P, pl.Z, n // 2)
    zs = o.z_grid(-z_max, z_max, 1)
    sums = o.harmonic_sums(plane, z_max, 16)
    tau = {H: o.threshold(H) for H in o.stages(16)}
    want = {(k.R, k.j): k for k in o.search(plane, zs, 16, r_lo=pl.hmax, h_max=pl.hmax)}
    got = {(int(k["R"]), int(k["j"])): k for k in c}
    assert len(got) == len(c)

    def borderline(R, j):
        return any(abs(sums[H][j, R] - tau[H]) <= 1e-5 * tau[H] for H in tau)

    for cell in set(got) ^ set(want):
        assert borderline(*cell), cell
    for cell in set(got) & set(want):
        g, w = got[cell], want[cell]
        assert int(g["harm"]) == w.harm or borderline(*cell), cell
        if int(g["harm"]) == w.harm:
            assert abs(float(g["power"]) - w.power) <= 1e-5 * w.power, cell
    assert len(want) >= 5


def test_harmonic_sum_ska_full_size_sampled(lib):
    """The timed configuration (one 2^23-sample series, 193 trials, L = 1024,
    bf16 storage and plane, harmonic sums to 16): every candidate record has
    the stage and power the oracle computes from the GPU's plane at its cell,
    and on 300 000 sampled cells plus every cell near the 8 injections the
    passing cells are exactly the records (up to sums within 1e-5 of a
    threshold)."""
    import torch
    x, inj, _ = synth.ska_single(seed=2, n=1 << 23)
    n = len(x)
    nb = n // 2
    say("fdas_harmonic_sum full size, bench configuration")
    pl = lib.Plan(store="bf16", plane="bf16", n_samples=n, z_min=-96.0, z_max=96.0, z_step=1.0, n_harmonics=16,
                  segment_len=1024)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
    cap = 1 << 22
    cands, count = pl.harmonic_sum(P, [n], capacity=cap)
    pl.check(count, cap)
    c = lib.candidates_to_numpy(cands, int(count.item()))
    plane = P.float().cpu().numpy().reshape(pl.Z, nb)
    j0 = 96
    tau = {H: o.threshold(H) for H in o.stages(16)}

    def oracle_at(rows, cols):
        S = o.harmonic_sum_cells(plane, j0, 16, rows, cols)
        h, _ = o.best_stage(S, cols, nb, r_lo=pl.hmax, h_max=pl.hmax)
        near = np.zeros(len(rows), bool)
        for H in S:
            near |= np.abs(S[H] - tau[H]) <= 1e-5 * tau[H]
        return S, h, near

    assert len(c) >= 100
    S, h, near = oracle_at(c["j"].astype(np.int64), c["R"].astype(np.int64))
    ok = (h == c["harm"]) | near
    assert ok.all(), np.nonzero(~ok)[0][:5]
    same = h == c["harm"]
    got_p = c["power"].astype(np.float64)[same]
    want_p = np.choose(np.searchsorted([1, 2, 4, 8, 16], h[same]), [S[H][same] for H in (1, 2, 4, 8, 16)])
    np.testing.assert_allclose(got_p, want_p, rtol=1e-5)
    # sampled cells: random ones and the neighbourhoods of the injections
    rng = np.random.default_rng(5)
    rows = [rng.integers(0, pl.Z, 300_000)]
    cols = [rng.integers(0, nb, 300_000)]
    for i in inj:
        for H in (1, 2, 4, 8, 16):  # where each stage's cell sees the injection as harmonic H
            rc, mc = int(round(i.r_mean * H)), int(round(i.z * H))
            if rc >= nb or abs(mc) > 96:
                continue
            jj, rr = np.meshgrid(np.arange(-4, 5) + j0 + mc, np.arange(-3, 4) + rc, indexing="ij")
            keep = (jj >= 0) & (jj < pl.Z) & (rr >= 0) & (rr < nb)
            rows.append(jj[keep])
            cols.append(rr[keep])
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    _, h, near = oracle_at(rows, cols)
    recorded = set(zip(c["j"].tolist(), c["R"].tolist()))
    got = np.array([(int(j), int(r)) in recorded for j, r in zip(rows, cols)])
    bad = (got != (h > 0)) & ~near
    assert not bad.any(), (rows[bad][:5], cols[bad][:5])
    assert (h > 0).sum() >= 50


def test_candidate_overflow_is_reported(lib):
    n = 1 << 17
    x = synth.make_series(n, [synth.Injection(0.1, 3000.0, 8.0, 0.1)], 8, 0)
    say("fdas_harmonic_sum overflow")
    pl, P, _ = gpu_plane(lib, x, small_params(1024))
    cands, count = pl.harmonic_sum(P, [n], capacity=3)
    with pytest.raises(lib.FdasError, match="overflow"):
        pl.check(count, 3)
    assert count.item() > 3


def test_counting_only_and_empty_batch(lib):
    """capacity = 0 counts the passing cells without storing any, the same
    count as with room for all of them; a batch of no series is refused."""
    import ctypes
    import torch
    n = 1 << 17
    x = synth.make_series(n, [synth.Injection(0.06, 3000.0, 8.0, 0.1)], 10, 0)
    say("fdas_harmonic_sum capacity 0")
    pl, P, _ = gpu_plane(lib, x, small_params(1024))
    _, full = pl.harmonic_sum(P, [n], capacity=1 << 16)
    _, none = pl.harmonic_sum(P, [n], capacity=0)
    pl.check(full, 1 << 16)
    assert int(none.item()) == int(full.item()) > 0
    lens = (ctypes.c_int64 * 1)(n)
    assert pl.lib.fdas_harmonic_sum(pl.handle, ctypes.c_void_p(P.data_ptr()), lens, 0, None, 0,
                                    ctypes.c_void_p(full.data_ptr())) == 1


def test_nonfinite_input_is_reported(lib):
    import torch
    n = 1 << 17
    x = synth.make_series(n, [], 9, 0)
    x[1234] = np.nan
    say("fdas_spectrum nonfinite")
    pl = lib.Plan(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, make_templates=False)
    pl.spectrum(torch.from_numpy(x).to("cuda"), [0], [n])
    with pytest.raises(lib.FdasError, match="NaN"):
        pl.check()
    pl.check()  # the latch clears


# ---------------------------------------------------------------- batch, graph, autotune

def test_search_graph_replays_match_eager(lib):
    """fdas_search captured into a HIP graph: every replay (with eager work and
    synchronisations in between) reproduces the eager result bit for bit."""
    import torch
    n = 1 << 19
    lens = [n, n // 2, n // 4, n]
    xs, truths = synth.batch_series(lens, seed=51, amp=(0.05, 0.08))
    flat, offs, lens_a = synth.concat(xs)
    say("fdas_search graph", lens)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pl = lib.Plan(n_samples=n, max_batch_samples=int(lens_a.sum()), z_min=-32.0, z_max=32.0, z_step=2.0,
                      n_harmonics=8, segment_len=1024, store="bf16", plane="bf16", stream=stream)
        xt = torch.from_numpy(flat).to("cuda")
        tot = int(lens_a.sum()) // 2
        P0, P1 = pl.new_plane(tot), pl.new_plane(tot)
        c0 = torch.zeros((1 << 15, 8), dtype=torch.int32, device="cuda")
        c1 = torch.zeros_like(c0)
        k0 = torch.zeros(1, dtype=torch.int64, device="cuda")
        k1 = torch.zeros_like(k0)
        pl.search(xt, offs, lens_a, P0, c0, k0, use_graph=False)
        pl.check(k0, c0.shape[0])
        want = sorted(map(tuple, lib.candidates_to_numpy(c0, int(k0.item())).tolist()))
        for rep in range(3):
            P1.fill_(0)
            k1.fill_(7)
            pl.search(xt, offs, lens_a, P1, c1, k1, use_graph=True)
            pl.check(k1, c1.shape[0])
            assert torch.equal(P0, P1), rep
            got = sorted(map(tuple, lib.candidates_to_numpy(c1, int(k1.item())).tolist()))
            assert got == want, rep
            torch.cuda.synchronize()
            _ = (P0.float().sum() + 1).item()   # eager work between replays
        assert len(want) > 0


@pytest.mark.parametrize("store,use_graph", [("f32", 1), ("bf16", 1), ("bf16", 0)])
def test_search_three_length_classes_match_oracle(lib, store, use_graph):
    """One batch holding all three length classes (N, N/2 and N/4 = 2^19,
    2^18 and 2^17 samples, as full-rate and 2x/4x decimated DM trials) through
    fdas_search, eager and captured in a HIP graph: every series' plane
    against the oracle's (FP32 storage: every cell within 1e-4 max(P, 1);
    BF16: 3e-2 at detections, 5e-2 max(P, 1) elsewhere), and its candidates
    against the oracle's search, of the GPU's own plane exactly (cell, stage,
    power, r = R/H, z = z_j/H, up to sums within 1e-5 of a threshold) and, for
    FP32, of the oracle's plane (up to sums within 2e-4 of a threshold)."""
    import torch
    n = 1 << 19
    lens = [n, n // 4, n // 2, n // 4, n]
    xs, truths = synth.batch_series(lens, seed=81, inj_per_series=(1, 2), amp=(0.05, 0.08), z_abs=28.0)
    flat, offs, lens_a = synth.concat(xs)
    say("fdas_search three length classes", store, "graph" if use_graph else "eager", lens)
    stream = torch.cuda.Stream()
    nh = 16
    zs = o.z_grid(-32, 32, 2)
    j0 = int(np.argmin(np.abs(zs)))
    tau = {H: o.threshold(H) for H in o.stages(nh)}
    with torch.cuda.stream(stream):
        pl = lib.Plan(n_samples=n, max_batch_samples=int(lens_a.sum()), z_min=-32.0, z_max=32.0, z_step=2.0,
                      n_harmonics=nh, segment_len=1024, store=store, plane=store, stream=stream)
        xt = torch.from_numpy(flat).to("cuda")
        P = pl.new_plane(int(lens_a.sum()) // 2)
        cap = 1 << 20
        cands = torch.zeros((cap, 8), dtype=torch.int32, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        for _ in range(2 if use_graph else 1):   # capture, then one replay
            pl.search(xt, offs, lens_a, P, cands, count, use_graph=bool(use_graph))
        pl.check(count, cap)
    c = lib.candidates_to_numpy(cands, int(count.item()))
    Pall = P.float().cpu().numpy().astype(np.float64)
    pos = 0
    for s_, x in enumerate(xs):
        nb = len(x) // 2
        g = Pall[pos: pos + pl.Z * nb].reshape(pl.Z, nb)
        pos += pl.Z * nb
        ref = o.power_plane(o.normalise(o.spectrum(x), "median"), zs)
        if store == "f32":
            bad = np.abs(g - ref) > 1e-4 * np.maximum(ref, 1.0)
            assert not bad.any(), (s_, np.argwhere(bad)[:5])
        else:
            e = o.power_errors(g, ref, tau1=o.threshold(1))
            assert e["max_rel_det"] < 3e-2, (s_, e)
            assert np.all(np.abs(g - ref) <= 5e-2 * np.maximum(ref, 1.0)), s_
        mine = c[c["series"] == s_]
        got = {(int(k["R"]), int(k["j"])): k for k in mine}
        assert len(got) == len(mine)
        sums = o.harmonic_sums(g, j0, nh)
        want = {(k.R, k.j): k for k in o.search(g, zs, nh, r_lo=pl.hmax, h_max=pl.hmax, series=s_)}

        def near(sm, R, j, tol):
            return any(abs(sm[H][j, R] - tau[H]) <= tol * tau[H] for H in tau)

        for cell in set(got) ^ set(want):
            assert near(sums, *cell, 1e-5), (s_, cell)
        for cell in set(got) & set(want):
            k, w = got[cell], want[cell]
            if int(k["harm"]) != w.harm:
                assert near(sums, *cell, 1e-5), (s_, cell)
                continue
            assert abs(float(k["power"]) - w.power) <= 1e-5 * w.power, (s_, cell)
            assert k["r"] == np.float32(w.r) and k["z"] == np.float32(w.z), (s_, cell)
        assert len(want) >= 20, (s_, len(want))
        if store == "f32":
            sums_o = o.harmonic_sums(ref, j0, nh)
            want_o = {(k.R, k.j) for k in o.search(ref, zs, nh, r_lo=pl.hmax, h_max=pl.hmax)}
            for cell in set(got) ^ want_o:
                assert near(sums_o, *cell, 2e-4), (s_, cell)
        # every injection of the series is among its candidates (within 1 bin, 1 z)
        for i in truths[s_]:
            assert np.any((np.abs(mine["r"] - i.r_mean) <= 1.0) & (np.abs(mine["z"] - i.z) <= 1.0)), (s_, i)


def test_workspace_rebind_drops_the_captured_graph(lib):
    """fdas_set_workspace onto a second workspace (the first still allocated,
    templates remade there) with the same search pointers: the graph replay
    that follows runs on the new workspace and equals the eager search bit
    for bit, also after the old workspace is overwritten."""
    import ctypes
    import torch
    n = 1 << 18
    lens = [n, n // 2]
    xs, _ = synth.batch_series(lens, seed=83, amp=(0.05, 0.08), z_abs=28.0)
    flat, offs, lens_a = synth.concat(xs)
    say("fdas_set_workspace rebind and graph", lens)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pl = lib.Plan(n_samples=n, max_batch_samples=int(lens_a.sum()), z_min=-32.0, z_max=32.0, z_step=2.0,
                      n_harmonics=8, segment_len=1024, store="bf16", plane="bf16", stream=stream)
        xt = torch.from_numpy(flat).to("cuda")
        tot = int(lens_a.sum()) // 2
        P0, P1 = pl.new_plane(tot), pl.new_plane(tot)
        c0 = torch.zeros((1 << 15, 8), dtype=torch.int32, device="cuda")
        c1 = torch.zeros_like(c0)
        k0 = torch.zeros(1, dtype=torch.int64, device="cuda")
        k1 = torch.zeros_like(k0)
        spec = pl.new_spectrum(tot)   # caller-owned: the graph's pointers stay the same across the rebind
        pl.search(xt, offs, lens_a, P0, c0, k0, use_graph=False)
        pl.search(xt, offs, lens_a, P1, c1, k1, spectrum=spec, use_graph=True)   # captured on the first workspace
        pl.check(k1, c1.shape[0])
        old_ws = pl.workspace
        new_ws = torch.empty_like(old_ws)
        assert pl.lib.fdas_set_workspace(pl.handle, ctypes.c_void_p(new_ws.data_ptr()), pl.ws_bytes) == 0
        pl.workspace = new_ws
        pl.make_templates()
        old_ws.fill_(0xFF)   # the old templates and descriptors are gone
        P1.fill_(0)
        spec.fill_(0)
        pl.search(xt, offs, lens_a, P1, c1, k1, spectrum=spec, use_graph=True)
        pl.check(k1, c1.shape[0])
        torch.cuda.synchronize()
    assert torch.equal(P0, P1)
    want = sorted(map(tuple, lib.candidates_to_numpy(c0, int(k0.item())).tolist()))
    got = sorted(map(tuple, lib.candidates_to_numpy(c1, int(k1.item())).tolist()))
    assert got == want and len(want) > 0
    del old_ws


def test_harmonic_sum_refuses_a_misaligned_plane(lib):
    """A plane pointer that is element- but not 16-byte aligned is an argument
    error before anything is enqueued (the count stays untouched)."""
    import ctypes
    import torch
    n = 1 << 17
    say("fdas_harmonic_sum misaligned plane")
    pl = lib.Plan(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, n_harmonics=4, store="bf16", plane="bf16",
                  make_templates=False)
    buf = torch.zeros(pl.Z * n // 2 + 64, dtype=torch.bfloat16, device="cuda")
    count = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    cands = torch.zeros((16, 8), dtype=torch.int32, device="cuda")
    lens = (ctypes.c_int64 * 1)(n)
    for shift in (1, 2, 7):   # bytes 2, 4, 14 past a 256-byte boundary
        st = pl.lib.fdas_harmonic_sum(pl.handle, ctypes.c_void_p(buf.data_ptr() + 2 * shift), lens, 1,
                                      ctypes.c_void_p(cands.data_ptr()), 16, ctypes.c_void_p(count.data_ptr()))
        assert st == 1, shift
        assert b"16-byte" in pl.lib.fdas_last_error(pl.handle)
    torch.cuda.synchronize()
    assert int(count.item()) == 5


@pytest.mark.parametrize("interbin", [0, 1])
def test_autotune_picks_a_valid_configuration(lib, interbin):
    import torch
    n = 1 << 18
    say("fdas_autotune", n, interbin)
    best = lib.autotune(cache="/tmp/fdas_tune_test.json", n_samples=n, z_min=-32.0, z_max=32.0, z_step=1.0,
                        store="bf16", plane="bf16", interbin=interbin)
    assert best.interbin == interbin
    assert best.segment_len in (1024, 2048, 4096, 8192)
    assert best.fft_radix in ((16, 8, 4) if best.segment_len == 1024 else (16,))
    x = synth.make_series(n, [synth.Injection(0.05, 7000.0, 21.0, 0.3)], 52, 0)
    pl = lib.Plan(params=best, n_samples=n)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
    zs = o.z_grid(-32, 32, 1)
    ref = o.power_plane(o.normalise(o.spectrum(x), "median"), zs, rows=[0, 25, 32, 53, 64])
    got = P.view(pl.Z, n // 2 * pl.res).float().cpu().numpy()[[0, 25, 32, 53, 64]][:, ::pl.res]
    e = o.power_errors(got, ref, tau1=o.threshold(1))
    assert e["max_rel_det"] < 3e-2


def test_search_chunked_equals_one_search(lib):
    """fdas_search_chunked over 6 series of the three length classes with a
    plane buffer that holds about two of them: several chunks, and exactly
    the records (global series indices) of one fdas_search over all six with
    a plane for all; a buffer smaller than one series' plane is refused
    before any work."""
    import ctypes
    import torch
    n = 1 << 19
    lens = [n, n // 2, n // 4, n, n // 2, n]
    xs, _ = synth.batch_series(lens, seed=85, inj_per_series=(1, 2), amp=(0.05, 0.08), z_abs=28.0)
    flat, offs, lens_a = synth.concat(xs)
    say("fdas_search_chunked", lens)
    pl = lib.Plan(n_samples=n, max_batch_samples=int(lens_a.sum()), z_min=-32.0, z_max=32.0, z_step=2.0,
                  n_harmonics=8, segment_len=1024, store="bf16", plane="bf16")
    xt = torch.from_numpy(flat).to("cuda")
    cap = 1 << 20
    P_all = pl.new_plane(int(lens_a.sum()) // 2)
    c0 = torch.zeros((cap, 8), dtype=torch.int32, device="cuda")
    k0 = torch.zeros(1, dtype=torch.int64, device="cuda")
    pl.search(xt, offs, lens_a, P_all, c0, k0)
    pl.check(k0, cap)
    want = np.sort(lib.candidates_to_numpy(c0, int(k0.item())), order=["series", "j", "R"])
    P_small = pl.new_plane(2 * n // 2)   # the plane of two full-length series
    c1 = torch.zeros_like(c0)
    k1 = torch.full((1,), 99, dtype=torch.int64, device="cuda")
    nch = pl.search_chunked(xt, offs, lens_a, P_small, c1, k1)
    pl.check(k1, cap)
    got = np.sort(lib.candidates_to_numpy(c1, int(k1.item())), order=["series", "j", "R"])
    assert nch >= 3, nch
    assert len(want) > 50 and np.array_equal(got, want)
    assert set(got["series"].tolist()) == set(range(len(lens)))
    # too small for the longest series: refused, nothing enqueued
    tiny = pl.new_plane(n // 4)
    k2 = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    with pytest.raises(lib.FdasError, match="plane_bytes"):
        pl.search_chunked(xt, offs, lens_a, tiny, c1, k2)
    torch.cuda.synchronize()
    assert int(k2.item()) == 7
