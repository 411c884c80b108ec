"""GPU parity of the half-bin (interbinned) plane and of the search on it,
through the C ABI, against the FP64 oracle: column 2r is the bin power
|y_r|^2 and column 2r + 1 the half-bin power |y_r - y_{r+1}|^2 / 2.

Tolerances as for the bin plane: FP32 storage 1e-4 max(P, 1); BF16/FP16
3e-2 relative on detections and 5e-2 max(P, 1) elsewhere.
"""
import math

import numpy as np
import pytest

import synth
from oracle import fdas64 as o

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def small_params(L):
    return dict(n_samples=1 << 17, z_min=-16.0, z_max=16.0, z_step=2.0, n_harmonics=4, segment_len=L, interbin=1)


def convolve(lib, x, params, store="f32", plane="f32"):
    import torch
    n = len(x)
    pl = lib.Plan(store=store, plane=plane, **params)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
    assert P.numel() == pl.Z * n
    return pl, P.float().cpu().numpy().astype(np.float64).reshape(pl.Z, n)


@pytest.mark.parametrize("L", [1024, 2048, 4096, 8192])
def test_interbin_plane_fp32_full_parity(lib, L):
    """Every column of a 2^17-sample series (h' = h_max rounded up to a
    multiple of 4, U the largest multiple of 4 <= L - 2 h' - 1: 68 to 9
    segments with a ragged tail), the one-wavefront and the block tiles."""
    x, inj, _ = synth.small_case(seed=1)
    say("fdas_convolve interbin f32 small case", L)
    pl, got = convolve(lib, x, small_params(L))
    assert pl.seg_margin == 24 and pl.U == (L - 49) // 4 * 4
    zs = o.z_grid(-16, 16, 2)
    ref = o.interbin_plane(o.normalise(o.spectrum(x), "median"), zs)
    bad = np.abs(got - ref) > 1e-4 * np.maximum(ref, 1.0)
    assert not bad.any(), (np.argwhere(bad)[:5], np.abs(got - ref).max())
    # the last half-bin column uses y at N/2 from the zero-extended spectrum
    assert np.all(np.abs(got[:, -1] - ref[:, -1]) <= 1e-4 * np.maximum(ref[:, -1], 1.0))


@pytest.mark.parametrize("store,plane,L", [("bf16", "bf16", 1024), ("f16", "f16", 2048), ("bf16", "bf16", 8192)])
def test_interbin_plane_reduced_precision(lib, store, plane, L):
    x, inj, _ = synth.small_case(seed=1)
    say("fdas_convolve interbin", store, plane, L)
    pl, got = convolve(lib, x, small_params(L), store=store, plane=plane)
    zs = o.z_grid(-16, 16, 2)
    ref = o.interbin_plane(o.normalise(o.spectrum(x), "median"), zs)
    e = o.power_errors(got, ref, tau1=o.threshold(1))
    assert e["max_rel_det"] < 3e-2, e
    assert np.all(np.abs(got - ref) < 5e-2 * np.maximum(ref, 1.0))


@pytest.mark.parametrize("plane_dt,nh", [("bf16", 16), ("f32", 4)])
def test_interbin_ragged_batch_search_matches_oracle(lib, plane_dt, nh):
    """Half-bin plane and harmonic sums over a ragged batch (2^18 and 2^17
    samples, 97 trials), against the oracle's half-bin search of the GPU's own
    plane: candidate cells, stages and powers agree except within 1e-5 of a
    threshold; fundamentals are R / (2H) bins.  The same batch through
    fdas_search (captured graph) gives the same records."""
    import torch
    n = 1 << 18
    lens = [n, n // 2, n, n // 2]
    xs, truths = synth.batch_series(lens, seed=71, inj_per_series=(1, 2), amp=(0.04, 0.07), z_abs=44.0)
    x, offs, _ = synth.concat(xs)
    say("fdas_harmonic_sum interbin ragged batch", plane_dt, nh)
    pl = lib.Plan(store=plane_dt, plane=plane_dt, n_samples=n, max_batch_samples=sum(lens), z_min=-48.0,
                  z_max=48.0, z_step=1.0, n_harmonics=nh, segment_len=1024, interbin=1)
    xt = torch.from_numpy(x).to("cuda")
    P = pl.convolve(xt, offs, lens)
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
        nc = L_                                   # 2 columns per bin
        plane = Pall[off: off + pl.Z * nc].reshape(pl.Z, nc)
        off += pl.Z * nc
        sums = o.harmonic_sums(plane, j0, nh)
        want = {(k.R, k.j): k for k in o.search(plane, zs, nh, r_lo=pl.hmax, h_max=pl.hmax, res=2)}
        mine = c[c["series"] == s_]
        got = {(int(k["R"]), int(k["j"])): k for k in mine}
        assert len(got) == len(mine)

        def borderline(R, j):
            return any(abs(sums[H][j, R] - tau[H]) <= 1e-5 * tau[H] for H in tau)

        for cell in set(got) ^ set(want):
            assert borderline(*cell), (s_, cell)
        for cell in set(got) & set(want):
            g, w = got[cell], want[cell]
            if int(g["harm"]) != w.harm:
                assert borderline(*cell), (s_, cell)
                continue
            assert abs(float(g["power"]) - w.power) <= 1e-5 * w.power, (s_, cell)
            assert float(g["r"]) == np.float32(w.r)
        assert len(want) >= 20, (s_, len(want))
        n_cells += len(want)
    assert abs(n_cells - len(c)) <= 0.001 * n_cells
    # whole search in one call, through a captured graph
    want = sorted(map(tuple, c.tolist()))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        pg = lib.Plan(store=plane_dt, plane=plane_dt, n_samples=n, max_batch_samples=sum(lens), z_min=-48.0,
                      z_max=48.0, z_step=1.0, n_harmonics=nh, segment_len=1024, interbin=1, stream=st)
        P2 = pg.new_plane(sum(lens) // 2)
        c2 = torch.zeros((cap, 8), dtype=torch.int32, device="cuda")
        n2 = torch.zeros(1, dtype=torch.int64, device="cuda")
        for rep in range(2):
            P2.fill_(0)
            pg.search(xt, offs, lens, P2, c2, n2, use_graph=True)
            pg.check(n2, cap)
            assert torch.equal(P2, P), rep
            got = sorted(map(tuple, lib.candidates_to_numpy(c2, int(n2.item())).tolist()))
            assert got == want, rep


def test_interbin_recovers_signals_midway_between_bins(lib):
    """96 injections of peak power 44 at mean frequencies exactly midway
    between bins (z on the grid): each bin keeps 0.405 x 44 = 17.8 < tau_1, the
    half-bin 0.81 x 44 = 35.7.  Recall of the half-bin search against the
    bin search on the same series (noise makes both statistical)."""
    import torch
    n = 1 << 19
    rng = np.random.default_rng(81)
    p0 = 44.0
    amp = math.sqrt(4 * p0 / n)
    inj = []
    for i in range(96):
        rbar = 3000 + 2500 * i + 0.5
        z = float(rng.integers(-40, 41))
        inj.append(synth.Injection(amp, rbar - z / 2, z, float(rng.uniform(0, 2 * np.pi))))
    x = synth.make_series(n, inj, 81, 0)
    say("interbin recall of midway signals", n, len(inj))
    found = {}
    for ib in (0, 1):
        pl = lib.Plan(store="bf16", plane="bf16", n_samples=n, z_min=-48.0, z_max=48.0, z_step=1.0,
                      n_harmonics=1, segment_len=1024, interbin=ib)
        P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
        cands, count = pl.harmonic_sum(P, [n], capacity=1 << 20)
        pl.check(count, 1 << 20)
        c = lib.candidates_to_numpy(cands, int(count.item()))
        hits = 0
        for s in inj:
            near = (np.abs(c["r"] - s.r_mean) <= 0.5) & (np.abs(c["z"] - s.z) <= 1.0)
            hits += bool(near.any())
        found[ib] = hits / len(inj)
    assert found[1] >= 0.9, found
    assert found[1] >= found[0] + 0.15, found


def test_interbin_ska_full_size_sampled(lib):
    """N = 2^23, 193 templates, BF16, L = 1024: sampled bin and half-bin
    columns and every injection's half-bin neighbourhood against the oracle's
    direct sums; then the search's records reach half-bin R up to 2^23 - 1 and
    their clustering equals the oracle's local maxima."""
    import torch
    x, inj, params = synth.ska_single(seed=2)
    params = dict(params)
    params.update(segment_len=1024, interbin=1)
    params.pop("norm")
    say("fdas_convolve interbin SKA single bf16")
    pl = lib.Plan(store="bf16", plane="bf16", **params)
    n = len(x)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), [0], [n])
    got = P.view(pl.Z, n)
    zs = o.z_grid(-96, 96, 1)
    taps, _ = o.template_taps(zs)
    a = o.normalise(o.spectrum(x), "median")
    rng = np.random.default_rng(6)
    rows = rng.integers(0, pl.Z, 3000)
    cols = rng.integers(0, n, 3000)
    cols[:50] = np.arange(50)
    cols[50:100] = n - 1 - np.arange(50)
    pk_c = np.concatenate([[2 * int(math.floor(i.r_mean)) + d for d in range(4)] for i in inj])
    pk_j = np.repeat([int(round(i.z - zs[0])) for i in inj], 4)
    rows = np.concatenate([rows, pk_j])
    cols = np.concatenate([cols, pk_c])
    ref = o.interbin_cells(a, taps, rows, cols)
    g = got[rows, cols].float().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g - ref) <= 3e-2 * np.maximum(ref, 1.0)), np.max(np.abs(g - ref) / np.maximum(ref, 1))
    # each injection's best of its bin / half-bin columns is far above threshold
    assert np.all(g[-4 * len(inj):].reshape(-1, 4).max(axis=1) > o.threshold(1))
    say("fdas_harmonic_sum + fdas_cluster interbin SKA single")
    cap = 1 << 22
    cands, count = pl.harmonic_sum(P, [n], capacity=cap)
    pl.check(count, cap)
    keep = pl.cluster(cands, count, 2, 2)
    c = lib.candidates_to_numpy(cands, int(count.item()))
    assert c["R"].max() >= (1 << 22) and c["R"].max() < (1 << 23)
    assert np.all(c["R"] < 2 * (n // 2 - pl.hmax))
    k = keep[: len(c)].cpu().numpy().astype(bool)
    assert np.array_equal(k, o.local_maxima(c["series"], c["R"], c["j"], c["sigma"], 2, 2))


def test_interbin_argument_errors_enqueue_nothing(lib):
    """Host-side checks of the half-bin path: a plane buffer sized for the bin
    plane, or not 16-byte aligned, is refused before any launch and leaves
    the buffer untouched."""
    import ctypes
    import torch
    n = 1 << 17
    say("interbin argument errors", n)
    pl = lib.Plan(store="f32", plane="f32", n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, segment_len=1024,
                  interbin=1)
    spec = pl.spectrum(torch.from_numpy(synth.make_series(n, [], 3, 0)).to("cuda"), [0], [n])
    small = torch.full((pl.Z * n // 2,), -1.0, device="cuda")            # bin-plane size: too small
    with pytest.raises(lib.FdasError, match="too small"):
        pl.convolve_spectrum(spec, [n], plane=small)
    need = pl.Z * n * 9 // 8                                              # values and column maxima
    big = torch.full((need + 4,), -1.0, device="cuda")
    lens = (ctypes.c_int64 * 1)(n)
    st = pl.lib.fdas_convolve_spectrum(pl.handle, ctypes.c_void_p(spec.data_ptr()), lens, 1,
                                       ctypes.c_void_p(big.data_ptr() + 8), need * 4)
    assert st == 1 and b"aligned" in pl.lib.fdas_last_error(pl.handle)
    torch.cuda.synchronize()
    assert bool((small == -1.0).all()) and bool((big == -1.0).all())


def test_refine_harmonics_argument_errors(lib):
    import ctypes
    import torch
    n = 1 << 17
    say("fdas_refine_harmonics argument errors", n)
    pl = lib.Plan(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, make_templates=False)
    spec = pl.spectrum(torch.from_numpy(synth.make_series(n, [], 4, 0)).to("cuda"), [0], [n])
    r = torch.tensor([1000.0], dtype=torch.float64, device="cuda")
    z = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = torch.zeros(1, dtype=torch.float64, device="cuda")
    f = pl.lib.fdas_refine_harmonics
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    assert f(pl.handle, vp(spec), n // 2, vp(r), vp(z), None, 1, 10, vp(p)) == 1          # no counts
    assert f(pl.handle, vp(spec), n // 2, vp(r), vp(z), vp(r), 1, -1, vp(p)) == 1         # n_iter < 0
    assert f(pl.handle, vp(spec), n, vp(r), vp(z), vp(r), 1, 10, vp(p)) == 1              # n_bins too large
    assert f(pl.handle, vp(spec), n // 2, vp(r), vp(z), None, 0, 10, vp(p)) == 0          # nothing to do
    with pytest.raises(ValueError):
        pl.refine_harmonics(spec, r, z, torch.tensor([1, 2]))
