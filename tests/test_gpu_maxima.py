"""GPU: the column maxima that follow the plane values in a plane buffer, and
the harmonic sum's bound-then-exact evaluation on planes where the bound
passes almost everywhere.

The maxima are compared bit for bit with the maximum over each run of 8
columns of the same buffer's values (numpy on the host); the harmonic-sum
records with the oracle's search over the values the GPU holds.
"""
import numpy as np
import pytest

import synth
from oracle import fdas64 as o

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def ref_maxima(v):
    """Largest of each run of 8 columns, a NaN or negative value (sign bit
    set, -0 included) counting as +inf."""
    w = np.where(np.isnan(v) | np.signbit(v), np.float32(np.inf), v).astype(np.float32)
    return w.reshape(v.shape[0], -1, 8).max(axis=2)


def series_rows(flat, Z, lens, res, div=1):
    """Splits a packed plane (or its maxima, div = 8) into per-series [Z][cols] arrays."""
    out, off = [], 0
    for L_ in lens:
        cols = L_ // 2 * res // div
        out.append(flat[off: off + Z * cols].reshape(Z, cols))
        off += Z * cols
    return out


@pytest.mark.parametrize("dt,interbin,L", [("f32", 0, 1024), ("bf16", 0, 1024), ("f16", 0, 1024), ("f32", 1, 1024),
                                           ("bf16", 1, 1024), ("bf16", 0, 4096), ("f32", 1, 2048)])
def test_column_maxima_are_maxima_of_runs_of_eight(lib, dt, interbin, L):
    """After the convolution of a ragged batch (2^18, 2^17 and 2^16 bins),
    every column maximum equals the largest of its 8 plane values (the
    one-wavefront and the block tiles, bin and half-bin planes); cleared and
    rebuilt by fdas_plane_maxima, they are the same again."""
    import torch
    n = 1 << 19
    lens = [n, n // 2, n // 4]
    xs, _ = synth.batch_series(lens, seed=71, inj_per_series=(1, 2), amp=(0.04, 0.07), z_abs=14.0)
    x, offs, _ = synth.concat(xs)
    say("column maxima", dt, "interbin", interbin, "L", L)
    pl = lib.Plan(store=dt, plane=dt, n_samples=n, max_batch_samples=sum(lens), z_min=-16.0, z_max=16.0,
                  z_step=2.0, n_harmonics=16, segment_len=L, interbin=interbin)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), offs, lens)
    M = pl.maxima(P)
    assert M.numel() == P.numel() // 8

    def check():
        vals = series_rows(P.float().cpu().numpy(), pl.Z, lens, pl.res)
        maxs = series_rows(M.float().cpu().numpy(), pl.Z, lens, pl.res, 8)
        for v, m in zip(vals, maxs):
            assert np.array_equal(m.view(np.uint32), ref_maxima(v).view(np.uint32))

    check()
    M.zero_()
    pl.plane_maxima(P, lens)
    check()


def planted_plane(rng, Z, nb, big, spikes):
    """Exp(1) noise with one value `big` at a random place in every run of 8
    columns (so every column maximum is at least `big`), plus `spikes` random
    cells of value 25 and a few NaN, -3 and -0 cells."""
    P = rng.exponential(1.0, (Z, nb))
    runs = nb // 8
    pos = rng.integers(0, 8, (Z, runs)) + 8 * np.arange(runs)[None, :]
    np.put_along_axis(P, pos, big, axis=1)
    P[rng.integers(0, Z, spikes), rng.integers(0, nb, spikes)] = 25.0
    for v in (np.nan, -3.0, -0.0):
        P[rng.integers(0, Z, 8), rng.integers(0, nb, 8)] = v
    return P


@pytest.mark.parametrize("dt,nh", [("bf16", 16), ("f32", 16), ("bf16", 8), ("f16", 4), ("f32", 1)])
def test_harmonic_sum_where_bounds_pass_everywhere_matches_oracle(lib, dt, nh):
    """A plane written by the caller (fdas_plane_maxima after the upload) in
    which every column maximum is at least 7: the bounds pass at nearly every
    cell, so nearly every cell sums exactly; the records are the oracle's
    search over the same values (cells, stages, powers, r and z), up to sums
    within 1e-5 of a threshold.  The maxima follow the convention (NaN and
    negative values count as +inf)."""
    import torch
    n = 1 << 17
    nb = n // 2
    say("harmonic sum, bound passing everywhere", dt, nh)
    pl = lib.Plan(store=dt, plane=dt, n_samples=n, z_min=-16.0, z_max=16.0, z_step=1.0, n_harmonics=nh,
                  segment_len=1024, make_templates=False)
    rng = np.random.default_rng(7 + nh)
    host = planted_plane(rng, pl.Z, nb, 7.0, 64)
    P = pl.new_plane(nb)
    P.copy_(torch.from_numpy(host.reshape(-1)).to(P.dtype))
    pl.plane_maxima(P, [n])
    vals = P.float().cpu().numpy().reshape(pl.Z, nb)
    assert np.array_equal(pl.maxima(P).float().cpu().numpy().reshape(pl.Z, -1).view(np.uint32),
                          ref_maxima(vals).view(np.uint32))
    cap = 1 << 20
    cands, count = pl.harmonic_sum(P, [n], capacity=cap)
    pl.check(count, cap)
    c = lib.candidates_to_numpy(cands, int(count.item()))
    plane = P.float().cpu().numpy().astype(np.float64).reshape(pl.Z, nb)
    zs = o.z_grid(-16, 16, 1)
    j0 = int(np.argmin(np.abs(zs)))
    tau = {H: o.threshold(H) for H in o.stages(nh)}
    sums = o.harmonic_sums(plane, j0, nh)
    want = {(k.R, k.j): k for k in o.search(plane, zs, nh, r_lo=pl.hmax, h_max=pl.hmax)}
    got = {(int(k["R"]), int(k["j"])): k for k in c}
    assert len(got) == len(c)

    def borderline(R, j):
        return any(abs(sums[H][j, R] - tau[H]) <= 1e-5 * tau[H] for H in tau)

    for cell in set(got) ^ set(want):
        assert borderline(*cell), cell
    for cell in set(got) & set(want):
        g, w = got[cell], want[cell]
        if int(g["harm"]) != w.harm:
            assert borderline(*cell), (cell, int(g["harm"]), w.harm)
            continue
        assert abs(float(g["power"]) - w.power) <= 1e-5 * w.power, cell
        assert g["r"] == np.float32(w.r) and g["z"] == np.float32(w.z), cell
    assert len(want) >= 30, len(want)


def test_plane_maxima_and_harmonic_sum_argument_errors(lib):
    """Host-side checks, nothing enqueued: fdas_plane_maxima refuses a plane
    that is not 16-byte aligned or too small for the batch's values and
    maxima; the harmonic sum refuses a plane buffer and batch for which the
    plan wrote no maxima (values uploaded without fdas_plane_maxima, or a
    batch other than the one convolved)."""
    import ctypes
    import torch
    n = 1 << 17
    say("column maxima argument errors")
    pl = lib.Plan(store="bf16", plane="bf16", n_samples=n, max_batch_samples=2 * n, z_min=-16.0, z_max=16.0,
                  z_step=2.0, n_harmonics=4, segment_len=1024)
    lens1 = (ctypes.c_int64 * 1)(n)
    need = pl.Z * (n // 2) * 9 // 8
    buf = torch.full((need + 64,), 3.0, dtype=torch.bfloat16, device="cuda")
    assert pl.lib.fdas_plane_maxima(pl.handle, ctypes.c_void_p(buf.data_ptr() + 2), lens1, 1, need * 2) == 1
    assert b"16-byte" in pl.lib.fdas_last_error(pl.handle)
    assert pl.lib.fdas_plane_maxima(pl.handle, ctypes.c_void_p(buf.data_ptr()), lens1, 1, need * 2 - 2) == 2
    torch.cuda.synchronize()
    assert bool((buf == 3.0).all())
    # values uploaded, no maxima written: refused, count untouched
    P = pl.new_plane(n // 2)
    P.fill_(1.0)
    count = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    cands = torch.zeros((16, 8), dtype=torch.int32, device="cuda")
    st = pl.lib.fdas_harmonic_sum(pl.handle, ctypes.c_void_p(P.data_ptr()), lens1, 1, ctypes.c_void_p(cands.data_ptr()),
                                  16, ctypes.c_void_p(count.data_ptr()))
    assert st == 7 and b"column maxima" in pl.lib.fdas_last_error(pl.handle)
    pl.plane_maxima(P, [n])
    _, c2 = pl.harmonic_sum(P, [n], capacity=16)
    assert int(c2.item()) == 0
    # a two-series convolution, then a harmonic sum of the first series alone
    x = torch.from_numpy(np.concatenate([synth.make_series(n, [], 4, 0), synth.make_series(n, [], 5, 0)])).to("cuda")
    P2 = pl.convolve(x, [0, n], [n, n])
    st = pl.lib.fdas_harmonic_sum(pl.handle, ctypes.c_void_p(P2.data_ptr()), lens1, 1, ctypes.c_void_p(cands.data_ptr()),
                                  16, ctypes.c_void_p(count.data_ptr()))
    assert st == 7
    torch.cuda.synchronize()
    assert int(count.item()) == 7
    _, c3 = pl.harmonic_sum(P2, [n, n], capacity=1 << 12)
    pl.check(c3, 1 << 12)
