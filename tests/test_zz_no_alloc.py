"""fdas_cluster_noalloc (static device table, no allocation by the library)
against fdas_cluster (caller scratch) through the C ABI: the same keep flags
on two calls in a row, the second with fewer records, and the record limit
refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import fdas64 as o

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def test_cluster_noalloc_matches_cluster(lib):
    import torch
    n = 1 << 18
    lens = [n, n // 2, n, n // 2]
    xs, _ = synth.batch_series(lens, seed=62, inj_per_series=(1, 2), amp=(0.04, 0.07), z_abs=44.0)
    x, offs, _ = synth.concat(xs)
    say("fdas_cluster_noalloc vs fdas_cluster", lens)
    pl = lib.Plan(store="bf16", plane="bf16", n_samples=n, max_batch_samples=sum(lens), z_min=-48.0, z_max=48.0,
                  z_step=1.0, n_harmonics=16, segment_len=1024)
    P = pl.convolve(torch.from_numpy(x).to("cuda"), offs, lens)
    cap = 1 << 20
    cands, count = pl.harmonic_sum(P, lens, capacity=cap)
    pl.check(count, cap)
    n_rec = int(count.item())
    assert 1000 < n_rec < cap
    c = lib.candidates_to_numpy(cands, n_rec)
    # first call: every record, the largest table the static array holds
    for rr, rj in ((2, 2), (5, 1)):
        want = pl.cluster(cands, count, rr, rj)[:n_rec].cpu().numpy()
        got = pl.cluster_noalloc(cands, count, rr, rj)[:n_rec].cpu().numpy()
        assert np.array_equal(got, want), (rr, rj)
        assert np.array_equal(got.astype(bool), o.local_maxima(c["series"], c["R"], c["j"], c["sigma"], rr, rj))
    # second call with a smaller input: 700 records, a smaller table over the
    # previous call's contents
    small = cands[:700].clone()
    want = pl.cluster(small, count, 2, 2).cpu().numpy()
    got = pl.cluster_noalloc(small, count, 2, 2).cpu().numpy()
    assert np.array_equal(got, want)
    c7 = c[:700]
    assert np.array_equal(got.astype(bool), o.local_maxima(c7["series"], c7["R"], c7["j"], c7["sigma"], 2, 2))


def test_cluster_noalloc_refuses_more_than_its_table_holds(lib):
    import torch
    n = 1 << 17
    say("fdas_cluster_noalloc limit")
    pl = lib.Plan(n_samples=n, z_min=-16.0, z_max=16.0, z_step=2.0, make_templates=False)
    cands = torch.zeros((4, 8), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    keep = torch.full((4,), 7, dtype=torch.uint8, device="cuda")
    st = pl.lib.fdas_cluster_noalloc(pl.handle, ctypes.c_void_p(cands.data_ptr()), ctypes.c_void_p(count.data_ptr()),
                                     (1 << 20) + 1, 2, 2, ctypes.c_void_p(keep.data_ptr()))
    assert st == 1 and b"at most" in pl.lib.fdas_last_error(pl.handle)
    torch.cuda.synchronize()
    assert keep.cpu().tolist() == [7, 7, 7, 7]
