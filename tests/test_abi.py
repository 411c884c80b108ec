"""The C-ABI library loads, exports every symbol include/fdas.h declares, and
rejects invalid parameters before touching a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

import paper_2211_13517_amd as fdas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdas.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdas_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fdas.LIB_PATH):
        pytest.fail("libfdas.so is not built; run `python -m paper_2211_13517_amd.build`")
    return fdas.load()


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for s in ["fdas_plan", "fdas_make_templates", "fdas_convolve", "fdas_harmonic_sum", "fdas_spectrum",
              "fdas_convolve_spectrum", "fdas_check", "fdas_plan_destroy", "fdas_last_error"]:
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(fdas.EXPORTS) <= set(declared_symbols())


def test_struct_sizes_match_the_header(lib):
    # fdas_params: 2 int64 + 4 double + 7 int32 (+4 pad) + 2 double + 4 int32
    assert ctypes.sizeof(fdas.Params) == 8 * 6 + 4 * 7 + 4 + 8 * 2 + 4 * 4


def test_default_params(lib):
    p = fdas.Params()
    assert lib.fdas_default_params(ctypes.byref(p)) == 0
    assert p.n_samples == 1 << 23 and p.z_max == 96.0 and p.z_step == 1.0 and p.n_harmonics == 16
    assert p.kernel_margin == 16 and p.norm == 2 and p.norm_block == 2048 and p.sigma_threshold == 6.0


BAD = [
    dict(n_samples=3 << 16),                    # not a power of two
    dict(n_samples=1 << 24),                    # above the supported range
    dict(z_min=-10.0, z_max=12.0),              # asymmetric grid
    dict(z_step=0.0),
    dict(z_max=95.5, z_min=-95.5, z_step=1.0),  # z_max/z_step not integral
    dict(n_harmonics=3),
    dict(segment_len=3000),
    dict(segment_len=1024, z_max=200.0, z_min=-200.0),  # L < 4 h_max
    dict(store_dtype=7),
    dict(norm=9),
    dict(norm_block=1000),
    dict(sigma_threshold=-1.0),
    dict(max_batch_samples=1 << 10),
    dict(interbin=2),
    dict(fft_radix=3),
    dict(fft_radix=8, segment_len=2048),
]


@pytest.mark.parametrize("kw", BAD)
def test_invalid_params_rejected_before_any_device_work(lib, kw):
    p = fdas.Params()
    lib.fdas_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    h = ctypes.c_void_p()
    st = lib.fdas_plan(ctypes.byref(p), 0, None, ctypes.byref(h))
    assert st == 1  # FDAS_ERR_ARG
    assert h.value is None
    assert len(lib.fdas_last_error(None)) > 0


def test_null_plan_calls_are_argument_errors(lib):
    assert lib.fdas_make_templates(None) == 1
    assert lib.fdas_query(None, None, None, None, None) == 1
    assert lib.fdas_plan_destroy(None) == 0


def test_binding_refuses_missing_library(tmp_path):
    saved = fdas._lib
    fdas._lib = None
    try:
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            fdas.load(str(tmp_path / "nope.so"))
    finally:
        fdas._lib = saved


def test_cluster_scratch_size_is_host_only(lib):
    L = lib
    assert L.fdas_cluster_scratch_bytes(-1) == -1
    # a power-of-two table of at least twice the records, 12 bytes a slot
    assert L.fdas_cluster_scratch_bytes(1000) == 2048 * 12
    assert L.fdas_cluster_scratch_bytes(1 << 20) == (1 << 21) * 12
    # record indices are 32-bit and the table at most 2^31 slots
    assert L.fdas_cluster_scratch_bytes(1 << 30) == (1 << 31) * 12
    assert L.fdas_cluster_scratch_bytes((1 << 30) + 1) == -1
