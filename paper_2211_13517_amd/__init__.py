"""Python binding of libfdas (MI355X Fourier Domain Acceleration Search hot path).

Argument marshalling only: every step of the search runs in the HIP kernels of
``libfdas.so``.  PyTorch supplies device memory and the HIP stream.  There is
no CPU fallback: if the shared library is missing, ``load()`` raises.

Layouts (see include/fdas.h):
  * series: float32 1-D device tensor, series i at offsets[i], length lengths[i]
  * spectrum: packed complex bins; F32 -> float32 [bins, 2], BF16 -> bfloat16
    [bins, 2], F16 -> float16 [bins, 2] (re, im)
  * plane: packed z-major power planes, F32/BF16/F16 1-D (two columns per
    bin, bin then half bin, for plans made with interbin=1)
  * candidates: int32 [capacity, 8] (series, harm, R, j, then r, z, power,
    sigma as float32 bits); ``candidates_to_numpy`` decodes them.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdas.so")

F32, BF16, F16 = 0, 1, 2
DTYPES = {"f32": F32, "bf16": BF16, "f16": F16}
NORMS = {"none": 0, "variance": 1, "median": 2, "rednoise": 3}

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_NOMEM", 3: "ERR_HIP", 4: "ERR_UNSUPPORTED",
          5: "ERR_OVERFLOW", 6: "ERR_NONFINITE", 7: "ERR_STATE"}


class FdasError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fdas {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("n_samples", c_int64), ("max_batch_samples", c_int64), ("tsamp", c_double),
                ("z_min", c_double), ("z_max", c_double), ("z_step", c_double),
                ("n_harmonics", c_int32), ("kernel_margin", c_int32), ("segment_len", c_int32),
                ("store_dtype", c_int32), ("plane_dtype", c_int32), ("norm", c_int32),
                ("norm_block", c_int32), ("noise_var", c_double), ("sigma_threshold", c_double),
                ("r_lo", c_int32), ("templates_per_tile", c_int32), ("interbin", c_int32), ("fft_radix", c_int32)]


EXPORTS = ["fdas_default_params", "fdas_plan", "fdas_query", "fdas_set_workspace", "fdas_make_templates",
           "fdas_spectrum", "fdas_convolve_spectrum", "fdas_convolve", "fdas_harmonic_sum", "fdas_check",
           "fdas_rz_power", "fdas_rz_power_grad", "fdas_refine", "fdas_search", "fdas_autotune",
           "fdas_copy_templates", "fdas_copy_thresholds", "fdas_test_fft", "fdas_plan_destroy",
           "fdas_last_error", "fdas_cluster_scratch_bytes", "fdas_cluster", "fdas_refine_harmonics",
           "fdas_cluster_noalloc", "fdas_search_chunked", "fdas_plane_maxima"]

_lib = None


def _buffer_bytes(t) -> int:
    """Bytes from a tensor's first element to the end of its allocation: a
    plane buffer's values view also reaches the column maxima after them."""
    return t.untyped_storage().nbytes() - t.storage_offset() * t.element_size()


def load(path: str = LIB_PATH):
    """Loads libfdas.so (built by ``paper_2211_13517_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2211_13517_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "fdas_default_params": ([POINTER(Params)], c_int),
        "fdas_plan": ([POINTER(Params), c_int, P, POINTER(P)], c_int),
        "fdas_query": ([P, POINTER(c_int64), POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)], c_int),
        "fdas_set_workspace": ([P, P, c_int64], c_int),
        "fdas_make_templates": ([P], c_int),
        "fdas_spectrum": ([P, P, POINTER(c_int64), POINTER(c_int64), c_int32, P], c_int),
        "fdas_convolve_spectrum": ([P, P, POINTER(c_int64), c_int32, P, c_int64], c_int),
        "fdas_convolve": ([P, P, POINTER(c_int64), POINTER(c_int64), c_int32, P, P, c_int64], c_int),
        "fdas_harmonic_sum": ([P, P, POINTER(c_int64), c_int32, P, c_int64, P], c_int),
        "fdas_plane_maxima": ([P, P, POINTER(c_int64), c_int32, c_int64], c_int),
        "fdas_check": ([P, P, c_int64], c_int),
        "fdas_rz_power": ([P, P, c_int64, P, P, c_int64, P, P], c_int),
        "fdas_rz_power_grad": ([P, P, c_int64, P, P, P, P, c_int64, P, P, P], c_int),
        "fdas_refine": ([P, P, c_int64, P, P, c_int64, c_int32, P], c_int),
        "fdas_refine_harmonics": ([P, P, c_int64, P, P, P, c_int64, c_int32, P], c_int),
        "fdas_search": ([P, P, POINTER(c_int64), POINTER(c_int64), c_int32, P, P, c_int64, P, c_int64, P, c_int32],
                        c_int),
        "fdas_search_chunked": ([P, P, POINTER(c_int64), POINTER(c_int64), c_int32, P, c_int64, P, c_int64, P,
                                 POINTER(c_int32)], c_int),
        "fdas_autotune": ([POINTER(Params), c_int, P, P, c_int64, POINTER(Params), POINTER(c_double)], c_int),
        "fdas_copy_templates": ([P, P, P], c_int),
        "fdas_copy_thresholds": ([P, POINTER(c_double)], c_int),
        "fdas_cluster_scratch_bytes": ([c_int64], c_int64),
        "fdas_cluster": ([P, P, P, c_int64, c_int32, c_int32, P, c_int64, P], c_int),
        "fdas_cluster_noalloc": ([P, P, P, c_int64, c_int32, c_int32, P], c_int),
        "fdas_test_fft": ([P, c_int32, c_int32, P, P, c_int64], c_int),
        "fdas_plan_destroy": ([P], c_int),
        "fdas_last_error": ([P], c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _i64(values: Sequence[int]):
    a = (c_int64 * len(values))(*[int(v) for v in values])
    return a


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def plane_torch_dtype(dt: int):
    import torch
    return {F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}[dt]


def spectrum_torch_dtype(dt: int):
    return plane_torch_dtype(dt)


class Plan:
    """One search configuration on one GPU (the torch current stream at creation).

    Keyword parameters follow ``fdas_params`` (include/fdas.h); ``store`` and
    ``plane`` take "f32"/"bf16"/"f16", ``norm`` takes "none"/"variance"/"median".
    """

    def __init__(self, device: int = 0, store: str = "f32", plane: str = "f32", norm: str = "median",
                 make_templates: bool = True, stream=None, params: Optional[Params] = None, **kw):
        import torch
        self.lib = load()
        p = Params()
        if params is not None:
            ctypes.memmove(byref(p), byref(params), ctypes.sizeof(Params))
        else:
            self._check(self.lib.fdas_default_params(byref(p)), None)
            p.store_dtype = DTYPES[store]
            p.plane_dtype = DTYPES[plane]
            p.norm = NORMS[norm]
        for k, v in kw.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(p, k, v)
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = c_void_p()
        st = self.lib.fdas_plan(byref(p), device, c_void_p(self.stream.cuda_stream), byref(h))
        if st != 0:
            raise FdasError(st, self.lib.fdas_last_error(None).decode())
        self.handle = h
        self.params = p
        ws, L, hmax, Z = c_int64(), c_int32(), c_int32(), c_int32()
        self._check(self.lib.fdas_query(h, byref(ws), byref(L), byref(hmax), byref(Z)))
        self.ws_bytes, self.L, self.hmax, self.Z = ws.value, L.value, hmax.value, Z.value
        # columns per bin of the plane: 2 on a half-bin (interbinned) plane,
        # which also gives up one output per segment.  Segment geometry as
        # fdas_plan sets it: the first output seg_margin = h_max rounded up to
        # a multiple of the bins per column maximum (8, or 4 on a half-bin
        # plane) into the FFT, U outputs, the largest such multiple with
        # U <= L - 2 seg_margin (- 1 on a half-bin plane)
        self.res = 2 if p.interbin else 1
        run = 8 // self.res
        self.seg_margin = -(-self.hmax // run) * run
        self.U = (self.L - 2 * self.seg_margin - (1 if p.interbin else 0)) // run * run
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self._check(self.lib.fdas_set_workspace(h, c_void_p(self.workspace.data_ptr()), self.ws_bytes))
        self.store_dtype, self.plane_dtype = p.store_dtype, p.plane_dtype
        self.n_harmonics = p.n_harmonics
        if make_templates:
            self.make_templates()

    # ------------------------------------------------------------------ plumbing
    def _check(self, st: int, h="self"):
        if st != 0:
            hh = self.handle if h == "self" else h
            raise FdasError(st, self.lib.fdas_last_error(hh).decode())

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.fdas_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_stages(self) -> int:
        return int(np.log2(self.n_harmonics)) + 1

    def z_values(self) -> np.ndarray:
        return self.params.z_min + self.params.z_step * np.arange(self.Z, dtype=np.float64)

    # ------------------------------------------------------------------ calls
    def make_templates(self):
        self._check(self.lib.fdas_make_templates(self.handle))

    def templates(self):
        """(taps complex128 [Z][2 h_max + 1], spectra [Z][L][2] in the storage dtype), on the GPU."""
        import torch
        taps = torch.empty((self.Z, 2 * self.hmax + 1), dtype=torch.complex128, device=self.device)
        spec = torch.empty((self.Z, self.L, 2), dtype=spectrum_torch_dtype(self.store_dtype), device=self.device)
        self._check(self.lib.fdas_copy_templates(self.handle, c_void_p(taps.data_ptr()), c_void_p(spec.data_ptr())))
        return taps, spec

    def thresholds(self) -> np.ndarray:
        out = (c_double * self.n_stages)()
        self._check(self.lib.fdas_copy_thresholds(self.handle, out))
        return np.array(out[:], dtype=np.float64)

    def new_spectrum(self, total_bins: int):
        import torch
        return torch.empty((total_bins, 2), dtype=spectrum_torch_dtype(self.store_dtype), device=self.device)

    def new_plane(self, total_bins: int):
        """A plane buffer for ``total_bins`` bins in all: returns the view of
        its Z * total_bins * res plane values; the column maxima (one eighth
        more) follow them in the same allocation (see ``maxima``)."""
        import torch
        n = self.Z * total_bins * self.res
        buf = torch.empty(n + n // 8, dtype=plane_torch_dtype(self.plane_dtype), device=self.device)
        return buf[:n]

    @staticmethod
    def maxima(plane):
        """The column-maxima section that follows a plane made by ``new_plane``."""
        return plane._base[plane.numel():]

    def plane_maxima(self, plane, lengths: Sequence[int]):
        """Writes the column maxima of plane values the caller wrote (fdas_plane_maxima)."""
        self._check(self.lib.fdas_plane_maxima(self.handle, c_void_p(plane.data_ptr()), _i64(lengths), len(lengths),
                                               _buffer_bytes(plane)))
        return plane

    def spectrum(self, series, offsets: Sequence[int], lengths: Sequence[int], out=None):
        total = int(sum(lengths)) // 2
        out = self.new_spectrum(total) if out is None else out
        self._check(self.lib.fdas_spectrum(self.handle, c_void_p(series.data_ptr()), _i64(offsets), _i64(lengths),
                                           len(lengths), c_void_p(out.data_ptr())))
        return out

    def convolve_spectrum(self, spectrum, lengths: Sequence[int], plane=None):
        total = int(sum(lengths)) // 2
        plane = self.new_plane(total) if plane is None else plane
        nbytes = _buffer_bytes(plane)
        self._check(self.lib.fdas_convolve_spectrum(self.handle, c_void_p(spectrum.data_ptr()), _i64(lengths),
                                                    len(lengths), c_void_p(plane.data_ptr()), nbytes))
        return plane

    def convolve(self, series, offsets: Sequence[int], lengths: Sequence[int], plane=None, spectrum=None):
        total = int(sum(lengths)) // 2
        plane = self.new_plane(total) if plane is None else plane
        nbytes = _buffer_bytes(plane)
        sp = None if spectrum is None else c_void_p(spectrum.data_ptr())
        self._check(self.lib.fdas_convolve(self.handle, c_void_p(series.data_ptr()), _i64(offsets), _i64(lengths),
                                           len(lengths), sp, c_void_p(plane.data_ptr()), nbytes))
        return plane

    def harmonic_sum(self, plane, lengths: Sequence[int], capacity: int = 1 << 20, cands=None, count=None):
        """Appends candidates; returns (cands int32 [capacity, 8], count int64 [1]) on the GPU."""
        import torch
        if cands is None:
            cands = torch.empty((max(capacity, 1), 8), dtype=torch.int32, device=self.device)
        if count is None:
            count = torch.zeros(1, dtype=torch.int64, device=self.device)
        self._check(self.lib.fdas_harmonic_sum(self.handle, c_void_p(plane.data_ptr()), _i64(lengths), len(lengths),
                                               c_void_p(cands.data_ptr()), capacity, c_void_p(count.data_ptr())))
        return cands, count

    def search(self, series, offsets: Sequence[int], lengths: Sequence[int], plane, cands, count,
               spectrum=None, use_graph: bool = False):
        """The whole search, spectrum to candidates, for one batch (optionally through a captured HIP graph)."""
        nbytes = _buffer_bytes(plane)
        self._check(self.lib.fdas_search(self.handle, c_void_p(series.data_ptr()), _i64(offsets), _i64(lengths),
                                         len(lengths), None if spectrum is None else c_void_p(spectrum.data_ptr()),
                                         c_void_p(plane.data_ptr()), nbytes, c_void_p(cands.data_ptr()),
                                         cands.shape[0], c_void_p(count.data_ptr()), 1 if use_graph else 0))

    def search_chunked(self, series, offsets: Sequence[int], lengths: Sequence[int], plane, cands, count) -> int:
        """The whole search over any number of series within ``plane``'s size
        (fdas_search_chunked); returns the number of chunks."""
        nbytes = _buffer_bytes(plane)
        nch = c_int32()
        self._check(self.lib.fdas_search_chunked(self.handle, c_void_p(series.data_ptr()), _i64(offsets),
                                                 _i64(lengths), len(lengths), c_void_p(plane.data_ptr()), nbytes,
                                                 c_void_p(cands.data_ptr()), cands.shape[0],
                                                 c_void_p(count.data_ptr()), byref(nch)))
        return nch.value

    def cluster(self, cands, count, radius_r: int = 2, radius_j: int = 2):
        """Local maxima among candidate records (see fdas_cluster): returns a
        uint8 device tensor [capacity], 1 for records to keep."""
        import torch
        cap = int(cands.shape[0])
        nbytes = int(self.lib.fdas_cluster_scratch_bytes(cap))
        if getattr(self, "_cluster_scratch", None) is None or self._cluster_scratch.numel() < nbytes:
            self._cluster_scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        keep = torch.empty(cap, dtype=torch.uint8, device=self.device)
        self._check(self.lib.fdas_cluster(self.handle, c_void_p(cands.data_ptr()), c_void_p(count.data_ptr()), cap,
                                          radius_r, radius_j, c_void_p(self._cluster_scratch.data_ptr()), nbytes,
                                          c_void_p(keep.data_ptr())))
        return keep

    def cluster_noalloc(self, cands, count, radius_r: int = 2, radius_j: int = 2, keep=None):
        """fdas_cluster through the library's static table (no device allocation
        by the library; at most 2^20 records).  ``keep``: optional uint8
        device tensor [capacity] to write into."""
        import torch
        cap = int(cands.shape[0])
        if keep is None:
            keep = torch.empty(cap, dtype=torch.uint8, device=self.device)
        self._check(self.lib.fdas_cluster_noalloc(self.handle, c_void_p(cands.data_ptr()), c_void_p(count.data_ptr()),
                                                  cap, radius_r, radius_j, c_void_p(keep.data_ptr())))
        return keep

    def check(self, count=None, capacity: int = 0):
        """Synchronises and raises FdasError for latched device conditions."""
        self._check(self.lib.fdas_check(self.handle, None if count is None else c_void_p(count.data_ptr()), capacity))

    # ------------------------------------------------------------ refinement
    def rz_power(self, spectrum, r, z, keep_y: bool = True):
        """P(r, z) (float64 [n]) and y (complex128 [n]) at off-grid candidates."""
        import torch
        r = r.contiguous().double()
        z = z.contiguous().double()
        n = r.numel()
        p = torch.empty(n, dtype=torch.float64, device=self.device)
        y = torch.empty(n, dtype=torch.complex128, device=self.device) if keep_y else None
        nb = spectrum.shape[0]
        self._check(self.lib.fdas_rz_power(self.handle, c_void_p(spectrum.data_ptr()), nb, c_void_p(r.data_ptr()),
                                           c_void_p(z.data_ptr()), n, c_void_p(p.data_ptr()),
                                           None if y is None else c_void_p(y.data_ptr())))
        return p, y

    def rz_power_grad(self, spectrum, r, z, grad_p, y=None, want_spectrum: bool = True):
        """(grad_r, grad_z, grad_spectrum complex64 [n_bins] or None) for upstream grad_p."""
        import torch
        r = r.contiguous().double()
        z = z.contiguous().double()
        gp = grad_p.contiguous().double()
        n = r.numel()
        gr = torch.empty(n, dtype=torch.float64, device=self.device)
        gz = torch.empty(n, dtype=torch.float64, device=self.device)
        nb = spectrum.shape[0]
        gs = torch.empty(nb, dtype=torch.complex64, device=self.device) if want_spectrum else None
        self._check(self.lib.fdas_rz_power_grad(
            self.handle, c_void_p(spectrum.data_ptr()), nb, c_void_p(r.data_ptr()), c_void_p(z.data_ptr()),
            None if y is None else c_void_p(y.data_ptr()), c_void_p(gp.data_ptr()), n, c_void_p(gr.data_ptr()),
            c_void_p(gz.data_ptr()), None if gs is None else c_void_p(gs.data_ptr())))
        return gr, gz, gs

    def refine(self, spectrum, r, z, n_iter: int = 30):
        """Gradient-ascent refinement: returns (r, z, p_final float64)."""
        import torch
        r = r.clone().contiguous().double()
        z = z.clone().contiguous().double()
        n = r.numel()
        pf = torch.empty(n, dtype=torch.float64, device=self.device)
        self._check(self.lib.fdas_refine(self.handle, c_void_p(spectrum.data_ptr()), spectrum.shape[0],
                                         c_void_p(r.data_ptr()), c_void_p(z.data_ptr()), n, n_iter,
                                         c_void_p(pf.data_ptr())))
        return r, z, pf

    def refine_harmonics(self, spectrum, r, z, n_harm, n_iter: int = 30):
        """Ascent of S = sum_{k<=H} P(k r, k z) at fundamentals (r, z), H per
        candidate (int tensor or scalar): returns (r, z, S float64)."""
        import torch
        r = r.clone().contiguous().double()
        z = z.clone().contiguous().double()
        n = r.numel()
        if not torch.is_tensor(n_harm):
            n_harm = torch.full((n,), int(n_harm), dtype=torch.int32, device=self.device)
        h = n_harm.to(device=self.device, dtype=torch.int32).contiguous()
        if h.numel() != n:
            raise ValueError("n_harm must hold one count per candidate")
        pf = torch.empty(n, dtype=torch.float64, device=self.device)
        self._check(self.lib.fdas_refine_harmonics(self.handle, c_void_p(spectrum.data_ptr()), spectrum.shape[0],
                                                   c_void_p(r.data_ptr()), c_void_p(z.data_ptr()),
                                                   c_void_p(h.data_ptr()), n, n_iter, c_void_p(pf.data_ptr())))
        return r, z, pf

    def test_fft(self, x, direction: int):
        """Batched complex FFT of length L through the library's FFT engine (self-test)."""
        import torch
        x = x.contiguous()
        out = torch.empty_like(x)
        L = x.shape[-1]
        self._check(self.lib.fdas_test_fft(self.handle, L, direction, c_void_p(x.data_ptr()),
                                           c_void_p(out.data_ptr()), x.numel() // L))
        return out


def autotune(device: int = 0, stream=None, cache: Optional[str] = None, **kw) -> Params:
    """Fastest (segment_len, templates_per_tile, fft_radix) for the given parameters, measured
    by fdas_autotune on this GPU; cached as JSON keyed by device and shape."""
    import json
    import torch
    lib = load()
    p = Params()
    lib.fdas_default_params(byref(p))
    for k, v in kw.items():
        if k in ("store", "plane"):
            setattr(p, k + "_dtype", DTYPES[v])
        elif k == "norm":
            p.norm = NORMS[v]
        else:
            setattr(p, k, v)
    name = torch.cuda.get_device_properties(device).gcnArchName if torch.cuda.is_available() else "none"
    key = (f"{name}|N={p.n_samples}|z={p.z_min},{p.z_max},{p.z_step}|m={p.kernel_margin}|s={p.store_dtype}"
           f"|p={p.plane_dtype}|ib={p.interbin}")
    cache = cache or os.environ.get("FDAS_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "fdas_tune.json"))
    table = {}
    if os.path.exists(cache):
        try:
            table = json.load(open(cache))
        except (OSError, ValueError):
            table = {}
    if key in table and "fft_radix" in table[key]:
        p.segment_len, p.templates_per_tile = table[key]["segment_len"], table[key]["templates_per_tile"]
        p.fft_radix = table[key]["fft_radix"]
        return p
    st = stream if stream is not None else torch.cuda.current_stream(device)
    nb = p.n_samples // 2
    z = int(round((p.z_max - p.z_min) / p.z_step)) + 1
    need = nb * 8 + nb * z * 4 * (2 if p.interbin else 1) * 9 // 8 + nb * 40 + (64 << 20)
    scratch = torch.empty(need, dtype=torch.uint8, device=f"cuda:{device}")
    best, ms = Params(), c_double()
    st_ = lib.fdas_autotune(byref(p), device, c_void_p(st.cuda_stream), c_void_p(scratch.data_ptr()), need,
                            byref(best), byref(ms))
    if st_ != 0:
        raise FdasError(st_, lib.fdas_last_error(None).decode())
    table[key] = {"segment_len": best.segment_len, "templates_per_tile": best.templates_per_tile,
                  "fft_radix": best.fft_radix, "conv_ms": ms.value}
    try:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        json.dump(table, open(cache, "w"), indent=1)
    except OSError:
        pass
    return best


def _rz_function():
    import torch

    class RZPower(torch.autograd.Function):
        """P(r, z) of a plan's spectrum with the library's hand-written adjoint.

        ``spectrum`` is complex64 [n_bins] (FP32 storage plans); gradients flow
        to it (PyTorch's d/dRe + i d/dIm convention), to r and to z."""

        @staticmethod
        def forward(ctx, spectrum, r, z, plan):
            spec = torch.view_as_real(spectrum)
            p, y = plan.rz_power(spec, r, z)
            ctx.plan = plan
            ctx.save_for_backward(spectrum, r, z, y)
            return p

        @staticmethod
        def backward(ctx, grad_p):
            spectrum, r, z, y = ctx.saved_tensors
            want = ctx.needs_input_grad[0]
            gr, gz, gs = ctx.plan.rz_power_grad(torch.view_as_real(spectrum), r, z, grad_p, y=y, want_spectrum=want)
            return gs, gr.to(r.dtype), gz.to(z.dtype), None

    return RZPower


_RZ = None


def rz_power(spectrum, r, z, plan):
    """Differentiable P(r, z) (see RZPower)."""
    global _RZ
    if _RZ is None:
        _RZ = _rz_function()
    return _RZ.apply(spectrum, r, z, plan)


CAND_FIELDS = ("series", "harm", "R", "j", "r", "z", "power", "sigma")


def candidates_to_numpy(cands, count: int) -> np.ndarray:
    """Decodes the first ``count`` records into a numpy structured array."""
    n = min(int(count), cands.shape[0])
    raw = cands[:n].cpu().numpy()
    dt = np.dtype([(f, "<i4") for f in CAND_FIELDS[:4]] + [(f, "<f4") for f in CAND_FIELDS[4:]])
    return raw.view(dt).reshape(-1)
