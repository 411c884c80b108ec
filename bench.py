"""FDAS hot-path benchmark on one MI355X.

One step = the whole hot path over one SKA-like series: real FFT and median
normalisation, overlap-save correlation with 193 acceleration templates and the
power plane, harmonic sums up to 16 and the 6-sigma threshold.  The series is
N = 2^23 float32 samples (536.9 s at 64 us) with 8 injected accelerated
sinusoids, already resident in HBM.  Throughput is bins x templates per second
(N/2 * 193 per step).  The headline path stores spectrum, templates and plane
in bfloat16; its arithmetic is FP32, except the two DFT-16 stages of each
1024-point inverse FFT, which run as FP16 matrix-core products with FP32 sums
(dtype "f32+f16"); the FP32-storage path (all FP32) is timed beside it.

Prints one JSON line.  Extra legs: the FP64 oracle timed on a bounded sample
of the same workload on the host's cores (cpu_baseline, the only use of the
oracle here), the power error of the BF16 path against the FP32-storage path
at detections (accuracy_vs_fp32_plane; the error against the FP64 oracle is
held by the GPU tests), the BF16 spectrum with an FP32 plane
(bf16_in_f32_plane), the recall of the injections, the energy per unit of
work, the same step on a half-bin plane, the refinement of 4096 off-grid
candidates on a 2^22-bin spectrum, and the 512-trial batch of uneven DM
trials (batch: autotuned, graph-replayed chunks).

Kernel durations come from HIP events recorded on the plan's stream around
each stage of every timed step.  The roofline object describes the kernel
with the largest share of the step; "kernels" holds both big ones.
"""
from __future__ import annotations

import argparse
import hashlib
import heapq
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
PEAK_FP32_VALU = 157.3e12  # flop/s, MI355X FP32 vector (packed; 78.6e12 unpacked)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--segment-len", type=int, default=1024)
    ap.add_argument("--store", default="bf16")
    ap.add_argument("--plane", default=None, help="plane dtype (default: same as --store)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-storage comparison leg")
    ap.add_argument("--no-check", action="store_true", help="skip the power error / recall leg")
    ap.add_argument("--no-refine", action="store_true", help="skip the candidate-refinement leg")
    ap.add_argument("--no-interbin", action="store_true", help="skip the half-bin plane leg")
    ap.add_argument("--no-energy", action="store_true", help="skip the energy-counter leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-trial batch leg")
    ap.add_argument("--interbin", action="store_true",
                    help="time the step on the half-bin plane (implies --only-step --no-fp32)")
    ap.add_argument("--only-step", action="store_true",
                    help="the timed step and the FP32 comparison only (no other leg): for profiler runs")
    ap.add_argument("--n", type=int, default=1 << 23)
    ap.add_argument("--calib-copy", action="store_true", help="also run a plain 1 GiB device copy (for counters)")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--workload", default="ska-single", choices=["ska-single", "ska-batch", "ska-full"],
                    help="ska-batch: 512 uneven DM trials (256 x 2^23, 128 x 2^22, 128 x 2^21) in chunks; "
                         "ska-full: 5925 trials with clustering and refinement")
    return ap.parse_args()


SOURCES = {"conv": ("k_conv.hip", "fft.hpp", "fft_mfma.hpp", "common.hpp", "launch.hpp"),
           "harmonic_sum": ("k_harmsum.hip", "fft.hpp", "common.hpp", "launch.hpp")}


def source_hash(kernel: str) -> str:
    """Hash of the sources a kernel is built from (a stored traffic figure is
    used only while it matches)."""
    h = hashlib.sha256()
    for f in SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2211_13517_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, key: str):
    """HBM-side bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE runs,
    each scaled by a plain 1 GiB copy's reading (profiles/traffic.json)."""
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tf):
        return None
    t = json.load(open(tf)).get(kernel, {})
    if t.get("source_hash") != source_hash(kernel):
        return None
    return t.get("per_launch_bytes", {}).get(key)


def algorithmic(L, U, hmax, Z, nbins, store_bytes, plane_bytes, interbin=False):
    """Per launch of the convolve->power kernel: bytes and flops the method needs.

    Bytes: the spectrum read once, the template spectra read once, the plane
    written once (plane_bytes per bin: both columns on a half-bin plane).
    Flops (FFT convention 5 L log2 L per complex FFT): one forward FFT per
    segment, and per segment and template a complex product (6 L), an inverse
    FFT and |y|^2 of the U useful outputs (3 U), plus the half-bin power
    |y_i - y_{i+1}|^2 / 2 (6 U) on a half-bin plane."""
    nseg = math.ceil(nbins / U)
    bytes_ = nbins * store_bytes + Z * L * store_bytes + Z * nbins * plane_bytes
    fft = 5.0 * L * math.log2(L)
    flops = nseg * fft + nseg * Z * (6.0 * L + fft + (9.0 if interbin else 3.0) * U)
    return bytes_, flops


def copy_probe(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy bandwidth on this GPU (read + write bytes / s),
    the practical HBM ceiling the kernels are also compared with."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3)


def harm_bytes(Z, nbins, plane_bytes):
    """Per launch of the harmonic sum: the plane read once (candidate records
    are a few KB)."""
    return Z * nbins * plane_bytes


def run_path(fdas, torch, xt, n, args, store, plane, interbin=0):
    pl = fdas.Plan(store=store, plane=plane, n_samples=n, z_min=-96.0, z_max=96.0, z_step=1.0, n_harmonics=16,
                   segment_len=args.segment_len, interbin=interbin)
    nb = n // 2
    spec = pl.new_spectrum(nb)
    P = pl.new_plane(nb)
    cap = 1 << 20
    cands = torch.empty((cap, 8), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        count.zero_()
        pl.spectrum(xt, [0], [n], out=spec)
        if ev is not None:
            ev[0].record(stream)
        pl.convolve_spectrum(spec, [n], plane=P)
        if ev is not None:
            ev[1].record(stream)
        pl.harmonic_sum(P, [n], capacity=cap, cands=cands, count=count)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    pl.check(count, cap)
    torch.cuda.synchronize()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    conv_ms = [a.elapsed_time(b) for a, b, _ in evs]
    harm_ms = [b.elapsed_time(c) for _, b, c in evs]
    pl.check(count, cap)
    return dict(plan=pl, plane=P, spec=spec, cands=cands, count=int(count.item()), step_s=dt / args.steps,
                conv_ms=float(np.mean(conv_ms)), harm_ms=float(np.mean(harm_ms)), step=step)


def spectrum_norm_timing(torch, fdas, xt, n, store, reps=20):
    """fdas_spectrum (real FFT + normalisation) of the bench series with the
    per-block median and with the rednoise sub-blocks, HIP-event timed."""
    out = {}
    for norm in ("median", "rednoise"):
        pl = fdas.Plan(store=store, n_samples=n, norm=norm, make_templates=False)
        spec = pl.new_spectrum(n // 2)
        for _ in range(3):
            pl.spectrum(xt, [0], [n], out=spec)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pl.spectrum(xt, [0], [n], out=spec)
        e1.record()
        torch.cuda.synchronize()
        out[norm] = e0.elapsed_time(e1) / reps
    return out


class EnergyMeter:
    """The GPU's energy counter (accumulator x resolution in microjoules) read
    through amdsmi, for the device torch calls cuda:0, matched by PCI address
    (or the only device amdsmi sees).  Reads only; no clock or power control."""

    def __init__(self, torch, smi=None):
        if smi is None:
            import amdsmi as smi
        self.smi = smi
        smi.amdsmi_init()
        props = torch.cuda.get_device_properties(0)
        want = (int(props.pci_domain_id), int(props.pci_bus_id), int(props.pci_device_id))
        handles = list(smi.amdsmi_get_processor_handles())
        match = []
        for h in handles:
            dom, bus, rest = smi.amdsmi_get_gpu_device_bdf(h).split(":")
            if (int(dom, 16), int(bus, 16), int(rest.split(".")[0], 16)) == want:
                match.append(h)
        if len(match) == 1:
            self.h, self.matched = match[0], "pci address"
        elif len(handles) == 1:
            self.h, self.matched = handles[0], "only device visible"
        else:
            raise RuntimeError(f"no unique amdsmi device for pci {want} among {len(handles)}")

    def joules(self) -> float:
        return self.read()[0]

    def read(self):
        """(joules, the counter's own timestamp in seconds, or None if it
        reports none).  The counter advances in steps (about once a second on
        MI355X), and its timestamp moves with each step."""
        e = self.smi.amdsmi_get_energy_count(self.h)
        ts = e.get("timestamp") or 0
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6, (ts * 1e-9 if ts else None)

    @staticmethod
    def power(r0, r1, wall_s):
        """Mean power between two reads: energy over the counter's own time
        between its updates (a window of wall time would see one, two or
        three one-second steps of the counter), else over the wall time."""
        (e0, ts0), (e1, ts1) = r0, r1
        if ts0 is not None and ts1 is not None and ts1 > ts0:
            return (e1 - e0) / (ts1 - ts0)
        return (e1 - e0) / wall_s

    def gfxclk_mhz(self):
        """Graphics clock from the metrics table: the average if reported,
        else the mean of the per-XCD current clocks (N/A fields skipped)."""
        try:
            m = self.smi.amdsmi_get_gpu_metrics_info(self.h)
        except Exception:
            return None
        for key in ("average_gfxclk_frequency", "current_gfxclk", "current_gfxclks"):
            v = m.get(key, "N/A")
            vals = v if isinstance(v, (list, tuple)) else [v]
            vals = [float(x) for x in vals if isinstance(x, (int, float)) and 0 < x < 65535]
            if vals:
                return sum(vals) / len(vals)
        return None

    def close(self):
        try:
            self.smi.amdsmi_shut_down()
        except Exception:
            pass


def energy_leg(torch, meter, runs, bt, seconds=2.0, preroll=3.0, reps=3):
    """Energy per 10^12 bins x templates of the whole step for each storage
    type: the mean power over a window of about `seconds` of back-to-back
    steps (energy over the counter's own time between its updates, so that
    the counter's one-second steps do not alias with the window) times the
    window's wall time per step.  Each window is preceded by `preroll`
    seconds of the same steps, so that the counter interval that reaches back
    before the window still sees only that load; the storage types alternate
    `reps` times and the median window is reported.  The idle power is taken
    over two seconds after a second of rest.  Clocks are whatever the GPU
    runs at (reported, not set)."""
    torch.cuda.synchronize()
    time.sleep(1.0)
    r0, t0 = meter.read(), time.perf_counter()
    for _ in range(2):
        time.sleep(1.0)
    r1, t1 = meter.read(), time.perf_counter()
    idle = meter.power(r0, r1, t1 - t0)
    out = {"idle_W": idle, "device": meter.matched, "clock_control": "none (default clocks)"}
    acc = {name: {"E": 0.0, "T": 0.0, "steps": 0, "J_per_1e12_bt_each": [], "ms_per_step_each": [], "W_each": []}
           for name in runs}
    for _ in range(reps):
        for name, r in runs.items():
            for _ in range(max(1, int(preroll / r["step_s"]))):
                r["step"]()
            torch.cuda.synchronize()  # the window must not inherit queued pre-roll work
            k = max(20, int(seconds / r["step_s"]))
            r0, t0 = meter.read(), time.perf_counter()
            for _ in range(k):
                r["step"]()
            torch.cuda.synchronize()
            r1, t1 = meter.read(), time.perf_counter()
            w = meter.power(r0, r1, t1 - t0)
            a = acc[name]
            a["E"] += w * (t1 - t0)
            a["T"] += t1 - t0
            a["steps"] += k
            a["J_per_1e12_bt_each"].append(w * (t1 - t0) / (k * bt) * 1e12)
            a["ms_per_step_each"].append((t1 - t0) / k * 1e3)
            a["W_each"].append(w)
    for name, a in acc.items():
        j = float(np.median(a["J_per_1e12_bt_each"]))
        w = float(np.median(a["W_each"]))
        ms = float(np.median(a["ms_per_step_each"]))
        out[name] = {"steps": a["steps"], "seconds": a["T"], "avg_W": w, "J_per_1e12_bt": j,
                     "J_per_1e12_bt_each": a["J_per_1e12_bt_each"], "ms_per_step_each": a["ms_per_step_each"],
                     "above_idle_J_per_1e12_bt": j - idle * ms * 1e-3 / bt * 1e12,
                     "avg_gfxclk_MHz": meter.gfxclk_mhz()}
    if "bf16" in out and "f32" in out:
        out["bf16_energy_saving"] = 1.0 - out["bf16"]["J_per_1e12_bt"] / out["f32"]["J_per_1e12_bt"]
    return out


def midway_recall(torch, fdas, synth, runs, n, n_inj=64, p0=44.0):
    """Recall of signals whose mean frequency lies exactly midway between two
    bins (z on the grid), at peak power p0: each bin keeps 0.405 p0, the
    half-bin column 0.81 p0.  Each plan in `runs` searches the same series
    once; a signal is recovered by a record within 0.5 bin and 1 z of it."""
    rng = np.random.default_rng(91)
    amp = math.sqrt(4 * p0 / n)
    inj = []
    for i in range(n_inj):
        rbar = 20000 + (n // 2 - 40000) // n_inj * i + 0.5
        z = float(rng.integers(-90, 91))
        inj.append(synth.Injection(amp, rbar - z / 2, z, float(rng.uniform(0, 2 * np.pi))))
    x2 = synth.make_series_device(n, inj, 91, 0)
    out = {"signals": n_inj, "peak_power": p0}
    for name, r in runs.items():
        pl, cands = r["plan"], r["cands"]
        cap = cands.shape[0]
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        pl.spectrum(x2, [0], [n], out=r["spec"])
        pl.convolve_spectrum(r["spec"], [n], plane=r["plane"])
        pl.harmonic_sum(r["plane"], [n], capacity=cap, cands=cands, count=count)
        pl.check(count, cap)
        c = fdas.candidates_to_numpy(cands, int(count.item()))
        hits = sum(bool(((np.abs(c["r"] - s.r_mean) <= 0.5) & (np.abs(c["z"] - s.z) <= 1.0)).any()) for s in inj)
        out[name] = hits / n_inj
    return out


def precision_checks(res, ref, inj, Z, tau1):
    """Relative power error of a reduced-precision plane at detections, against
    the FP32-storage plane of the same series on the same GPU (the parity
    tests hold that plane to 1e-4 of the FP64 oracle): every cell within
    +-3 bins and +-4 z of each injection's peak whose FP32 power is at least
    tau_1.  Plus the recall of the injections by each path's candidates."""
    nb = res["plane"].numel() // Z
    rows, cols = [], []
    for i in inj:
        rc, jc = int(round(i.r_mean)), int(round(i.z + 96))
        for dj in range(-4, 5):
            for dr in range(-3, 4):
                if 0 <= jc + dj < Z:
                    rows.append(jc + dj)
                    cols.append(rc + dr)
    ri, ci = torch_index(rows), torch_index(cols)
    got = res["plane"].view(Z, nb)[ri, ci].float().cpu().numpy().astype(np.float64)
    want = ref["plane"].view(Z, nb)[ri, ci].float().cpu().numpy().astype(np.float64)
    det = want >= tau1
    rel = np.abs(got - want) / want

    def recall(r):
        c = fdas_cands(r)
        return sum(bool(np.any((np.abs(c["r"] - i.r_mean) <= 1.0) & (np.abs(c["z"] - i.z) <= 1.0))) if len(c) else False
                   for i in inj) / len(inj)

    return dict(reference="FP32-storage plane of the same series", n_det=int(det.sum()),
                max_rel=float(rel[det].max()), median_rel=float(np.median(rel[det])),
                recall=recall(res), recall_reference=recall(ref))


_torch = None


def torch_index(a):
    return _torch.from_numpy(np.asarray(a)).to("cuda")


def fdas_cands(res):
    import paper_2211_13517_amd as fdas
    return fdas.candidates_to_numpy(res["cands"], res["count"])


# ------------------------------------------------------------ CPU baseline
# The oracle on the host's cores: a pool of worker processes (started with
# "spawn" before the first GPU call, so no worker inherits a GPU context),
# each holding the series' normalised spectrum and computing whole
# correlation rows of the plane with numpy's single-threaded FFT.

_ORACLE_A = None


def _oracle_worker_init(x, ready):
    global _ORACLE_A
    from oracle import fdas64 as o
    _ORACLE_A = o.normalise(o.spectrum(x), "median")
    ready.put(1)


def _oracle_rows(rows):
    from oracle import fdas64 as o
    zs = o.z_grid(-96, 96, 1)
    p = o.power_plane(_ORACLE_A, zs, rows=list(rows))
    return float(np.sum(p))


def cpu_pool_start(x):
    """Starts the oracle pool: one worker per core this process may use (at
    most 16, the host share of one GPU), each normalising the series once."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    ready = ctx.Queue()
    # one thread per worker: the oracle's quadratures call BLAS, whose own
    # thread pool in every worker would oversubscribe the cores many times
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    os.environ.update({k: "1" for k in saved})
    try:
        pool = ctx.Pool(cores, initializer=_oracle_worker_init, initargs=(x, ready))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return {"pool": pool, "ready": ready, "cores": cores}


def cpu_baseline(o, x, cp, rows_per_core=1):
    """The oracle as it stands, timed on a bounded sample of the step: the
    spectrum and median normalisation of the full series (one core, in this
    process), then `rows_per_core` correlation rows per worker spread over the
    pool (full-length FFT correlation per acceleration trial, FP64)."""
    cores = cp["cores"]
    for _ in range(cores):           # every worker has its spectrum
        cp["ready"].get(timeout=600)
    zs = o.z_grid(-96, 96, 1)
    rows = min(len(zs), rows_per_core * cores)
    sel = np.linspace(0, len(zs) - 1, rows).round().astype(int)
    t0 = time.perf_counter()
    o.normalise(o.spectrum(x), "median")
    t1 = time.perf_counter()
    cp["pool"].map(_oracle_rows, [[int(j)] for j in sel], chunksize=1)
    t2 = time.perf_counter()
    cp["pool"].close()
    cp["pool"].join()
    nb = len(x) // 2
    dt = t2 - t0
    return dict(value=rows * nb / dt, unit="bins*templates/s", cores=cores, kind="oracle",
                sample=f"spectrum+median normalisation of one N={len(x)} series on 1 core ({t1 - t0:.2f} s), then "
                       f"{rows} of its 193 template rows on {cores} worker processes ({t2 - t1:.2f} s); "
                       f"full-length FFT correlation, FP64, numpy single-threaded per process")


def refine_leg(torch, fdas, synth):
    """Refinement at its own workload: one 2^22-sample series, 4096 candidates
    perturbed by up to 0.5 bin and 1 z from injected truths, 40 ascent
    iterations each (FP64 positions, FP32 spectrum)."""
    n = 1 << 22
    truths, starts = synth.refine_candidates(4, 4096, r_gap=400.0)
    xt = synth.make_series_device(n, truths, 4, 0)
    pl = fdas.Plan(store="f32", n_samples=n, z_min=-96.0, z_max=96.0, z_step=1.0, make_templates=False)
    spec = pl.spectrum(xt, [0], [n])
    r = torch.tensor(starts[:, 0], dtype=torch.float64, device="cuda")
    z = torch.tensor(starts[:, 1], dtype=torch.float64, device="cuda")
    for _ in range(2):
        rr, zz, pf = pl.refine(spec, r, z, n_iter=40)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    K = 10
    e0.record()
    for _ in range(K):
        rr, zz, pf = pl.refine(spec, r, z, n_iter=40)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    tr = np.array([t.r_mean for t in truths])
    tz = np.array([t.z for t in truths])
    rr, zz = rr.cpu().numpy(), zz.cpu().numpy()
    # the same candidates as fundamentals of 16-harmonic sums (time only: the
    # series carries single sinusoids); z/16 keeps every harmonic's drift on
    # the grid's range
    r16, z16 = r / 16.0, z / 16.0
    pl.refine_harmonics(spec, r16, z16, 16, n_iter=40)
    torch.cuda.synchronize()
    e0.record()
    pl.refine_harmonics(spec, r16, z16, 16, n_iter=40)
    e1.record()
    torch.cuda.synchronize()
    ms16 = e0.elapsed_time(e1)
    return {"workload": "4096 candidates on one N=2^22 series, 40 ascent iterations", "ms": ms,
            "candidates_per_s": 4096 / (ms / 1e3),
            "within_1bin_1z_of_truth": float(np.mean((np.abs(rr - tr) < 1.0) & (np.abs(zz - tz) < 1.5))),
            "harmonics16_ms": ms16, "harmonics16_candidates_per_s": 4096 / (ms16 / 1e3)}


def full_leg(args, torch, fdas, synth):
    """The full SKA-like run: 5925 DM trials (3050 x 2^23, 1500 x 2^22,
    1375 x 2^21), 1 % carrying one injection; BF16 storage, harmonic sums to
    16, 6 sigma, in chunks of up to 16 + 8 + 8 series whose inputs are
    generated on the device before each chunk (untimed).  The search of each
    chunk is timed with HIP events.  Candidates are reduced to local maxima
    (fdas_cluster, +-2 bins, +-2 trials).  A maximum that can still be among
    the 1024 most significant so far is refined on its series' spectrum: the
    sum of its H harmonics, S = sum_k P(k r, k z), is climbed from its grid
    fundamental (R/H, z_j/H) (fdas_refine_harmonics); the top 1024 are
    reported."""
    N = 1 << 23
    lens_all, truths = synth.ska_full(seed=5, n=N)
    groups = [[i for i, L_ in enumerate(lens_all) if L_ == N // d] for d in (1, 2, 4)]
    per = (16, 8, 8)
    chunks = []
    while any(groups):
        c = []
        for g, k in zip(groups, per):
            c += g[:k]
            del g[:k]
        chunks.append(c)
    max_batch = 16 * N + 8 * (N // 2) + 8 * (N // 4)
    pl = fdas.Plan(store=args.store, plane=args.plane or args.store, n_samples=N, max_batch_samples=max_batch,
                   z_min=-96.0, z_max=96.0, z_step=1.0, n_harmonics=16, segment_len=args.segment_len)
    Z = pl.Z
    work = torch.empty(max_batch, dtype=torch.float32, device="cuda")
    plane = pl.new_plane(max_batch // 2)
    spec = pl.new_spectrum(max_batch // 2)
    cap = 1 << 23
    cands = torch.empty((cap, 8), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    search_ms, cluster_ms, refine_ms, n_cands = 0.0, 0.0, 0.0, 0
    found = {}       # trial -> list of (R, z_j) of local maxima
    refined = []     # (sigma, trial, R, zj, r_ref, z_ref, P_cell, P_ref)
    top_sig = []     # min-heap of the 1024 largest significances so far
    n_max, n_refined = 0, 0
    for ci, c in enumerate(chunks):
        if ci % 20 == 0:
            print(f"[full run] chunk {ci}/{len(chunks)}", file=sys.stderr, flush=True)
        lens = [lens_all[i] for i in c]
        offs = np.zeros(len(c), np.int64)
        offs[1:] = np.cumsum(lens)[:-1]
        for s_, i in enumerate(c):
            synth.fill_series_device(work[int(offs[s_]): int(offs[s_]) + lens[s_]], truths[i], 5, i)
        e0.record()
        pl.search(work, offs, lens, plane, cands, count, spectrum=spec)
        e1.record()
        torch.cuda.synchronize()
        search_ms += e0.elapsed_time(e1)
        pl.check(count, cap)
        n = int(count.item())
        n_cands += n
        if n == 0:
            continue
        e0.record()
        keep = pl.cluster(cands, count, 2, 2)
        e1.record()
        torch.cuda.synchronize()
        cluster_ms += e0.elapsed_time(e1)
        rec = fdas.candidates_to_numpy(cands, n)
        rec = rec[keep[:n].cpu().numpy().astype(bool)]
        n_max += len(rec)
        for s_ in np.unique(rec["series"]):
            zs_all = -96.0 + rec["j"][rec["series"] == s_].astype(np.float64)
            found[c[int(s_)]] = list(zip(rec["R"][rec["series"] == s_].tolist(), zs_all.tolist()))
        # only maxima that can still be in the final top 1024 are refined
        floor = top_sig[0] if len(top_sig) >= 1024 else -np.inf
        rec = rec[rec["sigma"] > floor]
        for v in rec["sigma"].tolist():
            if len(top_sig) < 1024:
                heapq.heappush(top_sig, v)
            elif v > top_sig[0]:
                heapq.heapreplace(top_sig, v)
        n_refined += len(rec)
        for s_ in np.unique(rec["series"]):
            m = rec[rec["series"] == s_]
            i = c[int(s_)]
            zj = -96.0 + m["j"].astype(np.float64)
            nb = lens[int(s_)] // 2
            sp = spec[int(offs[s_]) // 2: int(offs[s_]) // 2 + nb]
            hh = m["harm"].astype(np.float64)
            r0 = torch.tensor(m["R"].astype(np.float64) / hh, device="cuda")
            z0 = torch.tensor(zj / hh, device="cuda")
            hs = torch.tensor(m["harm"].astype(np.int32), device="cuda")
            e0.record()
            _, _, p_cell = pl.refine_harmonics(sp, r0, z0, hs, n_iter=0)
            rr, zz, pf = pl.refine_harmonics(sp, r0, z0, hs, n_iter=40)
            e1.record()
            torch.cuda.synchronize()
            refine_ms += e0.elapsed_time(e1)
            for k in range(len(m)):
                refined.append((float(m["sigma"][k]), i, int(m["R"][k]), float(zj[k]), float(rr[k]), float(zz[k]),
                                float(p_cell[k]), float(pf[k])))
    refined.sort(key=lambda t: -t[0])
    top = refined[:1024]
    bt = sum(lens_all) // 2 * Z
    det, hit, hit_ref = 0, 0, 0
    for i, tl in enumerate(truths):
        for t in tl:
            p_peak = lens_all[i] * t.amp ** 2 / 4 * 0.405
            if p_peak < 20.737 + 3 * math.sqrt(20.737):
                continue
            det += 1
            hit += any(abs(R - t.r_mean) <= 1.0 and abs(z - t.z) <= 1.0 for R, z in found.get(i, []))
            hit_ref += any(i == tr and abs(r - t.r_mean) <= 1.0 and abs(z - t.z) <= 1.5
                           for _, tr, _, _, r, z, _, _ in top)
    gain = [pr / pc for _, _, _, _, _, _, pc, pr in top if pc > 0]
    return {"workload": "5925 DM trials (3050 x 2^23, 1500 x 2^22, 1375 x 2^21), 1% with one injection, "
                        f"{len(chunks)} chunks of <= 16+8+8 series, 193 templates, harmonic sums to 16, 6 sigma, "
                        "local maxima (+-2 bins, +-2 trials) refined on their harmonic sums, top 1024 reported",
            "bt_per_s": bt / (search_ms / 1e3), "search_seconds": search_ms / 1e3, "bins_x_templates": bt,
            "candidates": n_cands, "local_maxima": n_max, "refined": n_refined, "cluster_seconds": cluster_ms / 1e3,
            "refine_seconds": refine_ms / 1e3,
            "detectable_injections": det, "injections": sum(len(t) for t in truths),
            "recall_detectable": (hit / det) if det else None,
            "recall_top1024_refined": (hit_ref / det) if det else None,
            "median_refined_power_gain_top1024": float(np.median(gain)) if gain else None}


def batch_leg(args, torch, fdas, synth):
    """Batching: 512 uneven DM trials, chunks of 16 x 2^23 + 8 x 2^22 + 8 x 2^21
    series (one HIP graph, replayed per chunk after the chunk's series are
    copied into the working buffer); BF16 storage, segment length and template
    grouping from the autotuner, harmonic sums to 16, 6 sigma."""
    N = 1 << 23
    per_chunk = [N] * 16 + [N // 2] * 8 + [N // 4] * 8
    n_chunks = 16
    lens_all = [N] * 256 + [N // 2] * 128 + [N // 4] * 128
    truths = synth.batch_injections(lens_all, seed=3)
    # series of chunk c: 16 full, 8 half, 8 quarter, in the order of lens_all
    idx = []
    for c in range(n_chunks):
        idx.append(list(range(16 * c, 16 * c + 16)) + list(range(256 + 8 * c, 256 + 8 * c + 8)) +
                   list(range(384 + 8 * c, 384 + 8 * c + 8)))
    chunk_samples = sum(per_chunk)
    offs = np.zeros(len(per_chunk), np.int64)
    offs[1:] = np.cumsum(per_chunk)[:-1]
    # all inputs resident in HBM before timing (11.8 GB float32)
    allx = torch.empty(n_chunks * chunk_samples, dtype=torch.float32, device="cuda")
    for c in range(n_chunks):
        for s_, i in enumerate(idx[c]):
            o0 = c * chunk_samples + int(offs[s_])
            synth.fill_series_device(allx[o0: o0 + per_chunk[s_]], truths[i], 3, i)
    # segment length and templates per tile from the autotuner (a full-length
    # series timed for every allowed L and template grouping on this GPU)
    tuned = fdas.autotune(cache=os.path.join("/tmp", "fdas_tune_bench.json"), n_samples=N, z_min=-96.0,
                          z_max=96.0, z_step=1.0, store=args.store, plane=args.plane or args.store)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        pl = fdas.Plan(store=args.store, plane=args.plane or args.store, n_samples=N, max_batch_samples=chunk_samples,
                       z_min=-96.0, z_max=96.0, z_step=1.0, n_harmonics=16, segment_len=tuned.segment_len,
                       templates_per_tile=tuned.templates_per_tile, fft_radix=tuned.fft_radix, stream=stream)
        work = torch.empty(chunk_samples, dtype=torch.float32, device="cuda")
        plane = pl.new_plane(chunk_samples // 2)
        cap = 1 << 23  # strong injections leave ~10^5 passing cells each
        cands = torch.empty((cap, 8), dtype=torch.int32, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        found = []

        def chunk(c, keep):
            work.copy_(allx[c * chunk_samples:(c + 1) * chunk_samples])
            pl.search(work, offs, per_chunk, plane, cands, count, use_graph=True)
            if keep:
                pl.check(count, cap)
                found.append(fdas.candidates_to_numpy(cands, int(count.item())))

        chunk(0, False)  # capture
        stream.synchronize()
        t0 = time.perf_counter()
        for c in range(n_chunks):
            chunk(c, False)
        stream.synchronize()
        dt = time.perf_counter() - t0
        for c in range(n_chunks):  # untimed pass keeping the candidates for recall
            chunk(c, True)
    bt = sum(lens_all) // 2 * pl.Z
    det, hit = 0, 0
    for c in range(n_chunks):
        cc = found[c]
        for s_, i in enumerate(idx[c]):
            sel = cc[cc["series"] == s_] if len(cc) else cc
            for j in truths[i]:
                n_s = lens_all[i]
                # detectable: oracle-free criterion, peak power above tau_1 + 3 sqrt(tau_1) at mid-bin scalloping
                p_peak = n_s * j.amp ** 2 / 4 * 0.405
                if p_peak < 20.737 + 3 * math.sqrt(20.737):
                    continue
                det += 1
                ok = len(sel) and np.any((np.abs(sel["r"] - j.r_mean) <= 1.0) & (np.abs(sel["z"] - j.z) <= 1.0))
                hit += bool(ok)
    return {"workload": "512 uneven DM trials (256 x 2^23, 128 x 2^22, 128 x 2^21), 16 graph replays of "
                        "32-series chunks, 193 templates, harmonic sums to 16, 6 sigma",
            "bt_per_s": bt / dt, "seconds": dt, "bins_x_templates": bt, "segment_len": pl.L,
            "templates_per_tile": int(tuned.templates_per_tile), "fft_radix": int(tuned.fft_radix), "autotuned": True,
            "recall_detectable": (hit / det) if det else None, "detectable_injections": det,
            "injections": sum(len(t) for t in truths)}


def main():
    global _torch
    args = parse()
    if args.interbin:
        args.only_step = args.no_fp32 = True
    if args.only_step:
        args.no_cpu_baseline = args.no_check = args.no_refine = args.no_interbin = args.no_energy = True
        args.no_batch = True
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (sharding over "
                                   "GPUs is designed but not built)"}))
        sys.exit(2)
    import synth
    cpu = None
    if args.workload == "ska-single":
        x, inj, _ = synth.ska_single(seed=2, n=args.n)
        if not args.no_cpu_baseline:
            cpu = cpu_pool_start(x)   # before torch or the library touch the GPU
    import torch
    _torch = torch
    import paper_2211_13517_amd as fdas
    fdas.load()
    if args.workload in ("ska-batch", "ska-full"):
        out = (batch_leg if args.workload == "ska-batch" else full_leg)(args, torch, fdas, synth)
        print(json.dumps(out), flush=True)
        if args.json_out:
            with open(args.json_out, "w") as f:
                f.write(json.dumps(out) + "\n")
        return
    n = args.n
    xt = torch.from_numpy(x).to("cuda")
    plane_dt = args.plane or args.store
    res = run_path(fdas, torch, xt, n, args, args.store, plane_dt, interbin=1 if args.interbin else 0)
    pl = res["plan"]
    Z, L, U, hmax = pl.Z, pl.L, pl.U, pl.hmax
    nb = n // 2
    bt = nb * Z
    sb = 8 if args.store == "f32" else 4
    pb = (4 if plane_dt == "f32" else 2) * pl.res   # plane bytes per bin (two columns on a half-bin plane)
    abytes, aflops = algorithmic(L, U, hmax, Z, nb, sb, pb, interbin=args.interbin)
    conv_s = res["conv_ms"] / 1e3
    harm_s = res["harm_ms"] / 1e3
    hbytes = harm_bytes(Z, nb, pb)
    key = f"{args.store}/{plane_dt}/{L}/{n}" + ("/interbin" if args.interbin else "")
    out = {
        "metric": "bins*templates/s for FDAS conv, BF16 vs FP32 at <=3% power err; HBM GB/s",
        "value": bt / res["step_s"],
        "unit": "bins*templates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["step_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # FP16 matrix-core DFT stages on the 1024-point, 16-bit-plane path
        "dtype": "f32+f16" if (L == 1024 and plane_dt != "f32") else "f32",
        "data": "synthetic",
        "config": {"workload": f"SKA-like single series: N=2^{int(math.log2(n))} float32, 8 injected accelerated "
                               f"sinusoids, 193 templates z in [-96,96] step 1, segment {L}, median normalisation, "
                               f"harmonic sums to 16, 6 sigma" + (", half-bin plane" if args.interbin else ""),
                   "storage": args.store, "plane": plane_dt, "segment_len": L, "templates": Z, "bins": nb},
    }
    # Both big kernels against their rooflines.  convolve->power is bound by
    # FP32 VALU issue (packed FP32 is not used, so 78.6 TFLOP/s is its real
    # ceiling; the published 157.3 is the peak quoted); the harmonic sum is
    # bound by HBM: one read of the plane is its algorithmic traffic.
    conv = {"bound": "alu", "achieved": aflops / conv_s / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
            "frac": aflops / conv_s / PEAK_FP32_VALU, "traffic": measured_traffic("conv", key),
            "ms": res["conv_ms"], "bt_per_s": bt / conv_s, "alg_bytes": abytes, "alg_flops": aflops,
            "hbm_alg_GBps": abytes / conv_s / 1e9}
    harm = {"bound": "hbm", "achieved": hbytes / harm_s / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": hbytes / harm_s / PEAK_HBM, "traffic": measured_traffic("harmonic_sum", key),
            "ms": res["harm_ms"], "alg_bytes": hbytes}
    copy_bw = copy_probe(torch)
    for kk, kb in (("harmonic_sum", harm), ("convolve_power", conv)):
        kb["copy_probe_GBps"] = copy_bw / 1e9
        alg_bps = kb["alg_bytes"] / (kb["ms"] / 1e3)
        kb["alg_frac_of_copy"] = alg_bps / copy_bw
        if kb["traffic"]:
            # FETCH_SIZE/WRITE_SIZE count the bytes leaving L2 for the memory
            # side (MALL hits included), not HBM bytes alone
            kb["l2_miss_GBps"] = kb["traffic"] / (kb["ms"] / 1e3) / 1e9
            kb["traffic_over_alg_bytes"] = kb["traffic"] / kb["alg_bytes"]
    out["kernels"] = {"convolve_power": conv, "harmonic_sum": harm}
    dom = harm if res["harm_ms"] > res["conv_ms"] else conv
    out["roofline"] = {k: dom[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    out["roofline"]["kernel"] = "harmonic_sum" if dom is harm else "convolve_power"
    if not args.no_fp32:
        r32 = run_path(fdas, torch, xt, n, args, "f32", "f32")
        out["fp32"] = {"value": bt / r32["step_s"], "ms_per_step": r32["step_s"] * 1e3,
                       "conv_bt_per_s": bt / (r32["conv_ms"] / 1e3), "conv_ms": r32["conv_ms"],
                       "harmonic_sum_ms": r32["harm_ms"]}
        out["speedup_vs_fp32"] = {"step": r32["step_s"] / res["step_s"], "conv": r32["conv_ms"] / res["conv_ms"],
                                  "harmonic_sum": r32["harm_ms"] / res["harm_ms"]}
    if not args.no_check and not args.no_fp32 and args.store != "f32":
        tau1 = float(res["plan"].thresholds()[0])
        out["accuracy_vs_fp32_plane"] = {args.store: precision_checks(res, r32, inj, Z, tau1)}
        if args.store == "bf16" and plane_dt == "bf16":
            # the third storage form: BF16 spectrum and templates, FP32 plane
            rbf = run_path(fdas, torch, xt, n, args, "bf16", "f32")
            out["bf16_in_f32_plane"] = {
                "value": bt / rbf["step_s"], "ms_per_step": rbf["step_s"] * 1e3, "conv_ms": rbf["conv_ms"],
                "harmonic_sum_ms": rbf["harm_ms"], "speedup_vs_fp32_step": r32["step_s"] / rbf["step_s"],
                "accuracy_vs_fp32_plane": precision_checks(rbf, r32, inj, Z, tau1)}
            del rbf
    if not args.no_energy and not args.no_fp32 and args.store == "bf16":
        try:
            meter = EnergyMeter(torch)
            try:
                out["energy"] = energy_leg(torch, meter, {"bf16": res, "f32": r32}, bt)
            finally:
                meter.close()
        except Exception as e:  # telemetry is optional: report, do not fail the bench
            out["energy"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.only_step:
        out["spectrum_ms_by_norm"] = spectrum_norm_timing(torch, fdas, xt, n, args.store)
    if L != 8192 and not args.only_step:
        # the segment length the SKA-like configuration names, for comparison
        a8 = argparse.Namespace(**vars(args))
        a8.segment_len = 8192
        r8 = run_path(fdas, torch, xt, n, a8, args.store, plane_dt)
        out["segment_8192"] = {"value": bt / r8["step_s"], "ms_per_step": r8["step_s"] * 1e3,
                               "conv_ms": r8["conv_ms"], "harmonic_sum_ms": r8["harm_ms"]}
        del r8
    if not args.no_interbin:
        rib = run_path(fdas, torch, xt, n, args, args.store, plane_dt, interbin=1)
        out["interbin"] = {
            "workload": "same series and step on the half-bin plane (bin and half-bin column per bin)",
            "value": bt / rib["step_s"], "ms_per_step": rib["step_s"] * 1e3, "conv_ms": rib["conv_ms"],
            "harmonic_sum_ms": rib["harm_ms"],
            "harmonic_sum_alg_GBps": 2 * hbytes / (rib["harm_ms"] / 1e3) / 1e9,
            "recall_midway": midway_recall(torch, fdas, synth, {"bins": res, "half_bins": rib}, n)}
    if not args.no_refine:
        out["refine"] = refine_leg(torch, fdas, synth)
    if not args.no_batch:
        b = batch_leg(args, torch, fdas, synth)
        out["batch"] = {k: b[k] for k in ("workload", "bt_per_s", "seconds", "recall_detectable",
                                          "detectable_injections", "segment_len", "templates_per_tile",
                                          "fft_radix")}
    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    if cpu is not None:
        from oracle import fdas64 as o
        out["cpu_baseline"] = cpu_baseline(o, x, cpu)
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
