"""Host-side logic of bench.py that needs no GPU: the energy counter's device
matching and unit scaling, and the energy-per-work arithmetic."""
import types

import pytest

import bench


class FakeSmi:
    """Two devices; the counter advances by `rate` units per fake second."""

    def __init__(self, bdfs, resolution=15.3):
        self.bdfs = bdfs
        self.res = resolution
        self.acc = {i: 1000 * i for i in range(len(bdfs))}
        self.inited = False

    def amdsmi_init(self):
        self.inited = True

    def amdsmi_shut_down(self):
        self.inited = False

    def amdsmi_get_processor_handles(self):
        return list(range(len(self.bdfs)))

    def amdsmi_get_gpu_device_bdf(self, h):
        return self.bdfs[h]

    def amdsmi_get_energy_count(self, h):
        return {"energy_accumulator": self.acc[h], "counter_resolution": self.res, "timestamp": 0}

    def amdsmi_get_gpu_metrics_info(self, h):
        return {"average_gfxclk_frequency": 2400}


def fake_torch(dom=0, bus=0x75, dev=0):
    props = types.SimpleNamespace(pci_domain_id=dom, pci_bus_id=bus, pci_device_id=dev)
    cuda = types.SimpleNamespace(get_device_properties=lambda i: props, synchronize=lambda: None)
    return types.SimpleNamespace(cuda=cuda)


def test_meter_matches_by_pci_address_and_scales_to_joules():
    smi = FakeSmi(["0000:05:00.0", "0000:75:00.0"])
    m = bench.EnergyMeter(fake_torch(bus=0x75), smi=smi)
    assert m.h == 1 and m.matched == "pci address"
    assert m.joules() == pytest.approx(1000 * 15.3e-6)
    assert m.gfxclk_mhz() == 2400.0
    m.close()
    assert not smi.inited


def test_meter_falls_back_to_the_only_device_and_refuses_ambiguity():
    m = bench.EnergyMeter(fake_torch(bus=0x11), smi=FakeSmi(["0000:05:00.0"]))
    assert m.h == 0 and m.matched == "only device visible"
    with pytest.raises(RuntimeError):
        bench.EnergyMeter(fake_torch(bus=0x11), smi=FakeSmi(["0000:05:00.0", "0000:06:00.0"]))


def test_gfxclk_falls_back_to_per_xcd_clocks():
    smi = FakeSmi(["0000:75:00.0"])
    smi.amdsmi_get_gpu_metrics_info = lambda h: {"average_gfxclk_frequency": "N/A", "current_gfxclk": "N/A",
                                                 "current_gfxclks": [2000, 2200, "N/A", 65535]}
    assert bench.EnergyMeter(fake_torch(), smi=smi).gfxclk_mhz() == 2100.0


def test_energy_leg_arithmetic(monkeypatch):
    """Idle 100 W; the bf16 step draws 600 W for 1 ms, the f32 step 500 W for
    2 ms: energy per 10^12 bt follows from the counter and the step count."""
    clock = {"t": 0.0}
    smi = FakeSmi(["0000:75:00.0"], resolution=1.0)       # 1 microjoule per unit
    meter = bench.EnergyMeter(fake_torch(), smi=smi)

    def advance(seconds, watts):
        clock["t"] += seconds
        smi.acc[0] += int(round(watts * seconds * 1e6))

    monkeypatch.setattr(bench.time, "sleep", lambda s: advance(s, 100.0))
    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock["t"])
    runs = {"bf16": {"step_s": 1e-3, "step": lambda: advance(1e-3, 600.0)},
            "f32": {"step_s": 2e-3, "step": lambda: advance(2e-3, 500.0)}}
    bt = 8.1e8
    out = bench.energy_leg(fake_torch(), meter, runs, bt, seconds=0.1, preroll=0.05, reps=2)
    assert out["idle_W"] == pytest.approx(100.0)
    assert out["bf16"]["steps"] == 200 and out["f32"]["steps"] == 100
    assert len(out["bf16"]["J_per_1e12_bt_each"]) == 2
    assert out["bf16"]["avg_W"] == pytest.approx(600.0)
    assert out["bf16"]["J_per_1e12_bt"] == pytest.approx(0.6 / bt * 1e12)
    assert out["f32"]["J_per_1e12_bt"] == pytest.approx(1.0 / bt * 1e12)
    assert out["f32"]["above_idle_J_per_1e12_bt"] == pytest.approx(0.8 / bt * 1e12)
    assert out["bf16_energy_saving"] == pytest.approx(0.4)


def test_energy_leg_is_exact_under_a_lagging_counter(monkeypatch):
    """A counter that reports the energy of 0.3 s ago: with a pre-roll of at
    least the lag, every window sees only its own load."""
    clock = {"t": 0.0}
    true = {"acc": 0.0}
    hist = [(0.0, 0.0)]
    lag = 0.3

    def advance(seconds, watts):
        clock["t"] += seconds
        true["acc"] += watts * seconds
        hist.append((clock["t"], true["acc"]))

    smi = FakeSmi(["0000:75:00.0"], resolution=1.0)

    def lagged(h):
        t = clock["t"] - lag
        e = max((a for (ts, a) in hist if ts <= t + 1e-12), default=0.0)
        return {"energy_accumulator": int(round(e * 1e6)), "counter_resolution": 1.0, "timestamp": 0}

    smi.amdsmi_get_energy_count = lagged
    meter = bench.EnergyMeter(fake_torch(), smi=smi)
    monkeypatch.setattr(bench.time, "sleep", lambda s: advance(s, 100.0))
    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock["t"])
    runs = {"bf16": {"step_s": 1e-3, "step": lambda: advance(1e-3, 600.0)},
            "f32": {"step_s": 2e-3, "step": lambda: advance(2e-3, 500.0)}}
    out = bench.energy_leg(fake_torch(), meter, runs, 1e9, seconds=1.0, preroll=0.5, reps=2)
    assert out["idle_W"] == pytest.approx(100.0, rel=1e-6)
    assert out["bf16"]["avg_W"] == pytest.approx(600.0, rel=1e-3)
    assert out["f32"]["avg_W"] == pytest.approx(500.0, rel=1e-3)
    # without the pre-roll the first bf16 window would straddle the idle second
    out0 = bench.energy_leg(fake_torch(), meter, runs, 1e9, seconds=1.0, preroll=0.0, reps=1)
    assert out0["bf16"]["avg_W"] < 560.0


def test_energy_leg_median_ignores_one_glitched_window(monkeypatch):
    """One window whose counter reading comes back halved does not move the
    reported energy: the median of three windows is taken."""
    clock = {"t": 0.0}
    smi = FakeSmi(["0000:75:00.0"], resolution=1.0)
    reads = {"n": 0}
    real = smi.amdsmi_get_energy_count

    def glitchy(h):
        reads["n"] += 1
        e = real(h)
        # the closing read of the second bf16 window (reads: 2 idle, then 2 per window, bf16 first)
        if reads["n"] == 2 + 2 * 2 + 2:
            e = dict(e, energy_accumulator=e["energy_accumulator"] - 300_000_000)   # half a window
        return e

    smi.amdsmi_get_energy_count = glitchy
    meter = bench.EnergyMeter(fake_torch(), smi=smi)

    def advance(seconds, watts):
        clock["t"] += seconds
        smi.acc[0] += int(round(watts * seconds * 1e6))

    monkeypatch.setattr(bench.time, "sleep", lambda s: advance(s, 100.0))
    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock["t"])
    runs = {"bf16": {"step_s": 1e-3, "step": lambda: advance(1e-3, 600.0)},
            "f32": {"step_s": 2e-3, "step": lambda: advance(2e-3, 500.0)}}
    out = bench.energy_leg(fake_torch(), meter, runs, 1e9, seconds=1.0, preroll=0.1, reps=3)
    each = out["bf16"]["J_per_1e12_bt_each"]
    assert min(each) < 0.9 * max(each)                         # the glitch is visible
    assert out["bf16"]["avg_W"] == pytest.approx(600.0, rel=1e-3)
    assert out["bf16"]["J_per_1e12_bt"] == pytest.approx(0.6 * 1e-3 / 1e9 * 1e12 * 1000, rel=1e-3)


def test_energy_leg_uses_the_counters_own_time_between_its_steps(monkeypatch):
    """A counter that advances only once per second (with its timestamp, as
    MI355X's does) makes a 2-second window see one, two or three steps; the
    power taken over the counter's own time between its steps is the true
    power in every window, and so is the energy per work."""
    clock = {"t": 0.0}
    true = {"acc": 0.0}
    smi = FakeSmi(["0000:75:00.0"], resolution=1.0)
    state = {"acc": 0.0, "ts": 0.0}

    def stepped(h):
        k = int(clock["t"])                      # the counter's last update, at a whole second
        if k > state["ts"]:
            # energy up to the update instant: the true accumulator then
            state["acc"], state["ts"] = energy_at(k), float(k)
        return {"energy_accumulator": int(round(state["acc"] * 1e6)), "counter_resolution": 1.0,
                "timestamp": int(state["ts"] * 1e9)}

    hist = [(0.0, 0.0)]

    def energy_at(t):
        # linear interpolation of the true accumulator at time t
        for (t0, a0), (t1, a1) in zip(hist, hist[1:]):
            if t0 <= t <= t1:
                return a0 + (a1 - a0) * (t - t0) / (t1 - t0) if t1 > t0 else a1
        return hist[-1][1]

    def advance(seconds, watts):
        clock["t"] += seconds
        true["acc"] += watts * seconds
        hist.append((clock["t"], true["acc"]))

    smi.amdsmi_get_energy_count = stepped
    meter = bench.EnergyMeter(fake_torch(), smi=smi)
    monkeypatch.setattr(bench.time, "sleep", lambda s: advance(s, 100.0))
    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock["t"])
    runs = {"bf16": {"step_s": 2e-3, "step": lambda: advance(2e-3, 600.0)},
            "f32": {"step_s": 3e-3, "step": lambda: advance(3e-3, 500.0)}}
    out = bench.energy_leg(fake_torch(), meter, runs, 1e9, seconds=2.0, preroll=3.0, reps=3)
    assert out["idle_W"] == pytest.approx(100.0, rel=1e-3)
    for name, w in (("bf16", 600.0), ("f32", 500.0)):
        each = out[name]["J_per_1e12_bt_each"]
        assert max(each) == pytest.approx(min(each), rel=1e-3), each
        assert out[name]["avg_W"] == pytest.approx(w, rel=1e-3)
    # J per 1e12 bt = W x step time / bt x 1e12
    assert out["bf16"]["J_per_1e12_bt"] == pytest.approx(600.0 * 2e-3 / 1e9 * 1e12, rel=1e-3)
