"""Host-side checks of the serving loop's scheduling (no GPU): a mock backend
with the device interface finishes each job after a known number of sweeps."""
import math

import pytest

from paper_2604_25876_amd.serve import Request, Server, percentile


class MockBackend:
    def __init__(self, max_jobs):
        self.max_jobs = max_jobs
        self.slots = {}
        self.free = list(range(max_jobs))
        self.log = []

    def footprint(self, desc):
        return desc["n"] ** 3

    def start(self, desc):
        slot = self.free.pop(0)
        self.slots[slot] = {"desc": desc, "sweeps": 0}
        self.log.append(("start", desc["name"], slot))
        return slot

    def run(self, sweeps):
        for s in self.slots.values():
            s["sweeps"] += sweeps

    def poll(self, slot):
        s = self.slots[slot]
        need = s["desc"]["need"]
        steps = min(s["sweeps"], need)
        return {"steps": steps, "done": s["sweeps"] >= need, "converged": s["sweeps"] >= need, "nonfinite": False}

    def finish(self, slot, keep_field=False):
        s = self.slots.pop(slot)
        self.free.append(slot)
        self.log.append(("finish", s["desc"]["name"], slot))
        return {"E": float(s["desc"]["need"])}


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t


def make(name, n, need, arrival=0.0):
    return Request({"name": name, "n": n, "need": need, "steps": 10 ** 6}, arrival=arrival)


def test_all_jobs_finish_and_budget_holds():
    be = MockBackend(4)
    srv = Server(be, max_jobs=4, hbm_budget=3 * 20 ** 3, sweeps_per_tick=8, clock=FakeClock())
    reqs = [make(f"j{i}", 20 if i % 2 else 10, need=8 * (1 + i % 5)) for i in range(17)]
    peak = 0
    orig_tick = srv.tick

    def tick():
        nonlocal peak
        orig_tick()
        peak = max(peak, srv.in_use)
        assert len(srv.active) <= 4

    srv.tick = tick
    rep = srv.serve(reqs)
    assert rep["jobs"] == 17 and rep["converged"] == 17
    assert peak <= 3 * 20 ** 3
    assert srv.in_use == 0 and not srv.active
    # FIFO: jobs start in submission order
    starts = [name for kind, name, _ in be.log if kind == "start"]
    assert starts == [f"j{i}" for i in range(17)]


def test_continuous_batching_reuses_slots_while_others_run():
    be = MockBackend(2)
    srv = Server(be, max_jobs=2, hbm_budget=10 ** 9, sweeps_per_tick=4, clock=FakeClock())
    reqs = [make("long", 10, 40), make("short1", 10, 4), make("short2", 10, 4), make("short3", 10, 4)]
    srv.serve(reqs)
    order = [(k, n) for k, n, _ in be.log]
    # the short jobs come and go while the long one keeps its slot
    assert order.index(("finish", "long")) > order.index(("start", "short3"))
    assert all(r.result["E"] == r.desc["need"] for r in srv.done)


def test_oversized_request_is_rejected():
    be = MockBackend(2)
    srv = Server(be, max_jobs=2, hbm_budget=10 ** 3, clock=FakeClock())
    with pytest.raises(ValueError):
        srv.submit(make("big", 20, 4))


def test_latencies_and_percentiles():
    assert percentile([3, 1, 2, 4], 50) == 2
    assert percentile([3, 1, 2, 4], 99) == 4
    assert math.isnan(percentile([], 50))
    be = MockBackend(1)
    srv = Server(be, max_jobs=1, hbm_budget=10 ** 9, sweeps_per_tick=4, clock=FakeClock())
    rep = srv.serve([make("a", 10, 4), make("b", 10, 4)])
    a, b = srv.done
    assert a.admitted <= b.admitted and b.latency >= b.service > 0
    assert rep["latency_p99_s"] >= rep["latency_p50_s"] > 0


def test_site_updates_and_sweep_bytes_are_counted_per_job():
    """The report's throughput counts every job's accepted steps over its interior sites,
    and its algorithmic bytes every sweep at 64 B (single) or 128 B (double) per interior
    site; the mock's sweeps are all accepted steps."""
    be = MockBackend(2)
    srv = Server(be, max_jobs=2, hbm_budget=10 ** 9, sweeps_per_tick=4, clock=FakeClock())
    reqs = [make("a", 10, 8), make("b", 14, 12)]
    reqs[1].desc["precision"] = "f64"
    rep = srv.serve(reqs)
    assert srv.site_updates == 8 * 6 ** 3 + 12 * 10 ** 3
    assert srv.sweep_bytes == 8 * 6 ** 3 * 64 + 12 * 10 ** 3 * 128
    assert rep["sweep_GBs"] == pytest.approx(srv.sweep_bytes / rep["wall_s"] / 1e9)
