"""Continuous-batching service for relaxation jobs.

Requests (initial-data descriptions with lattice, spacing, mass, time step,
tolerance, step cap and precision) arrive over time.  The server admits a
request when a batch slot is free and its HBM footprint (three fields plus
the workspace) fits the budget; admitted fields stay resident on the device
and step together with every other active field, one shared launch per sweep
slot (skyr_batch_run).  A finished field leaves the batch at once and its
memory and slot go to the next request, while the others keep stepping.
The server records arrival, admission and completion times, from which it
reports p50/p99 time-to-convergence beside throughput.

The device work goes through a backend object (GpuBackend drives the C ABI;
tests substitute a host-only mock with the same methods).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field


@dataclass
class Request:
    desc: dict                     # workload description (n, h, m, dt, tol, steps, precision, init, ...)
    arrival: float = 0.0           # seconds after the stream starts
    rid: int = -1
    admitted: float | None = None
    finished: float | None = None
    slot: int = -1
    state: dict = field(default_factory=dict)
    result: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def service(self) -> float:
        return self.finished - self.admitted


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return math.nan
    k = max(0, min(len(v) - 1, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


class GpuBackend:
    """Device side of the server: allocation, initial data, the batch, observables."""

    def __init__(self, max_jobs: int, device="cuda:0"):
        import torch

        from . import skyr
        self.torch = torch
        self.skyr = skyr
        self.device = torch.device(device)
        self.batch = skyr.Batch(max_jobs)
        self.bufs = {}

    def _model(self, desc):
        """The request's model: the pion mass "m" and, optionally, "m_y", "m_z",
        "m_w" and the sextic weight "c6"."""
        return self.skyr.Model(desc["m"], desc.get("m_y", 0.0), desc.get("m_z", 0.0), desc.get("m_w", 0.0),
                               desc.get("c6", 0.0))

    @staticmethod
    def _prec(desc):
        from . import skyr
        return skyr.F32_BULK if desc.get("precision", "f64") == "f32" else skyr.F64

    def footprint(self, desc) -> int:
        s = self.skyr
        n = desc["n"]
        lat = s.Lattice.cube(n, desc["h"])
        prec = self._prec(desc)
        elem = 4 if prec == s.F32_BULK else 8
        _, pitch = s.batch_layout(lat, prec)
        return 3 * 4 * n * n * pitch * elem + s.workspace_bytes(lat, prec)

    def start(self, desc) -> int:
        """The request's fields in the padded-row layout of batch fields (the initial data
        made dense, then copied in), and its flow added to the batch."""
        s = self.skyr
        n, h = desc["n"], desc["h"]
        prec = self._prec(desc)
        lat = s.Lattice.cube(n, h)
        dense = s.new_field(lat, prec, self.device)
        spec, keep = s.spec_from_description(desc["init"])
        s.init_field(lat, prec, spec, dense)
        layout = s.batch_layout(lat, prec)
        phi = s.to_padded(dense, layout)
        del dense
        alt, vel = self.torch.zeros_like(phi), self.torch.zeros_like(phi)
        work = s.new_workspace(lat, prec, self.device)
        flow = s.Flow(desc["dt"], desc["tol"], int(desc["steps"]), int(desc.get("renorm64_every", 16)),
                      s.flow_mode(desc.get("flow", "energy")))
        slot = self.batch.add_padded(lat, prec, self._model(desc), flow, phi, alt, vel, work, layout)
        self.bufs[slot] = (lat, prec, desc, phi, alt, vel, work, layout)
        return slot

    def site(self, slot: int, A: int, x: int, y: int, z: int):
        """The stored element of component A at lattice site (x, y, z) of a slot's field
        (a view, for checks and tests)."""
        lat, prec, desc, phi, alt, vel, work, (lead, pitch) = self.bufs[slot]
        return phi[x, y, A, lead + z]

    def run(self, sweeps: int) -> None:
        self.batch.run(sweeps)

    def poll(self, slot: int) -> dict:
        st = self.batch.poll(slot)
        return {"steps": st.steps, "arrests": st.arrests, "sweeps": st.sweeps, "E": st.E,
                "max_force": st.max_force, "converged": bool(st.converged), "nonfinite": bool(st.nonfinite),
                "done": bool(st.converged or st.nonfinite or st.steps >= self.bufs[slot][2]["steps"])}

    def finish(self, slot: int, keep_field: bool = False) -> dict:
        s = self.skyr
        lat, prec, desc, phi, alt, vel, work, layout = self.bufs.pop(slot)
        self.batch.remove(slot)
        field = s.from_padded(phi, layout, lat.shape[2])
        out = s.observables(lat, prec, self._model(desc), field, work)
        if keep_field:
            out["field"] = field
        return out

    def close(self) -> None:
        self.batch.close()


class Server:
    """FIFO admission by slot and HBM footprint; continuous batching."""

    def __init__(self, backend, max_jobs: int, hbm_budget: int, sweeps_per_tick: int = 32,
                 keep_fields: bool = False, clock=time.perf_counter, progress=None):
        self.backend = backend
        self.max_jobs = int(max_jobs)
        self.hbm_budget = int(hbm_budget)
        self.sweeps_per_tick = int(sweeps_per_tick)
        self.keep_fields = keep_fields
        self.clock = clock
        self.queue: deque[Request] = deque()
        self.active: dict[int, Request] = {}
        self.done: list[Request] = []
        self.in_use = 0
        self.t0 = None
        self.ticks = 0
        self.site_updates = 0
        # algorithmic HBM bytes of the sweeps run (read phi and v, write phi' and v' at every
        # interior site: 64 B in single, 128 B in double precision), redo sweeps included
        self.sweep_bytes = 0
        self.progress = progress  # called with the server after each finished request

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> None:
        if self.backend.footprint(req.desc) > self.hbm_budget:
            raise ValueError(f"request {req.rid} needs more than the whole HBM budget")
        self.queue.append(req)

    def _admit(self) -> None:
        while self.queue and len(self.active) < self.max_jobs:
            req = self.queue[0]
            if req.arrival > self.now():
                break
            need = self.backend.footprint(req.desc)
            if self.in_use + need > self.hbm_budget:
                break  # FIFO: the head waits for memory
            self.queue.popleft()
            req.slot = self.backend.start(req.desc)
            req.admitted = self.now()
            self.in_use += need
            self.active[req.slot] = req

    def tick(self) -> None:
        self._admit()
        if self.active:
            before = {s: (r.state.get("steps", 0), r.state.get("sweeps", r.state.get("steps", 0)))
                      for s, r in self.active.items()}
            self.backend.run(self.sweeps_per_tick)
            t = self.now()
            for slot, req in list(self.active.items()):
                st = self.backend.poll(slot)
                req.state = st
                n = req.desc["n"] - 4
                self.site_updates += (st["steps"] - before[slot][0]) * n ** 3
                site_bytes = 128 if req.desc.get("precision") == "f64" else 64
                self.sweep_bytes += (st.get("sweeps", st["steps"]) - before[slot][1]) * n ** 3 * site_bytes
                if st["done"]:
                    req.result = self.backend.finish(slot, self.keep_fields)
                    req.finished = t
                    self.in_use -= self.backend.footprint(req.desc)
                    del self.active[slot]
                    self.done.append(req)
                    if self.progress is not None:
                        self.progress(self)
        self.ticks += 1

    def serve(self, requests, idle_sleep: float = 1e-3, max_seconds: float | None = None) -> dict:
        """Feed `requests` (sorted by arrival) in real time until all finish."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = self.clock()
        total = len(pending)
        while len(self.done) < total:
            while pending and pending[0].arrival <= self.now():
                self.submit(pending.popleft())
            if not self.active and not self.queue:
                if pending:
                    time.sleep(min(idle_sleep, max(0.0, pending[0].arrival - self.now())))
                continue
            self.tick()
            if max_seconds is not None and self.now() > max_seconds:
                break
        return self.report()

    def report(self) -> dict:
        lat = [r.latency for r in self.done]
        svc = [r.service for r in self.done]
        conv = [r.latency for r in self.done if r.state.get("converged")]
        wall = self.now() if self.t0 is not None else math.nan
        return {
            "jobs": len(self.done),
            "wall_s": wall,
            "jobs_per_s": len(self.done) / wall if wall and wall > 0 else math.nan,
            "site_updates_per_s": self.site_updates / wall if wall and wall > 0 else math.nan,
            "sweep_GBs": self.sweep_bytes / wall / 1e9 if wall and wall > 0 else math.nan,
            "latency_p50_s": percentile(lat, 50), "latency_p99_s": percentile(lat, 99),
            "service_p50_s": percentile(svc, 50), "service_p99_s": percentile(svc, 99),
            "converged_latency_p50_s": percentile(conv, 50), "converged_latency_p99_s": percentile(conv, 99),
            "converged": sum(1 for r in self.done if r.state.get("converged")),
            "capped": sum(1 for r in self.done if not r.state.get("converged") and not r.state.get("nonfinite")),
            "nonfinite": sum(1 for r in self.done if r.state.get("nonfinite")),
            "ticks": self.ticks,
            "at_cap_fraction": (sum(1 for r in self.done if not r.state.get("converged")
                                    and not r.state.get("nonfinite")) / len(self.done)) if self.done else math.nan,
        }
