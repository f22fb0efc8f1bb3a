"""Throughput of the arrested Newton flow on one MI355X.

Workload: the 256^3 lattice (h = 0.1, m = 1) holding the product ansatz of
10 unit charges at seeded random centres in a radius-3 ball with Haar-random
isorotations (seed 1), profile f = pi exp(-r); time step dt = 0.01.  One
"step" is one accepted arrested-Newton-flow step over the whole lattice: the
fused sweep (derivatives, energy, exact gradient, projection, kick-drift,
renormalisation, FP64 partial sums) plus the device-side arrest decision.

The JSON line reports the FP32-bulk flow as `value` (site-updates/s, one
site-update = one interior site advanced by one accepted step) and the plain
FP64 flow beside it, the roofline of the sweep kernel (HBM bytes per site from
the algorithm, kernel time from HIP events around each sweep launch), and the
FP64 CPU oracle timed on a bounded sample on the host cores.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "site-updates/s FP32-bulk vs FP64 flow at 256³; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per interior site and sweep: read phi and v, write phi' and v'
BYTES_PER_SITE = {"f32": 4 * 4 * 4, "f64": 4 * 4 * 8}


def kernel_source_hash() -> str:
    """sha256 over the sources the sweep kernel is built from: its code and the list of
    compiled tile shapes (the host runtime around it does not change what it does)."""
    import hashlib
    hsh = hashlib.sha256()
    for f in ("sweep.hpp", "shapes.hpp"):
        with open(os.path.join(ROOT, "paper_2604_25876_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def _summary(name):
    """`key: value` lines of a committed profile summary, or None."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as fh:
            kv = dict(line.split(":", 1) for line in fh.read().splitlines()
                      if ":" in line and not line.startswith(("#", "|", "`", " ")))
    except OSError:
        return None
    return {k.strip(): v.strip() for k, v in kv.items()}


def recorded_traffic(prec_name, tile):
    """HBM bytes per sweep launch from the committed counter summary, or None.

    The summary holds `key: value` lines (FETCH_SIZE and WRITE_SIZE in KiB per
    dispatch per tile `<prec>_<variant>_<planes per slab>_...`, the scale factors a
    plain copy of known size gives for each counter and the kernel-source hash the
    counters were taken with).  Counters taken on other kernel sources or for another
    tile do not describe this launch and give None."""
    kv = _summary("sweep_traffic_random-b10-256.md")
    if not kv:
        return None
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    key = f"{prec_name}_{tile[0]}_{tile[1]}"
    try:
        fetch = float(kv[f"{key}_fetch_kib"]) * float(kv["fetch_scale"])
        write = float(kv[f"{key}_write_kib"]) * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return 1024.0 * (fetch + write)


# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 vector instruction per
# SIMD every 4 cycles (16 lanes per SIMD), in wave-instructions per second
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def recorded_valu(prec_name, tile):
    """VALU wave-instructions per sweep launch (SQ_INSTS_VALU) from the committed
    counter summary, or None when the kernel sources or the tile differ."""
    kv = _summary("sweep_instructions_random-b10-256.md")
    if not kv or kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv[f"{prec_name}_{tile[0]}_{tile[1]}_valu_per_launch"])
    except (KeyError, ValueError):
        return None


def valu_roofline(prec_name, tile, kernel_avg_s):
    """The sweep against the VALU issue rate: recorded instructions per launch
    over the live kernel time, as a fraction of the issue peak."""
    inst = recorded_valu(prec_name, tile)
    if inst is None:
        return None
    rate = inst / kernel_avg_s
    return {"bound": "alu", "achieved": rate / 1e9, "peak": VALU_ISSUE_PEAK / 1e9, "unit": "G wave-instructions/s",
            "frac": rate / VALU_ISSUE_PEAK, "valu_per_launch": inst}


def run_flow(skyr, torch, w, prec_name, steps, warmup, tile=None, masses=None, mode=None, form=0):
    """Time `steps` accepted flow steps of the workload after `warmup`.  The
    FP32-bulk flow uses the power arrest rule (its recommended setting), the
    FP64 flow the paper's energy rule; `masses` (m, m_y, m_z, m_w, c6) and
    `mode` override the workload's model and flow mode; form 1 takes the
    printed-form force."""
    prec = skyr.F32_BULK if prec_name == "f32" else skyr.F64
    n, h = w["n"], w["h"]
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description(w["init"])
    dev = torch.device("cuda:0")
    phi = skyr.new_field(lat, prec, dev)
    skyr.init_field(lat, prec, spec, phi)
    alt, vel = skyr.new_field(lat, prec, dev), skyr.new_field(lat, prec, dev)
    work = skyr.new_workspace(lat, prec, dev)
    model = skyr.Model(*(masses or (w["m"],)))
    model.form = form
    # tolerance 0: every call runs exactly its steps
    rule = mode or ("power" if prec_name == "f32" else "energy")
    flow = skyr.Flow(w["dt"], 0.0, 10 ** 12, 16, skyr.flow_mode(rule))
    # tile shape for this lattice and precision: measured once, before the timed region
    if tile is None:
        tile = skyr.autotune_cached(lat, prec, model, flow, phi, alt, vel, work)
    else:
        skyr.set_tile(lat, prec, *tile)
    st = skyr.anf_state()
    skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st, warmup, work)
    torch.cuda.synchronize()
    s0, sw0, ar0 = st.steps, st.sweeps, st.arrests
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    # the timed region: the flow as it runs in production (sweeps replayed from graphs)
    t0 = time.perf_counter()
    ev0.record()
    skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st, steps, work)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    done = st.steps - s0
    sweeps = st.sweeps - sw0
    arrests = st.arrests - ar0
    interior = (n - 4) ** 3
    elapsed = ev0.elapsed_time(ev1) / 1e3
    # the sweep kernel's own time: the same flow continued with a HIP event pair around every
    # sweep launch on the flow's stream (the launches are then direct, not from a graph)
    k_steps = max(1, min(steps, 200))
    skyr.timing_enable(True)
    skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st, k_steps, work)
    torch.cuda.synchronize()
    sweep_ms, sweep_n = skyr.timing_read()
    skyr.timing_enable(False)
    kernel_avg_s = sweep_ms / 1e3 / max(sweep_n, 1)
    bytes_launch = BYTES_PER_SITE[prec_name] * interior
    achieved = bytes_launch / kernel_avg_s / 1e9
    obs = skyr.observables(lat, prec, model, phi, work)
    return dict(
        prec=prec_name, steps=done, sweeps=sweeps, arrests=arrests, wall_s=wall,
        elapsed_s=elapsed, site_updates_per_s=done * interior / elapsed, ms_per_step=1e3 * elapsed / max(done, 1),
        ms_per_sweep=1e3 * elapsed / max(sweeps, 1),
        sweep_kernel_avg_us=kernel_avg_s * 1e6, sweep_launches=sweep_n, bytes_per_launch=bytes_launch,
        achieved_GBs=achieved, E=obs["E"], B=obs["B"], max_force=obs["max_force"],
        arrest=rule, tile={"variant": tile[0], "shape": skyr.tile_variants(prec)[tile[0]], "xchunk": tile[1]},
        traffic=recorded_traffic(prec_name, tile), valu=valu_roofline(prec_name, tile, kernel_avg_s))


def hedgehog_40_smoke(skyr, torch):
    """The hedgehog-40 configuration as specified (FP64, dt = 0.1, 300 arrested steps from
    the B = 1 hedgehog on 40^3 at h = 0.2): the arrests it takes, where its energy goes and
    the wall time of the 300 steps."""
    from skyr_inputs import HEDGEHOG_40 as w
    lat = skyr.Lattice.cube(w["n"], w["h"])
    spec, keep = skyr.spec_from_description(w["init"])
    dev = torch.device("cuda:0")
    phi = skyr.new_field(lat, skyr.F64, dev)
    skyr.init_field(lat, skyr.F64, spec, phi)
    alt, vel = skyr.new_field(lat, skyr.F64, dev), skyr.new_field(lat, skyr.F64, dev)
    work = skyr.new_workspace(lat, skyr.F64, dev)
    E0 = skyr.observables(lat, skyr.F64, skyr.Model(w["m"]), phi, work)["E"]
    flow = skyr.Flow(w["dt"], w["tol"], w["steps"], 0, skyr.flow_mode("energy"))
    st = skyr.anf_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    skyr.anf_step(lat, skyr.F64, skyr.Model(w["m"]), flow, phi, alt, vel, st, w["steps"], work)
    wall = time.perf_counter() - t0
    obs = skyr.observables(lat, skyr.F64, skyr.Model(w["m"]), phi, work)
    return {"workload": w["name"], "dt": w["dt"], "steps": st.steps, "arrests": st.arrests, "sweeps": st.sweeps,
            "E_start": E0, "E_end": obs["E"], "B_end": obs["B"], "max_force_end": obs["max_force"], "wall_s": wall}


def paper_size_layouts(skyr, torch, prec_name, steps=200, warmup=20):
    """The paper's own workload size (the O_h B = 4 cube on 151^3 at h = 0.107, dt = 0.1 h),
    whose 151-site rows are not whole 128-byte lines: the flow (tolerance 0, default tiles)
    on the dense field and on its padded, row-interleaved copy; site-updates/s of each."""
    from skyr_inputs import CUBE_B4_128
    prec = skyr.F32_BULK if prec_name == "f32" else skyr.F64
    n, h = 151, 0.107
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description(CUBE_B4_128["init"])
    dev = torch.device("cuda:0")
    phi = skyr.new_field(lat, prec, dev)
    skyr.init_field(lat, prec, spec, phi)
    layout = skyr.batch_layout(lat, prec)
    pphi = skyr.to_padded(phi, layout)
    work = skyr.new_workspace(lat, prec, dev)
    model = skyr.Model(1.0)
    flow = skyr.Flow(0.1 * h, 0.0, 10 ** 12, 16, skyr.flow_mode("power" if prec_name == "f32" else "energy"))
    out = {"workload": "cube-b4 at 151^3, h = 0.107", "layout": {"lead": layout[0], "pitch": layout[1]}}
    for name, f, run in (("dense", phi, skyr.anf_step), ("padded", pphi, skyr.anf_step_padded)):
        alt, vel = torch.zeros_like(f), torch.zeros_like(f)
        extra = (layout,) if name == "padded" else ()
        st = skyr.anf_state()
        run(lat, prec, model, flow, f, alt, vel, st, warmup, work, *extra)
        torch.cuda.synchronize()
        s0 = st.steps
        t0 = time.perf_counter()
        run(lat, prec, model, flow, f, alt, vel, st, steps, work, *extra)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[name] = {"site_updates_per_s": (st.steps - s0) * (n - 4) ** 3 / t, "ms_per_step": 1e3 * t / (st.steps - s0)}
    out["speedup"] = out["padded"]["site_updates_per_s"] / out["dense"]["site_updates_per_s"]
    return out


def block_share(skyr, torch, w, prec_name, reps=50):
    """One device's share of the workload's lattice split 2 x 2 x 2: the step sweep over the
    128^3 block at (128, 0, 128), its four-deep shell written from a separate buffer (what
    the neighbouring devices would send), timed with HIP events around the sweep launches
    (the shell fill is reported beside it)."""
    prec = skyr.F32_BULK if prec_name == "f32" else skyr.F64
    n, h = w["n"], w["h"]
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description(w["init"])
    dev = torch.device("cuda:0")
    full = skyr.new_field(lat, prec, dev)
    skyr.init_field(lat, prec, spec, full)
    origin, extent = (n // 2, 0, n // 2), (n // 2,) * 3
    blk = skyr.Block.of(lat, origin, extent)
    idx = [torch.clamp(torch.arange(e + 8, device=dev) + o - 4, 0, n - 1) for o, e in zip(origin, extent)]
    padded = full[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]].contiguous()
    own = torch.zeros(padded.shape[1:], dtype=torch.bool, device=dev)
    own[4:-4, 4:-4, 4:-4] = True
    shell = padded[:, ~own].contiguous()
    work = skyr.new_block_workspace(blk, prec, dev)

    def timed(phi, layout):
        out, vel = torch.zeros_like(phi), torch.zeros_like(phi)
        for _ in range(3):
            skyr.block_sweep(blk, prec, skyr.Model(w["m"]), skyr.BLOCK_STEP, phi, shell, out, vel=vel, work=work,
                             dt=w["dt"], want_sums=False, layout=layout)
        torch.cuda.synchronize()
        skyr.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            skyr.block_sweep(blk, prec, skyr.Model(w["m"]), skyr.BLOCK_STEP, phi, shell, out, vel=vel, work=work,
                             dt=w["dt"], want_sums=False, layout=layout)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms, cnt = skyr.timing_read()
        skyr.timing_enable(False)
        return 1e3 * ms / max(cnt, 1), 1e6 * wall / reps

    us, call_us = timed(padded, None)
    # the same block in padded, row-interleaved rows (skyr_block_sweep_padded)
    layout = skyr.block_layout(blk, prec)
    us_p, call_us_p = timed(skyr.to_padded(padded, layout), layout)
    # the block's own sites in I, per axis the overlap of [origin, origin + extent) with [2, n - 2)
    sites = 1
    for o, e in zip(origin, extent):
        sites *= max(0, min(o + e, n - 2) - max(o, 2))
    eb = 4 if prec_name == "f32" else 8
    return {"block": {"origin": list(origin), "extent": list(extent)}, "interior_sites": sites,
            "sweep_kernel_avg_us": us, "achieved_GBs": 16 * eb * sites / us / 1e3,
            "call_us": call_us, "site_updates_per_s": sites / (us / 1e6),
            "padded_rows": {"layout": {"lead": layout[0], "pitch": layout[1]}, "sweep_kernel_avg_us": us_p,
                            "call_us": call_us_p, "site_updates_per_s": sites / (us_p / 1e6)}}


def time_moments(skyr, torch, w, prec_name, reps=5):
    """Wall time of skyr_moments (an observables sweep, then the two FP64
    moment passes; each call synchronises) on the workload's initial field."""
    prec = skyr.F32_BULK if prec_name == "f32" else skyr.F64
    lat = skyr.Lattice.cube(w["n"], w["h"])
    spec, keep = skyr.spec_from_description(w["init"])
    dev = torch.device("cuda:0")
    phi = skyr.new_field(lat, prec, dev)
    skyr.init_field(lat, prec, spec, phi)
    work = skyr.new_workspace(lat, prec, dev)
    model = skyr.Model(w["m"])
    res = skyr.moments(lat, prec, model, phi, work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = skyr.moments(lat, prec, model, phi, work)
    ms = 1e3 * (time.perf_counter() - t0) / reps
    interior = (w["n"] - 4) ** 3
    return {"ms_per_call": ms, "interior_sites_per_s": interior / (ms / 1e3), "B": res["B"], "R": res["R"]}


def sweep_tiles(skyr, torch, w, prec_name, steps=20):
    """Time every compiled shape and slab length on the workload (flow steps
    from the initial field); one line per candidate."""
    prec = skyr.F32_BULK if prec_name == "f32" else skyr.F64
    n, h = w["n"], w["h"]
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description(w["init"])
    dev = torch.device("cuda:0")
    phi0 = skyr.new_field(lat, prec, dev)
    skyr.init_field(lat, prec, spec, phi0)
    phi, alt, vel = phi0.clone(), skyr.new_field(lat, prec, dev), skyr.new_field(lat, prec, dev)
    work = skyr.new_workspace(lat, prec, dev)
    model = skyr.Model(w["m"])
    flow = skyr.Flow(w["dt"], 0.0, 10 ** 12, 16, 0)
    rows = []
    nx = n - 4
    chunks = sorted({max(16, -(-nx // s)) for s in range(1, 13)}, reverse=True)
    for v, shape in enumerate(skyr.tile_variants(prec)):
        for xc in chunks:
            skyr.set_tile(lat, prec, v, xc)
            phi.copy_(phi0)
            vel.zero_()
            st = skyr.anf_state()
            skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st, 2, work)
            skyr.timing_enable(True)
            skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st, steps, work)
            ms, cnt = skyr.timing_read()
            skyr.timing_enable(False)
            us = 1e3 * ms / max(cnt, 1)
            rows.append({"prec": prec_name, "shape": shape, "xchunk": xc, "sweep_us": us,
                         "GBs": BYTES_PER_SITE[prec_name] * (n - 4) ** 3 / us / 1e3})
            print(json.dumps(rows[-1]), flush=True)
    return rows


def _job_buffers(skyr, torch, d):
    prec = skyr.F32_BULK if d["precision"] == "f32" else skyr.F64
    lat = skyr.Lattice.cube(d["n"], d["h"])
    dev = torch.device("cuda:0")
    phi = skyr.new_field(lat, prec, dev)
    spec, keep = skyr.spec_from_description(d["init"])
    skyr.init_field(lat, prec, spec, phi)
    alt, vel = skyr.new_field(lat, prec, dev), skyr.new_field(lat, prec, dev)
    work = skyr.new_workspace(lat, prec, dev)
    flow = skyr.Flow(d["dt"], 0.0, 10 ** 12, 16, skyr.flow_mode(d.get("flow", "energy")))
    return lat, prec, phi, alt, vel, work, flow


def tune_batch_tiles(skyr, torch, jobs):
    """The batch tile of every (lattice, precision) of `jobs`, by the batch autotuner
    on copies of the lattice's first job (before any timed region)."""
    tiles = {}
    for d in jobs:
        prec = skyr.F32_BULK if d["precision"] == "f32" else skyr.F64
        key = (d["n"], d["h"], prec)
        if key in tiles:
            continue
        lat, prec, phi, alt, vel, work, flow = _job_buffers(skyr, torch, d)
        v, xc, us = skyr.batch_autotune(lat, prec, skyr.Model(d["m"]), flow, phi)
        tiles[key] = {"n": d["n"], "precision": d["precision"], "variant": v, "xchunk": xc,
                      "us_per_slot": round(us, 1), "copies": skyr.batch_copies(lat, prec)}
        del phi, alt, vel, work
    return list(tiles.values())


def batch_throughput(skyr, torch, jobs, sweeps=64):
    """The same jobs stepped `sweeps` times (a) together in one batch (one
    launch per precision and tile shape and sweep slot, replayed from a captured
    graph; the fields in the padded rows of batch fields; the batch tiles set by
    the batch autotuner first) and (b) one at a time through skyr_anf_step;
    site-updates/s of each."""
    tiles = tune_batch_tiles(skyr, torch, jobs)
    bufs = [_job_buffers(skyr, torch, d) for d in jobs]
    with skyr.Batch(len(jobs)) as b:
        slots = []
        for d, (lat, prec, phi, alt, vel, work, flow) in zip(jobs, bufs):
            # the fields in the padded rows of batch fields
            layout = skyr.batch_layout(lat, prec)
            p = skyr.to_padded(phi, layout)
            slots.append(b.add_padded(lat, prec, skyr.Model(d["m"]), flow, p, torch.zeros_like(p),
                                      torch.zeros_like(p), work, layout))
        b.run(sweeps)  # warm-up: the graph of `sweeps` slots is captured here
        steps0 = [b.poll(s).steps for s in slots]
        sweeps0 = [b.poll(s).sweeps for s in slots]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(sweeps)
        t_batch = time.perf_counter() - t0
        upd_b = sum((b.poll(s).steps - s0) * (d["n"] - 4) ** 3 for s, s0, d in zip(slots, steps0, jobs))
        bytes_b = sum((b.poll(s).sweeps - s0) * (d["n"] - 4) ** 3 * BYTES_PER_SITE[d["precision"]]
                      for s, s0, d in zip(slots, sweeps0, jobs))
    bufs = [_job_buffers(skyr, torch, d) for d in jobs]
    for d, (lat, prec, phi, alt, vel, work, flow) in zip(jobs, bufs):
        skyr.anf_step(lat, prec, skyr.Model(d["m"]), flow, phi, alt, vel, skyr.anf_state(), 8, work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_s = 0
    for d, (lat, prec, phi, alt, vel, work, flow) in zip(jobs, bufs):
        st = skyr.anf_state()
        skyr.anf_step(lat, prec, skyr.Model(d["m"]), flow, phi, alt, vel, st, sweeps, work)
        steps_s += st.steps * (d["n"] - 4) ** 3
    t_seq = time.perf_counter() - t0
    return {"jobs": len(jobs), "sweeps": sweeps, "batched_site_updates_per_s": upd_b / t_batch,
            "sequential_site_updates_per_s": steps_s / t_seq, "batched_s": t_batch, "sequential_s": t_seq,
            "speedup": (upd_b / t_batch) / (steps_s / t_seq), "batch_tiles": tiles,
            "roofline": hbm_roofline(bytes_b / t_batch / 1e9)}


def copy_bandwidth(torch, gib=1, reps=5):
    """Attainable HBM bandwidth on this device: a device-to-device copy of `gib` GiB (read
    plus write, the sweep's own 1:1 mix), timed with events on the current stream; the
    median of `reps` copies after two untimed ones, in GB/s."""
    src = torch.ones(gib * 2 ** 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * gib * 2 ** 30 / sorted(ts)[reps // 2] / 1e9


def hbm_roofline(gbs):
    """Algorithmic bytes per second of a batched or served run (every sweep: read phi and
    v, write phi' and v' at each interior site) against the HBM peak."""
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


# mean accepted steps of a request of the served stream (measured over its first 128
# requests: 13,460, the requests stopped at the step cap included), used only to set the
# arrival rate
SERVE_STEPS_EST = 13500


def served_stream(skyr, torch, count=128, cap=20000, rate=None, bandwidth=None, sweeps_per_tick=32):
    """The served workload (Poisson arrivals, jobs of mixed size and precision).
    The arrival rate is 1.2 x the estimated service capacity, unless given: the batched
    algorithmic bandwidth (bytes/s) over the mean bytes of a request, SERVE_STEPS_EST
    sweeps of its interior sites at 64 B (FP32-bulk) or 128 B (FP64) each."""
    from paper_2604_25876_amd.serve import GpuBackend, Request, Server
    from skyr_inputs import served_stream as stream
    probe = stream(5, count, 1.0)
    mean_bytes = sum((d["n"] - 4) ** 3 * BYTES_PER_SITE[d["precision"]] for d in probe) / len(probe)
    capacity = None
    if rate is None:
        capacity = (bandwidth or 3e12) / (mean_bytes * SERVE_STEPS_EST)
        rate = 1.2 * capacity
    reqs = []
    for i, d in enumerate(stream(5, count, rate)):
        d = dict(d, steps=cap)
        reqs.append(Request(d, arrival=d["arrival"], rid=i))
    free, total = torch.cuda.mem_get_info()
    be = GpuBackend(max_jobs=32)

    def progress(srv):
        if len(srv.done) % 16 == 0 or len(srv.done) == count:
            print(f"# served {len(srv.done)}/{count} at {srv.now():.1f} s", file=sys.stderr, flush=True)

    srv = Server(be, max_jobs=32, hbm_budget=int(0.8 * free), sweeps_per_tick=sweeps_per_tick, progress=progress)
    rep = srv.serve(reqs)
    be.close()
    rep.update({"rate_per_s": rate, "capacity_est_jobs_per_s": capacity, "step_cap": cap,
                "tol": "1e-4 (FP64, energy arrest rule); max(1e-4, 2 x FP32 force floor) (FP32-bulk, power rule)",
                "roofline": hbm_roofline(rep["sweep_GBs"])})
    return rep


def host_cpu() -> dict:
    """The host's CPU model, sockets and logical CPUs (from /proc/cpuinfo)."""
    model, sockets, logical = None, set(), 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    logical += 1
                elif k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    sockets.add(v)
    except OSError:
        pass
    return {"model": model, "sockets": len(sockets) or None, "logical_cpus": logical or os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def _oracle_rate(oracle, np, phi, h, m, dt, budget_s, max_steps):
    """site-updates/s of the oracle's flow on phi: one untimed step, then as many steps as
    fit the budget (at least one); returns (rate, steps, seconds)."""
    vel = np.zeros_like(phi)
    st = oracle.AnfState.fresh()
    t0 = time.perf_counter()
    phi, vel, st, _, _ = oracle.anf(phi, vel, h, m, dt, 0.0, 1, st)
    t1 = time.perf_counter() - t0
    k = max(1, min(max_steps, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    phi, vel, st, _, _ = oracle.anf(phi, vel, h, m, dt, 0.0, 1 + k, st)
    tk = time.perf_counter() - t0
    interior = np.prod([s - 4 for s in phi.shape[1:]])
    return k * interior / tk, k, tk


def cpu_baseline(w, budget_s=12.0):
    """The FP64 oracle (as it stands) on the host: flow steps of the same 256^3 initial
    field with all its threads (the reported value), and of the cube-b4-128 input with all
    threads and with one; site-updates/s each."""
    import math

    import numpy as np

    import oracle
    n, h = w["n"], w["h"]
    init = w["init"]
    cs = oracle.random_constituents(init["seed"], init["B"], init["radius"], math.pi, init["prof_lambda"])
    phi = oracle.init_product((n, n, n), h, cs)
    threads = oracle.num_threads()
    rate, k, tk = _oracle_rate(oracle, np, phi, h, w["m"], w["dt"], budget_s, 20)
    from skyr_inputs import CUBE_B4_128 as c2
    phi2 = oracle.init_product((c2["n"],) * 3, c2["h"],
                               [oracle.cube_b4(prof_a=math.pi, prof_lambda=c2["init"]["prof_lambda"])])
    rate2, k2, tk2 = _oracle_rate(oracle, np, phi2, c2["h"], c2["m"], c2["dt"], 4.0, 50)
    # one thread, on the smaller field (the same work per site)
    oracle.set_num_threads(1)
    try:
        rate1, k1, tk1 = _oracle_rate(oracle, np, phi2, c2["h"], c2["m"], c2["dt"], 4.0, 4)
    finally:
        oracle.set_num_threads(threads)
    return {"value": rate, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} FP64 flow steps of the same {n}^3 random B=10 field after 1 untimed step "
                      f"({tk:.1f} s, {threads} threads)",
            "host": host_cpu(),
            "one_thread": {"value": rate1, "sample": f"{k1} FP64 flow steps of the cube-b4-128 field "
                                                     f"({tk1:.1f} s, 1 thread)"},
            "cube_b4_128": {"value": rate2, "sample": f"{k2} FP64 flow steps of the cube-b4-128 field "
                                                      f"({tk2:.1f} s, {threads} threads)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=64,
                    help="untimed steps before the timed region (64 also instantiate the flow's graph)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["f32", "f64"], default=None,
                    help="time one precision only (profiling runs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched and served workloads")
    ap.add_argument("--serve-jobs", type=int, default=128)
    ap.add_argument("--served-only", action="store_true",
                    help="run only the batched and served workloads and print the served record (profiling runs)")
    ap.add_argument("--sweep-tiles", action="store_true",
                    help="print the sweep time of every compiled tile shape and x-chunk, then exit")
    ap.add_argument("--batch-probe", action="store_true",
                    help="run 24 sweep slots of the 64-job batch (for counter runs of the batched kernel) and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="instead of the flow, copy a 1 GiB device buffer 5 times (reference for the HBM "
                         "byte counters: 1 GiB read + 1 GiB written per copy)")
    ap.add_argument("--tile-f32", default=None, metavar="V:X",
                    help="use tile variant V with X-plane slabs for the FP32 flow instead of the autotuner")
    ap.add_argument("--tile-f64", default=None, metavar="V:X", help="the same for the FP64 flow")
    args = ap.parse_args()
    tiles = {p: (tuple(int(t) for t in v.split(":")) if v else None)
             for p, v in (("f32", args.tile_f32), ("f64", args.tile_f64))}
    if args.batch_probe:
        # the 64-job mix on padded, row-interleaved fields with the default batch tiles: 24
        # sweep slots, for counter runs of the batched kernel
        import torch
        from paper_2604_25876_amd import skyr
        from skyr_inputs import batch_jobs
        skyr.lib()
        jobs = batch_jobs(4, 64)
        bufs = [_job_buffers(skyr, torch, d) for d in jobs]
        with skyr.Batch(len(jobs)) as b:
            for d, (lat, prec, phi, alt, vel, work, flow) in zip(jobs, bufs):
                layout = skyr.batch_layout(lat, prec)
                p = skyr.to_padded(phi, layout)
                b.add_padded(lat, prec, skyr.Model(d["m"]), flow, p, torch.zeros_like(p), torch.zeros_like(p), work,
                             layout)
            for _ in range(3):
                b.run(8)
        tiles = {n: skyr.get_batch_tile(skyr.Lattice.cube(n, 0.15), skyr.F32_BULK) for n in (48, 64, 96, 128)}
        print(json.dumps({"batch_probe_slots": 24, "algorithmic_bytes_per_slot":
                          sum((d["n"] - 4) ** 3 * BYTES_PER_SITE[d["precision"]] for d in jobs),
                          "tiles": {str(k): v for k, v in tiles.items()}}))
        return
    if args.copy_probe:
        import torch
        src = torch.ones(2 ** 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 2 ** 30, "copies": 5}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the flow of one lattice is not sharded across GPUs here "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_25876_amd import skyr
    from skyr_inputs import RANDOM_B10_256 as W

    skyr.lib()
    if args.served_only:
        from skyr_inputs import batch_jobs
        batch = batch_throughput(skyr, torch, batch_jobs(4, 64))
        serve = served_stream(skyr, torch, count=args.serve_jobs, bandwidth=batch["roofline"]["achieved"] * 1e9)
        print(json.dumps({"batched_64_jobs": batch, "served": serve}), flush=True)
        return
    if args.sweep_tiles:
        for p in ([args.only] if args.only else ["f32", "f64"]):
            sweep_tiles(skyr, torch, W, p)
        return
    if args.only:
        r = run_flow(skyr, torch, W, args.only, args.steps, args.warmup, tiles[args.only])
        print(json.dumps(r), flush=True)
        return
    r32 = run_flow(skyr, torch, W, "f32", args.steps, args.warmup, tiles["f32"])
    print(f"# f32-bulk: {r32}", file=sys.stderr, flush=True)
    r64 = run_flow(skyr, torch, W, "f64", args.steps, args.warmup, tiles["f64"])
    copy_gbs = copy_bandwidth(torch)
    print(f"# attainable (copy) bandwidth: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    print(f"# f64: {r64}", file=sys.stderr, flush=True)
    # the kernel variants with the program's other potentials, and with the sextic term too (Sec. 7.7), FP32-bulk
    pot_model = (W["m"], 0.5, 0.5, 0.5)
    rpot = run_flow(skyr, torch, W, "f32", max(args.steps // 5, 20), args.warmup, tiles["f32"], masses=pot_model)
    print(f"# f32-bulk, four potentials: {rpot}", file=sys.stderr, flush=True)
    ext_model = (W["m"], 0.5, 0.5, 0.5, 0.1)
    rext = run_flow(skyr, torch, W, "f32", max(args.steps // 5, 20), args.warmup, tiles["f32"], masses=ext_model)
    print(f"# f32-bulk, four potentials and sextic term: {rext}", file=sys.stderr, flush=True)
    # the printed-form force (one-stage stencil; its stiffer quartic term needs half the step)
    rform = run_flow(skyr, torch, {**W, "dt": 0.5 * W["dt"]}, "f32", max(args.steps // 5, 20), args.warmup,
                     (r32["tile"]["variant"], r32["tile"]["xchunk"]), mode="power", form=1)
    print(f"# f32-bulk, printed form: {rform}", file=sys.stderr, flush=True)
    moments = {p: time_moments(skyr, torch, W, p) for p in ("f32", "f64")}
    print(f"# moments: {moments}", file=sys.stderr, flush=True)
    c1 = hedgehog_40_smoke(skyr, torch)
    print(f"# hedgehog-40 as specified: {c1}", file=sys.stderr, flush=True)
    share = {p: block_share(skyr, torch, W, p) for p in ("f32", "f64")}
    print(f"# one device's block of a 2x2x2 split: {share}", file=sys.stderr, flush=True)
    paper151 = {p: paper_size_layouts(skyr, torch, p) for p in ("f32", "f64")}
    print(f"# paper-size lattice, dense vs padded rows: {paper151}", file=sys.stderr, flush=True)
    batch = serve = None
    if not args.no_batch:
        from skyr_inputs import batch_jobs
        batch = batch_throughput(skyr, torch, batch_jobs(4, 64))
        print(f"# batch: {batch}", file=sys.stderr, flush=True)
        serve = served_stream(skyr, torch, count=args.serve_jobs, bandwidth=batch["roofline"]["achieved"] * 1e9)
        print(f"# serve: {serve}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W)
        print(f"# cpu baseline: {cpu}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": r32["site_updates_per_s"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "ms_per_sweep": r32["ms_per_sweep"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": W["name"], "n": W["n"], "h": W["h"], "m": W["m"], "dt": W["dt"],
                   "init": W["init"], "precision": "f32-bulk (f64 sums and arrest test, renormalisation every 16)",
                   "arrest_f32": r32["arrest"], "arrest_f64": r64["arrest"],
                   "interior_sites": (W["n"] - 4) ** 3, "tile_f32": r32["tile"], "tile_f64": r64["tile"]},
        "f64_flow": {"value": r64["site_updates_per_s"], "ms_per_step": r64["ms_per_step"],
                     "ms_per_sweep": r64["ms_per_sweep"],
                     "sweep_kernel_avg_us": r64["sweep_kernel_avg_us"], "achieved_GBs": r64["achieved_GBs"],
                     "arrests": r64["arrests"], "sweeps": r64["sweeps"], "traffic": r64["traffic"]},
        "speedup_f32_over_f64": r32["site_updates_per_s"] / r64["site_updates_per_s"],
        "valu_issue": {"f32": r32["valu"], "f64": r64["valu"]},
        "sweeps_per_s": {"f32": r32["sweeps"] / r32["elapsed_s"], "f64": r64["sweeps"] / r64["elapsed_s"]},
        "f32_four_potentials": {"m_my_mz_mw": list(pot_model), "value": rpot["site_updates_per_s"],
                                "sweep_kernel_avg_us": rpot["sweep_kernel_avg_us"], "steps": rpot["steps"],
                                "E": rpot["E"]},
        "f32_extended_model": {"m_my_mz_mw_c6": list(ext_model), "value": rext["site_updates_per_s"],
                               "sweep_kernel_avg_us": rext["sweep_kernel_avg_us"], "steps": rext["steps"],
                               "E": rext["E"]},
        "f32_printed_form": {"dt": 0.5 * W["dt"], "arrest": "power", "value": rform["site_updates_per_s"],
                             "sweep_kernel_avg_us": rform["sweep_kernel_avg_us"], "steps": rform["steps"],
                             "E": rform["E"]},
        "moments": moments,
        "hedgehog_40_as_specified": c1,
        "block_128_of_256": share,
        "paper_size_151": paper151,
        "sweeps": r32["sweeps"],
        "arrests": r32["arrests"],
        "roofline": {"bound": "hbm", "achieved": r32["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r32["achieved_GBs"] / HBM_PEAK_GBS, "traffic": r32["traffic"],
                     "kernel": "sweep_kernel<float> (step mode)",
                     "kernel_avg_us": r32["sweep_kernel_avg_us"], "bytes_per_launch": r32["bytes_per_launch"],
                     "attainable": {"GBs": copy_gbs, "frac": r32["achieved_GBs"] / copy_gbs,
                                    "f64_frac": r64["achieved_GBs"] / copy_gbs,
                                    "probe": "device-to-device copy of 1 GiB (read + write), median of 5"}},
        "cpu_baseline": cpu,
        "batched_64_jobs": batch,
        "served": serve,
        "latency_p50_s": serve["latency_p50_s"] if serve else None,
        "latency_p99_s": serve["latency_p99_s"] if serve else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
