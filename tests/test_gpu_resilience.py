"""GPU: failure isolation and checkpoint / resume of flows.

A non-finite value planted from the host in one job's field stops that job only: its slot
reports SKYR_E_NONFINITE while every other job of the same batch (or served stream) ends
bit for bit as it does alone.  A flow checkpointed through the Sec. 7.4 binary field files
(field and velocity) plus its host state, and resumed in fresh buffers, ends bit for bit
as the uninterrupted flow, arrests and pending redo sweeps included."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def skyr():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2604_25876_amd import skyr as s
    s.lib()
    return s


def job(n, h, m, dt, prec, B, seed, tol=1e-3, steps=300, flow="energy"):
    return dict(n=n, h=h, m=m, dt=dt, tol=tol, steps=steps, precision=prec, flow=flow,
                init={"kind": "random_product", "B": B, "seed": seed, "radius": 1.5, "prof_lambda": 1.0})


JOBS = [job(24, 0.25, 1.0, 0.025, "f64", 1, 11), job(32, 0.2, 0.0, 0.02, "f32", 2, 12, flow="power"),
        job(28, 0.2, 1.0, 0.02, "f64", 3, 13, flow="power")]


def _setup(skyr, d):
    prec = skyr.F32_BULK if d["precision"] == "f32" else skyr.F64
    lat = skyr.Lattice.cube(d["n"], d["h"])
    phi = skyr.new_field(lat, prec, DEV)
    spec, keep = skyr.spec_from_description(d["init"])
    skyr.init_field(lat, prec, spec, phi)
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    flow = skyr.Flow(d["dt"], d["tol"], d["steps"], 16, skyr.flow_mode(d["flow"]))
    return lat, prec, phi, alt, vel, work, flow


def _batch(skyr, jobs, plant=None):
    """Run the jobs in one batch until each has stopped; plant(j, phi) may spoil job j's
    field after its initial data.  Returns per job (status of its last poll, state, field)."""
    bufs = [_setup(skyr, d) for d in jobs]
    if plant is not None:
        for j, b in enumerate(bufs):
            plant(j, b[2])
    L = skyr.lib()
    out = []
    with skyr.Batch(len(jobs)) as b:
        slots = [b.add(lat, prec, skyr.Model(d["m"]), flow, phi, alt, vel, work)
                 for d, (lat, prec, phi, alt, vel, work, flow) in zip(jobs, bufs)]
        for _ in range(100):
            b.run(16)
            sts = [b.poll(s) for s in slots]
            if all(st.converged or st.nonfinite or st.steps >= d["steps"] for st, d in zip(sts, jobs)):
                break
        for s, buf in zip(slots, bufs):
            st = skyr.AnfState()
            status = L.skyr_batch_poll(b._h, s, ctypes.byref(st))
            out.append((status, st, buf[2].cpu().numpy().copy()))
    return out


def test_nonfinite_job_stops_alone_in_a_batch(skyr):
    def plant(j, phi):
        if j == 1:
            phi[0, 9, 10, 11] = float("nan")  # an interior site

    mix = _batch(skyr, JOBS, plant)
    status, st, _ = mix[1]
    assert status == skyr.E_NONFINITE and st.nonfinite == 1 and st.steps == 0
    for j in (0, 2):
        alone = _batch(skyr, [JOBS[j]])[0]
        assert mix[j][0] == skyr.OK and alone[0] == skyr.OK
        assert (mix[j][1].steps, mix[j][1].arrests) == (alone[1].steps, alone[1].arrests)
        assert np.array_equal(mix[j][2], alone[2]), f"job {j} changed by its batch-mate's failure"


def test_nonfinite_request_stops_alone_in_the_server(skyr):
    from paper_2604_25876_amd.serve import GpuBackend, Request, Server

    class Planting(GpuBackend):
        def start(self, desc):
            slot = super().start(desc)
            if desc.get("plant_nan"):
                self.site(slot, 2, 12, 12, 12).fill_(float("inf"))
            return slot

    reqs = [dict(JOBS[0]), dict(JOBS[1], plant_nan=True), dict(JOBS[2])]
    be = Planting(max_jobs=3)
    srv = Server(be, max_jobs=3, hbm_budget=2 ** 30, sweeps_per_tick=16, keep_fields=True)
    rep = srv.serve([Request(d, arrival=0.0, rid=i) for i, d in enumerate(reqs)])
    be.close()
    assert rep["jobs"] == 3 and rep["nonfinite"] == 1
    for r in srv.done:
        if r.rid == 1:
            assert r.state["nonfinite"] and r.state["steps"] == 0
            continue
        alone = _batch(skyr, [JOBS[r.rid]])[0]
        assert r.state["steps"] == alone[1].steps
        assert np.array_equal(r.result["field"].cpu().numpy(), alone[2]), r.rid


@pytest.mark.parametrize("prec,rule", [(0, "energy"), (1, "power")], ids=["f64-energy", "f32-power"])
def test_checkpoint_resume_is_bitwise(skyr, prec, rule, tmp_path):
    """A hedgehog relaxed with arrests in segments of 13 steps, checkpointed after every
    segment to binary field files (phi and v) and a copy of the host state, each segment
    resumed in freshly allocated buffers: the end equals 78 uninterrupted steps."""
    lat = skyr.Lattice.cube(30, 0.2)
    spec, keep = skyr.spec_from_description({"kind": "hedgehog", "prof_lambda": 0.7})
    model = skyr.Model(1.0, 0.0, 0.0, 0.0, 0.05)
    flow = skyr.Flow(0.06, 0.0, 10 ** 9, 4, skyr.flow_mode(rule))

    def fresh():
        return skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV), \
            skyr.new_workspace(lat, prec, DEV)

    phi, alt, vel, work = fresh()
    skyr.init_field(lat, prec, spec, phi)
    phi0 = phi.clone()
    st = skyr.anf_state()
    skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st, 78, work)
    assert st.arrests > 0
    ref = (phi.cpu(), vel.cpu(), bytes(st))

    phi, alt, vel, work = fresh()
    phi.copy_(phi0)
    st = skyr.anf_state()
    for seg in range(6):
        skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st, 13, work)
        skyr.save_field(tmp_path / "phi.bin", lat, prec, model, phi, fmt="binary")
        skyr.save_field(tmp_path / "vel.bin", lat, prec, model, vel, fmt="binary")
        saved = bytes(st)
        del phi, alt, vel, work, st
        phi, alt, vel, work = fresh()
        skyr.load_field(tmp_path / "phi.bin", lat, prec, phi)
        skyr.load_field(tmp_path / "vel.bin", lat, prec, vel)
        st = skyr.AnfState.from_buffer_copy(saved)
    assert torch.equal(phi.cpu(), ref[0]) and torch.equal(vel.cpu(), ref[1])
    assert bytes(st) == ref[2]
