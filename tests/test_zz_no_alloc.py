"""The allocation-free flow entry point (skyr_anf_step_noalloc) against the
flow with a caller-owned workspace (skyr_anf_step), through the C ABI: the
same kernels run in both, so fields, velocities and flow states agree bit for
bit.  Two calls in a row share the library's fixed device scratch, the second
on a smaller lattice, so a stale control block or partial sum left by the
first call would show up in the second."""
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


def _start(skyr, n, h, prec, desc):
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description(desc)
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    torch.cuda.synchronize()
    return lat, phi


def _run(skyr, lat, prec, model, flow, phi0, steps, noalloc):
    phi = phi0.clone()
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    st = skyr.anf_state()
    if noalloc:
        skyr.anf_step_noalloc(lat, prec, model, flow, phi, alt, vel, st, steps)
    else:
        work = skyr.new_workspace(lat, prec, DEV)
        skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st, steps, work)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), vel.cpu().numpy(), st.as_dict()


# (lattice size, h, precision, arrest rule, steps, tolerance, initial data); the second is smaller
CASES = [
    (48, 0.2, 1, "power", 400, 1e-4, {"kind": "random_product", "B": 3, "seed": 5, "radius": 2.0, "prof_lambda": 1.0}),
    (28, 0.25, 0, "energy", 60, 0.0, {"kind": "hedgehog", "prof_lambda": 1.0}),
]


def test_noalloc_equals_anf_step_on_two_calls_in_a_row(skyr):
    for n, h, prec, rule, steps, tol, desc in CASES:
        print(f"noalloc case n={n} prec={prec} rule={rule} steps={steps}", flush=True)
        lat, phi0 = _start(skyr, n, h, prec, desc)
        model = skyr.Model(1.0)
        flow = skyr.Flow(0.1 * h, tol, 10 ** 6, 16, skyr.flow_mode(rule))
        ref = _run(skyr, lat, prec, model, flow, phi0, steps, noalloc=False)
        got = _run(skyr, lat, prec, model, flow, phi0, steps, noalloc=True)
        assert ref[2]["steps"] > 0 and not ref[2]["nonfinite"]
        assert got[2] == ref[2]
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
