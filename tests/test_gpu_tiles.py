"""GPU: every compiled tile shape of the fused sweep against the oracle, on
lattices whose (y, z) tiles and x-slabs are ragged: the gradient (plain,
projected, with every potential and the sextic term), the energy parts and
charge, and the arrested flow step by step.  The default tile choice covers one
shape per lattice; these tests set each shape explicitly."""
import numpy as np
import pytest

import oracle
from skyr_inputs import random_unit_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"
ALL = (0.9, 0.7, 1.3, 0.6, 0.1)  # m, m_y, m_z, m_w, c6


@pytest.fixture(scope="module")
def skyr():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2604_25876_amd import skyr as s
    s.lib()
    return s


def _lat(skyr, shape, h):
    lat = skyr.Lattice()
    lat.n[0], lat.n[1], lat.n[2] = shape
    lat.h = h
    return lat


def _rel_inf(got, ref):
    return np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)


def _with_tile(skyr, lat, prec, v, xchunk, fn):
    saved = skyr.get_tile(lat, prec)
    skyr.set_tile(lat, prec, v, xchunk)
    try:
        return fn()
    finally:
        skyr.set_tile(lat, prec, *saved)


# the compiled shapes (threads, output rows, output columns): FP64 (512, 16, 16), (512, 8, 32),
# (512, 12, 32); FP32 (768, 16, 32), (512, 12, 32), (1024, 24, 32)
SHAPES = {0: 3, 1: 3}
CASES = [(prec, v) for prec, n in SHAPES.items() for v in range(n)]


def test_every_compiled_shape_is_covered(skyr):
    assert {p: len(skyr.tile_variants(p)) for p in SHAPES} == SHAPES


@pytest.mark.parametrize("prec,v", CASES, ids=[f"{'f64' if p == 0 else 'f32'}-v{v}" for p, v in CASES])
@pytest.mark.parametrize("model", [(0.9,), ALL], ids=["pion", "all"])
def test_every_shape_gradient_matches_oracle(skyr, prec, v, model):
    shape, h = (37, 53, 70), 0.21
    phi = random_unit_field(shape, 23, 0.5)
    if prec == 1:
        phi = phi.astype(np.float32).astype(np.float64)
    lat = _lat(skyr, shape, h)
    t = torch.tensor(phi, dtype=skyr.field_dtype(prec), device=DEV)
    g, gp = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)

    def run():
        parts = skyr.energy_gradient(lat, prec, skyr.Model(*model), t, work, grad=g, projected=False)
        skyr.energy_gradient(lat, prec, skyr.Model(*model), t, work, grad=gp, projected=True)
        obs = skyr.observables(lat, prec, skyr.Model(*model), t, work)
        return parts, obs

    parts, obs = _with_tile(skyr, lat, prec, v, 21, run)
    ref = oracle.gradient(phi, h, model)
    refp, rmax = oracle.project(phi, ref)
    tol_g, tol_e = (1e-12, 1e-12) if prec == 0 else (2e-4, 2e-6)
    assert _rel_inf(g.double().cpu().numpy(), ref) <= tol_g
    assert _rel_inf(gp.double().cpu().numpy(), refp) <= tol_g
    assert parts["max_force"] == pytest.approx(rmax, rel=10 * tol_g)
    ro = oracle.observables(phi, h, model)
    for k in ("E", "E2", "E4", "E0", "E6"):
        assert obs[k] == pytest.approx(ro[k], rel=tol_e, abs=tol_e * abs(ro["E"])), k
    assert obs["B"] == pytest.approx(ro["B"], rel=10 * tol_e, abs=10 * tol_e * abs(ro["E"]))


@pytest.mark.parametrize("v", range(SHAPES[0]))
def test_every_f64_shape_flow_matches_oracle(skyr, v):
    """Hedgehog on 30 x 34 x 40 (ragged tiles, 16-plane slabs): 40 arrested-flow
    steps with every potential and the sextic term, fields, velocities and
    arrests as the oracle's."""
    shape, h, dt = (30, 34, 40), 0.25, 0.04
    lat = _lat(skyr, shape, h)
    spec, keep = skyr.spec_from_description({"kind": "hedgehog", "prof_lambda": 0.8})
    phi = skyr.new_field(lat, 0, DEV)
    skyr.init_field(lat, 0, spec, phi)
    ref0 = phi.cpu().numpy()
    alt, vel = skyr.new_field(lat, 0, DEV), skyr.new_field(lat, 0, DEV)
    work = skyr.new_workspace(lat, 0, DEV)
    st = skyr.anf_state()
    flow = skyr.Flow(dt, 0.0, 10 ** 9, 0, skyr.flow_mode("energy"))
    _with_tile(skyr, lat, 0, v, 16, lambda: skyr.anf_step(lat, 0, skyr.Model(*ALL), flow, phi, alt, vel, st, 40,
                                                          work))
    ref, rvel, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, ALL, dt, 0.0, 40)
    assert st.steps == 40 and st.arrests == rst.arrests
    assert np.abs(phi.cpu().numpy() - ref).max() < 1e-10
    assert np.abs(vel.cpu().numpy() - rvel).max() < 1e-9
