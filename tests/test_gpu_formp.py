"""GPU parity of the printed-form force (SKYR_FORM_PRINTED: the paper's
Euler-Lagrange expression of Sec. 3 with five-point second differences and
D_i D_j mixed derivatives) against the oracle's gradient_literal, on every
interior site, and of the flow that uses it against the oracle's flow with the
same force."""
import numpy as np
import pytest

import oracle
from skyr_inputs import random_unit_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"
MASS = (0.9, 0.7, 1.3, 0.6)


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


def _model(skyr, mass):
    m = skyr.Model(*mass)
    m.form = skyr.FORM_PRINTED
    return m


def _rel_inf(got, ref):
    return np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mass", [(1.0,), MASS], ids=["pion", "four"])
@pytest.mark.parametrize("shape", [(23, 29, 40), (40, 40, 40), (37, 20, 70)])
def test_printed_gradient_matches_oracle(skyr, prec, mass, shape):
    h = 0.2
    phi = random_unit_field(shape, 41, 0.5)
    if prec == 1:
        phi = phi.astype(np.float32).astype(np.float64)
    lat = _lat(skyr, shape, h)
    t = torch.tensor(phi, dtype=skyr.field_dtype(prec), device=DEV)
    g = skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    parts = skyr.energy_gradient(lat, prec, _model(skyr, mass), t, work, grad=g, projected=False)
    ref = oracle.gradient_literal(phi, h, mass)
    tol_g, tol_e = (1e-12, 1e-12) if prec == 0 else (3e-5, 2e-6)
    assert _rel_inf(g.double().cpu().numpy(), ref) <= tol_g
    E2, E4, E0, _ = oracle.energy_parts(phi, h, mass)
    assert parts["E"] == pytest.approx(E2 + E4 + E0, rel=tol_e)
    # projected output and the largest projected force
    gp = skyr.new_field(lat, prec, DEV)
    parts = skyr.energy_gradient(lat, prec, _model(skyr, mass), t, work, grad=gp, projected=True)
    refp, rmax = oracle.project(phi, ref)
    assert _rel_inf(gp.double().cpu().numpy(), refp) <= tol_g
    assert parts["max_force"] == pytest.approx(rmax, rel=10 * tol_g)


def _hedgehog_flow(skyr, prec, n, h, mass, dt, rule, steps):
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description({"kind": "hedgehog", "prof_lambda": 0.8})
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    ref0 = phi.double().cpu().numpy()
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    st = skyr.anf_state()
    skyr.anf_step(lat, prec, _model(skyr, mass), skyr.Flow(dt, 0.0, 10 ** 9, 0, skyr.flow_mode(rule)), phi, alt, vel,
                  st, steps, work)
    return ref0, phi.double().cpu().numpy(), vel.double().cpu().numpy(), st


@pytest.mark.parametrize("rule", ["energy", "power"])
def test_printed_flow_matches_oracle(skyr, rule):
    """80 arrested-flow steps with the printed force: the same arrests, fields
    and velocities as the oracle's flow with gradient_literal."""
    n, h, dt = 26, 0.25, 0.04
    ref0, phi, vel, st = _hedgehog_flow(skyr, 0, n, h, (1.0,), dt, rule, 80)
    ref, rvel, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, 1.0, dt, 0.0, 80, rule=rule, form="printed")
    assert st.steps == 80 and st.arrests == rst.arrests
    assert np.abs(phi - ref).max() < 1e-10
    assert np.abs(vel - rvel).max() < 1e-9


def test_printed_flow_fp32_bulk_tracks_fp64(skyr):
    n, h, dt = 26, 0.25, 0.04
    _, phi64, _, st64 = _hedgehog_flow(skyr, 0, n, h, MASS, dt, "power", 60)
    _, phi32, _, st32 = _hedgehog_flow(skyr, 1, n, h, MASS, dt, "power", 60)
    assert st32.steps == 60
    assert np.abs(phi32 - phi64).max() < 2e-4


def test_printed_form_is_rejected_where_unsupported(skyr):
    lat = skyr.Lattice.cube(24, 0.2)
    phi = skyr.new_field(lat, 0, DEV)
    phi[0] = 1.0
    work = skyr.new_workspace(lat, 0, DEV)
    m = _model(skyr, (1.0, 0.0, 0.0, 0.0, 0.1))
    with pytest.raises(skyr.SkyrError) as e:
        skyr.energy_gradient(lat, 0, m, phi, work)
    assert e.value.status == skyr.E_INVAL
    bad = skyr.Model(1.0)
    bad.form = 7
    with pytest.raises(skyr.SkyrError):
        skyr.observables(lat, 0, bad, phi, work)
    with skyr.Batch(4) as b:
        alt, vel = skyr.new_field(lat, 0, DEV), skyr.new_field(lat, 0, DEV)
        with pytest.raises(skyr.SkyrError) as e:
            b.add(lat, 0, _model(skyr, (1.0,)), skyr.Flow(0.02, 1e-4, 100, 0, 0), phi, alt, vel, work)
        assert e.value.status == skyr.E_INVAL


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", [(5, 5, 5), (5, 7, 6), (6, 5, 37)])
def test_printed_form_on_the_smallest_lattices(skyr, prec, shape):
    """One interior site (5^3), one interior row, a thin slab: every stencil
    reaches the frozen layers."""
    h = 0.3
    phi = random_unit_field(shape, 3, 0.8)
    if prec == 1:
        phi = phi.astype(np.float32).astype(np.float64)
    lat = _lat(skyr, shape, h)
    g = skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    t = torch.tensor(phi, dtype=skyr.field_dtype(prec), device=DEV)
    skyr.energy_gradient(lat, prec, _model(skyr, (0.7,)), t, work, grad=g)
    ref = oracle.gradient_literal(phi, h, 0.7)
    assert _rel_inf(g.double().cpu().numpy(), ref) <= (1e-12 if prec == 0 else 3e-5)


def test_printed_form_reports_nonfinite_input(skyr):
    lat = skyr.Lattice.cube(16, 0.2)
    phi = skyr.new_field(lat, 0, DEV)
    phi[0] = 1.0
    phi[1, 7, 9, 8] = float("nan")
    alt, vel = skyr.new_field(lat, 0, DEV), skyr.new_field(lat, 0, DEV)
    work = skyr.new_workspace(lat, 0, DEV)
    st = skyr.anf_state()
    with pytest.raises(skyr.SkyrError) as e:
        skyr.anf_step(lat, 0, _model(skyr, (1.0,)), skyr.Flow(0.02, 0.0, 10, 0, skyr.ARREST_POWER), phi, alt, vel,
                      st, 10, work)
    assert e.value.status == skyr.E_NONFINITE and st.nonfinite == 1
