"""GPU parity of the flow modes and model terms of the program (Sec. 7.5 and 7.7): the
modified pion mass, loosely and lightly bound potentials on top of the pion
mass, the sextic (BPS-Skyrme) term, the plain Newton flow and the first-order
gradient flow, against the FP64 oracle on identical inputs."""
import numpy as np
import pytest

import oracle
from skyr_inputs import random_unit_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"
MASS = (0.9, 0.7, 1.3, 0.6)  # m, m_y, m_z, m_w
SEXTIC = (1.0, 0.0, 0.0, 0.0, 0.1)  # the pion mass and the sextic term alone
ALL = MASS + (0.1,)  # m, m_y, m_z, m_w, c6


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


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", [(23, 29, 40), (40, 40, 40)])
def test_gradient_and_energy_with_all_potentials(skyr, prec, shape):
    h = 0.2
    phi = random_unit_field(shape, 31, 0.6)
    if prec == 1:
        phi = phi.astype(np.float32).astype(np.float64)
    lat = _lat(skyr, shape, h)
    t = torch.tensor(phi, dtype=skyr.field_dtype(prec), device=DEV)
    g = skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    parts = skyr.energy_gradient(lat, prec, skyr.Model(*MASS), t, work, grad=g, projected=False)
    ref = oracle.gradient(phi, h, MASS)
    E2, E4, E0, _ = oracle.energy_parts(phi, h, MASS)
    tol_g, tol_e = (1e-12, 1e-12) if prec == 0 else (2e-4, 2e-6)
    assert _rel_inf(g.double().cpu().numpy(), ref) <= tol_g
    assert parts["E0"] == pytest.approx(E0, rel=tol_e)
    assert parts["E"] == pytest.approx(E2 + E4 + E0, rel=tol_e)
    obs = skyr.observables(lat, prec, skyr.Model(*MASS), t, work)
    ro = oracle.observables(phi, h, MASS)
    assert obs["virial"] == pytest.approx(ro["virial"], rel=10 * tol_e, abs=10 * tol_e * abs(ro["E"]))


def _flow(skyr, n, h, mass, dt, mode, steps, prec=0):
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description({"kind": "hedgehog", "prof_lambda": 0.8})
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    ref0 = phi.double().cpu().numpy()
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    st = skyr.anf_state()
    skyr.anf_step(lat, prec, skyr.Model(*mass), skyr.Flow(dt, 0.0, 10 ** 9, 0, skyr.flow_mode(mode)), phi, alt, vel,
                  st, steps, work)
    return ref0, phi.double().cpu().numpy(), vel.double().cpu().numpy(), st


def test_newton_flow_matches_oracle(skyr):
    """Newton flow (never arrested): 60 steps, fields and velocities agree and
    no reset fires although the energy rises on the way."""
    n, h, dt = 24, 0.25, 0.03
    ref0, phi, vel, st = _flow(skyr, n, h, (1.0,), dt, "newton", 60)
    ref, rvel, rst, Et, _ = oracle.anf(ref0, np.zeros_like(ref0), h, 1.0, dt, 0.0, 60, arrest=False, trace=True)
    assert np.any(np.diff(Et) > 0)
    assert st.steps == 60 and st.arrests == 0 and rst.arrests == 0
    assert np.abs(phi - ref).max() < 1e-11
    assert np.abs(vel - rvel).max() < 1e-10


def test_gradient_flow_matches_oracle(skyr):
    """Gradient flow phi' = normalise(phi + dt F): 60 steps, the velocity stays
    zero, fields agree with the oracle; the same in FP32-bulk within rounding."""
    n, h, dt = 24, 0.25, 5e-4
    ref0, phi, vel, st = _flow(skyr, n, h, (1.0,), dt, "gradient", 60)
    ref, rvel, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, 1.0, dt, 0.0, 60, rule="gradient")
    assert st.steps == 60 and st.arrests == 0
    assert np.all(vel == 0.0)
    assert np.abs(phi - ref).max() < 1e-12
    ref0_32, phi32, vel32, st32 = _flow(skyr, n, h, (1.0,), dt, "gradient", 60, prec=1)
    assert np.all(vel32 == 0.0)
    assert np.abs(phi32 - ref).max() < 1e-5


def test_arrested_flow_with_potentials_matches_oracle(skyr):
    """The arrested Newton flow with all four potentials: 80 steps with resets,
    fields agree with the oracle."""
    n, h, dt = 24, 0.25, 0.05
    ref0, phi, vel, st = _flow(skyr, n, h, MASS, dt, "energy", 80)
    ref, rvel, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, MASS, dt, 0.0, 80)
    assert st.arrests == rst.arrests
    assert np.abs(phi - ref).max() < 1e-10


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("model", [SEXTIC, ALL], ids=["sextic", "all"])
@pytest.mark.parametrize("shape", [(23, 29, 40), (40, 40, 40)])
def test_gradient_energy_and_observables_with_sextic(skyr, prec, model, shape):
    """The sextic term (alone and with every potential): gradient element by
    element, E6 and E, the charge and the virial E2 - E4 + 3 E0 - 3 E6."""
    h = 0.2
    phi = random_unit_field(shape, 37, 0.6)
    if prec == 1:
        phi = phi.astype(np.float32).astype(np.float64)
    lat = _lat(skyr, shape, h)
    t = torch.tensor(phi, dtype=skyr.field_dtype(prec), device=DEV)
    g = skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    parts = skyr.energy_gradient(lat, prec, skyr.Model(*model), t, work, grad=g, projected=False)
    ref = oracle.gradient(phi, h, model)
    E2, E4, E0, E6 = oracle.energy_parts(phi, h, model)
    assert E6 > 0.1 * abs(E2)  # the term is not negligible on this field
    tol_g, tol_e = (1e-12, 1e-12) if prec == 0 else (2e-4, 2e-6)
    assert _rel_inf(g.double().cpu().numpy(), ref) <= tol_g
    assert parts["E6"] == pytest.approx(E6, rel=tol_e)
    assert parts["E"] == pytest.approx(E2 + E4 + E0 + E6, rel=tol_e)
    obs = skyr.observables(lat, prec, skyr.Model(*model), t, work)
    ro = oracle.observables(phi, h, model)
    for k in ("E", "E2", "E4", "E0", "E6"):
        assert obs[k] == pytest.approx(ro[k], rel=tol_e), k
    assert obs["B"] == pytest.approx(ro["B"], rel=10 * tol_e, abs=10 * tol_e * abs(ro["E"]))
    assert obs["virial"] == pytest.approx(ro["virial"], rel=10 * tol_e, abs=10 * tol_e * abs(ro["E"]))


def test_arrested_flow_with_sextic_matches_oracle(skyr):
    """The arrested Newton flow with the sextic term and every potential:
    80 steps with resets, fields and velocities agree with the oracle."""
    n, h, dt = 24, 0.25, 0.04
    model = MASS + (0.5,)
    ref0, phi, vel, st = _flow(skyr, n, h, model, dt, "energy", 80)
    ref, rvel, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, model, dt, 0.0, 80)
    assert st.arrests == rst.arrests
    assert np.abs(phi - ref).max() < 1e-10
    assert np.abs(vel - rvel).max() < 1e-9


@pytest.mark.parametrize("prec,rule,shape,tol", [(1, "power", (36, 33, 36), 0.0), (0, "energy", (26, 30, 26), 0.0),
                                                 (1, "power", (40, 40, 40), 2e-2), (0, "energy", (22, 24, 20), 0.0)],
                         ids=["f32-lead30", "f64-lead0", "f32-converging", "f64-lead14"])
def test_padded_flow_equals_dense(skyr, prec, rule, shape, tol):
    """skyr_anf_step_padded on the padded, row-interleaved copy of a field ends bitwise as
    skyr_anf_step on the dense field, over several calls (graph replays, arrests, and, with a
    tolerance, the stop with its restore sweep), and never writes the padding."""
    h = 0.2
    lat = _lat(skyr, shape, h)
    spec, keep = skyr.spec_from_description({"kind": "hedgehog", "prof_lambda": 0.8})
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    layout = skyr.batch_layout(lat, prec)
    lead, pitch = layout
    pphi = skyr.to_padded(phi, layout)
    palt, pvel = torch.zeros_like(pphi), torch.zeros_like(pphi)
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    flow = skyr.Flow(0.04, tol, 10 ** 6, 4, skyr.flow_mode(rule))
    model = skyr.Model(1.0, 0.0, 0.0, 0.0, 0.0)
    st_d, st_p = skyr.anf_state(), skyr.anf_state()
    for nsteps in (7, 150, 90):
        skyr.anf_step(lat, prec, model, flow, phi, alt, vel, st_d, nsteps, work)
        skyr.anf_step_padded(lat, prec, model, flow, pphi, palt, pvel, st_p, nsteps, work, layout)
        assert bytes(st_d) == bytes(st_p), nsteps
    assert st_d.arrests > 0
    if tol > 0:
        assert st_d.converged
    n2 = lat.shape[2]
    assert torch.equal(skyr.from_padded(pphi, layout, n2), phi)
    assert torch.equal(skyr.from_padded(pvel, layout, n2), vel)
    assert not pphi[..., :lead].any() and not pphi[..., lead + n2:].any()
    short = torch.zeros(lat.shape[:2] + (4, lead + n2 - 1), dtype=phi.dtype, device=DEV)
    with pytest.raises(skyr.SkyrError):
        skyr.anf_step_padded(lat, prec, model, flow, short, torch.zeros_like(short), torch.zeros_like(short),
                             skyr.anf_state(), 1, work, (lead, lead + n2 - 1))
