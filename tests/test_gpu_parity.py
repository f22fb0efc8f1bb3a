"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Every test builds identical seeded inputs for both sides, runs the library on
cuda:0 and the oracle on the host, and compares element by element (or on
sampled sites, for the full-size lattices).  Tolerances:
  * FP64 gradients / projected gradients: max-abs relative to max |g| <= 1e-12
  * FP64 energies, charge, virial: <= 1e-12 relative (1e-11 for the virial,
    a difference of parts)
  * FP32-bulk: inputs are the FP32 rounding of the same field; the gradient
    is compared at 2e-4 of max |g| (single-precision stencil cancellation
    ~ eps32 * 16/h^2), energies at 2e-6 relative
"""
import math

import numpy as np
import pytest

import oracle
from skyr_inputs import random_unit_field, HEDGEHOG_40_SMALLDT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def skyr():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2604_25876_amd import skyr as s
    s.lib()
    return s


DEV = "cuda:0"


def _tensor(a, prec, skyr):
    return torch.tensor(np.ascontiguousarray(a), dtype=skyr.field_dtype(prec), device=DEV)


def _lat(skyr, shape, h):
    lat = skyr.Lattice()
    lat.n[0], lat.n[1], lat.n[2] = shape
    lat.h = h
    return lat


def _rel_inf(got, ref):
    return np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)


# ----------------------------------------------------------- initial data
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("desc", [
    {"kind": "hedgehog", "prof_lambda": 1.0},
    {"kind": "cube_b4", "prof_lambda": 1.5},
    {"kind": "random_product", "B": 10, "seed": 1, "radius": 3.0, "prof_lambda": 1.0},
])
def test_init_matches_oracle(skyr, prec, desc):
    n, h = 40, 0.2
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description(desc)
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    if desc["kind"] == "hedgehog":
        cs = [oracle.hedgehog(prof_lambda=desc["prof_lambda"])]
    elif desc["kind"] == "cube_b4":
        cs = [oracle.cube_b4(prof_lambda=desc["prof_lambda"])]
    else:
        cs = oracle.random_constituents(desc["seed"], desc["B"], desc["radius"], math.pi, desc["prof_lambda"])
    ref = oracle.init_product((n, n, n), h, cs)
    got = phi.double().cpu().numpy()
    tol = 1e-13 if prec == 0 else 1e-7
    assert np.abs(got - ref).max() < tol


@pytest.mark.parametrize("prec", [0, 1])
def test_init_on_an_odd_lattice_matches_oracle(skyr, prec):
    """Odd lattice, constituents centred on sites: sites at each centre and on
    the negative x3 axis through it (z = infinity of the rational map, Sec. 4.1)
    stay finite and agree with the oracle."""
    n, h = 41, 0.2
    lat = skyr.Lattice.cube(n, h)
    q = (0.6, 0.0, 0.8, 0.0)
    cs = [skyr.cube_b4(X=(0.0, 0.0, 0.0), prof_lambda=1.2), skyr.constituent(1, [0, 1], [1], X=(1.0, -0.4, 0.6), quat=q)]
    spec, keep = skyr.init_spec(skyr.INIT_PRODUCT, cs)
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    got = phi.double().cpu().numpy()
    ref = oracle.init_product((n, n, n), h, [oracle.cube_b4(prof_lambda=1.2),
                                             oracle.constituent(1, [0, 1], [1], X=(1.0, -0.4, 0.6), quat=q)])
    assert np.all(np.isfinite(ref)) and np.all(np.isfinite(got))
    assert np.abs(got - ref).max() < (1e-13 if prec == 0 else 1e-7)


@pytest.mark.parametrize("prec", [0, 1])
def test_oriented_constituents_match_oracle(skyr, prec):
    """Constituents turned in space (Sec. 5.3) by Euler angles (Sec. 7.3.1):
    the two-cube chain of the program's example configuration and a turned,
    isorotated hedgehog, against the oracle on the same quaternions."""
    n, h = 48, 0.2
    lat = skyr.Lattice.cube(n, h)
    B = skyr.orientation_zyz(1.57079, 1.57079, -1.57079)
    Bh = skyr.orientation_zyz(0.3, -1.1, 2.0)
    q = (0.6, 0.0, 0.8, 0.0)
    lib_cs = [skyr.cube_b4(X=(-1.5, 0.0, 0.0)), skyr.cube_b4(X=(1.5, 0.0, 0.0), orient=B),
              skyr.constituent(1, [0, 1], [1], X=(0.3, 2.1, -0.7), quat=q, orient=Bh)]
    ora_cs = [oracle.cube_b4(X=(-1.5, 0.0, 0.0)), oracle.cube_b4(X=(1.5, 0.0, 0.0), orient=B),
              oracle.constituent(1, [0, 1], [1], X=(0.3, 2.1, -0.7), quat=q, orient=Bh)]
    spec, keep = skyr.init_spec(skyr.INIT_PRODUCT, lib_cs)
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    ref = oracle.init_product((n, n, n), h, ora_cs)
    assert np.abs(phi.double().cpu().numpy() - ref).max() < (1e-13 if prec == 0 else 1e-7)


def test_random_constituents_match_oracle(skyr):
    for seed, B in ((1, 10), (2**63 + 12345, 12), (7, 1)):
        a = skyr.random_constituents(seed, B, 3.0)
        b = oracle.random_constituents(seed, B, 3.0)
        for ca, cb in zip(a, b):
            assert list(ca.X) == list(cb.X)
            assert np.allclose(list(ca.quat), list(cb.quat), rtol=0, atol=1e-15)


# --------------------------------------------------------------- gradient
SHAPES = [(9, 9, 9), (40, 40, 40), (37, 53, 70), (5, 6, 7), (64, 20, 131)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("projected", [False, True])
def test_gradient_f64_matches_oracle(skyr, shape, projected):
    h, m = 0.21, 0.9
    phi = random_unit_field(shape, 17 + sum(shape), 0.5)
    lat = _lat(skyr, shape, h)
    t = _tensor(phi, 0, skyr)
    g = skyr.new_field(lat, 0, DEV)
    work = skyr.new_workspace(lat, 0, DEV)
    parts = skyr.energy_gradient(lat, 0, skyr.Model(m), t, work, grad=g, projected=projected)
    ref = oracle.gradient(phi, h, m)
    if projected:
        ref, _ = oracle.project(phi, ref)
    got = g.cpu().numpy()
    assert _rel_inf(got, ref) <= 1e-12
    E2, E4, E0, _ = oracle.energy_parts(phi, h, m)
    assert parts["E2"] == pytest.approx(E2, rel=1e-12)
    assert parts["E4"] == pytest.approx(E4, rel=1e-12)
    assert parts["E0"] == pytest.approx(E0, rel=1e-12)
    _, r = oracle.project(phi, oracle.gradient(phi, h, m))
    assert parts["max_force"] == pytest.approx(r, rel=1e-12)


@pytest.mark.parametrize("shape", [(40, 40, 40), (37, 53, 70)])
def test_gradient_f32_matches_oracle(skyr, shape):
    h, m = 0.2, 1.0
    phi = random_unit_field(shape, 3, 0.3).astype(np.float32).astype(np.float64)
    lat = _lat(skyr, shape, h)
    t = _tensor(phi, 1, skyr)
    g = skyr.new_field(lat, 1, DEV)
    work = skyr.new_workspace(lat, 1, DEV)
    parts = skyr.energy_gradient(lat, 1, skyr.Model(m), t, work, grad=g, projected=False)
    ref = oracle.gradient(phi, h, m)
    assert _rel_inf(g.double().cpu().numpy(), ref) <= 2e-4
    E = sum(oracle.energy_parts(phi, h, m))
    assert parts["E"] == pytest.approx(E, rel=2e-6)


def test_gradient_is_deterministic(skyr):
    """Two launches on the same input give bitwise identical outputs (a check
    for missing barriers and LDS races)."""
    shape, h, m = (48, 40, 100), 0.2, 1.0
    phi = random_unit_field(shape, 5, 0.5)
    lat = _lat(skyr, shape, h)
    for prec in (0, 1):
        t = _tensor(phi, prec, skyr)
        work = skyr.new_workspace(lat, prec, DEV)
        outs = []
        for _ in range(2):
            g = skyr.new_field(lat, prec, DEV)
            p = skyr.energy_gradient(lat, prec, skyr.Model(m), t, work, grad=g)
            outs.append((g.cpu().numpy(), p))
        assert np.array_equal(outs[0][0], outs[1][0])
        assert outs[0][1] == outs[1][1]


# ------------------------------------------------------------ observables
@pytest.mark.parametrize("desc", [
    {"kind": "hedgehog", "prof_lambda": 1.0},
    {"kind": "random_product", "B": 4, "seed": 3, "radius": 2.0, "prof_lambda": 1.0},
])
def test_observables_match_oracle(skyr, desc):
    n, h, m = 44, 0.2, 1.0
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description(desc)
    phi = skyr.new_field(lat, 0, DEV)
    skyr.init_field(lat, 0, spec, phi)
    work = skyr.new_workspace(lat, 0, DEV)
    got = skyr.observables(lat, 0, skyr.Model(m), phi, work)
    ref = oracle.observables(phi.cpu().numpy(), h, m)
    for k in ("E", "E2", "E4", "E0", "B", "max_force"):
        assert got[k] == pytest.approx(ref[k], rel=1e-12, abs=1e-13), k
    assert got["virial"] == pytest.approx(ref["virial"], rel=1e-11, abs=1e-12)


# ------------------------------------------------------------------- flow
def _flow_pair(skyr, n, h, m, dt, prec=0, desc=None):
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description(desc or {"kind": "hedgehog", "prof_lambda": 1.0})
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    return lat, phi, alt, vel, work


def test_flow_trajectory_matches_oracle_step_by_step(skyr):
    """Small-dt hedgehog (40^3, h = 0.2, dt = 0.025): fields and energies agree
    after every one of the first 30 steps."""
    w = HEDGEHOG_40_SMALLDT
    n, h, m, dt = w["n"], w["h"], w["m"], w["dt"]
    lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt)
    ref = phi.cpu().numpy()
    rvel = np.zeros_like(ref)
    st, rst = skyr.anf_state(), oracle.AnfState.fresh()
    flow = skyr.Flow(dt, 0.0, 10 ** 9, 0, 0)
    for k in range(30):
        skyr.anf_step(lat, 0, skyr.Model(m), flow, phi, alt, vel, st, 1, work)
        ref, rvel, rst, Et, _ = oracle.anf(ref, rvel, h, m, dt, 0.0, k + 1, rst, trace=True)
        assert st.steps == rst.steps == k + 1
        assert st.arrests == rst.arrests
        assert st.E_prev == pytest.approx(Et[-1], rel=1e-13)
        assert np.abs(phi.cpu().numpy() - ref).max() < 1e-12
        assert np.abs(vel.cpu().numpy() - rvel).max() < 1e-11


def test_flow_with_arrests_matches_oracle(skyr):
    """A step large enough to overshoot: the arrests fire on the same steps
    and the fields agree after 80 steps run in one call."""
    n, h, m, dt = 24, 0.25, 1.0, 0.06
    lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt)
    ref0 = phi.cpu().numpy()
    st = skyr.anf_state()
    skyr.anf_step(lat, 0, skyr.Model(m), skyr.Flow(dt, 0.0, 10 ** 9, 0, 0), phi, alt, vel, st, 80, work)
    ref, rvel, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, m, dt, 0.0, 80)
    assert rst.arrests > 0
    assert st.steps == 80 and st.arrests == rst.arrests and st.redo_sweeps == rst.arrests
    assert np.abs(phi.cpu().numpy() - ref).max() < 1e-10


def test_flow_power_rule_matches_oracle(skyr):
    """Power arrest rule (reset when h^3 sum F.v < 0): the resets fire on the
    same steps as in the oracle and the fields agree after 80 steps."""
    n, h, m, dt = 24, 0.25, 1.0, 0.06
    lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt)
    ref0 = phi.cpu().numpy()
    st = skyr.anf_state()
    flow = skyr.Flow(dt, 0.0, 10 ** 9, 0, skyr.ARREST_POWER)
    skyr.anf_step(lat, 0, skyr.Model(m), flow, phi, alt, vel, st, 80, work)
    ref, rvel, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, m, dt, 0.0, 80, rule="power")
    assert rst.arrests > 0
    assert st.steps == 80 and st.arrests == rst.arrests and st.redo_sweeps == rst.arrests
    assert np.abs(phi.cpu().numpy() - ref).max() < 1e-10
    assert np.abs(vel.cpu().numpy() - rvel).max() < 1e-9


def test_flow_resume_across_calls(skyr):
    """Chained calls (7 + 13 + 20 steps) equal one call of 40 steps, bitwise."""
    n, h, m, dt = 28, 0.25, 1.0, 0.05
    res = []
    for chunks in ((40,), (7, 13, 20)):
        lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt)
        st = skyr.anf_state()
        for c in chunks:
            skyr.anf_step(lat, 0, skyr.Model(m), skyr.Flow(dt, 0.0, 10 ** 9, 0, 0), phi, alt, vel, st, c, work)
        res.append((phi.cpu().numpy(), vel.cpu().numpy(), st.arrests))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]


def test_converged_energy_matches_oracle(skyr):
    """Relax the hedgehog to max|F| < 1e-5 on both sides: energies agree to
    1e-8 relative, B and virial to the same."""
    n, h, m, dt, tol = 40, 0.2, 1.0, 0.02, 1e-5
    lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt)
    ref0 = phi.cpu().numpy()
    st = skyr.anf_state()
    skyr.anf_step(lat, 0, skyr.Model(m), skyr.Flow(dt, tol, 20000, 0, 0), phi, alt, vel, st, 20000, work)
    assert st.converged == 1
    ref, _, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, m, dt, tol, 20000)
    assert rst.converged == 1
    got = skyr.observables(lat, 0, skyr.Model(m), phi, work)
    ro = oracle.observables(ref, h, m)
    assert got["E"] == pytest.approx(ro["E"], rel=1e-8)
    assert got["B"] == pytest.approx(ro["B"], rel=1e-8)


@pytest.mark.parametrize("rule", ["energy", "power"])
def test_velocity_after_convergence_matches_oracle(skyr, rule):
    """The velocity returned with a converged field is v_k of that field, as in
    the oracle (the in-place kick of the sweep that found convergence is undone),
    and its kinetic energy agrees; a flow then resumed with a tighter tolerance
    follows the oracle's uninterrupted flow to the tighter tolerance."""
    n, h, m, dt = 24, 0.25, 1.0, 0.03
    tol1, tol2 = 3e-3, 2e-4
    mode = skyr.flow_mode(rule)
    lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt)
    ref0 = phi.cpu().numpy()
    st = skyr.anf_state()
    skyr.anf_step(lat, 0, skyr.Model(m), skyr.Flow(dt, tol1, 10 ** 6, 0, mode), phi, alt, vel, st, 10 ** 6, work)
    ref, rvel, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, m, dt, tol1, 10 ** 6, rule=rule)
    assert st.converged == 1 and rst.converged == 1
    assert st.steps == rst.steps and st.arrests == rst.arrests
    assert np.abs(phi.cpu().numpy() - ref).max() < 1e-10
    vscale = max(np.abs(rvel).max(), 1e-300)
    assert np.abs(vel.cpu().numpy() - rvel).max() <= 1e-10 * vscale + 1e-300
    assert skyr.kinetic_energy(lat, 0, vel, work) == pytest.approx(oracle.kinetic(rvel, h), rel=1e-9, abs=1e-300)
    # resume with the tighter tolerance
    st.converged = 0
    skyr.anf_step(lat, 0, skyr.Model(m), skyr.Flow(dt, tol2, 10 ** 6, 0, mode), phi, alt, vel, st, 10 ** 6, work)
    ref2, rvel2, rst2, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, m, dt, tol2, 10 ** 6, rule=rule)
    print(f"{rule}: {rst.steps} steps to {tol1}, {rst2.steps} to {tol2}; arrests {st.arrests} / {rst2.arrests}")
    assert st.converged == 1 and st.steps == rst2.steps and st.arrests == rst2.arrests
    assert np.abs(phi.cpu().numpy() - ref2).max() < 1e-9


def test_converged_f32_bulk_against_oracle(skyr):
    """FP32-bulk relaxation of the same hedgehog: converged energy within 1e-6
    of the FP64 oracle's converged energy, B within 1e-3; the FP64 energy of
    the FP32 result (evaluated by the oracle) agrees even more closely."""
    n, h, m, dt, tol = 40, 0.2, 1.0, 0.02, 1e-4
    lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt, prec=1)
    ref0 = oracle.init_product((n, n, n), h, [oracle.hedgehog()])
    st = skyr.anf_state()
    skyr.anf_step(lat, 1, skyr.Model(m), skyr.Flow(dt, tol, 20000, 16, 0), phi, alt, vel, st, 20000, work)
    assert st.converged == 1
    ref, _, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, m, dt, 1e-5, 20000)
    got = skyr.observables(lat, 1, skyr.Model(m), phi, work)
    ro = oracle.observables(ref, h, m)
    e64 = oracle.energy(phi.double().cpu().numpy(), h, m)
    print(f"FP32-bulk: steps {st.steps} arrests {st.arrests} E32 {got['E']:.10f} E64(phi32) {e64:.10f} "
          f"oracle {ro['E']:.10f} B32 {got['B']:.8f} oracle B {ro['B']:.8f}")
    assert e64 == pytest.approx(ro["E"], rel=1e-6)
    assert got["E"] == pytest.approx(ro["E"], rel=1e-6)
    assert got["B"] == pytest.approx(ro["B"], abs=1e-3)


@pytest.mark.parametrize("prec", [0, 1])
def test_converged_power_rule_against_oracle(skyr, prec):
    """Power arrest rule, FP64 and FP32-bulk: the hedgehog relaxes to the same
    minimum as the oracle's energy-rule flow (energy within 1e-8 in FP64,
    1e-6 in FP32-bulk; B within 1e-3)."""
    n, h, m, dt = 40, 0.2, 1.0, 0.02
    tol = 1e-5 if prec == 0 else 1e-4
    lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt, prec=prec)
    ref0 = oracle.init_product((n, n, n), h, [oracle.hedgehog()])
    st = skyr.anf_state()
    skyr.anf_step(lat, prec, skyr.Model(m), skyr.Flow(dt, tol, 20000, 16, skyr.ARREST_POWER), phi, alt, vel, st,
                  20000, work)
    assert st.converged == 1
    ref, _, rst, _, _ = oracle.anf(ref0, np.zeros_like(ref0), h, m, dt, 1e-5, 20000)
    got = skyr.observables(lat, prec, skyr.Model(m), phi, work)
    ro = oracle.observables(ref, h, m)
    print(f"power rule prec {prec}: steps {st.steps} arrests {st.arrests} E {got['E']:.12f} oracle {ro['E']:.12f}")
    assert got["E"] == pytest.approx(ro["E"], rel=1e-8 if prec == 0 else 1e-6)
    assert got["B"] == pytest.approx(ro["B"], abs=1e-3)


@pytest.mark.parametrize("kr", [1, 16, 64])
def test_f32_bulk_norm_drift(skyr, kr):
    """FP32-bulk with the FP64 renormalisation every kr steps: after 640 steps
    of the random B = 4 product (64^3, h = 0.15) every interior site still has
    | |phi| - 1 | <= 1e-6 (the single-precision renormalisation keeps it at the
    rounding level between the double-precision ones), and the frozen layers
    are untouched."""
    n, h, m, dt = 64, 0.15, 1.0, 0.015
    desc = {"kind": "random_product", "B": 4, "seed": 3, "radius": 2.0, "prof_lambda": 1.0}
    lat, phi, alt, vel, work = _flow_pair(skyr, n, h, m, dt, prec=1, desc=desc)
    frozen0 = phi.clone()
    st = skyr.anf_state()
    skyr.anf_step(lat, 1, skyr.Model(m), skyr.Flow(dt, 0.0, 640, kr, skyr.ARREST_POWER), phi, alt, vel, st, 640, work)
    assert st.steps == 640 and not st.nonfinite
    p = phi.double().cpu().numpy()
    nrm = np.sqrt((p ** 2).sum(0))
    inner = np.zeros(p.shape[1:], dtype=bool)
    inner[2:-2, 2:-2, 2:-2] = True
    dev = np.abs(nrm[inner] - 1.0).max()
    print(f"kr {kr}: max | |phi| - 1 | = {dev:.3e}")
    assert dev <= 1e-6
    f0 = frozen0.cpu().numpy()
    assert np.array_equal(phi.cpu().numpy()[:, ~inner], f0[:, ~inner])


# ---------------------------------------------------------- edge cases
def test_smallest_lattice(skyr):
    """n = 5: a single interior site."""
    shape, h, m = (5, 5, 5), 0.3, 0.7
    phi = random_unit_field(shape, 2, 0.8)
    lat = _lat(skyr, shape, h)
    g = skyr.new_field(lat, 0, DEV)
    work = skyr.new_workspace(lat, 0, DEV)
    parts = skyr.energy_gradient(lat, 0, skyr.Model(m), _tensor(phi, 0, skyr), work, grad=g)
    ref = oracle.gradient(phi, h, m)
    assert _rel_inf(g.cpu().numpy(), ref) <= 1e-12
    assert parts["E"] == pytest.approx(oracle.energy(phi, h, m), rel=1e-12)


def test_vacuum_does_not_move(skyr):
    n, h = 20, 0.2
    lat = skyr.Lattice.cube(n, h)
    phi = skyr.new_field(lat, 0, DEV)
    phi[0] = 1.0
    alt, vel = skyr.new_field(lat, 0, DEV), skyr.new_field(lat, 0, DEV)
    work = skyr.new_workspace(lat, 0, DEV)
    st = skyr.anf_state()
    skyr.anf_step(lat, 0, skyr.Model(1.0), skyr.Flow(0.05, 1e-12, 100, 0, 0), phi, alt, vel, st, 100, work)
    assert st.converged == 1 and st.steps == 0 and st.E == 0.0
    assert bool((phi[0] == 1).all()) and bool((phi[1:] == 0).all())


def test_nonfinite_input_reports_error(skyr):
    n, h = 16, 0.2
    lat = skyr.Lattice.cube(n, h)
    phi = skyr.new_field(lat, 0, DEV)
    phi[0] = 1.0
    phi[2, 8, 8, 8] = float("nan")
    alt, vel = skyr.new_field(lat, 0, DEV), skyr.new_field(lat, 0, DEV)
    work = skyr.new_workspace(lat, 0, DEV)
    st = skyr.anf_state()
    with pytest.raises(skyr.SkyrError) as e:
        skyr.anf_step(lat, 0, skyr.Model(1.0), skyr.Flow(0.05, 0.0, 10, 0, 0), phi, alt, vel, st, 10, work)
    assert e.value.status == skyr.E_NONFINITE and st.nonfinite == 1


# ------------------------------------------------- full-size sampled checks
def _sample_sites(shape, count, seed):
    rng = np.random.default_rng(seed)
    pts = [tuple(rng.integers(2, s - 2) for s in shape) for _ in range(count)]
    # faces and corners of the interior
    n0, n1, n2 = shape
    pts += [(2, 2, 2), (n0 - 3, n1 - 3, n2 - 3), (2, n1 - 3, 2), (n0 // 2, 2, n2 - 3), (3, 3, 3)]
    return pts


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_random_b10_sampled(skyr, prec):
    """The 256^3 lattice, h = 0.1, random product of 10 unit charges (seed 1),
    in the launch configuration the benchmark times: gradient and one flow
    step on 400 sampled sites, and the total energy, against the oracle."""
    n, h, m, dt = 256, 0.1, 1.0, 0.01
    lat = skyr.Lattice.cube(n, h)
    spec, keep = skyr.spec_from_description({"kind": "random_product", "B": 10, "seed": 1, "radius": 3.0,
                                              "prof_lambda": 1.0})
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    host = phi.double().cpu().numpy()
    work = skyr.new_workspace(lat, prec, DEV)
    g = skyr.new_field(lat, prec, DEV)
    parts = skyr.energy_gradient(lat, prec, skyr.Model(m), phi, work, grad=g)
    gh = g.double().cpu().numpy()
    pts = _sample_sites((n, n, n), 400, 11)
    ref_g = np.array([oracle.gradient_at(host, h, m, *p) for p in pts])
    got_g = np.array([gh[:, p[0], p[1], p[2]] for p in pts])
    scale = np.abs(ref_g).max()
    tol = 1e-12 if prec == 0 else 2e-4
    assert np.abs(got_g - ref_g).max() <= tol * scale
    E = oracle.energy(host, h, m)
    assert parts["E"] == pytest.approx(E, rel=1e-12 if prec == 0 else 2e-6)
    # one flow step from rest
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    st = skyr.anf_state()
    skyr.anf_step(lat, prec, skyr.Model(m), skyr.Flow(dt, 0.0, 10 ** 9, 16, 0), phi, alt, vel, st, 1, work)
    ph = phi.double().cpu().numpy()
    vh = vel.double().cpu().numpy()
    gerr = tol * scale  # bound on the gradient error at a site
    for p, gr in zip(pts, ref_g):
        po, vo = oracle.update_at(host[:, p[0], p[1], p[2]], np.zeros(4), gr, dt)
        rnd = 1e-15 if prec == 0 else 2e-7
        assert np.abs(vh[:, p[0], p[1], p[2]] - vo).max() <= 2 * dt * gerr + rnd * (1 + np.abs(vo).max())
        assert np.abs(ph[:, p[0], p[1], p[2]] - po).max() <= 2 * dt * dt * gerr + 4 * rnd
    assert st.E_prev == pytest.approx(E, rel=1e-12 if prec == 0 else 2e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_largest_lattice_sampled(skyr, prec):
    """The largest cube the 32-bit component offsets allow (812^3 < 2^29 sites;
    813^3 is rejected), filled with 60 unit charges spread over the box:
    gradient and one flow step on sampled sites, the far corner included,
    against the oracle evaluated on 9^3 patches around them (the exact gradient
    at a site reads phi within four sites; patches are cut at the faces)."""
    n, h, m, dt = 812, 0.1, 1.0, 0.01
    assert skyr.workspace_bytes(skyr.Lattice.cube(n + 1, h), prec) == 0  # 813^3: rejected
    lat = skyr.Lattice.cube(n, h)
    assert skyr.workspace_bytes(lat, prec) > 0
    spec, keep = skyr.spec_from_description({"kind": "random_product", "B": 60, "seed": 9, "radius": 36.0,
                                              "prof_lambda": 1.0})
    print(f"largest lattice {n}^3 prec {prec}: init", flush=True)
    phi = skyr.new_field(lat, prec, DEV)
    skyr.init_field(lat, prec, spec, phi)
    work = skyr.new_workspace(lat, prec, DEV)
    g = skyr.new_field(lat, prec, DEV)
    skyr.energy_gradient(lat, prec, skyr.Model(m), phi, work, grad=g, want_parts=False)
    pts = _sample_sites((n, n, n), 120, 13) + [(n - 3, n - 3, n - 4), (n - 5, n - 3, n - 3), (n - 4, 2, n - 3)]

    def patch(t, p):
        lo = [max(0, c - 4) for c in p]
        hi = [min(n, c + 5) for c in p]
        a = t[:, lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].double().cpu().numpy()
        return np.ascontiguousarray(a), tuple(c - l for c, l in zip(p, lo))

    before = [patch(phi, p) for p in pts]
    ref_g = np.array([oracle.gradient_at(a, h, m, *q) for a, q in before])
    got_g = np.array([g[:, p[0], p[1], p[2]].double().cpu().numpy() for p in pts])
    assert np.abs(ref_g).max() > 1.0  # the samples see structure
    scale = np.abs(ref_g).max()
    tol = 1e-12 if prec == 0 else 2e-4
    assert np.abs(got_g - ref_g).max() <= tol * scale
    del g
    print("one flow step", flush=True)
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    st = skyr.anf_state()
    skyr.anf_step(lat, prec, skyr.Model(m), skyr.Flow(dt, 0.0, 10 ** 9, 16, 0), phi, alt, vel, st, 1, work)
    assert st.steps == 1 and np.isfinite(st.E_prev)
    gerr = tol * scale
    rnd = 1e-15 if prec == 0 else 2e-7
    for p, (a, q), gr in zip(pts, before, ref_g):
        po, vo = oracle.update_at(a[:, q[0], q[1], q[2]], np.zeros(4), gr, dt)
        vh = vel[:, p[0], p[1], p[2]].double().cpu().numpy()
        ph = phi[:, p[0], p[1], p[2]].double().cpu().numpy()
        assert np.abs(vh - vo).max() <= 2 * dt * gerr + rnd * (1 + np.abs(vo).max())
        assert np.abs(ph - po).max() <= 2 * dt * dt * gerr + 4 * rnd


@pytest.mark.parametrize("prec", [0, 1])
def test_kinetic_energy_matches_oracle(skyr, prec):
    """Kinetic energy of the velocity after a few flow steps on a ragged lattice
    against the oracle's definition on the same stored values."""
    shape, h = (29, 23, 41), 0.2
    lat = _lat(skyr, shape, h)
    phi = torch.tensor(random_unit_field(shape, 8, 0.3), dtype=skyr.field_dtype(prec), device=DEV)
    alt, vel = skyr.new_field(lat, prec, DEV), skyr.new_field(lat, prec, DEV)
    work = skyr.new_workspace(lat, prec, DEV)
    st = skyr.anf_state()
    skyr.anf_step(lat, prec, skyr.Model(1.0), skyr.Flow(0.01, 0.0, 10 ** 9, 0, skyr.NEWTON_FLOW), phi, alt, vel, st,
                  5, work)
    T = skyr.kinetic_energy(lat, prec, vel, work)
    ref = oracle.kinetic(vel.double().cpu().numpy(), h)
    assert ref > 0
    assert T == pytest.approx(ref, rel=1e-13 if prec == 0 else 1e-12)
