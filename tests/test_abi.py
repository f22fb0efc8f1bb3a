"""Host-side checks of the C ABI: the library loads, exports every symbol
include/skyr.h declares, and rejects invalid arguments before any device work
(no GPU needed: these paths never touch the device)."""
import ctypes
import math
import re
from pathlib import Path

import pytest

from paper_2604_25876_amd import skyr

ROOT = Path(__file__).resolve().parents[1]


def declared_symbols():
    text = (ROOT / "include" / "skyr.h").read_text()
    return sorted(set(re.findall(r"SKYR_API\s+[\w\s\*]+?\b(skyr_\w+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(skyr.exported_symbols())


def test_library_exports_every_declared_symbol():
    L = skyr.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert skyr.version().startswith("skyr")


def test_struct_layouts():
    assert ctypes.sizeof(skyr.Lattice) == 24
    assert ctypes.sizeof(skyr.Model) == 48
    assert ctypes.sizeof(skyr.Flow) == 32
    assert ctypes.sizeof(skyr.Constituent) == 8 + 2 * 9 * 16 + 3 * 8 + 4 * 8 + 16 + 4 * 8
    assert ctypes.sizeof(skyr.Obs) == 64
    assert ctypes.sizeof(skyr.AnfState) == 4 * 8 + 3 * 8 + 4 * 4
    assert ctypes.sizeof(skyr.MomentObs) == 43 * 8


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof of every public struct as the C compiler sees include/skyr.h equals
    the binding's ctypes layout."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    names = {"skyr_lattice": skyr.Lattice, "skyr_model": skyr.Model, "skyr_flow": skyr.Flow,
             "skyr_constituent": skyr.Constituent, "skyr_init_spec": skyr.InitSpec, "skyr_obs": skyr.Obs,
             "skyr_anf_state": skyr.AnfState, "skyr_moment_obs": skyr.MomentObs}
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "skyr.h"\nint main(void){\n' +
                   "".join(f'printf("%zu\\n", sizeof({n}));\n' for n in names) + "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", str(ROOT / "include"), "-o", str(exe), str(src)])
    sizes = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    for (n, cls), sz in zip(names.items(), sizes):
        assert ctypes.sizeof(cls) == sz, n


def test_workspace_bytes():
    lat = skyr.Lattice.cube(256, 0.1)
    for prec in (skyr.F64, skyr.F32_BULK):
        b = skyr.workspace_bytes(lat, prec)
        assert b >= 512 + 1024 * 32 * 8 and b % 64 == 0  # control, observables, moment partial sums
    assert skyr.workspace_bytes(skyr.Lattice.cube(4, 0.1), skyr.F64) == 0
    assert skyr.workspace_bytes(skyr.Lattice.cube(40, -1.0), skyr.F64) == 0
    assert skyr.workspace_bytes(lat, 7) == 0


def test_state_init():
    st = skyr.anf_state()
    assert st.steps == 0 and st.arrests == 0 and math.isinf(st.E_prev) and st.E_prev > 0


def _call(fn, *args):
    return fn(*args)


def test_invalid_arguments_rejected_without_device_work():
    L = skyr.lib()
    lat = skyr.Lattice.cube(40, 0.2)
    bad = skyr.Lattice.cube(4, 0.2)
    model, obs = skyr.Model(1.0), skyr.Obs()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    # null field / workspace
    assert L.skyr_observables(ctypes.byref(lat), 0, ctypes.byref(model), None, ctypes.byref(obs), fake, None) == skyr.E_INVAL
    assert L.skyr_observables(ctypes.byref(lat), 0, ctypes.byref(model), fake, ctypes.byref(obs), None, None) == skyr.E_INVAL
    # lattice too small, bad spacing, bad precision
    assert L.skyr_observables(ctypes.byref(bad), 0, ctypes.byref(model), fake, ctypes.byref(obs), fake, None) == skyr.E_INVAL
    assert "at least 5" in skyr.lib().skyr_last_error().decode()
    neg = skyr.Lattice.cube(40, 0.0)
    assert L.skyr_energy_gradient(ctypes.byref(neg), 0, ctypes.byref(model), fake, None, 0, None, fake, None) == skyr.E_INVAL
    assert L.skyr_energy_gradient(ctypes.byref(lat), 3, ctypes.byref(model), fake, None, 0, None, fake, None) == skyr.E_INVAL
    # misaligned workspace
    mis = ctypes.c_void_p(0x1008)
    assert L.skyr_energy_gradient(ctypes.byref(lat), 0, ctypes.byref(model), fake, None, 0, None, mis, None) == skyr.E_INVAL
    # flow arguments
    st = skyr.anf_state()
    for flow in (skyr.Flow(0.0, 0.0, 10, 0, 0), skyr.Flow(-1.0, 0.0, 10, 0, 0), skyr.Flow(0.1, -1.0, 10, 0, 0),
                 skyr.Flow(0.1, 0.0, -1, 0, 0), skyr.Flow(float("nan"), 0.0, 10, 0, 0),
                 skyr.Flow(0.1, 0.0, 10, 0, 4), skyr.Flow(0.1, 0.0, 10, 0, -1)):
        assert L.skyr_anf_step(ctypes.byref(lat), 0, ctypes.byref(model), ctypes.byref(flow), fake,
                               ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000), ctypes.byref(st), 1, fake,
                               None) == skyr.E_INVAL
    good = skyr.Flow(0.1, 0.0, 10, 0, 0)
    # aliasing buffers
    assert L.skyr_anf_step(ctypes.byref(lat), 0, ctypes.byref(model), ctypes.byref(good), fake, fake,
                           ctypes.c_void_p(0x3000), ctypes.byref(st), 1, fake, None) == skyr.E_INVAL
    assert st.steps == 0 and st.sweeps == 0
    # init spec checks
    spec, keep = skyr.init_spec(skyr.INIT_PRODUCT, [])
    assert L.skyr_init_field(ctypes.byref(lat), 0, ctypes.byref(spec), fake, None) == skyr.E_INVAL
    spec, keep = skyr.init_spec(skyr.INIT_RANDOM_PRODUCT, B=0, seed=1)
    assert L.skyr_init_field(ctypes.byref(lat), 0, ctypes.byref(spec), fake, None) == skyr.E_INVAL
    spec, keep = skyr.init_spec(9)
    assert L.skyr_init_field(ctypes.byref(lat), 0, ctypes.byref(spec), fake, None) == skyr.E_INVAL


def test_noalloc_flow_rejects_a_lattice_beyond_its_scratch():
    """skyr_anf_step_noalloc refuses, before any device work, a flow whose sweep
    has more blocks than its fixed scratch holds partial sums for (here 800^3 in
    single precision with 16-plane slabs: 50 x 25 tiles x 50 slabs, 62,500
    blocks against room for 4084), and checks its other arguments like
    skyr_anf_step."""
    L = skyr.lib()
    lat = skyr.Lattice.cube(800, 0.1)
    skyr.set_tile(lat, skyr.F32_BULK, 0, 16)
    st = skyr.anf_state()
    model, flow = skyr.Model(1.0), skyr.Flow(0.01, 0.0, 10, 0, 0)
    a, b, c = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    rc = L.skyr_anf_step_noalloc(ctypes.byref(lat), skyr.F32_BULK, ctypes.byref(model), ctypes.byref(flow), a, b, c,
                                 ctypes.byref(st), 1, None)
    assert rc == skyr.E_INVAL and "scratch" in L.skyr_last_error().decode()
    small = skyr.Lattice.cube(40, 0.2)
    bad_flow = skyr.Flow(0.0, 0.0, 10, 0, 0)
    assert L.skyr_anf_step_noalloc(ctypes.byref(small), skyr.F64, ctypes.byref(model), ctypes.byref(bad_flow), a, b,
                                   c, ctypes.byref(st), 1, None) == skyr.E_INVAL
    assert L.skyr_anf_step_noalloc(ctypes.byref(small), skyr.F64, ctypes.byref(model), ctypes.byref(flow), a, a, c,
                                   ctypes.byref(st), 1, None) == skyr.E_INVAL
    assert st.steps == 0 and st.sweeps == 0


class _FakeDeviceBuffer:
    """Stands in for a device tensor on the host: only what the binding's
    workspace check reads."""
    is_cuda = True

    def __init__(self, nbytes):
        self.nbytes = nbytes

    def is_contiguous(self):
        return True

    def numel(self):
        return self.nbytes

    def element_size(self):
        return 1

    def data_ptr(self):
        return 0x100000


def test_workspace_size_checked_before_the_call():
    """The C entry points cannot see the size of the workspace they are given;
    the binding refuses one smaller than skyr_workspace_bytes."""
    lat = skyr.Lattice.cube(40, 0.2)
    need = skyr.workspace_bytes(lat, skyr.F64)
    assert skyr._work_ptr(_FakeDeviceBuffer(need), lat, skyr.F64).value == 0x100000
    with pytest.raises(ValueError, match="workspace of"):
        skyr._work_ptr(_FakeDeviceBuffer(need - 1), lat, skyr.F64)
    with pytest.raises(ValueError):
        skyr._work_ptr(None, lat, skyr.F64)


def test_random_constituents_host_side():
    cs = skyr.random_constituents(1, 10, 3.0)
    assert len(cs) == 10
    for c in cs:
        assert sum(v * v for v in c.X) <= 9.0
        assert abs(sum(v * v for v in c.quat) - 1.0) < 1e-15
        assert c.degree == 1 and c.p[1][0] == 1.0 and c.q[0][0] == 1.0
    with pytest.raises(skyr.SkyrError):
        skyr.random_constituents(1, 0)
    with pytest.raises(skyr.SkyrError):
        skyr.random_constituents(1, 65)


def test_random_constituents_match_oracle_draws():
    """The library's SplitMix64 + Shoemake draws equal the oracle's (each side
    implements the generator from its published definition)."""
    import oracle
    for seed, B in ((1, 10), (4, 8), (2 ** 64 - 1, 12)):
        a = skyr.random_constituents(seed, B, 3.0)
        b = oracle.random_constituents(seed, B, 3.0)
        for ca, cb in zip(a, b):
            assert list(ca.X) == list(cb.X)
            assert list(ca.quat) == pytest.approx(list(cb.quat), abs=1e-15)


def test_orientation_zyz_is_the_product_of_axis_rotations():
    """skyr_orientation_zyz(a, b, c) = B with the printed D(B)_ij =
    (1/2) Tr(tau^i B tau^j B^dagger) equal to R_z(a) R_y(b) R_z(c)."""
    import numpy as np
    pauli = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]

    def rz(t):
        return np.array([[math.cos(t), -math.sin(t), 0], [math.sin(t), math.cos(t), 0], [0, 0, 1]])

    def ry(t):
        return np.array([[math.cos(t), 0, math.sin(t)], [0, 1, 0], [-math.sin(t), 0, math.cos(t)]])

    rng = np.random.default_rng(11)
    for a in [(1.57079, 1.57079, -1.57079), (3.14159, 0.0, 0.0)] + [tuple(rng.uniform(-4, 4, 3)) for _ in range(4)]:
        B = skyr.orientation_zyz(*a)
        assert abs(sum(v * v for v in B) - 1.0) < 1e-14 and B[0] >= 0.0
        Bm = B[0] * np.eye(2) + 1j * sum(B[k + 1] * pauli[k] for k in range(3))
        D = np.array([[0.5 * np.trace(pauli[i] @ Bm @ pauli[j] @ Bm.conj().T).real for j in range(3)]
                      for i in range(3)])
        np.testing.assert_allclose(D, rz(a[0]) @ ry(a[1]) @ rz(a[2]), atol=1e-14)


def _default_tile(n, prec):
    """The default tile rule, restated: over the compiled shapes and the even
    splits of x into 1 .. 8 slabs (of at least 16 planes), the pair of least
    estimated cost = rounds of the chip (one block per (slab, tile) item, 256
    CUs times the blocks a CU holds), times 1.15 beyond one round, x rows x
    columns x (slab planes + 4) x a per-shape price, the first on ties; z tiles
    start at z = 0 unless starting at z = 2 saves one."""
    import math
    # (interior waves, columns, blocks per CU), price
    shapes = {skyr.F64: [((4, 16, 1), 1.0), ((4, 32, 1), 1.02), ((6, 32, 1), 0.95)],
              skyr.F32_BULK: [((8, 32, 1), 1.0), ((6, 32, 2), 2.0), ((12, 32, 1), 0.9)]}[prec]
    i = n - 4
    best = None
    for v, ((nwi, oz, per_cu), price) in enumerate(shapes):
        oy = nwi * 64 // oz
        ty = math.ceil(i / oy)
        tz = min((n - 3) // oz + 1, math.ceil(i / oz))
        for sl in range(1, max(1, min(8, i // 16)) + 1):
            xc = math.ceil(i / sl)
            items = ty * tz * math.ceil(i / xc)
            rounds = math.ceil(items / (256 * per_cu))
            cost = rounds * (1.15 if rounds > 1 else 1.0) * oy * oz * (xc + 4) * price
            if best is None or cost < best[0] * (1 - 1e-9):
                best = (cost, v, xc)
    return best[1], max(1, best[2])


@pytest.mark.parametrize("n", [9, 24, 48, 66, 100, 118, 176, 182, 256, 400])
@pytest.mark.parametrize("prec", [0, 1])
def test_default_tile_choice(n, prec):
    """skyr_get_tile on a lattice never set or tuned (host logic only)."""
    lat = skyr.Lattice.cube(n, 0.1)
    assert skyr.get_tile(lat, prec) == _default_tile(n, prec)


def _batch_default_tile(n, prec):
    """The batch default tile rule, restated: the precision's first shape, x split
    evenly into the fewest slabs of at most 64 planes (at least 16 planes each)."""
    import math
    i = n - 4
    slabs = max(1, math.ceil(i / 64))
    return 0, max(min(16, i), math.ceil(i / slabs))


@pytest.mark.parametrize("n", [9, 24, 48, 64, 66, 96, 128, 150, 192, 256, 400])
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_default_tile_choice(n, prec):
    """skyr_get_batch_tile on a lattice never set or tuned for batches (host logic only),
    and a batch setting that changes neither the single-field setting nor the reverse."""
    lat = skyr.Lattice.cube(n, 0.1)
    want = _batch_default_tile(n, prec)
    assert skyr.get_batch_tile(lat, prec) == want
    if n == 150:
        solo = skyr.get_tile(lat, prec)
        skyr.set_batch_tile(lat, prec, 1, 20)
        assert skyr.get_batch_tile(lat, prec) == (1, 20) and skyr.get_tile(lat, prec) == solo
        skyr.set_tile(lat, prec, 2, 30)
        assert skyr.get_batch_tile(lat, prec) == (1, 20) and skyr.get_tile(lat, prec) == (2, 30)
        with pytest.raises(skyr.SkyrError):
            skyr.set_batch_tile(lat, prec, 3, 20)
        with pytest.raises(skyr.SkyrError):
            skyr.set_batch_tile(lat, prec, 0, 15)


@pytest.mark.parametrize("n", [9, 24, 48, 64, 66, 98, 100, 128, 150, 190])
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_layout(n, prec):
    """skyr_batch_layout restated (host logic only): the first tile column of the batch
    tile (z = 0, or z = 2 where that saves a tile) on a 128-byte line, rows of whole
    lines."""
    import math
    line = 16 if prec == skyr.F64 else 32
    oz = 16 if prec == skyr.F64 else 32  # the batch shape's columns
    aligned, inner = (n - 3) // oz + 1, math.ceil((n - 4) / oz)
    zstart = 0 if aligned <= inner else 2
    lead = (line - zstart % line) % line
    pitch = math.ceil((lead + n) / line) * line
    lat = skyr.Lattice((ctypes.c_int32 * 3)(n, n + 1, n), 0, 0.1)
    assert skyr.batch_layout(lat, prec) == (lead, pitch)
    assert (lead + zstart) % line == 0 and pitch % line == 0 and pitch >= lead + n
