"""Plain FP64 CPU oracle for the arrested Newton flow of the 3D Skyrme model.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package; the product library never does.  It
shares no code with the HIP path: the arithmetic lives in ``skyr_oracle.c``
(compiled with gcc, no fast-math, no FMA contraction) and this module only
marshals numpy arrays into it; ``moments.py`` evaluates the moment observables
of Sec. 5 (centre of mass, radius, inertia tensors, quadrupole, D-term) in
numpy on 2x2 complex matrices.

Paper: arXiv:2604.25876 (cuSkyrmion).  Each wrapped routine names the passage
it follows in the C source.  Field arrays are float64 of shape (4, n0, n1, n2),
z fastest; the two outer layers per face are frozen vacuum.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "skyr_oracle.c"
_LIB = _HERE / "liboracle.so"

_lib = None


def build(force: bool = True, sanitize: bool = False, out: Path | None = None) -> Path:
    """Compile the oracle with gcc (plain IEEE double, OpenMP over planes).  sanitize: with
    AddressSanitizer and UndefinedBehaviorSanitizer (into `out`; load that build with
    SKYR_ORACLE_LIB=<out> and gcc's libasan preloaded)."""
    lib = Path(out) if out is not None else (_HERE / "liboracle_san.so" if sanitize else _LIB)
    if force or not lib.exists() or lib.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = lib.with_suffix(".so.tmp")
        extra = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined"] if sanitize else []
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", *extra,
             "-o", str(tmp), str(_SRC), "-lm"])
        os.replace(tmp, lib)
    return lib


class AnfState(ctypes.Structure):
    """Mirror of ora_anf_state."""
    _fields_ = [("steps", ctypes.c_int64), ("arrests", ctypes.c_int64), ("E_prev", ctypes.c_double),
                ("E", ctypes.c_double), ("max_force", ctypes.c_double), ("converged", ctypes.c_int32),
                ("nonfinite", ctypes.c_int32)]

    @classmethod
    def fresh(cls) -> "AnfState":
        return cls(0, 0, math.inf, math.nan, math.nan, 0, 0)


class Constituent(ctypes.Structure):
    """Mirror of ora_constituent: a degree-d rational map p/q with profile
    f(r) = prof_a exp(-r/prof_lambda), centre X and isorotation quaternion."""
    _fields_ = [("degree", ctypes.c_int32), ("_pad", ctypes.c_int32),
                ("p", (ctypes.c_double * 2) * 9), ("q", (ctypes.c_double * 2) * 9),
                ("X", ctypes.c_double * 3), ("quat", ctypes.c_double * 4),
                ("prof_a", ctypes.c_double), ("prof_lambda", ctypes.c_double), ("orient", ctypes.c_double * 4)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    override = os.environ.get("SKYR_ORACLE_LIB")  # another build to load (the sanitizer runs)
    if override:
        lib = ctypes.CDLL(override)
    else:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        lib = ctypes.CDLL(str(_LIB))
    i3 = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
    sig = {
        "ora_first_derivatives": (None, [i3, d, dp, dp]),
        "ora_laplacian": (None, [i3, d, dp, dp]),
        "ora_energy_parts": (None, [i3, d, dp, dp, dp]),
        "ora_energy": (d, [i3, d, dp, dp]),
        "ora_flux": (None, [i3, d, dp, dp]),
        "ora_gradient": (None, [i3, d, dp, dp, dp]),
        "ora_project": (d, [i3, dp, dp, dp]),
        "ora_gradient_at": (None, [i3, d, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]),
        "ora_baryon": (d, [i3, d, dp]),
        "ora_observables": (None, [i3, d, dp, dp, dp]),
        "ora_update_at": (None, [dp, dp, dp, d, ctypes.c_int, dp, dp]),
        "ora_power": (d, [i3, d, dp, dp]),
        "ora_anf": (i64, [i3, d, dp, d, d, i64, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.POINTER(AnfState), dp,
                          ctypes.POINTER(i32)]),
        "ora_init_product": (None, [i3, d, i32, ctypes.POINTER(Constituent), dp]),
        "ora_splitmix64": (ctypes.c_uint64, [ctypes.c_uint64, i64]),
        "ora_random_constituents": (None, [ctypes.c_uint64, i32, d, d, d, ctypes.POINTER(Constituent)]),
        "ora_gradient_literal": (None, [i3, d, dp, dp, dp]),
        "ora_num_threads": (ctypes.c_int, []),
        "ora_set_num_threads": (None, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _mass(m) -> ctypes.Array:
    """Model constants {m, m_y, m_z, m_w, c6}: a float is the pion mass m alone;
    a sequence gives the potential masses and, fifth, the sextic coefficient."""
    vals = [float(m)] if np.isscalar(m) else [float(v) for v in m]
    if not 1 <= len(vals) <= 5:
        raise ValueError("give the pion mass, or up to four potential masses and c6")
    return (ctypes.c_double * 5)(*(vals + [0.0] * (5 - len(vals))))


def _dims(shape) -> ctypes.Array:
    return (ctypes.c_int * 3)(*[int(s) for s in shape])


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _field(phi) -> np.ndarray:
    a = np.ascontiguousarray(phi, dtype=np.float64)
    if a.ndim != 4 or a.shape[0] != 4:
        raise ValueError("field must have shape (4, n0, n1, n2)")
    return a


def num_threads() -> int:
    return _load().ora_num_threads()


def set_num_threads(t: int) -> None:
    _load().ora_set_num_threads(int(t))


# ---------------------------------------------------------------- derivatives
def first_derivatives(phi, h: float) -> np.ndarray:
    """D_i phi^A on the interior (zero elsewhere), shape (3, 4, n0, n1, n2)."""
    phi = _field(phi)
    a = np.empty((3,) + phi.shape, dtype=np.float64)
    _load().ora_first_derivatives(_dims(phi.shape[1:]), h, _ptr(phi), _ptr(a))
    return a


def laplacian(phi, h: float) -> np.ndarray:
    """Lap_h phi^A (five-point second differences summed over axes) on the
    interior, zero elsewhere, shape (4, n0, n1, n2)."""
    phi = _field(phi)
    lap = np.empty_like(phi)
    _load().ora_laplacian(_dims(phi.shape[1:]), h, _ptr(phi), _ptr(lap))
    return lap


# --------------------------------------------------------------------- energy
def energy_parts(phi, h: float, m) -> tuple[float, float, float, float]:
    """(E2, E4, E0, E6) of the discrete energy E_h = h^3 sum_I e."""
    phi = _field(phi)
    out = np.zeros(4)
    _load().ora_energy_parts(_dims(phi.shape[1:]), h, _mass(m), _ptr(phi), _ptr(out))
    return float(out[0]), float(out[1]), float(out[2]), float(out[3])


def energy(phi, h: float, m: float) -> float:
    phi = _field(phi)
    return float(_load().ora_energy(_dims(phi.shape[1:]), h, _mass(m), _ptr(phi)))


# ------------------------------------------------------------------- gradient
def flux(phi, h: float) -> np.ndarray:
    """Quartic flux Q_i^A = de4/da_i^A on the interior (zero elsewhere),
    shape (3, 4, n0, n1, n2)."""
    phi = _field(phi)
    P = np.empty((3,) + phi.shape, dtype=np.float64)
    _load().ora_flux(_dims(phi.shape[1:]), h, _ptr(phi), _ptr(P))
    return P


def gradient(phi, h: float, m: float) -> np.ndarray:
    """g = h^-3 dE_h/dphi on the interior, zero on the frozen layers."""
    phi = _field(phi)
    g = np.empty_like(phi)
    _load().ora_gradient(_dims(phi.shape[1:]), h, _mass(m), _ptr(phi), _ptr(g))
    return g


def project(phi, g) -> tuple[np.ndarray, float]:
    """Tangential part gT = g - (g.phi) phi and max over the interior of |gT|."""
    phi = _field(phi)
    g = _field(g)
    gT = np.empty_like(phi)
    r = _load().ora_project(_dims(phi.shape[1:]), _ptr(phi), _ptr(g), _ptr(gT))
    return gT, float(r)


def power(gT, vel, h: float) -> float:
    """h^3 sum over the interior of F . v with F = -gT (dE/dt along v is -power)."""
    gT = _field(gT)
    vel = _field(vel)
    return float(_load().ora_power(_dims(gT.shape[1:]), h, _ptr(gT), _ptr(vel)))


def gradient_at(phi, h: float, m: float, x: int, y: int, z: int) -> np.ndarray:
    """g at one interior site, from the flux at its stencil neighbours."""
    phi = _field(phi)
    g = np.zeros(4)
    _load().ora_gradient_at(_dims(phi.shape[1:]), h, _mass(m), _ptr(phi), int(x), int(y), int(z), _ptr(g))
    return g


def gradient_literal(phi, h: float, m: float) -> np.ndarray:
    """The paper's printed Euler-Lagrange expression (halved), five-point second
    derivatives and D_i D_j mixed derivatives, on the interior (zero on the
    frozen layers)."""
    phi = _field(phi)
    g = np.empty_like(phi)
    _load().ora_gradient_literal(_dims(phi.shape[1:]), h, _mass(m), _ptr(phi), _ptr(g))
    return g


def update_at(phi4, vel4, g4, dt: float, zero_v: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """One kick-drift-renormalise update at a single site."""
    p = np.ascontiguousarray(phi4, dtype=np.float64)
    v = np.ascontiguousarray(vel4, dtype=np.float64)
    g = np.ascontiguousarray(g4, dtype=np.float64)
    po, vo = np.zeros(4), np.zeros(4)
    _load().ora_update_at(_ptr(p), _ptr(v), _ptr(g), dt, int(bool(zero_v)), _ptr(po), _ptr(vo))
    return po, vo


# ---------------------------------------------------------------- observables
def baryon(phi, h: float) -> float:
    phi = _field(phi)
    return float(_load().ora_baryon(_dims(phi.shape[1:]), h, _ptr(phi)))


def observables(phi, h: float, m) -> dict:
    """{E, E2, E4, E0, B, virial, max_force, E6}; virial = E2 - E4 + 3 E0 - 3 E6."""
    phi = _field(phi)
    out = np.zeros(8)
    _load().ora_observables(_dims(phi.shape[1:]), h, _mass(m), _ptr(phi), _ptr(out))
    keys = ("E", "E2", "E4", "E0", "B", "virial", "max_force", "E6")
    return {k: float(v) for k, v in zip(keys, out)}


def kinetic(vel, h: float) -> float:
    """Kinetic energy of a flow velocity, (1/2) h^3 sum over I of |v|^2 (the
    definition; this library's normalisation)."""
    v = _field(vel)[:, 2:-2, 2:-2, 2:-2]
    return float(0.5 * h ** 3 * np.sum(v * v))


# ------------------------------------------------------------------------ ANF
def anf(phi, vel, h: float, m: float, dt: float, tol: float, target_steps: int, state: AnfState | None = None,
        arrest: bool = True, trace: bool = False, rule: str = "energy", form: str = "exact"):
    """Arrested Newton flow, in place on (phi, vel), until state.steps reaches
    target_steps, max|F| < tol, or a non-finite value.  rule = "energy"
    (arrest when E_n > E_{n-1}), "power" (arrest when h^3 sum F_n . v_n < 0)
    or "gradient" (the first-order gradient flow, no velocity); arrest=False
    with an arrest rule gives the plain Newton flow.  m: the pion mass, or the
    four potential masses (m_x, m_y, m_z, m_w).  form = "exact" (the derivative
    of the discrete energy) or "printed" (the printed Euler-Lagrange expression,
    gradient_literal) for the force.
    Returns (phi, vel, state, E_trace, arrest_trace); traces are None unless trace."""
    if rule not in ("energy", "power", "gradient"):
        raise ValueError(f"unknown flow rule {rule!r}")
    if form not in ("exact", "printed"):
        raise ValueError(f"unknown gradient form {form!r}")
    phi = _field(phi).copy()
    vel = _field(vel).copy()
    st = AnfState.fresh() if state is None else state
    n_max = max(int(target_steps) - int(st.steps), 0) + 1
    Et = np.full(n_max, np.nan) if trace else None
    At = np.zeros(n_max, dtype=np.int32) if trace else None
    mode = 3 if rule == "gradient" else (0 if not arrest else (1 if rule == "energy" else 2))
    nev = _load().ora_anf(_dims(phi.shape[1:]), h, _mass(m), dt, tol, int(target_steps), mode,
                          int(form == "printed"), _ptr(phi),
                          _ptr(vel), ctypes.byref(st), _ptr(Et) if trace else None,
                          At.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if trace else None)
    if trace:
        Et, At = Et[:nev], At[:nev]
    return phi, vel, st, Et, At


# ------------------------------------------------------------------------ init
def constituent(degree: int, p, q, X=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), prof_a: float = math.pi,
                prof_lambda: float = 1.0, orient=None) -> Constituent:
    """Build a constituent from complex coefficient lists p, q (index = power of z);
    orient: quaternion of its spatial rotation (None: unturned)."""
    c = Constituent()
    c.degree = int(degree)
    for k, v in enumerate(p):
        c.p[k][0], c.p[k][1] = complex(v).real, complex(v).imag
    for k, v in enumerate(q):
        c.q[k][0], c.q[k][1] = complex(v).real, complex(v).imag
    c.X[:] = list(map(float, X))
    c.quat[:] = list(map(float, quat))
    c.prof_a, c.prof_lambda = float(prof_a), float(prof_lambda)
    c.orient[:] = [0.0] * 4 if orient is None else list(map(float, orient))
    return c


def hedgehog(X=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), prof_a=math.pi, prof_lambda=1.0,
             orient=None) -> Constituent:
    """R(z) = z (Table RMA, B = 1)."""
    return constituent(1, [0, 1], [1], X, quat, prof_a, prof_lambda, orient)


def cube_b4(X=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), prof_a=math.pi, prof_lambda=1.0,
            orient=None) -> Constituent:
    """R(z) = (z^4 + 2 sqrt3 i z^2 + 1)/(z^4 - 2 sqrt3 i z^2 + 1) (Table RMA, B = 4, O_h)."""
    s = 2.0 * math.sqrt(3.0) * 1j
    return constituent(4, [1, 0, s, 0, 1], [1, 0, -s, 0, 1], X, quat, prof_a, prof_lambda, orient)


def init_product(shape, h: float, constituents) -> np.ndarray:
    """Product ansatz of the constituents, left to right; vacuum frozen layers."""
    cs = list(constituents)
    arr = (Constituent * max(len(cs), 1))(*cs)
    phi = np.empty((4,) + tuple(int(s) for s in shape), dtype=np.float64)
    _load().ora_init_product(_dims(shape), h, len(cs), arr, _ptr(phi))
    return phi


def random_constituents(seed: int, B: int, radius: float = 3.0, prof_a: float = math.pi,
                        prof_lambda: float = 1.0) -> list[Constituent]:
    """B hedgehogs with SplitMix64-drawn centres in a ball and Shoemake quaternions."""
    arr = (Constituent * int(B))()
    _load().ora_random_constituents(int(seed) & 0xFFFFFFFFFFFFFFFF, int(B), radius, prof_a, prof_lambda, arr)
    return list(arr)


def splitmix64(seed: int, k: int) -> int:
    """k-th (0-based) SplitMix64 output for the seed."""
    return int(_load().ora_splitmix64(int(seed) & 0xFFFFFFFFFFFFFFFF, int(k)))
