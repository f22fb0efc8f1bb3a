"""Thin ctypes binding of libskyr.so (include/skyr.h).

Argument marshalling only: every step of the flow runs in the HIP library.
Field tensors are torch tensors on a ROCm device, shape (4, n0, n1, n2),
contiguous, float64 (F64) or float32 (F32_BULK); workspaces are uint8 device
tensors of workspace_bytes(...) bytes.  Streams default to torch's current
stream.  Every function raises SkyrError when the library returns an error.
"""
from __future__ import annotations

import ctypes
import math
import os
from pathlib import Path

_PKG = Path(__file__).resolve().parent
# SKYR_LIB names another build of the library to load instead (the sanitizer runs of the
# CPU tests use it)
LIB_PATH = Path(os.environ.get("SKYR_LIB") or (_PKG / "libskyr.so"))

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NONFINITE, E_BUSY, E_IO = 0, -1, -2, -3, -4, -5, -6
FILE_BINARY, FILE_TEXT = 0, 1
FORM_EXACT, FORM_PRINTED = 0, 1
F64, F32_BULK = 0, 1
ARREST_ENERGY, ARREST_POWER, NEWTON_FLOW, GRADIENT_FLOW = 0, 1, 2, 3
_FLOW_MODES = {"energy": ARREST_ENERGY, "power": ARREST_POWER, "newton": NEWTON_FLOW, "gradient": GRADIENT_FLOW}


def flow_mode(mode) -> int:
    """skyr_flow_mode value of "energy" / "power" (arrested Newton flow with that
    arrest rule), "newton" or "gradient" (or of the value itself)."""
    if isinstance(mode, str):
        return _FLOW_MODES[mode]
    return int(mode)
INIT_HEDGEHOG, INIT_RATIONAL_MAP, INIT_PRODUCT, INIT_RANDOM_PRODUCT = 0, 1, 2, 3


class SkyrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"skyr status {status}: {msg}")
        self.status = status


class Lattice(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("_pad", ctypes.c_int32), ("h", ctypes.c_double)]

    @classmethod
    def cube(cls, n: int, h: float) -> "Lattice":
        return cls((ctypes.c_int32 * 3)(n, n, n), 0, float(h))

    @property
    def shape(self) -> tuple[int, int, int]:
        return tuple(int(v) for v in self.n)


class Model(ctypes.Structure):
    """Couplings: the pion mass m, the optional masses m_y, m_z, m_w, the sextic
    weight c6, and the form of the force (FORM_EXACT or FORM_PRINTED)."""
    _fields_ = [("m", ctypes.c_double), ("m_y", ctypes.c_double), ("m_z", ctypes.c_double),
                ("m_w", ctypes.c_double), ("c6", ctypes.c_double), ("form", ctypes.c_int32),
                ("_pad", ctypes.c_int32)]


class Flow(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("tol", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("renorm64_every", ctypes.c_int32), ("mode", ctypes.c_int32)]


class Constituent(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("_pad", ctypes.c_int32),
                ("p", (ctypes.c_double * 2) * 9), ("q", (ctypes.c_double * 2) * 9),
                ("X", ctypes.c_double * 3), ("quat", ctypes.c_double * 4),
                ("prof_a", ctypes.c_double), ("prof_lambda", ctypes.c_double), ("orient", ctypes.c_double * 4)]


class InitSpec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("count", ctypes.c_int32), ("c", ctypes.POINTER(Constituent)),
                ("B", ctypes.c_int32), ("_pad", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("ball_radius", ctypes.c_double), ("prof_a", ctypes.c_double), ("prof_lambda", ctypes.c_double)]


class Obs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("E", "E2", "E4", "E0", "B", "virial", "max_force", "E6")]

    def as_dict(self) -> dict:
        return {k: float(getattr(self, k)) for k, _ in self._fields_}


class MomentObs(ctypes.Structure):
    """Mirror of skyr_moment_obs: B, E (printed normalisation), X, R and the
    row-major 3x3 tensors U, V, W, Q, then D."""
    _fields_ = [("B", ctypes.c_double), ("E", ctypes.c_double), ("X", ctypes.c_double * 3), ("R", ctypes.c_double),
                ("U", ctypes.c_double * 9), ("V", ctypes.c_double * 9), ("W", ctypes.c_double * 9),
                ("Q", ctypes.c_double * 9), ("D", ctypes.c_double)]

    def as_dict(self) -> dict:
        import numpy as np
        out = {k: float(getattr(self, k)) for k in ("B", "E", "R", "D")}
        out["X"] = np.array(list(self.X))
        for k in ("U", "V", "W", "Q"):
            out[k] = np.array(list(getattr(self, k))).reshape(3, 3)
        return out


class AnfState(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("arrests", ctypes.c_int64), ("redo_sweeps", ctypes.c_int64),
                ("sweeps", ctypes.c_int64), ("E_prev", ctypes.c_double), ("E", ctypes.c_double),
                ("max_force", ctypes.c_double), ("converged", ctypes.c_int32), ("redo_pending", ctypes.c_int32),
                ("nonfinite", ctypes.c_int32), ("_pad", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: (getattr(self, k)) for k, _ in self._fields_ if not k.startswith("_")}


class Block(ctypes.Structure):
    """Mirror of skyr_block: the whole lattice, the block's first own site per axis and
    its own sites per axis.  Block fields are stored padded, extent + 8 sites per axis."""
    _fields_ = [("lattice", Lattice), ("origin", ctypes.c_int32 * 3), ("extent", ctypes.c_int32 * 3)]

    @classmethod
    def of(cls, lat: Lattice, origin, extent) -> "Block":
        return cls(lat, (ctypes.c_int32 * 3)(*origin), (ctypes.c_int32 * 3)(*extent))

    @property
    def padded_shape(self) -> tuple[int, int, int]:
        return tuple(int(e) + 8 for e in self.extent)


class BlockSums(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("E", "E2", "E4", "E0", "E6", "power", "max_force")]

    def as_dict(self) -> dict:
        return {k: float(getattr(self, k)) for k, _ in self._fields_}


BLOCK_GRADIENT, BLOCK_STEP = 0, 1

_lib = None

# exported symbols and their signatures (the list the ABI tests check)
_P = ctypes.c_void_p
_SIGNATURES = {
    "skyr_version": (ctypes.c_char_p, []),
    "skyr_last_error": (ctypes.c_char_p, []),
    "skyr_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Lattice), ctypes.c_int]),
    "skyr_random_constituents": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.POINTER(Constituent)]),
    "skyr_init_field": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(InitSpec), _P, _P]),
    "skyr_energy_gradient": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model), _P, _P,
                                            ctypes.c_int32, ctypes.POINTER(Obs), _P, _P]),
    "skyr_anf_state_init": (None, [ctypes.POINTER(AnfState)]),
    "skyr_anf_step": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model),
                                     ctypes.POINTER(Flow), _P, _P, _P, ctypes.POINTER(AnfState), ctypes.c_int64, _P,
                                     _P]),
    "skyr_anf_step_padded": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model),
                                            ctypes.POINTER(Flow), _P, _P, _P, ctypes.POINTER(AnfState),
                                            ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_int32, _P]),
    "skyr_anf_step_noalloc": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model),
                                             ctypes.POINTER(Flow), _P, _P, _P, ctypes.POINTER(AnfState),
                                             ctypes.c_int64, _P]),
    "skyr_write_field_host": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(Lattice),
                                             ctypes.POINTER(Model), _P]),
    "skyr_read_field_host": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(Lattice), ctypes.POINTER(Model), _P]),
    "skyr_file_info": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(Lattice), ctypes.POINTER(Model)]),
    "skyr_save_field": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(Lattice), ctypes.c_int,
                                       ctypes.POINTER(Model), _P, _P]),
    "skyr_load_field": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(Lattice), ctypes.c_int,
                                       ctypes.POINTER(Model), _P, _P]),
    "skyr_orientation_zyz": (None, [ctypes.POINTER(ctypes.c_double * 3), ctypes.POINTER(ctypes.c_double * 4)]),
    "skyr_kinetic_energy": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, _P, ctypes.POINTER(ctypes.c_double),
                                           _P, _P]),
    "skyr_moments": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model), _P,
                                    ctypes.POINTER(MomentObs), _P, _P]),
    "skyr_observables": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model), _P,
                                        ctypes.POINTER(Obs), _P, _P]),
    "skyr_tile_variants": (ctypes.c_int32, [ctypes.c_int]),
    "skyr_tile_variant_info": (ctypes.c_int, [ctypes.c_int, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "skyr_set_tile": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.c_int32, ctypes.c_int32]),
    "skyr_get_tile": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "skyr_autotune": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model),
                                     ctypes.POINTER(Flow), _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "skyr_set_batch_tile": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.c_int32, ctypes.c_int32]),
    "skyr_get_batch_tile": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]),
    "skyr_batch_autotune": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model),
                                           ctypes.POINTER(Flow), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32, _P,
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double)]),
    "skyr_batch_create": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_void_p)]),
    "skyr_batch_add": (ctypes.c_int, [_P, ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model),
                                      ctypes.POINTER(Flow), _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "skyr_batch_layout": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]),
    "skyr_batch_add_padded": (ctypes.c_int, [_P, ctypes.POINTER(Lattice), ctypes.c_int, ctypes.POINTER(Model),
                                             ctypes.POINTER(Flow), _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_int32)]),
    "skyr_batch_run": (ctypes.c_int, [_P, ctypes.c_int32]),
    "skyr_batch_poll": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(AnfState)]),
    "skyr_batch_remove": (ctypes.c_int, [_P, ctypes.c_int32]),
    "skyr_batch_active": (ctypes.c_int32, [_P]),
    "skyr_batch_destroy": (ctypes.c_int, [_P]),
    "skyr_block_sites": (ctypes.c_int64, [ctypes.POINTER(Block)]),
    "skyr_block_shell_sites": (ctypes.c_int64, [ctypes.POINTER(Block)]),
    "skyr_block_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Block), ctypes.c_int]),
    "skyr_block_sweep": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_int, ctypes.POINTER(Model), ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _P, _P, _P,
                                        _P, ctypes.POINTER(BlockSums), _P, _P]),
    "skyr_block_sweep_padded": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_int, ctypes.POINTER(Model),
                                               ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                               ctypes.c_int32, _P, _P, _P, _P, ctypes.POINTER(BlockSums), _P,
                                               ctypes.c_int32, ctypes.c_int32, _P]),
    "skyr_block_layout": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]),
    "skyr_timing_enable": (None, [ctypes.c_int32]),
    "skyr_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
}


def lib() -> ctypes.CDLL:
    """Load libskyr.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                               "python paper_2604_25876_amd/build.py")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    return list(_SIGNATURES)


def _check(status: int) -> None:
    if status != OK:
        msg = lib().skyr_last_error().decode(errors="replace")
        raise SkyrError(status, msg)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype=None, shape=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"tensor dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"tensor shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _work_ptr(work, lat: Lattice, prec: int):
    """The workspace pointer, after checking on the host that the tensor is a
    contiguous device buffer of at least workspace_bytes(lat, prec) bytes (the
    library cannot see the size of what it is given; it checks the alignment)."""
    if work is None:
        raise ValueError("a workspace is required")
    if not work.is_cuda or not work.is_contiguous():
        raise ValueError("workspace must be a contiguous GPU tensor")
    need = workspace_bytes(lat, prec)
    have = work.numel() * work.element_size()
    if have < need:
        raise ValueError(f"workspace of {have} bytes, this lattice and precision need {need}")
    return ctypes.c_void_p(work.data_ptr())


def field_dtype(prec: int):
    import torch
    return torch.float64 if prec == F64 else torch.float32


def version() -> str:
    return lib().skyr_version().decode()


def workspace_bytes(lat: Lattice, prec: int) -> int:
    return int(lib().skyr_workspace_bytes(ctypes.byref(lat), prec))


def new_field(lat: Lattice, prec: int, device="cuda"):
    import torch
    return torch.zeros((4,) + lat.shape, dtype=field_dtype(prec), device=device)


def new_workspace(lat: Lattice, prec: int, device="cuda"):
    import torch
    return torch.empty(workspace_bytes(lat, prec), dtype=torch.uint8, device=device)


def constituent(degree: int, p, q, X=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), prof_a: float = math.pi,
                prof_lambda: float = 1.0, orient=None) -> Constituent:
    """A rational-map constituent; orient: spatial orientation quaternion
    (None = unrotated), e.g. from orientation_zyz."""
    c = Constituent()
    c.degree = int(degree)
    for k, v in enumerate(p):
        c.p[k][0], c.p[k][1] = complex(v).real, complex(v).imag
    for k, v in enumerate(q):
        c.q[k][0], c.q[k][1] = complex(v).real, complex(v).imag
    c.X[:] = [float(v) for v in X]
    c.quat[:] = [float(v) for v in quat]
    c.prof_a, c.prof_lambda = float(prof_a), float(prof_lambda)
    c.orient[:] = [0.0] * 4 if orient is None else [float(v) for v in orient]
    return c


def orientation_zyz(a1: float, a2: float, a3: float) -> tuple:
    """Quaternion B with D(B) = R_z(a1) R_y(a2) R_z(a3) (skyr_orientation_zyz)."""
    ang, out = (ctypes.c_double * 3)(a1, a2, a3), (ctypes.c_double * 4)()
    lib().skyr_orientation_zyz(ang, out)
    return tuple(out)


def random_constituents(seed: int, B: int, radius: float = 3.0, prof_a: float = math.pi,
                        prof_lambda: float = 1.0) -> list[Constituent]:
    arr = (Constituent * int(B))()
    _check(lib().skyr_random_constituents(int(seed) & 0xFFFFFFFFFFFFFFFF, int(B), radius, prof_a, prof_lambda, arr))
    return list(arr)


def init_spec(kind: int, constituents=None, B: int = 0, seed: int = 0, ball_radius: float = 3.0,
              prof_a: float = math.pi, prof_lambda: float = 1.0):
    """Build an InitSpec; returns (spec, keepalive) -- keep the second value
    alive while the spec is in use."""
    cs = list(constituents or [])
    arr = (Constituent * max(len(cs), 1))(*cs) if cs else None
    spec = InitSpec(kind, len(cs), ctypes.cast(arr, ctypes.POINTER(Constituent)) if arr is not None else None,
                    int(B), 0, int(seed) & 0xFFFFFFFFFFFFFFFF, float(ball_radius), float(prof_a), float(prof_lambda))
    return spec, arr


def init_field(lat: Lattice, prec: int, spec: InitSpec, phi, stream=None) -> None:
    _check(lib().skyr_init_field(ctypes.byref(lat), prec, ctypes.byref(spec),
                                 _dev_ptr(phi, field_dtype(prec), (4,) + lat.shape), _stream(stream)))


def energy_gradient(lat: Lattice, prec: int, model: Model, phi, work, grad=None, projected: bool = False,
                    want_parts: bool = True, stream=None):
    obs = Obs()
    shape = (4,) + lat.shape
    _check(lib().skyr_energy_gradient(ctypes.byref(lat), prec, ctypes.byref(model),
                                      _dev_ptr(phi, field_dtype(prec), shape),
                                      _dev_ptr(grad, field_dtype(prec), shape), int(bool(projected)),
                                      ctypes.byref(obs) if want_parts else None, _work_ptr(work, lat, prec), _stream(stream)))
    return obs.as_dict() if want_parts else None


def anf_state() -> AnfState:
    st = AnfState()
    lib().skyr_anf_state_init(ctypes.byref(st))
    return st


def anf_step(lat: Lattice, prec: int, model: Model, flow: Flow, phi, phi_alt, vel, state: AnfState, nsteps: int,
             work, stream=None) -> AnfState:
    shape = (4,) + lat.shape
    dt = field_dtype(prec)
    _check(lib().skyr_anf_step(ctypes.byref(lat), prec, ctypes.byref(model), ctypes.byref(flow),
                               _dev_ptr(phi, dt, shape), _dev_ptr(phi_alt, dt, shape), _dev_ptr(vel, dt, shape),
                               ctypes.byref(state), int(nsteps), _work_ptr(work, lat, prec), _stream(stream)))
    return state


def anf_step_padded(lat: Lattice, prec: int, model: Model, flow: Flow, phi, phi_alt, vel, state: AnfState,
                    nsteps: int, work, layout: tuple[int, int], stream=None) -> AnfState:
    """skyr_anf_step on fields in the padded, row-interleaved layout (n0, n1, 4, pitch) of
    batch_layout / to_padded."""
    lead, pitch = (int(v) for v in layout)
    shape = lat.shape[:2] + (4, pitch)
    dt = field_dtype(prec)
    _check(lib().skyr_anf_step_padded(ctypes.byref(lat), prec, ctypes.byref(model), ctypes.byref(flow),
                                      _dev_ptr(phi, dt, shape), _dev_ptr(phi_alt, dt, shape),
                                      _dev_ptr(vel, dt, shape), ctypes.byref(state), int(nsteps),
                                      _work_ptr(work, lat, prec), lead, pitch, _stream(stream)))
    return state


def anf_step_noalloc(lat: Lattice, prec: int, model: Model, flow: Flow, phi, phi_alt, vel, state: AnfState,
                     nsteps: int, stream=None) -> AnfState:
    """skyr_anf_step_noalloc: the flow with the library's fixed device scratch as
    its workspace (nothing is allocated)."""
    shape = (4,) + lat.shape
    dt = field_dtype(prec)
    _check(lib().skyr_anf_step_noalloc(ctypes.byref(lat), prec, ctypes.byref(model), ctypes.byref(flow),
                                       _dev_ptr(phi, dt, shape), _dev_ptr(phi_alt, dt, shape),
                                       _dev_ptr(vel, dt, shape), ctypes.byref(state), int(nsteps), _stream(stream)))
    return state


def block_sites(blk: Block) -> int:
    return int(lib().skyr_block_sites(ctypes.byref(blk)))


def block_shell_sites(blk: Block) -> int:
    return int(lib().skyr_block_shell_sites(ctypes.byref(blk)))


def block_workspace_bytes(blk: Block, prec: int) -> int:
    return int(lib().skyr_block_workspace_bytes(ctypes.byref(blk), prec))


def new_block_field(blk: Block, prec: int, device="cuda"):
    import torch
    return torch.zeros((4,) + blk.padded_shape, dtype=field_dtype(prec), device=device)


def new_block_workspace(blk: Block, prec: int, device="cuda"):
    import torch
    return torch.zeros(block_workspace_bytes(blk, prec), dtype=torch.uint8, device=device)


def block_sweep(blk: Block, prec: int, model: Model, mode: int, phi, shell, out, vel=None, work=None,
                projected: bool = False, dt: float = 0.0, redo: bool = False, renorm64: bool = False,
                want_sums: bool = True, stream=None, layout: tuple[int, int] | None = None):
    """skyr_block_sweep: one sweep over a block's own interior sites (gradient or one
    kick-drift step) with its shell written from `shell`; returns the block's sums
    (a dict) when want_sums, else None.  With a layout (block_layout), phi, out and vel
    are in the padded, row-interleaved layout (P0, P1, 4, pitch) of skyr_block_sweep_padded."""
    shape = (4,) + blk.padded_shape if layout is None else blk.padded_shape[:2] + (4, int(layout[1]))
    dt_ = field_dtype(prec)
    if work is None or not work.is_cuda or work.numel() * work.element_size() < block_workspace_bytes(blk, prec):
        raise ValueError("a device workspace of block_workspace_bytes(blk, prec) bytes is required")
    sums = BlockSums()
    args = (ctypes.byref(blk), prec, ctypes.byref(model), int(mode), int(bool(projected)), float(dt),
            int(bool(redo)), int(bool(renorm64)), _dev_ptr(phi, dt_, shape),
            _dev_ptr(shell, dt_, (4, block_shell_sites(blk))), _dev_ptr(out, dt_, shape), _dev_ptr(vel, dt_, shape),
            ctypes.byref(sums) if want_sums else None, ctypes.c_void_p(work.data_ptr()))
    if layout is None:
        _check(lib().skyr_block_sweep(*args, _stream(stream)))
    else:
        _check(lib().skyr_block_sweep_padded(*args, int(layout[0]), int(layout[1]), _stream(stream)))
    return sums.as_dict() if want_sums else None


def block_layout(blk: Block, prec: int) -> tuple[int, int]:
    """(lead, pitch): the padded, row-interleaved layout of block fields for skyr_block_sweep_padded."""
    lead, pitch = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().skyr_block_layout(ctypes.byref(blk), prec, ctypes.byref(lead), ctypes.byref(pitch)))
    return int(lead.value), int(pitch.value)


def observables(lat: Lattice, prec: int, model: Model, phi, work, stream=None) -> dict:
    obs = Obs()
    _check(lib().skyr_observables(ctypes.byref(lat), prec, ctypes.byref(model),
                                  _dev_ptr(phi, field_dtype(prec), (4,) + lat.shape), ctypes.byref(obs),
                                  _work_ptr(work, lat, prec), _stream(stream)))
    return obs.as_dict()


def kinetic_energy(lat: Lattice, prec: int, vel, work, stream=None) -> float:
    """(1/2) h^3 sum over the interior of |v|^2 (skyr_kinetic_energy)."""
    out = ctypes.c_double()
    _check(lib().skyr_kinetic_energy(ctypes.byref(lat), prec, _dev_ptr(vel, field_dtype(prec), (4,) + lat.shape),
                                     ctypes.byref(out), _work_ptr(work, lat, prec), _stream(stream)))
    return float(out.value)


def moments(lat: Lattice, prec: int, model: Model, phi, work, stream=None) -> dict:
    """Centre of mass, RMS radius, inertia tensors U, V, W, quadrupole Q and
    D-term of phi (skyr_moments); tensors as 3x3 numpy arrays."""
    out = MomentObs()
    _check(lib().skyr_moments(ctypes.byref(lat), prec, ctypes.byref(model),
                              _dev_ptr(phi, field_dtype(prec), (4,) + lat.shape), ctypes.byref(out),
                              _work_ptr(work, lat, prec), _stream(stream)))
    return out.as_dict()


def _fmt(fmt) -> int:
    return {"binary": FILE_BINARY, "text": FILE_TEXT}[fmt] if isinstance(fmt, str) else int(fmt)


def write_field_host(path, lat: Lattice, model: Model, phi, fmt="binary") -> None:
    """Write a host field (numpy float64, shape (4, n0, n1, n2)) in the program's
    binary or text format (skyr_write_field_host)."""
    import numpy as np
    a = np.ascontiguousarray(phi, dtype=np.float64)
    if a.shape != (4,) + lat.shape:
        raise ValueError(f"field shape {a.shape}, expected {(4,) + lat.shape}")
    _check(lib().skyr_write_field_host(str(path).encode(), _fmt(fmt), ctypes.byref(lat), ctypes.byref(model),
                                       ctypes.c_void_p(a.ctypes.data)))


def read_field_host(path, lat: Lattice):
    """(field as numpy float64 (4, n0, n1, n2), Model) from a field file."""
    import numpy as np
    a = np.empty((4,) + lat.shape, dtype=np.float64)
    m = Model()
    _check(lib().skyr_read_field_host(str(path).encode(), ctypes.byref(lat), ctypes.byref(m),
                                      ctypes.c_void_p(a.ctypes.data)))
    return a, m


def file_info(path):
    """(Lattice, Model) stored in a field file."""
    lat, m = Lattice(), Model()
    _check(lib().skyr_file_info(str(path).encode(), ctypes.byref(lat), ctypes.byref(m)))
    return lat, m


def save_field(path, lat: Lattice, prec: int, model: Model, phi, fmt="binary", stream=None) -> None:
    _check(lib().skyr_save_field(str(path).encode(), _fmt(fmt), ctypes.byref(lat), prec, ctypes.byref(model),
                                 _dev_ptr(phi, field_dtype(prec), (4,) + lat.shape), _stream(stream)))


def load_field(path, lat: Lattice, prec: int, phi, stream=None) -> Model:
    m = Model()
    _check(lib().skyr_load_field(str(path).encode(), ctypes.byref(lat), prec, ctypes.byref(m),
                                 _dev_ptr(phi, field_dtype(prec), (4,) + lat.shape), _stream(stream)))
    return m


def cube_b4(X=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), prof_a: float = math.pi,
            prof_lambda: float = 1.0, orient=None) -> Constituent:
    """R(z) = (z^4 + 2 sqrt3 i z^2 + 1) / (z^4 - 2 sqrt3 i z^2 + 1): the O_h map of Table RMA."""
    s = 2.0 * math.sqrt(3.0) * 1j
    return constituent(4, [1, 0, s, 0, 1], [1, 0, -s, 0, 1], X, quat, prof_a, prof_lambda, orient)


def spec_from_description(init: dict):
    """InitSpec (and its keepalive) for an initial-data description
    {"kind": "hedgehog" | "cube_b4" | "random_product", ...}; a cube_b4 takes an
    optional centre "X" and isorotation quaternion "quat"."""
    kind = init["kind"]
    lam = float(init.get("prof_lambda", 1.0))
    a = float(init.get("prof_a", math.pi))
    if kind == "hedgehog":
        return init_spec(INIT_HEDGEHOG, prof_a=a, prof_lambda=lam)
    if kind == "cube_b4":
        return init_spec(INIT_RATIONAL_MAP, [cube_b4(X=tuple(init.get("X", (0.0, 0.0, 0.0))),
                                                     quat=tuple(init.get("quat", (1.0, 0.0, 0.0, 0.0))),
                                                     prof_a=a, prof_lambda=lam)])
    if kind == "random_product":
        return init_spec(INIT_RANDOM_PRODUCT, B=int(init["B"]), seed=int(init["seed"]),
                         ball_radius=float(init.get("radius", 3.0)), prof_a=a, prof_lambda=lam)
    raise ValueError(f"unknown initial data {kind!r}")


def timing_enable(on: bool) -> None:
    """Start (reset) or stop the event timing of sweep launches on this thread."""
    lib().skyr_timing_enable(int(bool(on)))


def timing_read() -> tuple[float, int]:
    """(summed sweep-kernel event time in ms, number of timed sweep launches)."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().skyr_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


# ------------------------------------------------------------------ tiles
def tile_variants(prec: int) -> list[tuple[int, int, int]]:
    """Compiled sweep shapes: (threads per block, output rows, output columns) of each."""
    out = []
    for v in range(lib().skyr_tile_variants(prec)):
        info = (ctypes.c_int32 * 3)()
        _check(lib().skyr_tile_variant_info(prec, v, info))
        out.append(tuple(int(x) for x in info))
    return out


def set_tile(lat: Lattice, prec: int, variant: int, xchunk: int) -> None:
    _check(lib().skyr_set_tile(ctypes.byref(lat), prec, int(variant), int(xchunk)))


def get_tile(lat: Lattice, prec: int) -> tuple[int, int]:
    v, x = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().skyr_get_tile(ctypes.byref(lat), prec, ctypes.byref(v), ctypes.byref(x)))
    return int(v.value), int(x.value)


def set_batch_tile(lat: Lattice, prec: int, variant: int, xchunk: int) -> None:
    """The tile of this lattice's fields in batches."""
    _check(lib().skyr_set_batch_tile(ctypes.byref(lat), prec, int(variant), int(xchunk)))


def get_batch_tile(lat: Lattice, prec: int) -> tuple[int, int]:
    v, x = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().skyr_get_batch_tile(ctypes.byref(lat), prec, ctypes.byref(v), ctypes.byref(x)))
    return int(v.value), int(x.value)


def batch_copies(lat: Lattice, prec: int, fill: int = 512, most: int = 64) -> int:
    """Fields for skyr_batch_autotune: enough that the candidate with the fewest blocks
    (one slab of the largest tile) still has `fill` blocks, 2 .. `most`."""
    ny, nz = lat.shape[1] - 4, lat.shape[2] - 4
    fewest = min(-(-ny // oy) * -(-nz // oz) for _, oy, oz in tile_variants(prec))
    return max(2, min(most, -(-fill // max(fewest, 1))))


def batch_autotune(lat: Lattice, prec: int, model: Model, flow: Flow, phi0, copies: int | None = None,
                   padded: bool = True, stream=None):
    """Time every slab split for this lattice's fields in a batch of `copies` copies of
    the dense field phi0 (default batch_copies), stored in the padded rows of
    batch_layout (or densely), and keep the fastest as its batch tile.  Returns
    (variant, planes per slab, microseconds per sweep slot of the batch).  The copies
    are allocated here and freed on return; phi0 is not changed."""
    import torch
    n = copies or batch_copies(lat, prec)
    dev = phi0.device
    layout = batch_layout(lat, prec) if padded else (0, 0)
    first = to_padded(phi0, layout) if padded else phi0
    phis = [first.clone() for _ in range(n)]
    alts = [torch.zeros_like(first) for _ in range(n)]
    vels = [torch.zeros_like(first) for _ in range(n)]
    works = [new_workspace(lat, prec, dev) for _ in range(n)]
    shape, dt = tuple(first.shape), field_dtype(prec)
    arr = lambda ts, f: (ctypes.c_void_p * n)(*[f(t).value for t in ts])
    v, x, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().skyr_batch_autotune(ctypes.byref(lat), prec, ctypes.byref(model), ctypes.byref(flow), n,
                                     arr(phis, lambda t: _dev_ptr(t, dt, shape)),
                                     arr(alts, lambda t: _dev_ptr(t, dt, shape)),
                                     arr(vels, lambda t: _dev_ptr(t, dt, shape)),
                                     arr(works, lambda t: _work_ptr(t, lat, prec)), layout[0], layout[1],
                                     _stream(stream), ctypes.byref(v), ctypes.byref(x), ctypes.byref(us)))
    return int(v.value), int(x.value), float(us.value)


def autotune(lat: Lattice, prec: int, model: Model, flow: Flow, phi, phi_alt, vel, work, stream=None):
    """Measure every shape / slab length on this lattice and keep the fastest.
    Returns (variant, planes per slab, sweep microseconds).  vel is zeroed."""
    shape = (4,) + lat.shape
    dt = field_dtype(prec)
    v, x, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().skyr_autotune(ctypes.byref(lat), prec, ctypes.byref(model), ctypes.byref(flow),
                               _dev_ptr(phi, dt, shape), _dev_ptr(phi_alt, dt, shape), _dev_ptr(vel, dt, shape),
                               _work_ptr(work, lat, prec), _stream(stream), ctypes.byref(v), ctypes.byref(x), ctypes.byref(us)))
    return int(v.value), int(x.value), float(us.value)


def _cache_path():
    import os
    return os.environ.get("SKYR_TUNE_CACHE")


def autotune_cached(lat: Lattice, prec: int, model: Model, flow: Flow, phi, phi_alt, vel, work, stream=None):
    """autotune() with a JSON cache keyed by lattice dimensions and precision
    (file named by the SKYR_TUNE_CACHE environment variable; no cache if unset)."""
    import json
    import os
    path = _cache_path()
    key = f"{lat.shape[0]}x{lat.shape[1]}x{lat.shape[2]}:{'f64' if prec == F64 else 'f32'}"
    table = {}
    if path and os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
        if key in table:
            v, x = table[key]["variant"], table[key]["xchunk"]
            set_tile(lat, prec, v, x)
            return v, x, table[key].get("us")
    v, x, us = autotune(lat, prec, model, flow, phi, phi_alt, vel, work, stream)
    if path:
        table[key] = {"variant": v, "xchunk": x, "us": us}
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return v, x, us


# ---------------------------------------------------------------- batches
def batch_layout(lat: Lattice, prec: int) -> tuple[int, int]:
    """(lead, pitch): the padded-row layout of batch fields on this lattice."""
    lead, pitch = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().skyr_batch_layout(ctypes.byref(lat), prec, ctypes.byref(lead), ctypes.byref(pitch)))
    return int(lead.value), int(pitch.value)


def to_padded(t, layout: tuple[int, int]):
    """A dense (4, n0, n1, n2) field copied into the zeroed, row-interleaved padded layout
    of batch fields, (n0, n1, 4, pitch) with z = 0 at element lead of a row."""
    import torch
    lead, pitch = layout
    out = torch.zeros(t.shape[1:3] + (4, pitch), dtype=t.dtype, device=t.device)
    out[..., lead:lead + t.shape[3]] = t.permute(1, 2, 0, 3)
    return out


def from_padded(t, layout: tuple[int, int], n2: int):
    """The dense (4, n0, n1, n2) field of a padded one."""
    lead, _ = layout
    return t[..., lead:lead + n2].permute(2, 0, 1, 3).contiguous()


class Batch:
    """Owner of a skyr_batch (many flows advanced by shared launches).  Field,
    velocity and workspace tensors belong to the caller; the batch keeps a
    reference to each flow's tensors until the flow is removed, so that their
    memory is not reused while its launches still write to it."""

    def __init__(self, max_jobs: int, stream=None):
        h = ctypes.c_void_p()
        _check(lib().skyr_batch_create(int(max_jobs), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.max_jobs = int(max_jobs)
        self._tensors = {}

    def add(self, lat: Lattice, prec: int, model: Model, flow: Flow, phi, phi_alt, vel, work) -> int:
        shape = (4,) + lat.shape
        dt = field_dtype(prec)
        slot = ctypes.c_int32()
        _check(lib().skyr_batch_add(self._h, ctypes.byref(lat), prec, ctypes.byref(model), ctypes.byref(flow),
                                    _dev_ptr(phi, dt, shape), _dev_ptr(phi_alt, dt, shape),
                                    _dev_ptr(vel, dt, shape), _work_ptr(work, lat, prec), ctypes.byref(slot)))
        self._tensors[int(slot.value)] = (phi, phi_alt, vel, work)
        return int(slot.value)

    def add_padded(self, lat: Lattice, prec: int, model: Model, flow: Flow, phi, phi_alt, vel, work,
                   layout: tuple[int, int]) -> int:
        """add() for fields in the padded, row-interleaved layout of batch fields (batch_layout,
        to_padded): tensors of shape (n0, n1, 4, pitch)."""
        lead, pitch = (int(v) for v in layout)
        shape = lat.shape[:2] + (4, pitch)
        dt = field_dtype(prec)
        slot = ctypes.c_int32()
        _check(lib().skyr_batch_add_padded(self._h, ctypes.byref(lat), prec, ctypes.byref(model),
                                           ctypes.byref(flow), _dev_ptr(phi, dt, shape),
                                           _dev_ptr(phi_alt, dt, shape), _dev_ptr(vel, dt, shape),
                                           _work_ptr(work, lat, prec), lead, pitch, ctypes.byref(slot)))
        self._tensors[int(slot.value)] = (phi, phi_alt, vel, work)
        return int(slot.value)

    def run(self, sweeps: int) -> None:
        _check(lib().skyr_batch_run(self._h, int(sweeps)))

    def poll(self, slot: int) -> AnfState:
        st = AnfState()
        status = lib().skyr_batch_poll(self._h, int(slot), ctypes.byref(st))
        if status not in (OK, E_NONFINITE):
            _check(status)
        return st

    def remove(self, slot: int) -> None:
        _check(lib().skyr_batch_remove(self._h, int(slot)))
        self._tensors.pop(int(slot), None)

    def active(self) -> int:
        return int(lib().skyr_batch_active(self._h))

    def close(self) -> None:
        if self._h:
            _check(lib().skyr_batch_destroy(self._h))
            self._h = ctypes.c_void_p()
            self._tensors.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
