"""Oracle for the observables of Sec. 5 beyond energy, charge and virial:
centre of mass (eq. CoM), RMS radius (eq. RMS radius), the isospin, spin and
mixed inertia tensors (eqs. U, V, W inertia tensor), the isospin-0 electric
quadrupole (eq. Q tensor, rho = B0/2) and the monopole D-term (eq. D-term with
the static stress tensor of eq. Stress tensor).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.

The formulas are evaluated literally on 2x2 complex matrices, site by site:
U = phi0 + i phi.tau, d_i U = a_i^0 + i a_i.tau with a_i = D_i phi the
fourth-order first difference of Sec. 3, L_i = U^dagger d_i U,
T_j = (i/2) U^dagger [tau^j, U], commutators and traces as printed.  Integrals
are h^3 sums over the interior I (the same sites as the energy and the charge).

Readings (the paper leaves them open):
* B0 is the charge density b = -(1/2 pi^2) det[phi, a_1, a_2, a_3], the sign
  that gives the hedgehog with f(0) = pi charge +1; B in eqs. CoM and RMS
  radius is h^3 sum b.
* The tensors and the D-term use the printed (un-halved) normalisation of the
  Lagrangian, so they compare with the paper's printed values; E in the D-term
  is the total static energy in that normalisation, twice the library's E.
* L_i keeps its identity part phi . a_i, which vanishes in the continuum and is
  O(h^4) on the lattice (traces as printed include it).
* The sextic term and the extra potentials do not enter: the printed tensors
  contain the quadratic and quartic terms only (a potential has no time
  derivative and cancels from the D-term).
"""
from __future__ import annotations

import math

import numpy as np

from . import energy, first_derivatives

_TAU = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128)
_ONE = np.eye(2, dtype=np.complex128)


def _levi_civita() -> np.ndarray:
    eps = np.zeros((3, 3, 3))
    for i, j, k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        eps[i, j, k], eps[i, k, j] = 1.0, -1.0
    return eps


_EPS = _levi_civita()


def _su2(q) -> np.ndarray:
    """q^0 + i q.tau for q of shape (4, N): (N, 2, 2) complex."""
    return (q[0][:, None, None] * _ONE + 1j * np.einsum("an,auv->nuv", q[1:], _TAU))


def _dag(M) -> np.ndarray:
    return np.conj(np.swapaxes(M, -1, -2))


def _tr(M) -> np.ndarray:
    return np.real(np.trace(M, axis1=-2, axis2=-1))


def _comm(X, Y) -> np.ndarray:
    return X @ Y - Y @ X


def interior_coordinates(shape, h: float) -> np.ndarray:
    """x_i = (idx - (n_i - 1)/2) h on the interior I, shape (3, N), z fastest."""
    axes = [(np.arange(2, n - 2) - (n - 1) / 2.0) * h for n in shape]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()])


def moments(phi, h: float, m=1.0) -> dict:
    """{B, E, X (3,), R, U, V, W, Q (3x3), D} of the field (Sec. 5)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    shape = phi.shape[1:]
    a = first_derivatives(phi, h)[:, :, 2:-2, 2:-2, 2:-2].reshape(3, 4, -1)
    p = phi[:, 2:-2, 2:-2, 2:-2].reshape(4, -1)
    x = interior_coordinates(shape, h)
    h3 = h ** 3

    # charge density and centre of mass (eq. CoM)
    cols = np.stack([p, a[0], a[1], a[2]], axis=-1)  # (4, N, 4): columns phi, a_1, a_2, a_3
    b = -np.linalg.det(np.moveaxis(cols, 1, 0)) / (2.0 * math.pi ** 2)
    B = h3 * b.sum()
    X = h3 * (x * b).sum(axis=1) / B
    r = x - X[:, None]
    r2 = (r * r).sum(axis=0)

    # RMS radius and quadrupole (eqs. RMS radius, Q tensor)
    R = math.sqrt(h3 * (r2 * b).sum() / B)
    Q = np.empty((3, 3))
    for i in range(3):
        for j in range(3):
            Q[i, j] = h3 * ((3.0 * r[i] * r[j] - r2 * (i == j)) * 0.5 * b).sum()

    # currents
    Um = _su2(p)
    Ud = _dag(Um)
    L = [Ud @ _su2(a[k]) for k in range(3)]
    T = [0.5j * (Ud @ _comm(_TAU[j], Um)) for j in range(3)]

    # inertia tensors (eqs. U, V, W inertia tensor)
    CT = [[_comm(L[k], T[i]) for i in range(3)] for k in range(3)]  # [L_k, T_i]
    CL = [[_comm(L[k], L[mm]) for mm in range(3)] for k in range(3)]  # [L_k, L_m]
    Uij = np.empty((3, 3))
    for i in range(3):
        for j in range(3):
            dens = _tr(T[i] @ T[j]) + 0.25 * sum(_tr(CT[k][i] @ CT[k][j]) for k in range(3))
            Uij[i, j] = -h3 * dens.sum()
    # K_mp = Tr(L_m L_p + 1/4 sum_k [L_k, L_m][L_k, L_p]) per site
    K = [[_tr(L[mm] @ L[pp]) + 0.25 * sum(_tr(CL[k][mm] @ CL[k][pp]) for k in range(3)) for pp in range(3)]
         for mm in range(3)]
    Vij = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            acc = np.zeros_like(b)
            for l in range(3):
                for mm in range(3):
                    if _EPS[i, l, mm] == 0.0:
                        continue
                    for n in range(3):
                        for pp in range(3):
                            if _EPS[j, n, pp] == 0.0:
                                continue
                            acc += _EPS[i, l, mm] * _EPS[j, n, pp] * r[l] * r[n] * K[mm][pp]
            Vij[i, j] = -h3 * acc.sum()
    Wij = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            acc = np.zeros_like(b)
            for l in range(3):
                for mm in range(3):
                    if _EPS[j, l, mm] == 0.0:
                        continue
                    dens = _tr(T[i] @ L[mm]) + 0.25 * sum(_tr(CT[k][i] @ CL[k][mm]) for k in range(3))
                    acc += _EPS[j, l, mm] * r[l] * dens
            Wij[i, j] = h3 * acc.sum()

    # D-term (eq. D-term) with the static stress tensor T_ij = -Tr(L_i L_j)
    # - 1/4 sum_k Tr([L_i, L_k][L_j, L_k]) + delta_ij Lag, Lag = -(static energy density)
    e_stat = (-0.5 * sum(_tr(L[k] @ L[k]) for k in range(3))
              - (1.0 / 16.0) * sum(_tr(_comm(L[i], L[j]) @ _comm(L[i], L[j])) for i in range(3) for j in range(3))
              + _mass_term(p, m))
    S = [[-_tr(L[i] @ L[j]) - 0.25 * sum(_tr(_comm(L[i], L[k]) @ _comm(L[j], L[k])) for k in range(3))
          - (i == j) * e_stat for j in range(3)] for i in range(3)]
    trS = S[0][0] + S[1][1] + S[2][2]
    mom = sum(r[i] * r[j] * S[i][j] for i in range(3) for j in range(3)) - r2 * trS / 3.0
    E = 2.0 * energy(phi, h, m)
    D = -(2.0 * E / 5.0) * h3 * mom.sum()
    return {"B": float(B), "E": float(E), "X": X, "R": R, "U": Uij, "V": Vij, "W": Wij, "Q": Q, "D": float(D)}


def _mass_term(p, m) -> np.ndarray:
    """m^2 Tr(1 - U) = 2 m^2 (1 - phi0), the pion-mass potential in the printed normalisation."""
    mm = float(m if np.isscalar(m) else m[0])
    return 2.0 * mm * mm * (1.0 - p[0])
