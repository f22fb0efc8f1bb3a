"""One-dimensional references for spherically symmetric (hedgehog) fields.

For phi = (cos f(r), sin f(r) x/r) the energy of the sigma-model form
(Sec. 2.1, one half of the printed normalisation) reduces to

  E2 = 4 pi int ( r^2 f'^2 / 2 + sin^2 f ) dr
  E4 = 4 pi int ( f'^2 sin^2 f + sin^4 f / (2 r^2) ) dr
  E0 = 4 pi m^2 int r^2 (1 - cos f) dr
  B  = -(2/pi) int f' sin^2 f dr        (= 1 for f(0) = pi, f(inf) = 0)

(the strain eigenvalues of a hedgehog are f'^2 and twice sin^2 f / r^2).
These are independent of the lattice code: quadrature of a given profile, and
a minimiser of the radial functional on a fine radial grid.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def hedgehog_parts(f, fp, m: float, R: float = 40.0) -> dict:
    """E2, E4, E0, B of the hedgehog with profile f (derivative fp) on [0, R]."""
    def q(fun):
        val, _ = integrate.quad(fun, 0.0, R, limit=400, epsabs=1e-13, epsrel=1e-13)
        return val

    E2 = 4 * math.pi * q(lambda r: 0.5 * r * r * fp(r) ** 2 + math.sin(f(r)) ** 2)
    E4 = 4 * math.pi * q(lambda r: fp(r) ** 2 * math.sin(f(r)) ** 2
                         + (math.sin(f(r)) ** 4 / (2 * r * r) if r > 0 else 0.0))
    E0 = 4 * math.pi * m * m * q(lambda r: r * r * (1 - math.cos(f(r))))
    B = -(2 / math.pi) * q(lambda r: fp(r) * math.sin(f(r)) ** 2)
    return dict(E2=E2, E4=E4, E0=E0, E=E2 + E4 + E0, B=B)


def _radial_terms(f_int: np.ndarray, dr: float, m: float):
    """Midpoint-rule radial energy with f(0) = pi and f(R) = 0 fixed: energy,
    gradient and the tridiagonal Hessian (as banded rows) with respect to the
    interior profile values.  Interval k couples f_k and f_{k+1} through
    fm = (f_k + f_{k+1})/2 and fp = (f_{k+1} - f_k)/dr at r = (k + 1/2) dr."""
    f = np.concatenate([[math.pi], f_int, [0.0]])
    r = (np.arange(len(f) - 1) + 0.5) * dr
    fm = 0.5 * (f[1:] + f[:-1])
    fp = (f[1:] - f[:-1]) / dr
    s, c = np.sin(fm), np.cos(fm)
    s2f, c2f = np.sin(2 * fm), np.cos(2 * fm)
    dens = 0.5 * r * r * fp ** 2 + s ** 2 + fp ** 2 * s ** 2 + s ** 4 / (2 * r * r) + m * m * r * r * (1 - c)
    w = 4 * math.pi * dr
    E = w * dens.sum()
    d_fm = s2f * (1 + fp ** 2) + 2 * s ** 3 * c / (r * r) + m * m * r * r * s
    d_fp = r * r * fp + 2 * fp * s ** 2
    h_mm = 2 * c2f * (1 + fp ** 2) + (2 / (r * r)) * (3 * s * s * c * c - s ** 4) + m * m * r * r * c
    h_mp = 2 * fp * s2f
    h_pp = r * r + 2 * s ** 2
    # chain rule with d fm/d(f_k, f_k+1) = (1/2, 1/2), d fp/d(f_k, f_k+1) = (-1/dr, 1/dr)
    g_left = w * (0.5 * d_fm - d_fp / dr)     # d/d f_k of interval k
    g_right = w * (0.5 * d_fm + d_fp / dr)    # d/d f_{k+1} of interval k
    H_ll = w * (0.25 * h_mm - h_mp / dr + h_pp / dr ** 2)
    H_rr = w * (0.25 * h_mm + h_mp / dr + h_pp / dr ** 2)
    H_lr = w * (0.25 * h_mm - h_pp / dr ** 2)
    n = len(f)
    grad = np.zeros(n)
    grad[:-1] += g_left
    grad[1:] += g_right
    diag = np.zeros(n)
    diag[:-1] += H_ll
    diag[1:] += H_rr
    off = H_lr  # couples k and k+1
    # restrict to the interior unknowns 1..n-2
    return E, grad[1:-1], diag[1:-1], off[1:-1]


def minimise_radial(m: float, R: float = 20.0, dr: float = 0.01, iters: int = 200) -> float:
    """Minimum of the radial energy on [0, R] with f(0) = pi, f(R) = 0, by
    damped Newton iteration on the tridiagonal Hessian."""
    from scipy.linalg import solve_banded

    M = int(round(R / dr))
    r = np.arange(1, M) * dr
    f = math.pi * np.exp(-r)
    E, g, d, o = _radial_terms(f, dr, m)
    for _ in range(iters):
        ab = np.zeros((3, len(f)))
        ab[0, 1:] = o
        ab[1] = d
        ab[2, :-1] = o
        step = solve_banded((1, 1), ab, -g)
        t = 1.0
        while True:
            En, gn, dn, on = _radial_terms(f + t * step, dr, m)
            if En <= E or t < 1e-6:
                break
            t *= 0.5
        f = f + t * step
        done = abs(E - En) <= 1e-15 * abs(E) and np.max(np.abs(t * step)) < 1e-12
        E, g, d, o = En, gn, dn, on
        if done:
            break
    return float(E)


def radial_minimum(m: float, R: float = 20.0, dr: float = 0.01) -> float:
    """Richardson-extrapolated (second order in dr) minimum of the radial energy."""
    e1 = minimise_radial(m, R, dr)
    e2 = minimise_radial(m, R, dr / 2)
    return (4 * e2 - e1) / 3
