"""Pins of the moment observables of the oracle (Sec. 5: centre of mass, RMS
radius, inertia tensors U, V, W, quadrupole Q, D-term) against facts that do
not come from the oracle's own formulas:

* the hedgehog's radial integrals, derived by hand from the printed traces
  (U = V = W = Lambda 1, Lambda = (16 pi/3) int r^2 sin^2 f (1 + f'^2 + sin^2 f/r^2) dr;
  R^2 = -(2/pi) int r^2 f' sin^2 f dr; the D-term from the radial and tangential
  stresses), approached at fourth order in h;
* exact lattice symmetries: translation by whole sites, a global isorotation
  (U -> D U D^T, W -> D W, V unchanged, with D(A)_ij = (1/2) Tr(tau^i A tau^j A^dagger)
  evaluated here from its printed definition), the 90-degree rotation that maps
  a pair along x to a pair along y, and the vanishing of Q for a spherical
  charge distribution.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.moments import moments

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")
scipy_integrate = pytest.importorskip("scipy.integrate")

LAM = 0.7  # profile length of the test hedgehogs, f = pi exp(-r / LAM)


def _radial(lam=LAM, m=1.0):
    quad = scipy_integrate.quad
    f = lambda r: math.pi * math.exp(-r / lam)
    fp = lambda r: -f(r) / lam
    s2 = lambda r: math.sin(f(r)) ** 2 / (r * r)
    lam_iso = 16 * math.pi / 3 * quad(lambda r: r * r * math.sin(f(r)) ** 2 * (1 + fp(r) ** 2)
                                      + math.sin(f(r)) ** 4, 0, 60, limit=400)[0]
    r2 = -(2 / math.pi) * quad(lambda r: r * r * fp(r) * math.sin(f(r)) ** 2, 0, 60, limit=400)[0]
    E = 4 * math.pi * quad(lambda r: r * r * (fp(r) ** 2 + 2 * s2(r) + 2 * fp(r) ** 2 * s2(r) + s2(r) ** 2
                                              + 2 * m * m * (1 - math.cos(f(r)))), 1e-12, 60, limit=400)[0]
    # r_i r_j (T_ij - delta_ij T/3) = (2/3) r^2 (tau_r - tau_t), tau_r - tau_t = 2 (f'^2 - s^2)(1 + s^2)
    shear = 4 * math.pi * quad(lambda r: r ** 4 * (2 / 3) * 2 * (fp(r) ** 2 - s2(r)) * (1 + s2(r)),
                               1e-12, 60, limit=400)[0]
    return {"Lambda": lam_iso, "R": math.sqrt(r2), "E": E, "D": -(2 * E / 5) * shear}


def _hedgehog(n, h, **kw):
    return oracle.init_product((n, n, n), h, [oracle.hedgehog(prof_lambda=LAM, **kw)])


def _d_of(A):
    """D(A)_ij = (1/2) Tr(tau^i A tau^j A^dagger), A = a0 + i a.tau."""
    tau = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]])
    Am = A[0] * np.eye(2) + 1j * sum(A[k + 1] * tau[k] for k in range(3))
    return np.array([[0.5 * np.trace(tau[i] @ Am @ tau[j] @ Am.conj().T).real for j in range(3)]
                     for i in range(3)])


@pytest.fixture(scope="module")
def hedgehogs():
    return {h: moments(_hedgehog(n, h), h) for n, h in ((48, 0.2), (64, 0.15))}


def test_hedgehog_tensors_approach_the_radial_integral_at_fourth_order(hedgehogs):
    rad = _radial()
    lam = rad["Lambda"]
    for k in "UVW":
        coarse, fine = hedgehogs[0.2][k], hedgehogs[0.15][k]
        for M in (coarse, fine):
            assert np.abs(M - np.diag(np.diag(M))).max() < 1e-10 * lam  # isotropic, no off-diagonal part
            assert np.ptp(np.diag(M)) < 1e-10 * lam
        e_coarse, e_fine = abs(coarse[0, 0] - lam), abs(fine[0, 0] - lam)
        assert e_fine < 6e-3 * lam, k
        assert e_coarse / e_fine > 2.6, k  # (0.2 / 0.15)^4 = 3.16


def test_hedgehog_radius_energy_and_d_term(hedgehogs):
    rad = _radial()
    fine, coarse = hedgehogs[0.15], hedgehogs[0.2]
    assert fine["R"] == pytest.approx(rad["R"], rel=6e-3)
    assert abs(coarse["R"] - rad["R"]) > 2.5 * abs(fine["R"] - rad["R"])
    assert fine["E"] == pytest.approx(rad["E"], rel=2e-2)
    assert fine["D"] == pytest.approx(rad["D"], rel=2e-2)
    assert abs(coarse["D"] - rad["D"]) > 2.5 * abs(fine["D"] - rad["D"])
    assert fine["D"] < 0
    for M in (fine, coarse):
        assert np.abs(M["Q"]).max() < 1e-12  # spherical charge distribution
        assert np.abs(M["X"]).max() < 1e-12


def test_translation_by_whole_sites():
    n, h = 48, 0.2
    shift = np.array([2, -3, 1]) * h
    base = moments(_hedgehog(n, h), h)
    moved = moments(_hedgehog(n, h, X=tuple(shift)), h)
    # equal up to the truncation of the tails at the frozen boundary, which the
    # shift brings 0.6 closer (moving the frame instead would change V by O(1))
    assert np.abs(moved["X"] - shift).max() < 1e-6
    for k, tol in (("U", 1e-4), ("V", 5e-4), ("W", 1e-4), ("Q", 1e-7)):
        assert np.abs(moved[k] - base[k]).max() < tol * np.abs(base["U"]).max(), k
    assert moved["R"] == pytest.approx(base["R"], rel=1e-6)
    assert moved["D"] == pytest.approx(base["D"], rel=3e-3)


def test_global_isorotation_rotates_the_isospin_index():
    """phi -> A phi A^dagger: U -> D U D^T, W -> D W, V and Q unchanged, and for
    the hedgehog W = Lambda D(A) is not symmetric (catches a transposed W)."""
    n, h = 40, 0.2
    A = np.array([0.8, 0.2, -0.5, 0.4])
    A /= np.linalg.norm(A)
    pair = [((-0.8, 0.0, 0.0), np.array([1.0, 0.0, 0.0, 0.0])),
            ((0.8, 0.2, 0.0), np.array([0.9, 0.3, 0.1, -0.3]) / np.linalg.norm([0.9, 0.3, 0.1, -0.3]))]
    mk = lambda cs: oracle.init_product((n, n, n), h, [oracle.hedgehog(X=X, quat=tuple(q), prof_lambda=LAM)
                                                       for X, q in cs])
    base = moments(mk(pair), h)
    turned = moments(mk([(X, _qmul(A, q)) for X, q in pair]), h)
    D = _d_of(A)
    scale = np.abs(base["U"]).max()
    assert np.abs(turned["U"] - D @ base["U"] @ D.T).max() < 1e-9 * scale
    assert np.abs(turned["W"] - D @ base["W"]).max() < 1e-9 * scale
    assert np.abs(turned["V"] - base["V"]).max() < 1e-9 * scale
    assert np.abs(turned["Q"] - base["Q"]).max() < 1e-9 * np.abs(base["Q"]).max()
    assert np.abs(base["W"] - base["W"].T).max() > 1e-3 * scale  # the test can see a transposition
    hh = moments(oracle.init_product((n, n, n), h, [oracle.hedgehog(quat=tuple(A), prof_lambda=LAM)]), h)
    # the centred hedgehog's W is w 1 on the cubic lattice (w within O(h^4) of U's
    # Lambda), so the isorotated one is w D(A) exactly, and not w D(A)^T
    w = np.trace(D.T @ hh["W"]) / 3.0
    assert w == pytest.approx(hh["U"][0, 0], rel=1e-2)
    assert np.abs(hh["W"] - w * D).max() < 1e-9 * w
    assert np.abs(hh["W"] - w * D.T).max() > 0.1 * w


def _qmul(a, b):
    """Quaternion product (a0 + i a.tau)(b0 + i b.tau) as 4-vectors (appendix identity)."""
    a0, av, b0, bv = a[0], a[1:], b[0], b[1:]
    return np.concatenate([[a0 * b0 - av @ bv], a0 * bv + b0 * av - np.cross(av, bv)])


def test_pair_along_x_and_along_y():
    """Two unrotated hedgehogs on the x axis, then on the y axis: the second is
    the first turned by 90 degrees about z and isorotated, so Q and V have their
    x and y entries swapped; both are diagonal, Q traceless and axially
    symmetric about the pair's axis (Q_yy = Q_zz = -Q_xx/2)."""
    n, h, d = 40, 0.2, 0.9
    mk = lambda X1, X2: oracle.init_product((n, n, n), h, [oracle.hedgehog(X=X1, prof_lambda=LAM),
                                                            oracle.hedgehog(X=X2, prof_lambda=LAM)])
    px = moments(mk((-d, 0, 0), (d, 0, 0)), h)
    py = moments(mk((0, -d, 0), (0, d, 0)), h)
    perm = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]])
    q = px["Q"]
    assert q[0, 0] > 0.1
    assert np.abs(q - np.diag(np.diag(q))).max() < 1e-10 * q[0, 0]
    assert q[1, 1] == pytest.approx(-q[0, 0] / 2, rel=1e-9) and q[2, 2] == pytest.approx(-q[0, 0] / 2, rel=1e-9)
    for k in ("Q", "V"):
        assert np.abs(py[k] - perm @ px[k] @ perm.T).max() < 1e-9 * np.abs(px[k]).max(), k
    assert px["V"][1, 1] > px["V"][0, 0]  # rotating about the pair's axis costs least
    assert py["R"] == pytest.approx(px["R"], rel=1e-10)
    assert py["D"] == pytest.approx(px["D"], rel=1e-9)
