"""Pins of the oracle's kernel formulas (no GPU).

* Ein / E1 against scipy's exponential integral (A&S 5.1.11 / 5.1.22);
* U^eps(0) against the r -> 0 limit; U - U^eps vanishing at the far field
  (condition (b) of eq. ApproxProp, Theorem 2);
* every W = FT(U - U^eps) of Table 1 (and the Yukawa split) against direct
  quadrature of eq. Fourier-Symmetric.
"""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import oracle as O

KINDS = ["coulomb3d", "yukawa3d", "log2d", "coulomb2d", "biharmonic3d", "biharmonic2d"]


def test_e1_matches_library():
    x = np.concatenate([np.geomspace(1e-8, 1.0, 60), np.linspace(1.0, 60.0, 120)])
    got = O.e1(x)
    ref = special.exp1(x)
    assert np.max(np.abs(got - ref) / ref) <= 5e-15


def test_ein_relation():
    x = np.geomspace(1e-6, 1.0, 50)
    assert np.max(np.abs(O.ein(x) - (special.exp1(x) + np.euler_gamma + np.log(x)))) <= 2e-15
    assert O.ein([0.0])[0] == 0.0


@pytest.mark.parametrize("kind", KINDS)
def test_ueps_limit_at_zero(kind):
    eps = 0.7
    lam = 1.3 if kind == "yukawa3d" else 0.0
    r = np.array([0.0, 1e-7, 1e-6])
    v = O.ueps(kind, r, eps, lam)
    assert np.isfinite(v[0])
    assert abs(v[0] - v[1]) <= 1e-6 * max(1.0, abs(v[0]))
    assert abs(v[1] - v[2]) <= 1e-5 * max(1.0, abs(v[0]))


@pytest.mark.parametrize("kind", KINDS)
def test_far_field_agreement(kind):
    """U^eps = U to double precision beyond ~6 eps (Sec. 1, Theorem 2)."""
    eps = 0.5
    lam = 0.8 if kind == "yukawa3d" else 0.0
    r = np.linspace(6.5 * eps, 30 * eps, 50)
    u = O.u(kind, r, lam)
    ue = O.ueps(kind, r, eps, lam)
    assert np.max(np.abs(u - ue) / np.abs(u)) <= 1e-15


def what_quadrature(kind, k, eps, lam):
    """eq. Fourier-Symmetric: radial Hankel (2D) / sinc (3D) transform of U - U^eps."""
    d = O.KIND_DIM[kind]
    rmax = 12.0 * eps

    def diff(r):
        return O.u(kind, np.array([r]), lam)[0] - O.ueps(kind, np.array([r]), eps, lam)[0]

    if d == 3:
        f = lambda r: 4 * np.pi * diff(r) * r * r * (np.sinc(k * r / np.pi))
    else:
        f = lambda r: 2 * np.pi * diff(r) * r * special.j0(k * r)
    val, _ = integrate.quad(f, 1e-300, rmax, limit=500, epsabs=1e-16, epsrel=1e-13)
    return val


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k", [0.0, 1e-3, 0.37, 1.0, 2.9, 7.5])
def test_what_matches_fourier_symmetric_quadrature(kind, k):
    eps = 0.8
    lam = 1.1 if kind == "yukawa3d" else 0.0
    got = O.what(kind, [k], eps, lam)[0]
    ref = what_quadrature(kind, k, eps, lam)
    assert abs(got - ref) <= 1e-11 * max(abs(ref), 1e-3 * eps ** 4)


def test_yukawa_reduces_to_coulomb():
    r = np.linspace(0.0, 5.0, 40)
    k = np.linspace(0.0, 9.0, 40)
    assert np.allclose(O.ueps("yukawa3d", r, 0.6, 1e-9), O.ueps("coulomb3d", r, 0.6), rtol=1e-8)
    assert np.allclose(O.what("yukawa3d", k, 0.6, 1e-9), O.what("coulomb3d", k, 0.6), rtol=1e-8)


def test_small_k_branches_against_mpmath():
    """The series branches of the biharmonic W (x = k^2 eps^2/4 < 1/2) and the
    closed forms beyond agree with a 40-digit evaluation of Table 1."""
    import mpmath as mp
    mp.mp.dps = 40
    eps = 1.3
    for x in (1e-6, 0.1, 0.4999, 0.5001, 2.0):
        k = 2.0 * np.sqrt(x) / eps
        kk, e = mp.mpf(k), mp.mpf(eps)
        X = kk * kk * e * e / 4
        ref3 = (-8 + mp.e ** (-X) * (8 + 2 * kk**2 * e**2 + kk**4 * e**4)) / (8 * kk**4)
        ref2 = (-16 + mp.e ** (-X) * (16 + 4 * kk**2 * e**2 + kk**4 * e**4)) / (16 * kk**4)
        assert abs(O.what("biharmonic3d", [k], eps)[0] - float(ref3)) <= 1e-14 * abs(float(ref3))
        assert abs(O.what("biharmonic2d", [k], eps)[0] - float(ref2)) <= 1e-14 * abs(float(ref2))
