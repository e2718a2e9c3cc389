"""Pins of the oracle's building blocks against facts fixed outside it.

* Boys function (the radial factor of Eq. 12) against mpmath's incomplete gamma function,
  F_m(0) = 1/(2m+1), the downward recursion identity and the large-T asymptote.
* Complex and real solid harmonics (Eq. 2, Condon-Shortley) against scipy's spherical
  harmonics, harmonicity, and S^1 = (y, z, x).
* Clebsch-Gordan coefficients against sympy.
* The vector-coupling shift (Eqs. 7-8, with the shift vector P - A = (beta/p)(B - A)) as the
  addition theorem at random points, evaluated against direct harmonics of the sum.
* The product rule (supplement Eq. 4) at random points.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import special

import oracle
import xcheck


def boys_ref(m, T):
    mpmath.mp.dps = 40
    if T == 0:
        return mpmath.mpf(1) / (2 * m + 1)
    a = mpmath.mpf(m) + mpmath.mpf(1) / 2
    return mpmath.gammainc(a, 0, mpmath.mpf(T)) / (2 * mpmath.mpf(T) ** a)


T_GRID = [0.0, 1e-12, 1e-6, 1e-3, 0.05, 0.3, 1.0, 2.5, 7.0, 12.0, 19.9, 25.0, 33.3, 39.99, 40.01,
          45.0, 60.0, 100.0, 250.0, 1000.0, 6.4e4]


@pytest.mark.parametrize("T", T_GRID)
def test_boys_against_incomplete_gamma(T):
    F = oracle.boys(15, T)
    for m in range(16):
        ref = float(boys_ref(m, T))
        assert abs(F[m] - ref) <= 2e-14 * abs(ref), (m, T, F[m], ref)


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("T", [0.7, 17.0, 39.0, 41.0, 120.0])
def test_boys_extended_precision(T, prec):
    # long double / __float128 builds must track the reference well below double rounding
    F = oracle.boys(12, T, precision=prec)
    for m in range(13):
        ref = float(boys_ref(m, T))
        assert abs(F[m] - ref) <= 2e-16 * abs(ref)


def test_boys_identities():
    for m in range(16):
        assert oracle.boys(15, 0.0)[m] == pytest.approx(1.0 / (2 * m + 1), rel=1e-15)
    for T in [0.2, 3.0, 30.0, 80.0]:
        F = oracle.boys(15, T)
        for m in range(15):
            # (2m+1) F_m = 2T F_{m+1} + exp(-T)
            lhs = (2 * m + 1) * F[m]
            rhs = 2 * T * F[m + 1] + math.exp(-T)
            assert lhs == pytest.approx(rhs, rel=1e-13)
    # F_0 = sqrt(pi/T)/2 erf(sqrt T)
    for T in [1e-3, 0.5, 8.0, 55.0]:
        assert oracle.boys(0, T)[0] == pytest.approx(0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T)), rel=1e-14)
    # large-T asymptote (2m-1)!!/2^{m+1} sqrt(pi/T^{2m+1})
    T = 2000.0
    F = oracle.boys(10, T)
    for m in range(11):
        df = 1.0
        for i in range(2 * m - 1, 1, -2):
            df *= i
        assert F[m] == pytest.approx(df / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1)), rel=1e-14)


def _sph(l, m, theta, phi):
    if hasattr(special, "sph_harm_y"):
        return special.sph_harm_y(l, m, theta, phi)
    return special.sph_harm(m, l, phi, theta)


def test_complex_solid_harmonics_against_scipy():
    rng = np.random.default_rng(7)
    for _ in range(20):
        v = rng.normal(size=3) * 1.3
        r = np.linalg.norm(v)
        theta, phi = math.acos(v[2] / r), math.atan2(v[1], v[0])
        Y = oracle.solid_complex(12, *v)
        for l in range(13):
            for m in range(-l, l + 1):
                ref = math.sqrt(4 * math.pi / (2 * l + 1)) * r ** l * _sph(l, m, theta, phi)
                assert abs(Y[l * l + m + l] - ref) <= 1e-12 * max(1.0, r ** l), (l, m)


def test_real_solid_harmonics():
    rng = np.random.default_rng(8)
    for _ in range(10):
        x, y, z = rng.normal(size=3)
        S = oracle.solid_real(6, x, y, z)
        assert np.allclose(S[1:4], [y, z, x], rtol=0, atol=1e-15)
        s3 = math.sqrt(3)
        assert np.allclose(S[4:9], [s3 * x * y, s3 * y * z, (3 * z * z - (x * x + y * y + z * z)) / 2, s3 * x * z,
                                    s3 / 2 * (x * x - y * y)], atol=1e-14)
        for l in range(7):
            assert np.allclose(S[l * l:(l + 1) ** 2], xcheck.eval_real_solid(l, x, y, z), atol=1e-12)


def test_solid_harmonics_are_harmonic():
    # Laplacian by a fourth-order central-difference stencil must vanish (Laplace equation),
    # while a single second derivative does not
    h = 1e-2
    v = np.array([0.4, -0.3, 0.6])

    def d2(k):
        e = np.zeros(3)
        e[k] = h
        f = lambda s: oracle.solid_real(6, *(v + s * e))
        return (-f(2) + 16 * f(1) - 30 * f(0) + 16 * f(-1) - f(-2)) / (12 * h * h)

    parts = [d2(k) for k in range(3)]
    lap = parts[0] + parts[1] + parts[2]
    assert np.abs(lap).max() < 1e-7
    assert np.abs(parts[2][4:]).max() > 0.5


def test_clebsch_gordan_against_sympy():
    from sympy.physics.wigner import clebsch_gordan
    rng = np.random.default_rng(9)
    cases = 0
    for j1 in range(0, 7):
        for j2 in range(0, 7):
            for J in range(abs(j1 - j2), j1 + j2 + 1):
                m1 = int(rng.integers(-j1, j1 + 1))
                m2s = [m for m in range(-j2, j2 + 1) if abs(m1 + m) <= J]
                m2 = m2s[int(rng.integers(len(m2s)))]
                ref = float(clebsch_gordan(j1, j2, J, m1, m2, m1 + m2))
                assert oracle.cg(j1, m1, j2, m2, J, m1 + m2) == pytest.approx(ref, abs=1e-14)
                cases += 1
    assert cases == 231  # every (j1, j2, J) with j1, j2 <= 6


def test_addition_theorem_with_eps():
    # Y^l_m(u + v) = sum_{lam, mu} eps_{l lam m mu} Y^{l-lam}_{m-mu}(u) Y^{lam}_{mu}(v)   (Eqs. 7, 8)
    rng = np.random.default_rng(10)
    for _ in range(5):
        u, v = rng.normal(size=3), rng.normal(size=3)
        Yu = oracle.solid_complex(6, *u)
        Yv = oracle.solid_complex(6, *v)
        Ys = oracle.solid_complex(6, *(u + v))
        for l in range(7):
            for m in range(-l, l + 1):
                s = 0j
                for lam in range(l + 1):
                    for mu in range(-lam, lam + 1):
                        if abs(m - mu) <= l - lam:
                            s += oracle.eps(l, lam, m, mu) * Yu[(l - lam) ** 2 + (m - mu) + (l - lam)] * Yv[lam * lam + mu + lam]
                assert abs(s - Ys[l * l + m + l]) <= 1e-11 * max(1.0, abs(Ys[l * l + m + l]))


def test_shift_matrix_reproduces_centered_harmonic():
    # Eq. 7 with the corrected vector: Y^{la}(r - A) = sum S[ma, l1 m1] Y^{l1}(r - P), P - A = (b/p)(B - A)
    rng = np.random.default_rng(11)
    A, B, r = rng.normal(size=3), rng.normal(size=3), rng.normal(size=3)
    a, b = 0.8, 1.9
    P = (a * A + b * B) / (a + b)
    for la in range(7):
        S = oracle.shift_matrix(la, b / (a + b), B - A)
        YP = oracle.solid_complex(la, *(r - P))
        lhs = oracle.solid_complex(la, *(r - A))[la * la:]
        assert np.allclose(S @ YP, lhs, rtol=1e-12, atol=1e-12)
        # the printed sign (vector A - B) is wrong once la - l1 is odd
        if la >= 1:
            Sw = oracle.shift_matrix(la, b / (a + b), A - B)
            assert not np.allclose(Sw @ YP, lhs, rtol=1e-6, atol=1e-6)


def test_product_rule():
    # Y^{l1}_{m1} Y^{l2}_{m2} = sum_L <l1 0 l2 0|L0><l1 m1 l2 m2|LM> r^{l1+l2-L} Y^L_M
    rng = np.random.default_rng(12)
    v = rng.normal(size=3)
    r2 = float(v @ v)
    Y = oracle.solid_complex(12, *v)
    for l1 in range(7):
        for l2 in range(7):
            for m1 in range(-l1, l1 + 1):
                for m2 in range(-l2, l2 + 1):
                    M = m1 + m2
                    s = 0j
                    for L in range(abs(l1 - l2), l1 + l2 + 1, 2):
                        if abs(M) <= L:
                            k = (l1 + l2 - L) // 2
                            s += (oracle.cg(l1, 0, l2, 0, L, 0) * oracle.cg(l1, m1, l2, m2, L, M) * r2 ** k
                                  * Y[L * L + M + L])
                    ref = Y[l1 * l1 + m1 + l1] * Y[l2 * l2 + m2 + l2]
                    assert abs(s - ref) <= 1e-11 * max(1.0, abs(ref))
