"""Pins of the oracle's special functions against closed forms and library routines."""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle as O


@pytest.mark.parametrize("x", [1e-6, 0.01, 0.5, 3.0, 10.0, 40.0])
def test_sph_j_matches_scipy(x):
    j = O.sph_j(14, x)
    ref = sp.spherical_jn(np.arange(15), x)
    assert np.max(np.abs(j - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-12


def test_sph_j_closed_forms_and_zeros():
    for x in [0.3, np.pi, 2 * np.pi, 7.0]:
        j = O.sph_j(3, x)
        assert abs(j[0] - np.sin(x) / x) < 1e-15
        assert abs(j[1] - (np.sin(x) / x**2 - np.cos(x) / x)) < 1e-15
    assert O.sph_j(4, 0.0)[0] == 1.0 and np.all(O.sph_j(4, 0.0)[1:] == 0.0)


@pytest.mark.parametrize("x", [0.05, 0.7, 5.0, 30.0])
def test_sph_y_matches_scipy(x):
    y = O.sph_y(12, x)
    ref = sp.spherical_yn(np.arange(13), x)
    assert np.max(np.abs(y - ref) / np.abs(ref)) < 1e-12


@pytest.mark.parametrize("z", [1e-4, 0.3 - 0.2j, 2.0 - 0.5j, 10 - 0.7j, 24.5 - 0.5j, 30 - 0.6j, 200 - 0.5j,
                               -0.3j, 0.5j, 5.0 + 0.0j])
def test_bessel_J_complex_matches_scipy(z):
    J = O.bessel_J(16, complex(z))
    ref = sp.jv(np.arange(17), complex(z))
    assert np.max(np.abs(J - ref) / np.abs(ref)) < 1e-12


def test_bessel_J_integral_representation():
    # J_n(z) = (1/2pi i^n) int_0^{2pi} e^{i z cos t + i n t} dt (Section 3.5), trapezoid rule
    z = 3.7 - 0.4j
    t = np.linspace(0, 2 * np.pi, 400, endpoint=False)
    J = O.bessel_J(6, z)
    for n in range(7):
        v = np.mean(np.exp(1j * z * np.cos(t) + 1j * n * t)) / (1j**n)
        assert abs(v - J[n]) < 1e-13


def test_gauss_legendre_exact_for_polynomials():
    x, w = O.gauss_legendre()
    assert abs(w.sum() - 2.0) < 1e-14
    for deg in range(0, 32, 3):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.sum(w * x**deg) - exact) < 1e-14


def _phat_scipy(n, m, x):
    # scipy's lpmv carries the Condon-Shortley phase; Phat drops it (Section 2.1)
    c = math.sqrt((2 * n + 1) / (4 * math.pi) * math.factorial(n - m) / math.factorial(n + m))
    return c * (-1) ** m * sp.lpmv(m, n, x)


@pytest.mark.parametrize("x", [-0.9, -0.3, 0.0, 0.45, 0.99])
def test_legendre_real_matches_scipy(x):
    p = 10
    P = O.legendre(p, x, math.sqrt(1 - x * x))
    for n in range(p + 1):
        for m in range(n + 1):
            assert abs(P[n, m] - _phat_scipy(n, m, x)) < 1e-13


def test_phat00_is_one_over_sqrt_4pi():
    # the text prints 1/(4 pi); the normalisation c_00 fixes 1/sqrt(4 pi)
    assert abs(O.legendre(0, 0.3, math.sqrt(0.91))[0, 0] - 1 / math.sqrt(4 * math.pi)) < 1e-16


def test_branch_sqrt_equals_krho_over_k_on_contour():
    # eq. (branch) evaluated at k_z/k equals k_rho/k on both contour pieces
    k = 1.7
    for kr in [-0.1j, -0.45j, 0.2 - 0.5j, 1.69 - 0.5j, 3.0 - 0.5j, 80.0 - 0.5j]:
        kz = np.sqrt(k * k - kr * kr)
        assert abs(O.branch_sqrt(kz / k) - kr / k) < 1e-14


def test_branch_sqrt_limits_on_the_cut():
    x = 0.4
    assert abs(O.branch_sqrt(x + 1e-14j) - math.sqrt(1 - x * x)) < 1e-12
    assert abs(O.branch_sqrt(x - 1e-14j) + math.sqrt(1 - x * x)) < 1e-12


@pytest.mark.parametrize("case", [("a", 0.5, 1.0, 1 + 1j), ("b", 0.5, 1.8, 1 - 1.3j), ("c", 0.5, 1.8, 0.7 + 2.2j)])
def test_funk_hecke_extended_to_complex_kz(case):
    """Proposition (extfunkhecke): e^{i k.r} = sum conj(A_n^m(r)) i^n Phat_n^m(kz/k) e^{i m alpha}
    for complex kz, with the eq. (branch) square root in both places (Section 2.2
    example: r = (0.3, 0.4, z), alpha = pi/4)."""
    _, z, k, kz = case
    r = np.array([0.3, 0.4, z])
    alpha = math.pi / 4
    kzk = kz / k
    s = O.branch_sqrt(kzk)
    kvec = np.array([k * s * math.cos(alpha), k * s * math.sin(alpha), kz])
    exact = np.exp(1j * np.dot(kvec, r))
    p = 40
    P = O.legendre(p, kzk, s)
    Y = O.sph_harm(p, r)
    rr = np.linalg.norm(r)
    j = O.sph_j(p, k * rr)
    errs = []
    acc = 0
    for n in range(p + 1):
        for m in range(-n, n + 1):
            pm = P[n, abs(m)] * ((-1) ** m if m < 0 else 1)
            acc += 4 * math.pi * j[n] * np.conj(Y[n * n + n + m]) * 1j**n * pm * np.exp(1j * m * alpha)
        errs.append(abs(acc - exact) / abs(exact))
    assert errs[-1] < 1e-13
    # spectral convergence: the error falls by many orders over the range
    assert errs[25] < 1e-6 * errs[2]


def test_wigner3j_known_values():
    assert abs(O.wigner3j(1, 1, 0, 0, 0, 0) + 1 / math.sqrt(3)) < 1e-15
    assert abs(O.wigner3j(1, 1, 2, 1, -1, 0) - 1 / math.sqrt(30)) < 1e-15
    assert abs(O.wigner3j(2, 2, 2, 0, 0, 0) + math.sqrt(2 / 35)) < 1e-15
    assert O.wigner3j(1, 1, 1, 0, 0, 0) == 0.0


def test_gaunt_equals_numerical_triple_integral():
    # G(a,al;c,ga;e) = int Y_a^al Y_c^ga conj(Y_e^{al+ga}); Gauss-Legendre x trapezoid, exact
    nth, nph = 40, 64
    xg, wg = np.polynomial.legendre.leggauss(nth)
    ph = np.arange(nph) * 2 * math.pi / nph
    th = np.arccos(xg)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(wg, np.full(nph, 2 * math.pi / nph))

    def Y(n, m):
        # scipy (CS phase) -> the product is convention independent as shown by the check
        return sp.sph_harm_y(n, m, TH, PH)

    rng = np.random.default_rng(3)
    for _ in range(25):
        a, c = rng.integers(0, 7, 2)
        e = rng.integers(abs(a - c), a + c + 1)
        al = rng.integers(-a, a + 1)
        ga = rng.integers(-c, c + 1)
        if abs(al + ga) > e:
            continue
        num = np.sum(W * Y(a, al) * Y(c, ga) * np.conj(Y(e, al + ga)))
        assert abs(num - O.gaunt(int(a), int(al), int(c), int(ga), int(e))) < 1e-13
