"""Pins of the oracle's expansions and translation operators (Sections 2.1, 3.3, 3.5)."""
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def h0(x):
    return np.exp(1j * x) / (1j * x)


@pytest.mark.parametrize("kind", [0, 1])
def test_point_expansions_converge_to_h0(kind):
    """h-expansion (eq. (freespace3dmulexp)) and j-expansion (eq. (freespace3dlocexp))."""
    k = 1.3
    r = np.array([1.5, -1.0, 0.8])
    s = np.array([0.1, 0.05, -0.1])
    R = np.linalg.norm(r - s)
    errs = []
    for p in (4, 8, 14):
        if kind == 0:
            c = O.point_expansion(0, k, s, p)
            v = O.eval_expansion(0, k, c, r, p)
        else:
            c = O.point_expansion(1, k, r, p)
            v = O.eval_expansion(1, k, c, s, p)
        errs.append(abs(v - h0(k * R)) / abs(h0(k * R)))
    assert errs[0] > 1e-8 and errs[1] < 1e-9 and errs[2] < 1e-13


def test_m2l_maps_point_multipole_to_point_local():
    k, p, P2 = 1.3, 5, 14
    cs = np.array([0.1, -0.2, 0.05])
    ct = np.array([1.1, 0.9, 1.3])
    src = cs + np.array([0.12, -0.05, 0.08])
    M = O.point_expansion(0, k, src - cs, P2)
    L = O.translation(1, k, ct - cs, P2, cached=True) @ M
    ref = O.point_expansion(1, k, src - ct, P2)
    nc = (p + 1) ** 2
    assert np.max(np.abs(L[:nc] - ref[:nc])) < 1e-12 * np.max(np.abs(ref[:nc]))


def test_m2m_and_l2l_shift_point_expansions():
    k, p, P2 = 1.3, 5, 14
    nc = (p + 1) ** 2
    c = np.array([0.2, 0.2, 0.2])
    P = np.zeros(3)
    src = c + np.array([0.05, -0.07, 0.03])
    Mc = O.point_expansion(0, k, src - c, P2)
    Mp = O.translation(0, k, P - c, P2, cached=True) @ Mc
    ref = O.point_expansion(0, k, src - P, P2)
    assert np.max(np.abs(Mp[:nc] - ref[:nc])) < 1e-13 * np.max(np.abs(ref[:nc]))
    far = np.array([7.0, -5.0, 6.5])
    LP = O.point_expansion(1, k, far - P, P2)
    Lc = O.translation(0, k, c - P, P2, cached=True) @ LP
    ref = O.point_expansion(1, k, far - c, P2)
    assert np.max(np.abs(Lc[:nc] - ref[:nc])) < 1e-12 * np.max(np.abs(ref[:nc]))


def test_translation_cache_is_the_same_operator():
    k, p = 0.9, 4
    b = [0.3, -0.7, 1.1]
    for kind in (0, 1):
        A = O.translation(kind, k, b, p)
        B = O.translation(kind, k, b, p, cached=True)
        assert np.max(np.abs(A - B)) <= 1e-15 * np.max(np.abs(A))


def test_reaction_m2l_equal_k_is_free_m2l():
    """sigma = 1 and k_l = k_l' reduce the reaction M2L integral operator to the
    free-space one for the image displacement (the spectral form of S in Section 2.2)."""
    kk = 1.4
    d = (0.0, -1.2)
    k = (kk, kk, kk)
    p = 5
    for dx, dy, zt, zs in [(0.7, -0.4, 0.3, 0.45), (0.0, 0.0, 0.5, 0.5), (-1.1, 0.2, 0.15, 0.9)]:
        T = O.reaction_T(d, k, 0, 0, 1, 1, dx, dy, zt, zs, p)
        S = O.translation(1, kk, [dx, dy, zt + zs], p, cached=True)
        assert np.max(np.abs(T - S)) < 1e-12 * np.max(np.abs(S))


def test_reaction_m2l_against_two_dimensional_quadrature():
    """The alpha integral of eq. (metoleimage2) done numerically (trapezoid in alpha,
    the same k_rho nodes) must equal the Bessel-reduced form for distinct k_l, k_l'."""
    d = (0.0, -1.2)
    k = (0.8, 1.5, 2.0)
    l, a, lp, b = 0, 0, 1, 0
    p = 3
    dx, dy, zt, zs = 0.55, -0.3, 0.4, 0.5
    T = O.reaction_T(d, k, l, a, lp, b, dx, dy, zt, zs, p)
    # 2-D reference: same contour with plain Gauss panels, alpha by trapezoid
    xg, wg = O.gauss_legendre()
    nodes, weights = [], []
    for s0 in (0.0, 0.25):
        for g in range(16):
            nodes.append(-1j * (s0 + 0.125 + 0.125 * xg[g]))
            weights.append(-1j * 0.125 * wg[g])
    t0 = 0.0
    while t0 < 160.0:
        h = 0.25 if t0 < 6 else 1.0
        for g in range(16):
            nodes.append(t0 + h / 2 + h / 2 * xg[g] - 0.5j)
            weights.append(h / 2 * wg[g])
        t0 += h
    nal = 96
    al = np.arange(nal) * 2 * math.pi / nal
    kt, ks = k[l], k[lp]
    ref = np.zeros_like(T)
    nc = (p + 1) ** 2
    for kr, w in zip(nodes, weights):
        kzt, kzs = np.sqrt(kt**2 - kr**2), np.sqrt(ks**2 - kr**2)
        sig = O.densities(d, k, kr, l, lp)[a, b]
        Pt = O.legendre(p, kzt / kt, kr / kt)
        Ps = O.legendre(p, kzs / ks, kr / ks)
        ez = np.exp(1j * kzt * zt + 1j * kzs * zs)
        ea = np.exp(1j * kr * (dx * np.cos(al) + dy * np.sin(al)))
        base = w * kr * ez * sig / kzt
        for n in range(p + 1):
            for m in range(-n, n + 1):
                pt = Pt[n, abs(m)] * ((-1) ** m if m < 0 else 1)
                for n2 in range(p + 1):
                    for m2 in range(-n2, n2 + 1):
                        ps = Ps[n2, abs(m2)] * ((-1) ** m2 if m2 < 0 else 1)
                        ang = np.mean(ea * np.exp(1j * (m2 - m) * al)) * 2 * math.pi
                        # T = (-1)^{n'} / (2 pi) int int ... Q e^{i(m'-m) alpha}, Q = i^{n+n'+1} Phat Phat,
                        # in the Phi normalisation (times 4 pi / (i k_l))
                        Q = 1j ** (n + n2 + 1) * pt * ps
                        ref[n * n + n + m, n2 * n2 + n2 + m2] += (-1) ** n2 / (2 * math.pi) * base * Q * ang
    ref *= 4 * math.pi / (1j * kt)
    assert np.max(np.abs(T - ref)) < 1e-10 * np.max(np.abs(ref))


def _me_errors(b, z, zp, pmax):
    d = (0.0, -2.0)
    k = (0.8, 1.5, 2.0)
    ht = z - d[1]
    hs = (zp - d[1]) if b == 0 else (d[0] - zp)
    exact = O.reaction_kernel(d, k, 1, 0, 1, b, 0.0, ht, hs)
    errs = []
    for p in range(1, pmax + 1):
        M = O.point_expansion(0, k[1], [-0.375, 0.0, 0.0], p)
        F = O.reaction_me_basis(d, k, 1, 0, 1, b, 0.625 - 1.0, 0.0, ht, hs, p)
        errs.append(abs(np.sum(M * F) - exact) / abs(exact))
    return np.array(errs)


def test_reaction_me_convergence_rates_match_paper():
    """ME convergence experiment of Section 3.3: fitted a in err ~ a^p."""
    rows = [l.split() for l in open(os.path.join(GOLD, "me_convergence_rates.txt"))
            if l.strip() and not l.startswith("#")]
    for comp, z, zp, a_printed in rows:
        b = 0 if comp == "up_up" else 1
        e = _me_errors(b, float(z), float(zp), 14)
        ps = np.arange(1, len(e) + 1)
        ok = e > 1e-14
        a = math.exp(np.polyfit(ps[ok], np.log(e[ok]), 1)[0])
        a_printed = float(a_printed)
        if comp == "up_up" or a_printed > 0.12:
            # the captions' fits: reproduced within 25 %
            assert abs(a - a_printed) <= 0.25 * a_printed, (comp, z, zp, a)
        else:
            # printed 0.10 where the plotted error meets its floor: at least as fast
            assert a <= 1.05 * a_printed, (comp, z, zp, a)
        assert e[-1] < 0.05 * e[0]
