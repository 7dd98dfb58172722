"""End-to-end pins of the oracle's potentials and of its rounding scale.

These fix the oracle's assembled quantities against what mathematics fixes,
independently of the oracle's own formulas:
- equal wavenumbers in every layer make the whole layered sum a free-space sum
  over all particles (the interface conditions are then trivially met by the free
  wave; Section 3.1 densities);
- reciprocity of the layered Green's function under the interface conditions
  [u] = 0, [k u_z] = 0: k_l^2 G_{l l'}(r, r') = k_l'^2 G_{l' l}(r', r) in the
  normalisation of eq. (totalinteraction);
- the reaction operators (Section 3.3 eq. (metoleimage2)) are contour integrals,
  so by Cauchy's theorem two contours (different depth b, hence different node
  sets) must give the same matrix up to rounding, in the norm that weighs entries
  by their effect on expansions of boxes of size h;
- reaction_T_mass is the sum of the moduli of the quadrature terms: it bounds
  |T| entrywise, vanishes where the integrand does, and on the equal-k adjacent
  component (sigma = 1) its (0,0;0,0) entry is the integral of |integrand| along
  the contour, computed here by adaptive quadrature.
"""
import numpy as np
import pytest
import scipy.integrate as si

import oracle as O


def _particles(d, counts, seed):
    """A few particles per layer, at least 0.08 from every interface."""
    rng = np.random.default_rng(seed)
    xs, ys, zs, ls = [], [], [], []
    L = len(d)
    for l, n in enumerate(counts):
        if l == 0:
            lo, hi = d[0] + 0.08, d[0] + 0.9
        elif l == L:
            lo, hi = d[-1] - 0.9, d[-1] - 0.08
        else:
            lo, hi = d[l] + 0.08, d[l - 1] - 0.08
        xs.append(rng.uniform(-0.5, 0.5, n))
        ys.append(rng.uniform(-0.5, 0.5, n))
        zs.append(rng.uniform(lo, hi, n))
        ls.append(np.full(n, l, dtype=np.int32))
    nt = sum(counts)
    q = rng.uniform(-1, 1, nt) + 1j * rng.uniform(-1, 1, nt)
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), np.concatenate(ls), q)


@pytest.mark.parametrize("d,kk", [((0.0, -1.2), 1.3), ((0.0, -0.6, -1.2, -1.8), 0.9)])
def test_equal_k_direct_sum_is_free_sum_over_all_layers(d, kk):
    """All layers with the same k: Phi(r_i) = sum over every j != i of Q_j h0(k R_ij),
    whatever the layers of i and j (the reaction part then carries exactly the
    cross-layer free interaction and nothing within a layer)."""
    L = len(d)
    k = (kk,) * (L + 1)
    x, y, z, lay, q = _particles(d, [7] * (L + 1), seed=21)
    n = len(x)
    phi = O.direct(d, k, x, y, z, lay, q, np.arange(n))
    R = np.sqrt((x[:, None] - x[None]) ** 2 + (y[:, None] - y[None]) ** 2 + (z[:, None] - z[None]) ** 2)
    np.fill_diagonal(R, 1.0)
    H = np.exp(1j * kk * R) / (1j * kk * R)
    np.fill_diagonal(H, 0.0)
    ref = H @ q
    err = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    assert err < 1e-12, err


@pytest.mark.parametrize("d,k", [((0.0, -1.2), (0.8, 1.5, 2.0)),
                                 ((0.0, -0.6, -1.2, -1.8), (0.5, 1.2, 2.0, 2.8, 3.0))])
def test_reciprocity_of_direct_sum(d, k):
    """One unit charge at r' in layer l' seen at r in layer l, and the reverse:
    k_l^2 G_{l l'}(r, r') = k_l'^2 G_{l' l}(r', r) for every layer pair."""
    L = len(d)
    rng = np.random.default_rng(22)
    x, y, z, lay, _ = _particles(d, [1] * (L + 1), seed=23)
    for l in range(L + 1):
        for lp in range(L + 1):
            i = l
            if l == lp:
                # a second particle in the same layer
                xx = np.array([x[i], x[i] + rng.uniform(-0.4, 0.4)])
                yy = np.array([y[i], y[i] + rng.uniform(-0.4, 0.4)])
                zz = np.array([z[i], z[i]])
                # move the second one vertically within the layer
                zz[1] = z[i] + (0.05 if (l == 0 or l == L or z[i] + 0.05 < d[l - 1] - 0.08) else -0.05)
                ll = np.array([l, l], dtype=np.int32)
            else:
                xx, yy, zz = np.array([x[l], x[lp]]), np.array([y[l], y[lp]]), np.array([z[l], z[lp]])
                ll = np.array([l, lp], dtype=np.int32)
            g_ab = O.direct(d, k, xx, yy, zz, ll, np.array([0.0, 1.0 + 0j]), [0])[0]
            g_ba = O.direct(d, k, xx, yy, zz, ll, np.array([1.0 + 0j, 0.0]), [1])[0]
            lhs, rhs = k[l] ** 2 * g_ab, k[lp] ** 2 * g_ba
            assert abs(lhs - rhs) <= 1e-12 * abs(lhs), (l, lp, lhs, rhs)


def _gate_weights(p, kt, ks, h):
    n = np.array([int(np.sqrt(i)) for i in range((p + 1) ** 2)])
    df = np.array([np.prod(np.arange(1, 2 * v + 2, 2, dtype=float)) for v in range(p + 1)])
    return np.outer((kt * h) ** n / df[n], (ks * h) ** n / df[n])


def gate_norm_rel(A, B, p, kt, ks, h):
    """Relative error of A against B in the norm weighing entry (n, n') by
    (k_t h)^n (k_s h)^n' / ((2n+1)!! (2n'+1)!!)."""
    W = _gate_weights(p, kt, ks, h)
    return np.sqrt(np.sum(W ** 2 * np.abs(A - B) ** 2) / np.sum(W ** 2 * np.abs(B) ** 2))


STACK3 = ((0.0, -1.2), (0.8, 1.5, 2.0))
# (l, a, l', b, dx, dy, zt, zs): the deep classes are the ones close to the interface
DEEP = [(0, 0, 0, 0, 0.2, 0.0, 0.05, 0.05), (2, 1, 2, 1, 0.6, -0.6, 0.1, 0.1), (1, 1, 0, 0, -0.35, 0.3, 0.2, 0.06),
        (1, 0, 1, 1, 0.275, 0.55, 0.1375, 0.4125)]


@pytest.mark.parametrize("p", [8, 10])
def test_reaction_operator_independent_of_contour_depth(p):
    """Cauchy's theorem: contours of depth b = 0.5 and b = 0.3 give the same
    operator; in the gate norm (h = twice the smaller centre distance) the two
    agree to 1e-11 even on the deepest classes, where individual high-order
    entries carry cancellation errors of order eps times the sum of |terms|."""
    d, k = STACK3
    for l, a, lp, b, dx, dy, zt, zs in DEEP:
        R1 = O.reaction_T(d, k, l, a, lp, b, dx, dy, zt, zs, p, qb=0.5)
        R2 = O.reaction_T(d, k, l, a, lp, b, dx, dy, zt, zs, p, qb=0.3)
        e = gate_norm_rel(R2, R1, p, k[l], k[lp], 2 * min(zt, zs))
        assert e < 1e-11, (p, l, a, lp, b, e)


def test_reaction_mass_bounds_the_operator():
    """|T| <= mass entrywise (triangle inequality, up to rounding), with a
    non-trivial ratio somewhere (the integrals do cancel)."""
    d, k = STACK3
    p = 5
    for l, a, lp, b, dx, dy, zt, zs in DEEP:
        T = O.reaction_T(d, k, l, a, lp, b, dx, dy, zt, zs, p)
        M = O.reaction_T_mass(d, k, l, a, lp, b, dx, dy, zt, zs, p)
        assert np.all(np.abs(T) <= M * (1 + 1e-13) + 1e-300)
        assert np.max(M / np.maximum(np.abs(T), 1e-300)) > 10.0


def test_reaction_mass_vanishes_where_the_integrand_does():
    """At rho = 0 the Bessel factor J_{m'-m}(0) vanishes for m' != m: those entries
    of T are zero, and so are their masses."""
    d, k = STACK3
    p = 4
    T = O.reaction_T(d, k, 1, 0, 1, 1, 0.0, 0.0, 0.3, 0.4, p)
    M = O.reaction_T_mass(d, k, 1, 0, 1, 1, 0.0, 0.0, 0.3, 0.4, p)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            for n2 in range(p + 1):
                for m2 in range(-n2, n2 + 1):
                    i, j = n * n + n + m, n2 * n2 + n2 + m2
                    if m2 != m:
                        assert M[i, j] == 0.0 and T[i, j] == 0.0
                    else:
                        assert M[i, j] > 0.0


@pytest.mark.parametrize("zt,zs", [(0.3, 0.2), (0.1, 0.15)])
def test_reaction_mass_is_the_integral_of_the_modulus(zt, zs):
    """Equal k = kk in every layer, component (0, up; 1, down): sigma = 1, so at
    rho = 0 the (0,0;0,0) integrand of T is (4 pi / k) Phat_0^0^2 k_rho e^{i kz H}/kz
    with H = zt + zs and Phat_0^0 = 1/sqrt(4 pi).  Its mass is the integral of the
    modulus along Gamma1 (k_rho = -i s, s in [0, b]) and Gamma2 (k_rho = t - i b),
    and the (1,0;1,0) entry carries the extra factor |Phat_1^0(kz/k)|^2 / Phat_0^0^2
    = 3 |kz/k|^2."""
    kk, b = 1.4, 0.5
    d, k = (0.0, -1.2), (kk, kk, kk)
    p = 1
    M = O.reaction_T_mass(d, k, 0, 0, 1, 1, 0.0, 0.0, zt, zs, p, qb=b)
    H = zt + zs

    def kz(kr):
        v = np.sqrt(complex(kk * kk - kr * kr))
        return v if v.imag >= 0 else -v

    def f1(s, extra):
        kr = -1j * s
        z = kz(kr)
        g = abs(kr * np.exp(1j * z * H) / z) / kk
        return g * (3 * abs(z / kk) ** 2 if extra else 1.0)

    def f2(t, extra):
        kr = t - 1j * b
        z = kz(kr)
        g = abs(kr * np.exp(1j * z * H) / z) / kk
        return g * (3 * abs(z / kk) ** 2 if extra else 1.0)

    for extra, ij in ((False, (0, 0)), (True, (2, 2))):
        a1, _ = si.quad(f1, 0.0, b, args=(extra,), epsabs=0, epsrel=1e-13, limit=200)
        tmax = 80.0 / H + 10.0
        pts = np.linspace(0.0, 2 * kk, 9)[1:]
        a2, _ = si.quad(f2, 0.0, tmax, args=(extra,), epsabs=0, epsrel=1e-13, limit=2000, points=pts)
        ref = a1 + a2
        assert abs(M[ij] - ref) <= 1e-11 * ref, (extra, M[ij], ref)
