"""Pins of the oracle's layered-medium machinery: densities and contour quadrature."""
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _printed(kr, k, d1):
    k0, k1, k2 = k
    kz = [np.sqrt(kk**2 - kr**2) for kk in k]
    a0, a1, a2 = [k[i] * kz[i] for i in range(3)]
    kz0, kz1, kz2 = kz
    E = np.exp(-1j * d1 * kz1)
    E2 = E * E
    kappa11 = (a1 - a2) / 2 * E2 + (a1 + a2) / 2
    kappa12 = 1j * ((a2 - a1) / 2 * E2 + (a1 + a2) / 2)
    den = k0 * kz0 * kappa11 - 1j * k1 * kz1 * kappa12
    env = dict(k0=k0, k1=k1, k2=k2, kz0=kz0, kz1=kz1, kz2=kz2, a0=a0, a1=a1, a2=a2, E=E, den=den)
    rows = []
    for line in open(os.path.join(GOLD, "three_layer_densities.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, l, a, b, formula = line.split()
        rows.append((name, int(l), 0 if a == "up" else 1, 0 if b == "up" else 1, eval(formula, {}, env)))
    return rows


@pytest.mark.parametrize("kr", [0.3 - 0.5j, 1.7 - 0.5j, 5.0 - 0.5j, 40.0 - 0.5j, -0.2j, -0.5j])
def test_densities_match_printed_three_layer_forms(kr):
    k = (0.8, 1.5, 2.0)
    d = (0.0, -1.2)
    for name, l, a, b, val in _printed(kr, k, d[1]):
        s = O.densities(d, k, kr, l, 1)
        assert abs(s[a, b] - val) <= 1e-13 * abs(val), name


def test_densities_fresnel_two_layers():
    k = (1.1, 2.3)
    for kr in [0.4 - 0.5j, 3.0 - 0.5j, -0.3j]:
        kz = [np.sqrt(kk * kk - kr * kr) for kk in k]
        a = [k[i] * kz[i] for i in range(2)]
        s00 = O.densities([0.0], k, kr, 0, 0)
        # reflection of the source's down-going wave back into layer 0
        assert abs(s00[0, 0] - (a[0] - a[1]) / (a[0] + a[1])) < 1e-14
        s11 = O.densities([0.0], k, kr, 1, 1)
        assert abs(s11[1, 1] - (a[1] - a[0]) / (a[0] + a[1])) < 1e-14


STACK5 = dict(d=(0.0, -0.6, -1.2, -1.8), k=(0.5, 1.2, 2.0, 2.8, 3.0))


def _z_in(l, d, rng):
    if l == 0:
        return d[0] + rng.uniform(0.05, 1.0)
    if l == len(d):
        return d[-1] - rng.uniform(0.05, 1.0)
    return rng.uniform(d[l] + 0.02, d[l - 1] - 0.02)


def test_reciprocity_five_layers():
    """k_l g_{l,lp}(z, z') = k_lp g_{lp,l}(z', z): the interface conditions
    [u] = 0, [k u_z] = 0 make k * (Green's function) symmetric."""
    d, k = STACK5["d"], STACK5["k"]
    rng = np.random.default_rng(0)
    for kr in [0.7 - 0.5j, 2.9 - 0.5j, 6.0 - 0.5j, -0.3j]:
        for l in range(5):
            for lp in range(5):
                z, zp = _z_in(l, d, rng), _z_in(lp, d, rng)
                g1 = O.spectral_g(d, k, kr, l, z, lp, zp, with_free=True)
                g2 = O.spectral_g(d, k, kr, lp, zp, l, z, with_free=True)
                assert abs(k[l] * g1 - k[lp] * g2) <= 1e-12 * abs(k[l] * g1)


def test_equal_wavenumbers_give_free_field():
    """Equal k everywhere: the total spectral Green's function is the free wave
    e^{i kz |z-z'|}/kz for every layer pair (same-layer reaction vanishes)."""
    d = STACK5["d"]
    k = (1.3,) * 5
    rng = np.random.default_rng(1)
    for kr in [0.7 - 0.5j, 4.0 - 0.5j, -0.3j]:
        kz = np.sqrt(1.3**2 - kr**2)
        for l in range(5):
            for lp in range(5):
                z, zp = _z_in(l, d, rng), _z_in(lp, d, rng)
                g = O.spectral_g(d, k, kr, l, z, lp, zp, with_free=True)
                assert abs(g - np.exp(1j * kz * abs(z - zp)) / kz) < 1e-13
                if l == lp:
                    s = O.densities(d, k, kr, l, lp)
                    assert np.max(np.abs(s)) < 1e-14


def test_layer_merge():
    """Setting k_{j+1} = k_j must reproduce the stack with interface d_j removed."""
    d, k = list(STACK5["d"]), list(STACK5["k"])
    j = 1
    k2 = list(k)
    k2[j + 1] = k2[j]
    dm = d[:j] + d[j + 1:]
    km = k2[:j + 1] + k2[j + 2:]

    def merged_layer(l):
        return l if l <= j else l - 1

    rng = np.random.default_rng(2)
    for kr in [0.9 - 0.5j, 3.5 - 0.5j]:
        for l in range(5):
            for lp in range(5):
                z, zp = _z_in(l, d, rng), _z_in(lp, d, rng)
                g = O.spectral_g(d, k2, kr, l, z, lp, zp, with_free=True)
                gm = O.spectral_g(dm, km, kr, merged_layer(l), z, merged_layer(lp), zp, with_free=True)
                assert abs(g - gm) <= 1e-12 * max(abs(gm), 1e-300)


@pytest.mark.parametrize("k,rho,dz", [(1.5, 0.3, 0.5), (0.8, 1.2, 0.2), (2.0, 0.0, 0.1), (2.5, 2.0, 1.0),
                                      (3.0, 0.05, 0.05)])
def test_sommerfeld_identity(k, rho, dz):
    """eq. (sommerfeldid): (1/k) int k_rho J0(k_rho rho) e^{i kz dz}/kz = h0(k R)."""
    v, _ = O.sommerfeld_h0(k, rho, dz)
    R = np.hypot(rho, dz)
    ref = np.exp(1j * k * R) / (1j * k * R)
    assert abs(v - ref) <= 1e-12 * abs(ref)


def test_contour_independence_and_refinement():
    """Cauchy: the value must not depend on the contour depth b; halving the panels
    and lengthening the contour must not change it."""
    k, rho, dz = 1.7, 0.8, 0.3
    v0, n0 = O.sommerfeld_h0(k, rho, dz, b=0.5)
    for b in (0.25, 1.0):
        v, _ = O.sommerfeld_h0(k, rho, dz, b=b)
        assert abs(v - v0) < 1e-13 * abs(v0)
    v2, n2 = O.sommerfeld_h0(k, rho, dz, b=0.5, scale=2.0)
    assert n2 > n0 and abs(v2 - v0) < 1e-13 * abs(v0)


def test_reaction_kernel_equal_k_adjacent_is_free_space():
    """Equal k: the component (l, up; l+1, down) has sigma = 1 and the polarisation
    source sits at the mirror distance, so its kernel is h0 of the image distance
    (the Remark after eq. (redefinedist))."""
    kk = 1.4
    d = (0.0, -1.2)
    k = (kk, kk, kk)
    for kr in [0.3 - 0.5j, 3 - 0.5j, -0.2j]:
        s = O.densities(d, k, kr, 0, 1)
        assert abs(s[0, 1] - 1) < 1e-14
    for rho, ht, hs in [(0.5, 0.3, 0.2), (0.0, 0.1, 0.15), (1.3, 0.6, 0.4)]:
        g = O.reaction_kernel(d, k, 0, 0, 1, 1, rho, ht, hs)
        R = np.hypot(rho, ht + hs)
        assert abs(g - np.exp(1j * kk * R) / (1j * kk * R)) < 1e-13 * abs(g)
