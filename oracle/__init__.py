"""FP64 CPU oracle for the layered-media Helmholtz FMM -- test infrastructure only.

Plain, slow reference implementations written from the paper (Wang, Zhang & Cai,
SISC 2019).  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package; the HIP library never does, and this
package never imports the HIP library.  Everything here is a thin ctypes layer over
``oracle.c`` (argument marshalling only).

Functions that are pinned by tests against values fixed by the paper or by
mathematics are listed in ``tests/test_oracle_*.py``; the pins are:
  special functions      -> closed forms / scipy / mpmath reference values
  Legendre on C + branch -> Funk-Hecke identity on complex k_z (Section 2.2)
  contour quadrature     -> Sommerfeld identity (eq. (sommerfeldid)) closed form
  densities              -> printed three-layer closed forms (Section 3.1),
                            Fresnel two-layer form, reciprocity, equal-k, layer merge
  translations           -> addition theorems vs. point-source closed forms
  reaction M2L           -> sigma = 1, equal k reduces to the free-space operator;
                            brute-force 2-D (k_rho, alpha) quadrature
  reaction ME            -> printed convergence rates (Section 3.3 figure captions)
  plain FMM              -> direct summation (exponential decay of the error in p)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    """Compile oracle.c into liboracle.so (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-o", _LIB_PATH, os.path.join(_HERE, "oracle.c"), "-lm"]
    subprocess.check_call(cmd)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _declare(L):
    c_int, c_double = ctypes.c_int, ctypes.c_double
    sig = {
        "orc_sph_j": [c_int, c_double, _D],
        "orc_sph_y": [c_int, c_double, _D],
        "orc_legendre": None,
        "orc_gauss_legendre": [_D, _D],
        "orc_densities": [c_int, _D, _D, c_double, c_double, c_int, c_int, _D],
        "orc_spectral_g": [c_int, _D, _D, c_double, c_double, c_int, c_double, c_int, c_double, c_int, _D],
        "orc_sommerfeld_h0": [c_double, c_double, c_double, c_double, c_double, _D],
        "orc_direct": [c_int, _D, _D, c_int, _D, _D, _D, _I, _D, c_int, _I, c_double, c_int, _D],
        "orc_wigner3j": [c_int] * 6,
        "orc_gaunt": [c_int] * 5,
        "orc_translation": [c_int, c_double, _D, c_int, _D],
        "orc_translation_cached": [c_int, c_double, _D, c_int, _D],
        "orc_point_expansion": [c_int, c_double, _D, c_int, _D],
        "orc_eval_expansion": [c_int, c_double, _D, _D, c_int, _D],
        "orc_reaction_T": [c_int, _D, _D, c_int, c_int, c_int, c_int, c_double, c_double, c_double, c_double,
                           c_int, c_double, _D],
        "orc_reaction_T_mass": [c_int, _D, _D, c_int, c_int, c_int, c_int, c_double, c_double, c_double,
                                c_double, c_int, c_double, _D],
        "orc_reaction_kernel": [c_int, _D, _D, c_int, c_int, c_int, c_int, c_double, c_double, c_double,
                                c_double, _D],
        "orc_reaction_me_basis": [c_int, _D, _D, c_int, c_int, c_int, c_int, c_double, c_double, c_double,
                                  c_double, c_int, c_double, _D],
        "orc_fmm": [c_int, _D, _D, c_int, c_int, c_int, c_double, c_int, _D, _D, _D, _I, _D, c_int, _D, _I],
        "orc_num_threads": [],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        if args is not None:
            f.argtypes = args
    L.orc_wigner3j.restype = ctypes.c_double
    L.orc_gaunt.restype = ctypes.c_double
    L.orc_num_threads.restype = ctypes.c_int


def _dp(a):
    return a.ctypes.data_as(_D)


def _ip(a):
    return a.ctypes.data_as(_I)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _cplx(buf):
    return buf[0::2] + 1j * buf[1::2]


# ---------------------------------------------------------------- special functions
def sph_j(nmax, x):
    out = np.zeros(nmax + 1)
    lib().orc_sph_j(nmax, float(x), _dp(out))
    return out


def sph_y(nmax, x):
    out = np.zeros(nmax + 1)
    lib().orc_sph_y(nmax, float(x), _dp(out))
    return out


class _C(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


def bessel_J(nmax, z):
    """J_0..J_nmax at complex z."""
    L = lib()
    f = L.orc_bessel_J
    f.argtypes = [ctypes.c_int, _C, _D]
    out = np.zeros(2 * (nmax + 1))
    f(nmax, _C(z.real, z.imag), _dp(out))
    return _cplx(out)


def branch_sqrt(z):
    L = lib()
    f = L.orc_branch_sqrt
    f.argtypes = [_C]
    f.restype = _C
    r = f(_C(complex(z).real, complex(z).imag))
    return complex(r.re, r.im)


def legendre(p, x, s):
    """Phat_n^m(x), 0 <= m <= n <= p, with s = sqrt(1-x^2) on the chosen branch.
    Returns dict-like 2-D array P[n, m] (m <= n), complex."""
    L = lib()
    f = L.orc_legendre
    f.argtypes = [ctypes.c_int, _C, _C, _D]
    nt = (p + 1) * (p + 2) // 2
    out = np.zeros(2 * nt)
    f(p, _C(complex(x).real, complex(x).imag), _C(complex(s).real, complex(s).imag), _dp(out))
    t = _cplx(out)
    P = np.zeros((p + 1, p + 1), dtype=complex)
    for n in range(p + 1):
        for m in range(n + 1):
            P[n, m] = t[n * (n + 1) // 2 + m]
    return P


def sph_harm(p, v):
    L = lib()
    f = L.orc_sph_harm
    f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
    out = np.zeros(2 * (p + 1) ** 2)
    f(p, float(v[0]), float(v[1]), float(v[2]), _dp(out))
    return _cplx(out)


def gauss_legendre():
    x = np.zeros(16)
    w = np.zeros(16)
    lib().orc_gauss_legendre(_dp(x), _dp(w))
    return x, w


# ---------------------------------------------------------------- layered medium
def densities(d, k, kr, l, lp):
    """sigma^{ab}_{l,lp}(kr) as a 2x2 complex array [a][b], a/b = 0 up, 1 down."""
    d = _f64(d)
    k = _f64(k)
    out = np.zeros(8)
    lib().orc_densities(len(d), _dp(d), _dp(k), float(np.real(kr)), float(np.imag(kr)), l, lp, _dp(out))
    return _cplx(out).reshape(2, 2)


def spectral_g(d, k, kr, l, z, lp, zp, with_free=True):
    d = _f64(d)
    k = _f64(k)
    out = np.zeros(2)
    lib().orc_spectral_g(len(d), _dp(d), _dp(k), float(np.real(kr)), float(np.imag(kr)), l, float(z), lp,
                         float(zp), int(with_free), _dp(out))
    return complex(out[0], out[1])


def sommerfeld_h0(k, rho, dz, b=0.5, scale=1.0):
    """Contour quadrature of (1/k) int k_rho J0(k_rho rho) e^{i kz dz}/kz dk_rho.
    scale shrinks the panels and extends t_max (scale > 1) for convergence checks.
    Returns (value, number of nodes)."""
    out = np.zeros(3)
    lib().orc_sommerfeld_h0(float(k), float(rho), float(dz), float(b), float(scale), _dp(out))
    return complex(out[0], out[1]), int(out[2])


def direct(d, k, x, y, z, layer, q, targets, b=0.5, what=3):
    """Phi_l(r_i) at the listed target indices by direct summation (exact quantity)."""
    d = _f64(d)
    k = _f64(k)
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = _i32(layer)
    q = np.ascontiguousarray(np.asarray(q, dtype=np.complex128)).view(np.float64)
    tg = _i32(targets)
    out = np.zeros(2 * len(tg))
    lib().orc_direct(len(d), _dp(d), _dp(k), len(x), _dp(x), _dp(y), _dp(z), _ip(layer), _dp(q), len(tg),
                     _ip(tg), float(b), int(what), _dp(out))
    return _cplx(out)


# ---------------------------------------------------------------- translations
def wigner3j(j1, j2, j3, m1, m2, m3):
    return lib().orc_wigner3j(j1, j2, j3, m1, m2, m3)


def gaunt(a, al, c, ga, e):
    return lib().orc_gaunt(a, al, c, ga, e)


def translation(kind, k, b, p, cached=False):
    """Op[new (n,m), old (nu,mu)]; kind 0 regular (M2M/L2L), 1 singular (M2L)."""
    nc = (p + 1) ** 2
    out = np.zeros(2 * nc * nc)
    bv = _f64(b)
    fn = lib().orc_translation_cached if cached else lib().orc_translation
    fn(int(kind), float(k), _dp(bv), p, _dp(out))
    return _cplx(out).reshape(nc, nc)


def point_expansion(kind, k, rv, p):
    out = np.zeros(2 * (p + 1) ** 2)
    lib().orc_point_expansion(int(kind), float(k), _dp(_f64(rv)), p, _dp(out))
    return _cplx(out)


def eval_expansion(kind, k, coef, rv, p):
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.complex128)).view(np.float64)
    out = np.zeros(2)
    lib().orc_eval_expansion(int(kind), float(k), _dp(c), _dp(_f64(rv)), p, _dp(out))
    return complex(out[0], out[1])


# ---------------------------------------------------------------- reaction components
def reaction_T(d, k, l, a, lp, b, dx, dy, zt, zs, p, qb=0.5):
    nc = (p + 1) ** 2
    d = _f64(d)
    k = _f64(k)
    out = np.zeros(2 * nc * nc)
    lib().orc_reaction_T(len(d), _dp(d), _dp(k), l, a, lp, b, float(dx), float(dy), float(zt), float(zs), p,
                         float(qb), _dp(out))
    return _cplx(out).reshape(nc, nc)


def reaction_T_mass(d, k, l, a, lp, b, dx, dy, zt, zs, p, qb=0.5):
    """Per-entry sum of |quadrature terms| of reaction_T (its rounding scale)."""
    nc = (p + 1) ** 2
    d = _f64(d)
    k = _f64(k)
    out = np.zeros(nc * nc)
    lib().orc_reaction_T_mass(len(d), _dp(d), _dp(k), l, a, lp, b, float(dx), float(dy), float(zt), float(zs), p,
                              float(qb), _dp(out))
    return out.reshape(nc, nc)


def reaction_kernel(d, k, l, a, lp, b, rho, ht, hs, qb=0.5):
    d = _f64(d)
    k = _f64(k)
    out = np.zeros(2)
    lib().orc_reaction_kernel(len(d), _dp(d), _dp(k), l, a, lp, b, float(rho), float(ht), float(hs), float(qb),
                              _dp(out))
    return complex(out[0], out[1])


def reaction_me_basis(d, k, l, a, lp, b, dx, dy, ht, hc, p, qb=0.5):
    d = _f64(d)
    k = _f64(k)
    out = np.zeros(2 * (p + 1) ** 2)
    lib().orc_reaction_me_basis(len(d), _dp(d), _dp(k), l, a, lp, b, float(dx), float(dy), float(ht), float(hc),
                                p, float(qb), _dp(out))
    return _cplx(out)


# ---------------------------------------------------------------- plain FMM
def fmm(d, k, p, leaf_max, x, y, z, layer, q, what=3, qb=0.5, max_depth=8):
    """Plain FMM potentials for every particle; returns (phi, info) with info =
    [free-tree depth per layer..., reaction-tree depth].  Tree depths are capped at
    max_depth (1..8)."""
    d = _f64(d)
    k = _f64(k)
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = _i32(layer)
    q = np.ascontiguousarray(np.asarray(q, dtype=np.complex128)).view(np.float64)
    n = len(x)
    out = np.zeros(2 * n)
    info = np.zeros(len(d) + 2, dtype=np.int32)
    lib().orc_fmm(len(d), _dp(d), _dp(k), int(p), int(leaf_max), int(max_depth), float(qb), n, _dp(x), _dp(y),
                  _dp(z), _ip(layer), _dp(q), int(what), _dp(out), _ip(info))
    return _cplx(out), info


def num_threads():
    return lib().orc_num_threads()
