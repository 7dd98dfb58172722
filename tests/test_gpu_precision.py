"""Mixed-precision path (plan option precision = 1): near field in FP32 and the
M2L on FP32 matrix cores with per-level rescaled expansions, everything else in
FP64.  Its result is compared with the FP64 path of the same plan parameters
(same trees, same p); the bar is a relative error of at most 1e-6 (Err2), the
accuracy the FP32 form has to keep to replace the FP64 one.
"""
import numpy as np
import pytest

from paper_1902_05132_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-6


def _both(w, p, leaf, quad_tol=0.0):
    from paper_1902_05132_amd import lfmm
    a = lfmm.Plan(w["d"], w["k"], p=p, leaf_max=leaf)
    b = lfmm.Plan(w["d"], w["k"], p=p, leaf_max=leaf, precision=1, quad_tol=quad_tol)
    phi64 = a.eval_torch(w["x"], w["y"], w["z"], w["q"])
    phi32 = b.eval_torch(w["x"], w["y"], w["z"], w["q"])
    ra, rb = a.report(), b.report()
    assert ra["free_depth"] == rb["free_depth"] and ra["reaction_depth"] == rb["reaction_depth"]
    assert ra["precision"] == 0 and rb["precision"] == 1
    e2 = np.linalg.norm(phi32 - phi64) / np.linalg.norm(phi64)
    emax = np.max(np.abs(phi32 - phi64)) / np.max(np.abs(phi64))
    return e2, emax


def test_mixed_precision_three_layer_3k():
    w = W.three_layer_3k()
    e2, emax = _both(w, w["p"], w["leaf"])
    print("three layers, N = 3000, mixed vs FP64: Err2 %.2e Errmax %.2e" % (e2, emax))
    assert e2 < TOL_MIXED and emax < TOL_MIXED


def test_mixed_precision_with_truncated_contour():
    """The benchmark's mixed setting: FP32 parts and the Sommerfeld contour truncated at
    1e-10, against the FP64 path with the default contour."""
    w = W.three_layer_3k()
    e2, emax = _both(w, w["p"], w["leaf"], quad_tol=1e-10)
    print("mixed, contour at 1e-10, vs FP64: Err2 %.2e Errmax %.2e" % (e2, emax))
    assert e2 < TOL_MIXED and emax < TOL_MIXED


@pytest.mark.parametrize("p", [8, 10])
def test_mixed_precision_high_order_deep_tree(p):
    """Order 8 and 10 on a tree deep enough that unscaled FP32 M2L operators
    would overflow at order 10 (h_20 of small arguments)."""
    w = W.layered_cubes(W.THREE_LAYER_D, W.THREE_LAYER_K, [4000, 4000, 4000], W.THREE_LAYER_CENTERS, seed=31)
    e2, emax = _both(w, p, 24)
    print("p = %d mixed vs FP64: Err2 %.2e Errmax %.2e" % (p, e2, emax))
    assert np.isfinite(e2) and e2 < TOL_MIXED and emax < TOL_MIXED


def test_mixed_precision_near_field_library_path():
    """k r > 1 on some pairs: the FP32 near field falls back to sincosf."""
    w = W.layered_cubes(W.THREE_LAYER_D, (3.0, 5.0, 7.0), [3000, 3000, 3000], W.THREE_LAYER_CENTERS, seed=37)
    e2, emax = _both(w, 6, 400)
    print("sincos path mixed vs FP64: Err2 %.2e Errmax %.2e" % (e2, emax))
    assert e2 < TOL_MIXED


@pytest.mark.parametrize("side,k,form", [(0.05, 2.0, 2), (0.1, 2.0, 1), (1.0, 2.0, 0)])
def test_mixed_near_field_forms_against_oracle(side, k, form):
    """One medium, every particle in one leaf: the FP32 near field alone against the
    oracle's direct sum, in each form of h0.  The host bounds k r by 2 k side sqrt(3):
    0.35 <= 1/2 at side 0.05 (fitted cubics), 0.69 <= 1 at side 0.1 (fitted quartics),
    6.9 at side 1 (sincosf)."""
    import oracle as O
    from paper_1902_05132_amd import lfmm
    n = 700
    rng = np.random.default_rng(41)
    pts = np.array([0.2, -0.1, 0.3]) + side * (rng.random((n, 3)) - 0.5)
    x, y, z = pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy()
    q = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    P = lfmm.Plan((), (k,), p=4, leaf_max=1000, precision=1)
    phi = P.eval_torch(x, y, z, q)
    rep = P.report()
    assert rep["free_depth"][0] == 0 and rep["p2p_pairs"] == n * (n - 1)
    assert rep["p2p_series"] == form
    ref = O.direct((), (k,), x, y, z, np.zeros(n, np.int32), q, np.arange(n))
    e2 = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    emax = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    print("form %d: Err2 %.2e Errmax %.2e vs the oracle's direct sum" % (form, e2, emax))
    assert e2 < TOL_MIXED and emax < TOL_MIXED
