"""Pre-computed tables of the reaction M2L integrals on the GPU.

* Build: every geometry combination of the medium is tabulated by the library's
  quadrature and validated against it halfway between nodes; the bounds are finite
  and at the FP64 level.
* Gate closed: bit-identical to an evaluation without tables.
* Gate open: every class inside the tabulated range takes the tables; the potential
  matches the oracle's FMM to the FP64 parity tolerance of the quadrature path
  (1e-10), and the quadrature path to within the largest bound; the reaction
  integrals cost a fraction of the quadrature's time.
* Box sizes between the nodes (the same particles spread laterally), precedence
  over the surrogate, save / load round trip and rejections, release.
"""
import numpy as np
import pytest

import oracle as O
from paper_1902_05132_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FMM = 1e-10
H_RANGE = (0.03, 1.0)


def _lfmm():
    from paper_1902_05132_amd import lfmm
    return lfmm


def _rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _eval(P, w):
    return P.eval_torch(w["x"], w["y"], w["z"], w["q"])


@pytest.fixture(scope="module")
def built():
    lf = _lfmm()
    w = W.three_layer_3k()
    P = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], profile=True)
    rep = P.tables_build(h_min=H_RANGE[0], h_max=H_RANGE[1])
    print("table report:", rep)
    ref = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], profile=True)
    _eval(ref, w)  # first evaluation sizes the workspaces
    phi_ref = _eval(ref, w)
    return dict(lf=lf, w=w, P=P, rep=rep, phi_ref=phi_ref, rep_ref=ref.report())


def test_build_report_and_bounds(built):
    r, P = built["rep"], built["P"]
    assert r["n_combos"] == 16 * 37
    assert r["n_slots"] == r["n_combos"] * r["npanel"] * r["nnode"]
    assert r["n_validation"] == r["n_combos"] * r["npanel"] * 4
    assert r["bytes"] == r["n_slots"] * 21 * 36 * 16
    b = P.tables_bounds()
    assert b.size == 16 * 37
    # interpolation of smooth functions on 16 Chebyshev points per panel: the
    # validated error sits at the quadrature's own noise level
    assert np.all(np.isfinite(b)) and np.all(b > 0) and b.max() < 1e-8, (b.min(), b.max())
    assert r["err_max"] * 2 == pytest.approx(b.max())


def test_gate_closed_is_bit_identical(built):
    P, w = built["P"], built["w"]
    P.tables_gate(0.0)
    phi = _eval(P, w)
    assert P.report()["n_react_table"] == 0
    assert np.array_equal(phi, built["phi_ref"])


def _oracle_fmm(w):
    ref, _ = O.fmm(w["d"], w["k"], w["p"], w["leaf"], w["x"], w["y"], w["z"], w["layer"], w["q"])
    return ref


def test_gate_open_matches_oracle_and_quadrature(built):
    P, w = built["P"], built["w"]
    P.tables_gate(1e300)
    _eval(P, w)
    phi = _eval(P, w)
    rep = P.report()
    P.tables_gate(0.0)
    n_tab, n_cls = rep["n_react_table"], rep["n_react_classes"]
    assert n_tab == n_cls > 0
    e_quad = _rel2(phi, built["phi_ref"])
    ref = _oracle_fmm(w)
    e2, emax = _rel2(phi, ref), _relmax(phi, ref)
    st, st0 = rep["stage_ms"], built["rep_ref"]["stage_ms"]
    t_tab = st["react_tables"] + st["react_mfma"] + st["react_table"]
    t_quad = st0["react_tables"] + st0["react_mfma"]
    print("tables: %d of %d classes; Err2 vs quadrature %.2e, vs oracle FMM %.2e (max %.2e); "
          "reaction integrals %.3f ms (quadrature %.3f ms)" % (n_tab, n_cls, e_quad, e2, emax, t_tab, t_quad))
    assert e_quad <= max(P.tables_bounds().max(), 1e-14)
    assert e2 < TOL_FMM and emax < TOL_FMM
    assert t_tab < 0.5 * t_quad


def test_box_sizes_between_nodes(built):
    # spreading the particles laterally changes the root and so every box size
    P, lf = built["P"], built["lf"]
    w = dict(built["w"])
    w["x"] = w["x"] * 2.37
    w["y"] = w["y"] * 2.37
    Q = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"])
    phi_q = _eval(Q, w)
    P.tables_gate(1e300)
    phi = _eval(P, w)
    rep = P.report()
    P.tables_gate(0.0)
    assert rep["n_react_table"] == rep["n_react_classes"] > 0
    ref = _oracle_fmm(w)
    print("spread x2.37: Err2 vs quadrature %.2e, vs oracle FMM %.2e" % (_rel2(phi, phi_q), _rel2(phi, ref)))
    assert _rel2(phi, phi_q) <= max(P.tables_bounds().max(), 1e-14)
    assert _rel2(phi, ref) < TOL_FMM and _relmax(phi, ref) < TOL_FMM


def test_partial_range_mixes_tables_and_quadrature(built):
    """Tables covering only some of the box sizes: the other classes fall back to the
    quadrature in the same evaluation, and the result still matches the oracle."""
    lf, w = built["lf"], built["w"]
    Q = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"])
    Q.tables_build(h_min=0.1, h_max=0.3)
    Q.tables_gate(1e300)
    phi = _eval(Q, w)
    rep = Q.report()
    assert 0 < rep["n_react_table"] < rep["n_react_classes"], rep
    ref = _oracle_fmm(w)
    print("partial range: %d of %d classes from the tables, Err2 vs oracle FMM %.2e"
          % (rep["n_react_table"], rep["n_react_classes"], _rel2(phi, ref)))
    assert _rel2(phi, built["phi_ref"]) <= max(Q.tables_bounds().max(), 1e-14)
    assert _rel2(phi, ref) < TOL_FMM and _relmax(phi, ref) < TOL_FMM


def test_tables_need_a_layered_medium(built):
    lf, w = built["lf"], built["w"]
    H = lf.Plan([], [w["k"][0]], p=4, leaf_max=16)
    with pytest.raises(lf.LfmmError) as e:
        H.tables_build()
    assert e.value.code == 1


def test_tables_take_precedence_over_surrogate(built):
    P, w = built["P"], built["w"]
    P.surrogate_train(seed=3, epochs=2)
    P.surrogate_gate(1e300)
    P.tables_gate(1e300)
    a = _eval(P, w)
    ra = P.report()
    P.tables_gate(0.0)
    _eval(P, w)
    rb = P.report()
    P.surrogate_gate(0.0)
    assert ra["n_react_table"] == ra["n_react_classes"] and ra["n_react_surrogate"] == 0
    assert rb["n_react_surrogate"] == rb["n_react_classes"] and rb["n_react_table"] == 0
    P.tables_gate(1e300)
    b = _eval(P, w)
    P.tables_gate(0.0)
    assert np.array_equal(a, b)


def test_save_load_roundtrip_rejections_release(built, tmp_path):
    lf, w = built["lf"], built["w"]
    Q = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"])
    with pytest.raises(lf.LfmmError) as e:
        Q.tables_save(str(tmp_path / "none.bin"))
    assert e.value.code == 1
    r = Q.tables_build(h_min=0.1, h_max=0.6, nnode=8, du=3.0)
    assert r["npanel"] == 2 and r["nnode"] == 8
    path = str(tmp_path / "tables.bin")
    Q.tables_save(path)
    R = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"])
    R.tables_load(path)
    assert np.array_equal(Q.tables_bounds(), R.tables_bounds())
    Q.tables_gate(1e300)
    R.tables_gate(1e300)
    a = _eval(Q, w)
    b = _eval(R, w)
    assert R.report()["n_react_table"] > 0
    assert np.array_equal(a, b)
    other = lf.Plan(w["d"], (0.8, 1.5, 2.1), p=w["p"], leaf_max=w["leaf"])
    with pytest.raises(lf.LfmmError) as e:
        other.tables_load(path)
    assert e.value.code == 5
    with pytest.raises(lf.LfmmError) as e:
        R.tables_load(str(tmp_path / "missing.bin"))
    assert e.value.code == 5
    data = open(path, "rb").read()
    cut = tmp_path / "cut.bin"
    cut.write_bytes(data[:len(data) - 1000])
    with pytest.raises(lf.LfmmError) as e:
        R.tables_load(str(cut))
    assert e.value.code == 5
    # a failed load leaves no tables behind; release frees them
    phi0 = _eval(lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"]), w)
    assert np.array_equal(_eval(R, w), phi0) and R.report()["n_react_table"] == 0
    Q.tables_release()
    assert np.array_equal(_eval(Q, w), phi0) and Q.report()["n_react_table"] == 0
