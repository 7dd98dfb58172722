"""Pins of the oracle's plain FMM against the oracle's direct summation."""
import numpy as np
import pytest

import oracle as O
from paper_1902_05132_amd import workloads as W


@pytest.fixture(scope="module")
def small():
    w = W.small_three_layer(n_per_layer=120, seed=5)
    tg = np.arange(0, len(w["x"]), 9)
    ref = O.direct(w["d"], w["k"], w["x"], w["y"], w["z"], w["layer"], w["q"], tg)
    reff = O.direct(w["d"], w["k"], w["x"], w["y"], w["z"], w["layer"], w["q"], tg, what=1)
    return w, tg, ref, reff


def test_fmm_error_decays_exponentially_in_p(small):
    """Truncation error of the plain FMM vs the exact sum falls geometrically in p
    (exponential convergence of MEs/LEs, Section 3.3 and Section 4)."""
    w, tg, ref, _ = small
    errs = []
    for p in (2, 4, 6, 8):
        phi, info = O.fmm(w["d"], w["k"], p, 12, w["x"], w["y"], w["z"], w["layer"], w["q"])
        errs.append(np.linalg.norm(phi[tg] - ref) / np.linalg.norm(ref))
        assert info[-1] >= 2  # reaction trees deep enough to use M2L
    errs = np.array(errs)
    assert np.all(np.diff(np.log(errs)) < -1.0)  # each +2 in p gains > e
    assert errs[-1] < 1e-4


def test_fmm_free_and_reaction_parts_separately(small):
    w, tg, ref, reff = small
    p = 8
    phf, _ = O.fmm(w["d"], w["k"], p, 12, w["x"], w["y"], w["z"], w["layer"], w["q"], what=1)
    phr, _ = O.fmm(w["d"], w["k"], p, 12, w["x"], w["y"], w["z"], w["layer"], w["q"], what=2)
    assert np.linalg.norm(phf[tg] - reff) / np.linalg.norm(reff) < 1e-4
    assert np.linalg.norm(phr[tg] - (ref - reff)) / np.linalg.norm(ref - reff) < 1e-4


def test_fmm_without_far_field_is_exact():
    """A single leaf per tree (leaf_max >= N) leaves only direct interactions, so the
    plain FMM equals the direct sum to quadrature accuracy."""
    w = W.small_three_layer(n_per_layer=30, seed=6)
    n = len(w["x"])
    phi, info = O.fmm(w["d"], w["k"], 3, 1000, w["x"], w["y"], w["z"], w["layer"], w["q"])
    assert list(info[:3]) == [0, 0, 0] and info[3] == 1
    ref = O.direct(w["d"], w["k"], w["x"], w["y"], w["z"], w["layer"], w["q"], np.arange(n))
    assert np.max(np.abs(phi - ref)) < 1e-11 * np.max(np.abs(ref))
