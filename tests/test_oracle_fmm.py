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
    """A single leaf per free tree (leaf_max >= N) and reaction trees of depth 1
    (max_depth = 1: every target box touches every image box) leave only direct
    interactions, so the plain FMM equals the direct sum to quadrature accuracy."""
    w = W.small_three_layer(n_per_layer=30, seed=6)
    n = len(w["x"])
    phi, info = O.fmm(w["d"], w["k"], 3, 1000, w["x"], w["y"], w["z"], w["layer"], w["q"], max_depth=1)
    assert list(info[:3]) == [0, 0, 0] and info[3] == 1
    ref = O.direct(w["d"], w["k"], w["x"], w["y"], w["z"], w["layer"], w["q"], np.arange(n))
    assert np.max(np.abs(phi - ref)) < 1e-11 * np.max(np.abs(ref))


def test_reaction_depth_reaches_below_the_interface_gap():
    """The reaction trees are deep enough that the finest boxes are no thicker than
    the smallest particle-to-interface distance (here 0.1), leaving the reaction
    near field empty."""
    w = W.small_three_layer(n_per_layer=30, seed=6)
    _, info = O.fmm(w["d"], w["k"], 3, 1000, w["x"], w["y"], w["z"], w["layer"], w["q"], what=2)
    gap = min(np.min(w["z"][w["layer"] == 0] - 0.0), np.min(0.0 - w["z"][w["layer"] == 1]),
              np.min(w["z"][w["layer"] == 1] + 1.2), np.min(-1.2 - w["z"][w["layer"] == 2]))
    z0, z1, z2 = (w["z"][w["layer"] == l] for l in range(3))
    H = max(np.max(z0), np.max(-z1), np.max(z1 + 1.2), np.max(-1.2 - z2))
    S = max(np.ptp(w["x"]), np.ptp(w["y"]), 2 * H)
    D = int(info[3])
    assert S / 2 ** D <= gap < S / 2 ** (D - 1)
