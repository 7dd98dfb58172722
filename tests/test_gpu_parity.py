"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Tolerances: implementation parity of the same truncated algorithm (same trees,
same order p, same operators up to quadrature and rounding) is held to 1e-10
relative, the FP64 target; component operators to 1e-11 relative to their
largest entry (different quadrature node sets on the two sides).
"""
import hashlib

import numpy as np
import pytest

import oracle as O
from paper_1902_05132_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FMM = 1e-10
TOL_OP = 1e-11


def _lfmm():
    from paper_1902_05132_amd import lfmm
    return lfmm


def gate_norm_rel(A, B, p, kt, ks, h):
    """Relative error of A against B in the norm weighing entry (n, n') by
    (k_t h)^n (k_s h)^n' / ((2n+1)!! (2n'+1)!!)."""
    n = np.array([int(np.sqrt(i)) for i in range((p + 1) ** 2)])
    df = np.array([np.prod(np.arange(1, 2 * v + 2, 2, dtype=float)) for v in range(p + 1)])
    W = np.outer((kt * h) ** n / df[n], (ks * h) ** n / df[n])
    return np.sqrt(np.sum(W ** 2 * np.abs(A - B) ** 2) / np.sum(W ** 2 * np.abs(B) ** 2))


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


STACKS = [
    ("three_layer", (0.0, -1.2), (0.8, 1.5, 2.0)),
    ("five_layer", (0.0, -0.6, -1.2, -1.8), (0.5, 1.2, 2.0, 2.8, 3.0)),
    ("two_layer", (0.3,), (2.3, 1.1)),
]


@pytest.mark.parametrize("name,d,k", STACKS)
def test_densities_match_oracle(name, d, k):
    lf = _lfmm()
    P = lf.Plan(d, k, p=3, leaf_max=16)
    kr = np.concatenate([-1j * np.linspace(0.01, 0.5, 7), np.linspace(0.0, 6.0, 25) - 0.5j,
                         np.linspace(10, 300, 9) - 0.5j])
    for l in range(len(k)):
        for lp in range(len(k)):
            g = P.densities(kr, l, lp)
            ref = np.array([O.densities(d, k, z, l, lp) for z in kr])
            scale = np.maximum(np.abs(ref), 1e-300)
            mask = np.abs(ref) > 1e-200
            err = np.abs(g - ref)[mask] / scale[mask]
            assert np.all(err < 1e-12), (name, l, lp, err.max())
            assert np.all(np.abs(g[~mask]) < 1e-200)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("p", [3, 5, 8, 10])
def test_translation_operators_match_oracle(kind, p):
    lf = _lfmm()
    P = lf.Plan((0.0,), (1.0, 1.0), p=p, leaf_max=16)
    for kw, b in [(1.3, (0.3, -0.7, 1.1)), (0.8, (-0.125, 0.125, -0.125)), (2.0, (0.0, 0.0, 0.6)),
                  (1.5, (0.9, 0.0, 0.0))]:
        G = P.translation(kind, kw, b)
        R = O.translation(kind, kw, b, p, cached=True)
        assert rel(G, R) < TOL_OP, (kind, p, kw, b, rel(G, R))


@pytest.mark.parametrize("p", [3, 5, 8, 10])
def test_reaction_operators_match_oracle(p):
    lf = _lfmm()
    d, k = (0.0, -1.2), (0.8, 1.5, 2.0)
    P = lf.Plan(d, k, p=p, leaf_max=16)
    cases = [(0, 0, 1, 0, 0.55, -0.3, 0.4, 0.5), (1, 1, 2, 1, 0.0, 0.0, 0.3, 0.3), (2, 1, 0, 0, -1.1, 0.6, 0.15, 0.9),
             (1, 0, 1, 1, 0.275, 0.55, 0.1375, 0.4125), (0, 0, 0, 0, 0.2, 0.0, 0.05, 0.05),
             (2, 1, 2, 1, 0.6, -0.6, 0.1, 0.1), (1, 1, 0, 0, -0.35, 0.3, 0.2, 0.06)]
    for l, a, lp, b, dx, dy, zt, zs in cases:
        G = P.reaction_operator(l, a, lp, b, dx, dy, zt, zs)
        R = O.reaction_T(d, k, l, a, lp, b, dx, dy, zt, zs, p)
        # two correct quadratures of these oscillatory integrals differ by rounding of
        # the order of eps times the sum of |terms| (plus a tiny relative floor)
        mass = O.reaction_T_mass(d, k, l, a, lp, b, dx, dy, zt, zs, p)
        bound = 64 * 2.2e-16 * mass + TOL_OP * np.max(np.abs(R))
        assert np.all(np.abs(G - R) <= bound), (l, a, lp, b, rel(G, R), np.max(np.abs(G - R) / bound))
        # entrywise, deep classes at p >= 8 carry cancellation errors far above 1e-11 of
        # max|T| in their highest orders (the bound above admits them); what an operator
        # does to expansions of boxes of size h is measured by the gate norm, which
        # weighs entry (n, n') by (k_t h)^n (k_s h)^n' / ((2n+1)!! (2n'+1)!!): there the
        # two quadratures must agree to 1e-11 (the oracle's two contours agree to 3e-12)
        h = 2 * min(zt, zs)
        eg = gate_norm_rel(G, R, p, k[l], k[lp], h)
        assert eg < TOL_OP, (l, a, lp, b, p, eg)


_ORACLE_FMM = {}


def _oracle_fmm(w, p, leaf):
    """The oracle's FMM of a workload, kept for the tests that share it."""
    h = hashlib.sha256()
    for a in (w["d"], w["k"], w["x"], w["y"], w["z"], w["layer"], w["q"]):
        h.update(np.ascontiguousarray(a).tobytes())
    key = (h.hexdigest(), p, leaf)
    if key not in _ORACLE_FMM:
        _ORACLE_FMM[key] = O.fmm(w["d"], w["k"], p, leaf, w["x"], w["y"], w["z"], w["layer"], w["q"])
    return _ORACLE_FMM[key]


def _check_fmm(w, p, leaf, tol=TOL_FMM):
    lf = _lfmm()
    P = lf.Plan(w["d"], w["k"], p=p, leaf_max=leaf)
    phi = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
    rep = P.report()
    ref, info = _oracle_fmm(w, p, leaf)
    L = len(w["d"])
    assert rep["free_depth"][:L + 1] == [int(v) for v in info[:L + 1]]
    assert rep["reaction_depth"] == int(info[L + 1])
    e = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    emax = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    assert e < tol and emax < tol, (e, emax)
    return phi, ref, rep


def test_fmm_small_three_layer():
    w = W.small_three_layer(n_per_layer=60, seed=11)
    _check_fmm(w, p=4, leaf=12)


def test_fmm_three_layer_ragged():
    w = W.layered_cubes(W.THREE_LAYER_D, W.THREE_LAYER_K, [211, 97, 143], W.THREE_LAYER_CENTERS, seed=12)
    _check_fmm(w, p=5, leaf=9)


def test_fmm_three_layer_3k_full():
    """Config 1: 3 x 1000 particles, p = 5, leaf <= 50; every target against the oracle FMM."""
    w = W.three_layer_3k()
    phi, ref, rep = _check_fmm(w, p=w["p"], leaf=w["leaf"])
    # and against the exact sum on a sample: the FMM truncation error at p = 5
    tg = np.arange(0, len(w["x"]), 97)
    ex = O.direct(w["d"], w["k"], w["x"], w["y"], w["z"], w["layer"], w["q"], tg)
    assert np.linalg.norm(phi[tg] - ex) / np.linalg.norm(ex) < 1e-3


@pytest.mark.parametrize("p", [8, 10])
def test_fmm_bench_tree_shape(p):
    """The benchmark's launch configuration at a size the oracle's FMM finishes in
    seconds: three-layer cubes, leaf bound 256 (about 128 particles per leaf, the
    full-size run has about 85), reaction trees of depth 5 (the interface gap rule,
    as at full size), p = 8 (the bench's order: the (p+1)^2 = 81 row tiles, P2M and
    L2P at order 8) and p = 10; FP64 path against the oracle's FMM on the same trees."""
    w = W.three_layer_cubes(n=24576, seed=2, p=p, leaf=256)
    phi, ref, rep = _check_fmm(w, p=p, leaf=256)
    assert rep["free_depth"][:3] == [2, 2, 2] and rep["reaction_depth"] == 5


@pytest.mark.parametrize("p", [8, 10])
def test_fmm_bench_tree_shape_mixed(p):
    """The same in mixed precision against the oracle's FMM: the FP32 kernels the
    bench times at its launch configuration, within the 1e-6 bar."""
    lf = _lfmm()
    w = W.three_layer_cubes(n=24576, seed=2, p=p, leaf=256)
    P = lf.Plan(w["d"], w["k"], p=p, leaf_max=256, precision=1, quad_tol=1e-10)
    phi = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
    ref, _ = _oracle_fmm(w, p, 256)
    e = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    emax = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    assert e < 1e-6 and emax < 1e-6, (e, emax)


@pytest.mark.parametrize("p", [1, 2, 3, 6, 7, 9])
def test_fmm_every_order(p):
    """The expansion orders no other end-to-end test takes: every compiled P2M / L2P
    order and every M2L tile shape (one tile at p <= 3, three plus a vector-ALU row at
    6, four at 7, seven at 9), FP64 against the oracle's FMM at 1e-10 and mixed
    precision within the 1e-6 bar."""
    w = W.small_three_layer(n_per_layer=150, seed=13)
    _, ref, rep = _check_fmm(w, p=p, leaf=10)
    assert rep["free_depth"][:3] == [2, 2, 2]  # free-space M2L too, not only the reaction part
    assert rep["m2l_ks"] == 8  # few tiles: eight waves share each tile's operators
    P = _lfmm().Plan(w["d"], w["k"], p=p, leaf_max=10, precision=1, quad_tol=1e-10)
    phi = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
    e = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    emax = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    assert e < 1e-6 and emax < 1e-6, (e, emax)


def test_stage_events_levels():
    """Stage times: every stage at profile 1, only the roofline stages (M2L, near field,
    node sums, P2M, L2P) at profile 2, none at 0; the potentials are the same bits."""
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=150, seed=13)
    out = {}
    for level in (0, 1, 2):
        P = lf.Plan(w["d"], w["k"], p=5, leaf_max=10, profile=level)
        out[level] = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
        st = P.report()["stage_ms"]
        light = {"m2l", "p2p_free", "react_mfma", "p2m", "l2p"}
        if level == 0:
            assert all(v == 0 for v in st.values()), st
        elif level == 1:
            assert st["tree"] > 0 and st["m2l"] > 0 and st["jobs"] > 0, st
        else:
            assert all(st[k] > 0 for k in light), st
            assert all(v == 0 for k, v in st.items() if k not in light), st
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def _cube(n, side, centre, seed):
    rng = np.random.default_rng(seed)
    pts = centre + side * (rng.random((n, 3)) - 0.5)
    q = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    return pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(), q


@pytest.mark.parametrize("side,k,form", [(0.05, 2.0, 2), (0.1, 2.0, 1), (1.0, 2.0, 0), (0.05, 9.0, 0)])
def test_near_field_only_free_space(side, k, form):
    """One medium, every particle in one leaf: the result is the plain pair sum.
    The host bounds k r by 2 k side sqrt(3): side 0.05 with k = 2 (0.35 <= 1/2)
    takes the shorter series for sin(x)/x and cos(x), side 0.1 with k = 2 (0.69 <= 1)
    the full series; side 1 with k = 2 (6.9) and side 0.05 with k = 9 (1.56) exceed
    the bound and take the library sincos path."""
    lf = _lfmm()
    x, y, z, q = _cube(700, side, np.array([0.2, -0.1, 0.3]), seed=21)
    P = lf.Plan((), (k,), p=4, leaf_max=1000)
    phi = P.eval_torch(x, y, z, q)
    rep = P.report()
    assert rep["free_depth"][0] == 0 and rep["p2p_series"] == form
    assert rep["p2p_pairs"] == 700 * 699
    ref = O.direct((), (k,), x, y, z, np.zeros(700, np.int32), q, np.arange(700))
    assert rel(phi, ref) < 1e-12, rel(phi, ref)


def test_free_space_fmm_single_layer():
    """L = 0 (homogeneous medium): free-space FMM only, against the oracle's FMM."""
    rng = np.random.default_rng(5)
    n = 1500
    x, y, z = rng.random(n), rng.random(n), rng.random(n)
    q = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    w = dict(d=(), k=(1.7,), x=x, y=y, z=z, layer=np.zeros(n, np.int32), q=q)
    _check_fmm(w, p=6, leaf=20)


def _m2l_list_count(level):
    """Interaction-list entries at one level of a full uniform tree: pairs of cells
    whose parents are adjacent (or equal) and which are not adjacent themselves,
    counted by brute force over the grid."""
    n = 1 << level
    c = np.arange(n)
    total = 0
    for ix in range(n):
        ax = (np.abs(c // 2 - ix // 2) <= 1)
        nx = (np.abs(c - ix) <= 1)
        for iy in range(n):
            ay = (np.abs(c // 2 - iy // 2) <= 1)
            ny = (np.abs(c - iy) <= 1)
            for iz in range(n):
                az = (np.abs(c // 2 - iz // 2) <= 1)
                nz = (np.abs(c - iz) <= 1)
                par = ax[:, None, None] & ay[None, :, None] & az[None, None, :]
                adj = nx[:, None, None] & ny[None, :, None] & nz[None, None, :]
                total += int(np.count_nonzero(par & ~adj))
    return total


def test_translation_pair_counts_full_tree():
    """Homogeneous medium, 20,000 uniform particles, leaf <= 100: the depth rule gives
    depth 3 (level 2 holds about 312 particles per cell, level 3 about 39) and every
    level-3 cell is occupied (a Poisson(39) cell is empty with probability e^-39).
    The tree is then the full octree: 585 boxes, one M2M and one L2L per level-3
    box, and the M2L products of the full interaction lists at levels 2 and 3."""
    lf = _lfmm()
    rng = np.random.default_rng(17)
    n = 20000
    x, y, z = rng.random(n), rng.random(n), rng.random(n)
    q = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    P = lf.Plan((), (1.1,), p=4, leaf_max=100)
    P.eval_torch(x, y, z, q)
    rep = P.report()
    assert rep["free_depth"][0] == 3
    assert rep["n_boxes"] == 1 + 8 + 64 + 512
    assert rep["m2m_pairs"] == 512 and rep["l2l_pairs"] == 512
    assert rep["m2l_pairs"] == _m2l_list_count(2) + _m2l_list_count(3)


def test_empty_and_single_particle():
    lf = _lfmm()
    d, k = W.THREE_LAYER_D, W.THREE_LAYER_K
    P = lf.Plan(d, k, p=4, leaf_max=16)
    assert len(P.eval_torch([], [], [], [])) == 0
    one = ([0.1], [0.2], [0.5], [1.0 + 2.0j])
    phi = P.eval_torch(*one)
    # a lone particle sees only its own reaction field
    ref, _ = O.fmm(d, k, 4, 16, *one[:3], [0], one[3])
    assert abs(phi[0] - ref[0]) <= 1e-10 * abs(ref[0])
    ex = O.direct(d, k, *one[:3], [0], one[3], [0])
    assert abs(phi[0] - ex[0]) <= 1e-3 * abs(ex[0])


def test_empty_layer():
    """Particles in the top and bottom layers only: the middle layer has no tree."""
    w = W.layered_cubes(W.THREE_LAYER_D, W.THREE_LAYER_K, [300, 0, 250], W.THREE_LAYER_CENTERS, seed=13)
    _check_fmm(w, p=4, leaf=12)


def test_given_layers_match_derived_and_permutation():
    """Passing layer ids gives the same result as deriving them from z, and a
    permutation of the particles permutes the potentials."""
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=80, seed=17)
    P = lf.Plan(w["d"], w["k"], p=4, leaf_max=12)
    a = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
    b = P.eval_torch(w["x"], w["y"], w["z"], w["q"], layer=w["layer"])
    assert np.array_equal(a, b)
    perm = np.random.default_rng(3).permutation(len(a))
    c = P.eval_torch(w["x"][perm], w["y"][perm], w["z"][perm], w["q"][perm])
    assert rel(c, a[perm]) < 1e-13


def test_particle_on_interface_rejected():
    lf = _lfmm()
    P = lf.Plan(W.THREE_LAYER_D, W.THREE_LAYER_K, p=4, leaf_max=12)
    with pytest.raises(lf.LfmmError) as e:
        P.eval_torch([0.1, 0.2], [0.0, 0.1], [0.5, 0.0], [1.0, 1.0])
    assert e.value.code == 1


def test_host_entry_point_matches_device():
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=50, seed=19)
    P = lf.Plan(w["d"], w["k"], p=4, leaf_max=12)
    a = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
    b = P.eval_host(w["x"], w["y"], w["z"], w["q"])
    assert np.array_equal(a, b)


def test_five_layer_fmm():
    d, k = (0.0, -0.6, -1.2, -1.8), (0.5, 1.2, 2.0, 2.8, 3.0)
    cen = (0.35, -0.3, -0.9, -1.5, -2.15)
    w = W.layered_cubes(d, k, [90, 70, 70, 70, 90], cen, side=0.5, seed=23)
    _check_fmm(w, p=4, leaf=10)


def test_five_interface_fmm():
    """Five interfaces, the shallowest stack whose densities come from the per-node
    layer tables (uneven counts per layer), against the oracle's FMM."""
    d = tuple(-0.6 * i for i in range(5))
    k = tuple(0.6 + 0.4 * i for i in range(6))
    w = W.layered_cubes(d, k, [30, 25, 30, 25, 30, 35], (0.3, -0.3, -0.9, -1.5, -2.1, -2.7), side=0.3, seed=41)
    _check_fmm(w, p=4, leaf=10)


def test_ten_interface_fmm():
    """Ten interfaces, eleven layers: 400 reaction components, against the oracle's FMM."""
    w = W.ten_layer(n=330, seed=31, p=4, leaf=10)
    _check_fmm(w, p=4, leaf=10)


def test_separate_targets():
    """Targets apart from the sources (every layer, one on a source position):
    against the oracle's FMM on the union with zero target charges (same trees,
    1e-10) and against the exact sum (truncation)."""
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=120, seed=41)
    rng = np.random.default_rng(42)
    tx = rng.uniform(-0.5, 0.5, 30)
    ty = rng.uniform(-0.5, 0.5, 30)
    tz = np.concatenate([rng.uniform(0.1, 1.1, 10), rng.uniform(-1.1, -0.1, 10), rng.uniform(-2.3, -1.3, 10)])
    tx[0], ty[0], tz[0] = w["x"][0], w["y"][0], w["z"][0]  # coincides with a source
    P = lf.Plan(w["d"], w["k"], p=5, leaf_max=12)
    phi = P.eval_targets_torch(w["x"], w["y"], w["z"], w["q"], tx, ty, tz)
    assert np.array_equal(phi, P.eval_targets_host(w["x"], w["y"], w["z"], w["q"], tx, ty, tz))
    ns = len(w["x"])
    ux, uy, uz = np.concatenate([w["x"], tx]), np.concatenate([w["y"], ty]), np.concatenate([w["z"], tz])
    ul = np.concatenate([w["layer"], (tz < 0).astype(np.int32) + (tz < -1.2).astype(np.int32)])
    uq = np.concatenate([w["q"], np.zeros(30, complex)])
    ref, _ = O.fmm(w["d"], w["k"], 5, 12, ux, uy, uz, ul, uq)
    assert rel(phi, ref[ns:]) < TOL_FMM, rel(phi, ref[ns:])
    ex = O.direct(w["d"], w["k"], ux, uy, uz, ul, uq, np.arange(ns, ns + 30))
    assert np.linalg.norm(phi - ex) / np.linalg.norm(ex) < 1e-3


def test_batch_matches_single_and_oracle():
    """lfmm_eval_batch over independent media (the batching workload's recipe,
    smaller N): every problem equals its own single evaluation bit for bit, and
    the smallest problem matches the oracle's FMM (same trees, 1e-10)."""
    import torch
    lf = _lfmm()
    probs = W.batch_three_layer(seed=5, nprob=12, nmin=1500, nmax=6000)
    dev = torch.device("cuda")
    plans, xyzs, qs, phis, singles = [], [], [], [], []
    for w in probs:
        P = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"])
        xyz = torch.tensor(np.stack([w["x"], w["y"], w["z"]]), dtype=torch.float64, device=dev).contiguous()
        q = torch.tensor(w["q"], dtype=torch.complex128, device=dev)
        plans.append(P)
        xyzs.append(xyz)
        qs.append(q)
        phis.append(torch.empty_like(q))
        s1 = torch.empty_like(q)
        P.eval_device(xyz, q, s1)
        singles.append(s1)
    torch.cuda.synchronize()
    st = lf.eval_batch(plans, xyzs, qs, phis, nworkers=4)
    torch.cuda.synchronize()
    assert st == [0] * len(probs)
    for a, b in zip(phis, singles):
        assert torch.equal(a, b)
    i = int(np.argmin([len(w["x"]) for w in probs]))
    w = probs[i]
    ref, _ = O.fmm(w["d"], w["k"], w["p"], w["leaf"], w["x"], w["y"], w["z"], w["layer"], w["q"])
    assert rel(phis[i].cpu().numpy(), ref) < TOL_FMM


def test_batch_rejects_repeated_plan():
    import torch
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=30, seed=43)
    P = lf.Plan(w["d"], w["k"], p=4, leaf_max=12)
    dev = torch.device("cuda")
    xyz = torch.tensor(np.stack([w["x"], w["y"], w["z"]]), dtype=torch.float64, device=dev).contiguous()
    q = torch.tensor(w["q"], dtype=torch.complex128, device=dev)
    with pytest.raises(lf.LfmmError):
        lf.eval_batch([P, P], [xyz, xyz], [q, q], [torch.empty_like(q), torch.empty_like(q)])


def test_reaction_near_field_only():
    """Reaction trees of depth 1 (max_depth = 1): every reaction interaction is in
    the near field, summed pair by pair with the Sommerfeld quadrature; against
    the oracle's FMM with the same cap (1e-10) and the exact sum."""
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=40, seed=47)
    P = lf.Plan(w["d"], w["k"], p=4, leaf_max=1000, max_depth=1)
    phi = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
    rep = P.report()
    assert rep["reaction_depth"] == 1 and rep["nf_react_pairs"] > 0
    ref, info = O.fmm(w["d"], w["k"], 4, 1000, w["x"], w["y"], w["z"], w["layer"], w["q"], max_depth=1)
    assert int(info[3]) == 1
    assert rel(phi, ref) < TOL_FMM, rel(phi, ref)
    ex = O.direct(w["d"], w["k"], w["x"], w["y"], w["z"], w["layer"], w["q"], np.arange(len(w["x"])))
    assert rel(phi, ex) < 1e-11, rel(phi, ex)


def test_five_layer_clustered():
    """The five-layer Gaussian-cluster workload (its recipe, N = 5000, p = 5):
    clustered particles 0.05 from the interfaces give uneven, deeper trees."""
    w = W.five_layer_clusters(n=5000, p=5, leaf=64)
    phi, ref, rep = _check_fmm(w, p=5, leaf=64)
    assert rep["reaction_depth"] >= 5


def test_five_layer_clusters_p10():
    """Config 5's recipe at N = 24,000 (seed 11), p = 10, leaf <= 64: clusters 0.05 from
    the interfaces (reaction trees six levels deep), every reaction component of the
    five layers, the order-10 kernels.  FP64 against the oracle's FMM at 1e-10 (depths
    equal); the mixed path within 1e-6 of the FP64 path."""
    lf = _lfmm()
    w = W.five_layer_clusters(n=24000, seed=11, p=10, leaf=64)
    phi, ref, rep = _check_fmm(w, p=10, leaf=64)
    assert rep["reaction_depth"] >= 6
    pm = lf.Plan(w["d"], w["k"], p=10, leaf_max=64, precision=1, quad_tol=1e-10).eval_torch(
        w["x"], w["y"], w["z"], w["q"])
    e2 = np.linalg.norm(pm - phi) / np.linalg.norm(phi)
    emax = np.max(np.abs(pm - phi)) / np.max(np.abs(phi))
    print("five-layer clusters, p = 10: mixed vs FP64 Err2 %.2e, Errmax %.2e" % (e2, emax))
    assert e2 < 1e-6 and emax < 1e-6, (e2, emax)


def test_physical_normalisation():
    lf = _lfmm()
    # one homogeneous layer, two particles: the physical potential is the closed form
    k = 1.3
    x, y, z = np.array([0.1, 0.4]), np.array([-0.2, 0.3]), np.array([0.0, 0.25])
    q = np.array([1.0 + 0.5j, -0.3 + 2.0j])
    P = lf.Plan([], [k], p=4, leaf_max=8, physical=True)
    phi = P.eval_torch(x, y, z, q)
    r = np.sqrt((x[0] - x[1]) ** 2 + (y[0] - y[1]) ** 2 + (z[0] - z[1]) ** 2)
    g = np.exp(1j * k * r) / (4 * np.pi * r)
    assert np.allclose(phi, [q[1] * g, q[0] * g], rtol=1e-14, atol=0)
    # three layers: Phi times i k_l / (4 pi), layer by layer
    w = W.small_three_layer(n_per_layer=80, seed=5)
    a = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"]).eval_torch(w["x"], w["y"], w["z"], w["q"])
    b = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], physical=True).eval_torch(w["x"], w["y"], w["z"], w["q"])
    kl = np.asarray(w["k"])[w["layer"]]
    assert np.allclose(b, a * 1j * kl / (4 * np.pi), rtol=1e-15, atol=0)


def test_operator_reuse_on_unchanged_trees():
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=300, seed=11)
    for prec in (0, 1):
        P = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=prec, reuse_operators=True)
        a = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
        assert P.report()["ops_reused"] == 0
        b = P.eval_torch(w["x"], w["y"], w["z"], 2.0 * w["q"])  # same trees, other charges
        assert P.report()["ops_reused"] == 1
        assert np.array_equal(b, 2.0 * a) or np.allclose(b, 2.0 * a, rtol=1e-14, atol=0)
        # moved particles: whatever the plan reuses must give the result of a fresh plan
        # (operators depend only on the trees' box sizes, so a shift inside the same
        # roots may keep them)
        fresh_plan = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=prec)
        x2 = w["x"] * 0.9
        c = P.eval_torch(x2, w["y"], w["z"], w["q"])
        assert np.array_equal(c, fresh_plan.eval_torch(x2, w["y"], w["z"], w["q"]))
        # stretched laterally: larger roots, so the operators are generated again
        x3, y3 = w["x"] * 1.3, w["y"] * 1.3
        d = P.eval_torch(x3, y3, w["z"], w["q"])
        assert P.report()["ops_reused"] == 0
        assert np.array_equal(d, fresh_plan.eval_torch(x3, y3, w["z"], w["q"]))


def test_quadrature_tolerance_option():
    """quad_tol ends the Sommerfeld contour earlier: fewer nodes, and a potential that
    moves by at most a small multiple of the tolerance from the default contour's;
    values outside (0, 1) are rejected."""
    lf = _lfmm()
    w = W.three_layer_3k()
    a = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"])
    pa = a.eval_torch(w["x"], w["y"], w["z"], w["q"])
    na = a.report()["n_react_nodes"]
    for tol in (1e-6, 1e-10):
        b = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], quad_tol=tol)
        pb = b.eval_torch(w["x"], w["y"], w["z"], w["q"])
        nb = b.report()["n_react_nodes"]
        e = float(np.linalg.norm(pb - pa) / np.linalg.norm(pa))
        print("quad_tol %.0e: %d of %d class-nodes, Err2 vs the default contour %.2e" % (tol, nb, na, e))
        assert nb < na
        assert e < 10 * tol
    for bad in (-1.0, 1.0, 1.5):
        with pytest.raises(lf.LfmmError) as ex:
            lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], quad_tol=bad)
        assert ex.value.code == 1


def test_quadrature_node_budget():
    """A plan whose node budget is below what the workload's reaction classes need fails
    the evaluation with LFMM_ENOCONV (no output claimed); the same plan parameters with
    the default budget evaluate, and the budget equal to the largest class's count passes."""
    lf = _lfmm()
    w = W.three_layer_3k()
    a = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"])
    pa = a.eval_torch(w["x"], w["y"], w["z"], w["q"])
    b = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], quad_max_nodes=64)
    with pytest.raises(lf.LfmmError) as ex:
        b.eval_torch(w["x"], w["y"], w["z"], w["q"])
    assert ex.value.code == lf.LFMM_ENOCONV
    c = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], quad_max_nodes=1 << 16)
    assert np.array_equal(c.eval_torch(w["x"], w["y"], w["z"], w["q"]), pa)


def test_autotune_keeps_results():
    import torch
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=400, seed=13)
    dev = torch.device("cuda")
    xyz = torch.tensor(np.stack([w["x"], w["y"], w["z"]]), dtype=torch.float64, device=dev).contiguous()
    q = torch.tensor(w["q"], dtype=torch.complex128, device=dev)
    for prec in (0, 1):
        ref = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=prec).eval_torch(
            w["x"], w["y"], w["z"], w["q"])
        P = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=prec)
        phi = torch.empty_like(q)
        r = P.autotune(xyz, q, phi)
        torch.cuda.synchronize()
        assert r["gemm_ks"] in (1, 2, 4, 8) and r["trials"] >= 3 and r["ms_best"] <= r["ms_default"]
        after = P.eval_torch(w["x"], w["y"], w["z"], w["q"])
        # a different tile shape changes the summation order only
        assert rel(after, ref) < (1e-13 if prec == 0 else 1e-6)
        assert rel(phi.cpu().numpy(), ref) < (1e-13 if prec == 0 else 1e-6)
