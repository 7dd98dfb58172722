"""Positions prepared once, charges applied many times (lfmm_prepare / lfmm_apply), in
a captured HIP graph, and the batch of independent problems launched as one graph
(lfmm_batch_*).  Each result must equal lfmm_eval_device's bit for bit (the same
kernels in the same order on the same data); the oracle's FMM pins the batch's
smallest, median and largest problem at the FP64 bar (same trees, 1e-10)."""
import numpy as np
import pytest

import oracle as O
from paper_1902_05132_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FMM = 1e-10


def _lfmm():
    from paper_1902_05132_amd import lfmm
    return lfmm


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def _dev(w):
    import torch
    dev = torch.device("cuda")
    xyz = torch.tensor(np.stack([w["x"], w["y"], w["z"]]), dtype=torch.float64, device=dev).contiguous()
    q = torch.tensor(w["q"], dtype=torch.complex128, device=dev)
    return xyz, q


def _charges(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    q = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    return torch.tensor(q, dtype=torch.complex128, device="cuda")


CASES = [("three_layer_3k", 0), ("three_layer_3k", 1), ("five_layer_small", 0)]


def _workload(name):
    if name == "three_layer_3k":
        return W.three_layer_3k()
    return W.five_layer_clusters(n=6000, seed=9, p=5, leaf=40)


@pytest.mark.parametrize("name,precision", CASES)
def test_apply_equals_eval_bitwise(name, precision):
    import torch
    lf = _lfmm()
    w = _workload(name)
    xyz, q = _dev(w)
    n = xyz.shape[1]
    A = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=precision)
    ref = A.eval_device(xyz, q, torch.empty_like(q))
    q2 = _charges(n, 77)
    ref2 = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=precision).eval_device(
        xyz, q2, torch.empty_like(q2))
    # after lfmm_eval_device on the same plan
    out = A.apply(q, torch.full_like(q, 7.0))
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # after lfmm_prepare on a fresh plan, two charge sets, twice each
    B = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=precision)
    B.prepare(xyz)
    rep = B.report()
    assert rep["n_boxes"] > 0 and rep["m2l_pairs"] == A.report()["m2l_pairs"]
    for _ in range(2):
        a = B.apply(q2, torch.empty_like(q2))
        b = B.apply(q, torch.empty_like(q))
        torch.cuda.synchronize()
        assert torch.equal(a, ref2) and torch.equal(b, ref)


def test_apply_rejected_without_prepared_positions():
    import torch
    lf = _lfmm()
    w = W.small_three_layer(n_per_layer=40, seed=3)
    xyz, q = _dev(w)
    P = lf.Plan(w["d"], w["k"], p=4, leaf_max=16)
    with pytest.raises(lf.LfmmError):
        P.apply(q, torch.empty_like(q))
    # an evaluation on a lent workspace (allocation-free entry point) leaves nothing to apply
    P.eval_device_noalloc(xyz, q, torch.empty_like(q))
    rc = P.lib.lfmm_apply(P.h, q.data_ptr(), torch.empty_like(q).data_ptr(), None)
    assert rc == 1


@pytest.mark.parametrize("precision", [0, 1])
def test_apply_in_captured_graph(precision):
    """lfmm_apply captured into a HIP graph (torch's capture): every replay, with new
    charges written into the captured input between replays and eager work and
    synchronisations in between, equals the eager result bit for bit."""
    import torch
    lf = _lfmm()
    w = W.three_layer_3k()
    xyz, q = _dev(w)
    n = xyz.shape[1]
    P = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=precision)
    P.prepare(xyz)
    qbuf = q.clone()
    phibuf = torch.zeros_like(q)
    P.apply(qbuf, phibuf)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=s):
        P.apply(qbuf, phibuf)
    for trial in range(4):
        qn = _charges(n, 100 + trial)
        qbuf.copy_(qn)
        g.replay()
        torch.cuda.synchronize()
        got = phibuf.clone()
        eager = P.apply(qn, torch.empty_like(qn))
        torch.cuda.synchronize()
        assert torch.equal(got, eager), trial


def test_batch_graph_matches_single_and_oracle():
    """The batching workload's recipe at smaller N (12 problems, 1.5k-6k particles):
    one graph launch gives every problem its own single evaluation bit for bit, again
    after the charges change in place; the smallest, median and largest problems match
    the oracle's FMM (same trees, 1e-10)."""
    import torch
    lf = _lfmm()
    probs = W.batch_three_layer(seed=5, nprob=12, nmin=1500, nmax=6000)
    plans, xyzs, qs, phis = [], [], [], []
    for w in probs:
        xyz, q = _dev(w)
        plans.append(lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"]))
        xyzs.append(xyz)
        qs.append(q)
        phis.append(torch.zeros_like(q))
    assert lf.batch_prepare(plans, xyzs, nworkers=4) == [0] * len(probs)
    B = lf.Batch(plans, qs, phis, nbranch=4)
    r = B.report()
    print("batch: %d particles, %d graph nodes, %d branches, capture %.1f ms"
          % (r["n_total"], r["graph_nodes"], r["branches"], r["capture_ms"]), flush=True)
    assert r["n_total"] == sum(len(w["x"]) for w in probs) and r["graph_nodes"] > len(probs)
    for trial in range(2):
        if trial:
            for i, q in enumerate(qs):
                q.copy_(_charges(q.numel(), 200 + i))
        B.launch()
        torch.cuda.synchronize()
        for i, w in enumerate(probs):
            ref = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"]).eval_device(
                xyzs[i], qs[i], torch.empty_like(qs[i]))
            torch.cuda.synchronize()
            assert torch.equal(phis[i], ref), (trial, i)
    sizes = np.array([len(w["x"]) for w in probs])
    order = np.argsort(sizes)
    for i in (order[0], order[len(order) // 2], order[-1]):
        w = probs[i]
        qh = qs[i].cpu().numpy()
        ref, _ = O.fmm(w["d"], w["k"], w["p"], w["leaf"], w["x"], w["y"], w["z"], w["layer"], qh)
        assert rel(phis[i].cpu().numpy(), ref) < TOL_FMM, (i, rel(phis[i].cpu().numpy(), ref))
    B.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_m2l_split_one_on_long_operator_lists(precision):
    """M2L K-split 1 on a problem whose reaction groups list the most operators (every
    source slab occupied, reaction depth 6): one wave holds a target tile's whole list
    in LDS (above 64 KB).  K-split 8 there: eight waves of a 512-thread workgroup share
    each tile's list.  Same potentials as split 4 up to summation order."""
    import torch
    lf = _lfmm()
    probs = W.batch_three_layer(seed=3)
    w = probs[int(np.argmin([len(v["x"]) for v in probs]))]
    xyz, q = _dev(w)
    out = {}
    for ks in (1, 4, 8):
        P = lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=precision)
        P.set_tiles(ks, 8, 256)
        out[ks] = P.eval_device(xyz, q, torch.empty_like(q))
        torch.cuda.synchronize()
    b = out[4].cpu().numpy()
    for ks in (1, 8):
        a = out[ks].cpu().numpy()
        assert rel(a, b) < (1e-13 if precision == 0 else 1e-6), (ks, rel(a, b))


def test_repeated_batches_on_worker_streams():
    """lfmm_eval_batch twice on the same plans (each call's worker streams are gone by the
    next), then lfmm_batch_prepare, a plain evaluation and destruction of the plans:
    nothing waits on an event recorded on a stream that no longer exists."""
    import torch
    lf = _lfmm()
    probs = W.batch_three_layer(seed=8, nprob=6, nmin=1500, nmax=3000)
    plans, xyzs, qs = [], [], []
    for w in probs:
        xyz, q = _dev(w)
        plans.append(lf.Plan(w["d"], w["k"], p=w["p"], leaf_max=w["leaf"], precision=1))
        xyzs.append(xyz)
        qs.append(q)
    outs = []
    for r in range(2):
        phis = [torch.empty_like(q) for q in qs]
        assert lf.eval_batch(plans, xyzs, qs, phis, nworkers=3) == [0] * len(probs)
        torch.cuda.synchronize()
        outs.append(phis)
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    assert lf.batch_prepare(plans, xyzs, nworkers=3) == [0] * len(probs)
    for i, P in enumerate(plans):
        c = P.eval_device(xyzs[i], qs[i], torch.empty_like(qs[i]))
        torch.cuda.synchronize()
        assert torch.equal(c, outs[0][i])
        P.close()
