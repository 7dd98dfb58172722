"""Python binding of liblfmm.so (argument marshalling only).

Every stage of the evaluation runs in the HIP library; PyTorch only provides
device memory and the stream.  Loading fails loudly when the library is missing:
there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblfmm.so")

LFMM_OK = 0
NOALLOC_BYTES = 512 << 20  # LFMM_NOALLOC_BYTES of include/lfmm.h
_STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "HIP runtime error", 4: "not supported",
           5: "surrogate or table file error", 6: "Sommerfeld quadrature over its node budget"}
LFMM_ENOCONV = 6


class LfmmError(RuntimeError):
    def __init__(self, code, what, detail=""):
        super().__init__("%s failed: %s (status %d)%s" % (what, _STATUS.get(code, "?"), code,
                                                           ": " + detail if detail else ""))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("contour_b", ctypes.c_double), ("max_depth", ctypes.c_int), ("min_gap", ctypes.c_double),
                ("profile", ctypes.c_int), ("precision", ctypes.c_int), ("physical", ctypes.c_int),
                ("reuse_operators", ctypes.c_int), ("quad_tol", ctypes.c_double),
                ("quad_max_nodes", ctypes.c_int64)]


class Report(ctypes.Structure):
    _fields_ = [("n_trees", ctypes.c_int), ("free_depth", ctypes.c_int * 17), ("reaction_depth", ctypes.c_int),
                ("n_boxes", ctypes.c_int64), ("n_ops_free", ctypes.c_int64), ("n_react_classes", ctypes.c_int64),
                ("n_react_nodes", ctypes.c_int64), ("n_ops_react", ctypes.c_int64), ("m2l_pairs", ctypes.c_int64),
                ("m2l_slots", ctypes.c_int64), ("m2m_pairs", ctypes.c_int64), ("l2l_pairs", ctypes.c_int64),
                ("p2p_pairs", ctypes.c_int64), ("nf_react_pairs", ctypes.c_int64),
                ("p2p_series", ctypes.c_int), ("precision", ctypes.c_int),
                ("stage_ms", ctypes.c_double * 24), ("n_react_surrogate", ctypes.c_int64), ("ops_reused", ctypes.c_int),
                ("n_react_table", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("p2m_points", ctypes.c_int64), ("p2m_leaves", ctypes.c_int64),
                ("l2p_points", ctypes.c_int64), ("l2p_leaves", ctypes.c_int64), ("m2l_ks", ctypes.c_int)]


class BatchReport(ctypes.Structure):
    _fields_ = [("n_total", ctypes.c_int64), ("graph_nodes", ctypes.c_int64), ("branches", ctypes.c_int),
                ("capture_ms", ctypes.c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("gemm_ks", ctypes.c_int), ("p2p_ta", ctypes.c_int), ("p2p_ch", ctypes.c_int),
                ("trials", ctypes.c_int), ("ms_default", ctypes.c_double), ("ms_best", ctypes.c_double)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("h_min", ctypes.c_double), ("h_max", ctypes.c_double), ("epochs", ctypes.c_int),
                ("batch", ctypes.c_int), ("lr", ctypes.c_double), ("holdout", ctypes.c_double),
                ("width", ctypes.c_int), ("nhidden", ctypes.c_int)]


class TrainReport(ctypes.Structure):
    _fields_ = [("n_train", ctypes.c_int64), ("n_holdout", ctypes.c_int64), ("n_values", ctypes.c_int64),
                ("n_combos", ctypes.c_int), ("nin", ctypes.c_int), ("nout", ctypes.c_int),
                ("epochs", ctypes.c_int), ("steps", ctypes.c_int),
                ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("err_median", ctypes.c_double), ("err_max", ctypes.c_double),
                ("ms_labels", ctypes.c_double), ("ms_train", ctypes.c_double)]


class TableOpts(ctypes.Structure):
    _fields_ = [("h_min", ctypes.c_double), ("h_max", ctypes.c_double), ("nnode", ctypes.c_int),
                ("du", ctypes.c_double), ("nval", ctypes.c_int)]


class TableReport(ctypes.Structure):
    _fields_ = [("n_combos", ctypes.c_int), ("npanel", ctypes.c_int), ("nnode", ctypes.c_int),
                ("n_slots", ctypes.c_int64), ("n_validation", ctypes.c_int64), ("bytes", ctypes.c_int64),
                ("err_median", ctypes.c_double), ("err_max", ctypes.c_double),
                ("ms_build", ctypes.c_double), ("ms_validate", ctypes.c_double)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def load():
    """Load liblfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes liblfmm.so bind to that single runtime
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblfmm.so not found at %s: build it first (python -m paper_1902_05132_amd.build "
                          "or __graft_entry__.build())" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.lfmm_plan.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Options),
                            ctypes.POINTER(vp)]
    L.lfmm_eval_device.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp]
    L.lfmm_eval_device_noalloc.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp]
    L.lfmm_eval.argtypes = [vp, ctypes.c_int64, _D, ctypes.c_void_p, _D, _D]
    L.lfmm_eval_targets_device.argtypes = [vp, ctypes.c_int64, vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp]
    L.lfmm_eval_targets.argtypes = [vp, ctypes.c_int64, _D, vp, _D, ctypes.c_int64, _D, vp, _D]
    L.lfmm_eval_batch.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.lfmm_prepare.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
    L.lfmm_apply.argtypes = [vp, vp, vp, vp]
    L.lfmm_batch_prepare.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.lfmm_batch_capture.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(BatchReport)]
    L.lfmm_set_tiles.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.lfmm_batch_launch.argtypes = [vp, vp]
    L.lfmm_batch_destroy.argtypes = [vp]
    L.lfmm_batch_destroy.restype = None
    L.lfmm_last_report.argtypes = [vp, ctypes.POINTER(Report)]
    L.lfmm_stage_name.argtypes = [ctypes.c_int]
    L.lfmm_stage_name.restype = ctypes.c_char_p
    L.lfmm_destroy.argtypes = [vp]
    L.lfmm_destroy.restype = None
    L.lfmm_status_string.argtypes = [ctypes.c_int]
    L.lfmm_status_string.restype = ctypes.c_char_p
    L.lfmm_last_hip_error.argtypes = []
    L.lfmm_last_hip_error.restype = ctypes.c_char_p
    L.lfmm_quad_nodes.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, ctypes.POINTER(Options), ctypes.c_double,
                                  ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]
    L.lfmm_translation.argtypes = [vp, ctypes.c_int, ctypes.c_double, _D, _D]
    L.lfmm_reaction_operator.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
    L.lfmm_densities.argtypes = [vp, ctypes.c_int, _D, ctypes.c_int, ctypes.c_int, _D]
    L.lfmm_autotune.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.POINTER(TuneReport)]
    L.lfmm_surrogate_train.argtypes = [vp, ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(TrainOpts),
                                       ctypes.POINTER(TrainReport)]
    L.lfmm_surrogate_save.argtypes = [vp, ctypes.c_char_p]
    L.lfmm_surrogate_load.argtypes = [vp, ctypes.c_char_p]
    L.lfmm_surrogate_gate.argtypes = [vp, ctypes.c_double]
    L.lfmm_surrogate_bounds.argtypes = [vp, ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int)]
    L.lfmm_tables_build.argtypes = [vp, ctypes.POINTER(TableOpts), ctypes.POINTER(TableReport)]
    L.lfmm_tables_gate.argtypes = [vp, ctypes.c_double]
    L.lfmm_tables_bounds.argtypes = [vp, ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int)]
    L.lfmm_tables_release.argtypes = [vp]
    L.lfmm_tables_save.argtypes = [vp, ctypes.c_char_p]
    L.lfmm_tables_load.argtypes = [vp, ctypes.c_char_p]
    _F = ctypes.POINTER(ctypes.c_float)
    L.lfmm_mlp_forward_backward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            _F, _F, _F, _F, _F, _D]
    _lib = L
    return L


def _check(rc, what):
    if rc != LFMM_OK:
        detail = ""
        if rc == 3 and _lib is not None:
            detail = (_lib.lfmm_last_hip_error() or b"").decode(errors="replace")
        raise LfmmError(rc, what, detail)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dev_arg(t, name, dtype, numel, device=None):
    """Check a torch tensor handed to the library by address: on the GPU, contiguous,
    of the given dtype and with at least `numel` elements (and on `device` if given).
    A wrong argument would otherwise become an out-of-bounds device access."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise LfmmError(1, "%s: a torch tensor is required" % name)
    if not t.is_cuda:
        raise LfmmError(1, "%s: must be on the GPU" % name)
    if t.dtype != dtype:
        raise LfmmError(1, "%s: dtype %s, expected %s" % (name, t.dtype, dtype))
    if not t.is_contiguous():
        raise LfmmError(1, "%s: must be contiguous" % name)
    if t.numel() < numel:
        raise LfmmError(1, "%s: %d elements, at least %d needed" % (name, t.numel(), numel))
    if device is not None and t.device != device:
        raise LfmmError(1, "%s: on %s, the other arguments are on %s" % (name, t.device, device))
    return t.data_ptr()


def _xyz_arg(xyz, name):
    import torch
    if not isinstance(xyz, torch.Tensor) or xyz.dim() != 2 or xyz.shape[0] != 3:
        raise LfmmError(1, "%s: a (3, n) tensor is required" % name)
    n = int(xyz.shape[1])
    return n, _dev_arg(xyz, name, torch.float64, 3 * n)


def quad_nodes(d, k, p, dz, rho, contour_b=0.5, quad_tol=0.0, quad_max_nodes=0):
    """lfmm_quad_nodes: contour nodes of one reaction class at image distance dz and
    horizontal distance rho, for the medium (d, k) and order p.  Host only (no device).
    Returns (status, nodes): status 0, or LFMM_ENOCONV over quad_max_nodes."""
    lib = load()
    d = _f64(d)
    k = _f64(k)
    opt = Options(contour_b, 8, 1e-9, 0, 0, 0, 0, float(quad_tol), int(quad_max_nodes))
    out = ctypes.c_int64(0)
    rc = lib.lfmm_quad_nodes(len(d), d.ctypes.data_as(_D) if len(d) else None, k.ctypes.data_as(_D), int(p),
                             ctypes.byref(opt), float(dz), float(rho), ctypes.byref(out))
    if rc not in (LFMM_OK, LFMM_ENOCONV):
        raise LfmmError(rc, "lfmm_quad_nodes")
    return rc, int(out.value)


class Plan:
    """lfmm_plan wrapper: d (L interfaces, decreasing), k (L+1 wavenumbers), order p, leaf size."""

    def __init__(self, d, k, p, leaf_max, contour_b=0.5, max_depth=8, min_gap=1e-9, profile=False, precision=0,
                 physical=False, reuse_operators=False, quad_tol=0.0, quad_max_nodes=0):
        """precision 0: FP64 throughout; 1: mixed (FP32 near field and FP32-MFMA M2L).
        physical: return physical potentials (Phi times i k_l / (4 pi)) instead of Phi.
        reuse_operators: keep the previous evaluation's operators when its trees are the same.
        quad_tol: truncation of the Sommerfeld contour (0: the default e^-40).
        quad_max_nodes: contour nodes one reaction class may take (0: 2^20); more is LFMM_ENOCONV."""
        self.lib = load()
        self.d = _f64(d)
        self.k = _f64(k)
        self.p = int(p)
        self.L = len(self.d)
        opt = Options(contour_b, max_depth, min_gap, int(profile), int(precision), 1 if physical else 0,
                      1 if reuse_operators else 0, float(quad_tol), int(quad_max_nodes))
        h = ctypes.c_void_p()
        dptr = self.d.ctypes.data_as(_D) if self.L else None
        _check(self.lib.lfmm_plan(self.L, dptr, self.k.ctypes.data_as(_D), self.p, int(leaf_max),
                                  ctypes.byref(opt), ctypes.byref(h)), "lfmm_plan")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.lfmm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- device evaluation (torch tensors on the GPU) ----
    def eval_device(self, xyz, q, phi, layer=None, stream=None):
        """xyz: float64 (3, n) contiguous; q, phi: complex128 (n,) contiguous; layer: int32 (n,) or None."""
        import torch
        n, xp = _xyz_arg(xyz, "xyz")
        qp = _dev_arg(q, "q", torch.complex128, n, xyz.device)
        fp = _dev_arg(phi, "phi", torch.complex128, n, xyz.device)
        lp = _dev_arg(layer, "layer", torch.int32, n, xyz.device) if layer is not None else None
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(self.lib.lfmm_eval_device(self.h, n, xp, lp, qp, fp, ctypes.c_void_p(s.cuda_stream)),
               "lfmm_eval_device")
        self._prep_n = n
        return phi

    def prepare(self, xyz, layer=None, stream=None):
        """lfmm_prepare: trees, lists and operators for these positions (no charges)."""
        import torch
        n, xp = _xyz_arg(xyz, "xyz")
        lp = _dev_arg(layer, "layer", torch.int32, n, xyz.device) if layer is not None else None
        s = stream if stream is not None else torch.cuda.current_stream()
        self._prep_n = None
        _check(self.lib.lfmm_prepare(self.h, n, xp, lp, ctypes.c_void_p(s.cuda_stream)), "lfmm_prepare")
        self._prep_n = n
        return self

    def apply(self, q, phi, stream=None):
        """lfmm_apply: Phi for charges q (complex128 (n,)) at the prepared positions into
        phi; queued on the stream, no synchronisation (capturable into a graph)."""
        import torch
        n = getattr(self, "_prep_n", None)
        if n is None:
            raise LfmmError(1, "lfmm_apply: the plan has no prepared positions")
        qp = _dev_arg(q, "q", torch.complex128, n)
        fp = _dev_arg(phi, "phi", torch.complex128, n, q.device)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(self.lib.lfmm_apply(self.h, qp, fp, ctypes.c_void_p(s.cuda_stream)), "lfmm_apply")
        return phi

    def set_tiles(self, gemm_ks, p2p_ta, p2p_ch):
        """lfmm_set_tiles: tile shapes for later evaluations and preparations."""
        _check(self.lib.lfmm_set_tiles(self.h, int(gemm_ks), int(p2p_ta), int(p2p_ch)), "lfmm_set_tiles")

    def eval_device_noalloc(self, xyz, q, phi, layer=None, stream=None):
        """lfmm_eval_device_noalloc: as eval_device, with the workspace taken from the
        library's static device scratch (no allocation); synchronous."""
        import torch
        n, xp = _xyz_arg(xyz, "xyz")
        qp = _dev_arg(q, "q", torch.complex128, n, xyz.device)
        fp = _dev_arg(phi, "phi", torch.complex128, n, xyz.device)
        lp = _dev_arg(layer, "layer", torch.int32, n, xyz.device) if layer is not None else None
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(self.lib.lfmm_eval_device_noalloc(self.h, n, xp, lp, qp, fp, ctypes.c_void_p(s.cuda_stream)),
               "lfmm_eval_device_noalloc")
        return phi

    def eval_torch(self, x, y, z, q, layer=None):
        import torch
        dev = torch.device("cuda")
        xyz = torch.stack([torch.as_tensor(np.asarray(v, dtype=np.float64)) for v in (x, y, z)]).to(dev)
        qq = torch.as_tensor(np.asarray(q, dtype=np.complex128)).to(dev)
        lt = None if layer is None else torch.as_tensor(np.asarray(layer, dtype=np.int32)).to(dev)
        phi = torch.empty(len(x), dtype=torch.complex128, device=dev)
        self.eval_device(xyz.contiguous(), qq.contiguous(), phi, lt)
        torch.cuda.synchronize()
        return phi.cpu().numpy()

    def eval_targets_device(self, src_xyz, q, tgt_xyz, phi, src_layer=None, tgt_layer=None, stream=None):
        """Phi at separate targets.  src_xyz (3, ns), tgt_xyz (3, nt) float64 contiguous on the
        GPU; q (ns,), phi (nt,) complex128; layer ids int32 or None (both or neither)."""
        import torch
        ns, sp = _xyz_arg(src_xyz, "src_xyz")
        nt, tp = _xyz_arg(tgt_xyz, "tgt_xyz")
        dev = src_xyz.device
        if tgt_xyz.device != dev:
            raise LfmmError(1, "tgt_xyz: on %s, the sources are on %s" % (tgt_xyz.device, dev))
        qp = _dev_arg(q, "q", torch.complex128, ns, dev)
        fp = _dev_arg(phi, "phi", torch.complex128, nt, dev)
        if (src_layer is None) != (tgt_layer is None):
            raise LfmmError(1, "src_layer and tgt_layer: give both or neither")
        sl = _dev_arg(src_layer, "src_layer", torch.int32, ns, dev) if src_layer is not None else None
        tl = _dev_arg(tgt_layer, "tgt_layer", torch.int32, nt, dev) if tgt_layer is not None else None
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(self.lib.lfmm_eval_targets_device(self.h, ns, sp, sl, qp, nt, tp, tl, fp,
                                                 ctypes.c_void_p(s.cuda_stream)), "lfmm_eval_targets_device")
        return phi

    def eval_targets_torch(self, sx, sy, sz, q, tx, ty, tz):
        import torch
        dev = torch.device("cuda")
        S = torch.stack([torch.as_tensor(np.asarray(v, dtype=np.float64)) for v in (sx, sy, sz)]).to(dev)
        T = torch.stack([torch.as_tensor(np.asarray(v, dtype=np.float64)) for v in (tx, ty, tz)]).to(dev)
        qq = torch.as_tensor(np.asarray(q, dtype=np.complex128)).to(dev)
        phi = torch.empty(len(tx), dtype=torch.complex128, device=dev)
        self.eval_targets_device(S.contiguous(), qq.contiguous(), T.contiguous(), phi)
        torch.cuda.synchronize()
        return phi.cpu().numpy()

    def eval_targets_host(self, sx, sy, sz, q, tx, ty, tz):
        S = np.ascontiguousarray(np.concatenate([_f64(sx), _f64(sy), _f64(sz)]))
        T = np.ascontiguousarray(np.concatenate([_f64(tx), _f64(ty), _f64(tz)]))
        qq = np.ascontiguousarray(np.asarray(q, dtype=np.complex128)).view(np.float64)
        out = np.zeros(2 * len(tx))
        _check(self.lib.lfmm_eval_targets(self.h, len(sx), S.ctypes.data_as(_D), None, qq.ctypes.data_as(_D),
                                          len(tx), T.ctypes.data_as(_D), None, out.ctypes.data_as(_D)),
               "lfmm_eval_targets")
        return out[0::2] + 1j * out[1::2]

    # ---- host evaluation ----
    def eval_host(self, x, y, z, q, layer=None):
        n = len(x)
        xyz = np.ascontiguousarray(np.concatenate([_f64(x), _f64(y), _f64(z)]))
        qq = np.ascontiguousarray(np.asarray(q, dtype=np.complex128)).view(np.float64)
        out = np.zeros(2 * n)
        lay = None if layer is None else np.ascontiguousarray(np.asarray(layer, dtype=np.int32))
        lp = lay.ctypes.data_as(ctypes.c_void_p) if lay is not None else None
        _check(self.lib.lfmm_eval(self.h, n, xyz.ctypes.data_as(_D), lp, qq.ctypes.data_as(_D),
                                  out.ctypes.data_as(_D)), "lfmm_eval")
        return out[0::2] + 1j * out[1::2]

    def report(self):
        r = Report()
        _check(self.lib.lfmm_last_report(self.h, ctypes.byref(r)), "lfmm_last_report")
        stages = {}
        i = 0
        while True:
            nm = self.lib.lfmm_stage_name(i)
            if nm is None:
                break
            stages[nm.decode()] = r.stage_ms[i]
            i += 1
        return dict(n_trees=r.n_trees, free_depth=[r.free_depth[i] for i in range(self.L + 1)],
                    reaction_depth=r.reaction_depth, n_boxes=r.n_boxes, n_ops_free=r.n_ops_free,
                    n_react_classes=r.n_react_classes, n_react_nodes=r.n_react_nodes, n_ops_react=r.n_ops_react,
                    m2l_pairs=r.m2l_pairs, m2l_slots=r.m2l_slots,
                    m2m_pairs=r.m2m_pairs, l2l_pairs=r.l2l_pairs, p2p_pairs=r.p2p_pairs, nf_react_pairs=r.nf_react_pairs,
                    p2p_series=r.p2p_series, precision=r.precision,
                    n_react_surrogate=r.n_react_surrogate, ops_reused=r.ops_reused,
                    n_react_table=r.n_react_table, workspace_bytes=r.workspace_bytes,
                    p2m_points=r.p2m_points, p2m_leaves=r.p2m_leaves, l2p_points=r.l2p_points,
                    l2p_leaves=r.l2p_leaves, m2l_ks=r.m2l_ks, stage_ms=stages)

    def autotune(self, xyz, q, phi, layer=None, stream=None):
        """lfmm_autotune on torch device tensors (as eval_device); returns the tuning report."""
        import torch
        n, xp = _xyz_arg(xyz, "xyz")
        qp = _dev_arg(q, "q", torch.complex128, n, xyz.device)
        fp = _dev_arg(phi, "phi", torch.complex128, n, xyz.device)
        lp = _dev_arg(layer, "layer", torch.int32, n, xyz.device) if layer is not None else None
        s = stream if stream is not None else torch.cuda.current_stream()
        r = TuneReport()
        _check(self.lib.lfmm_autotune(self.h, n, xp, lp, qp, fp, ctypes.c_void_p(s.cuda_stream), ctypes.byref(r)),
               "lfmm_autotune")
        return {f: getattr(r, f) for f, _ in TuneReport._fields_}

    # ---- learned surrogate of the reaction integrals ----
    def surrogate_train(self, n_samples=0, seed=0, h_min=0.0, h_max=0.0, epochs=0, batch=0, lr=0.0, holdout=0.0,
                        width=0, nhidden=0):
        """Train on quadrature labels (zeros select the library defaults); returns the training report."""
        o = TrainOpts(h_min, h_max, epochs, batch, lr, holdout, width, nhidden)
        r = TrainReport()
        _check(self.lib.lfmm_surrogate_train(self.h, int(n_samples), int(seed), ctypes.byref(o), ctypes.byref(r)),
               "lfmm_surrogate_train")
        return {f: getattr(r, f) for f, _ in TrainReport._fields_}

    def surrogate_save(self, path):
        _check(self.lib.lfmm_surrogate_save(self.h, os.fsencode(path)), "lfmm_surrogate_save")

    def surrogate_load(self, path):
        _check(self.lib.lfmm_surrogate_load(self.h, os.fsencode(path)), "lfmm_surrogate_load")

    def surrogate_gate(self, tol):
        _check(self.lib.lfmm_surrogate_gate(self.h, float(tol)), "lfmm_surrogate_gate")

    def surrogate_bounds(self):
        cnt = ctypes.c_int()
        _check(self.lib.lfmm_surrogate_bounds(self.h, 0, None, ctypes.byref(cnt)), "lfmm_surrogate_bounds")
        out = np.zeros(max(cnt.value, 1))
        _check(self.lib.lfmm_surrogate_bounds(self.h, cnt.value, out.ctypes.data_as(_D), ctypes.byref(cnt)),
               "lfmm_surrogate_bounds")
        return out[:cnt.value]

    # ---- pre-computed tables of the reaction integrals ----
    def tables_build(self, h_min=0.0, h_max=0.0, nnode=0, du=0.0, nval=0):
        """Tabulate by quadrature and validate (zeros select the library defaults); returns the report."""
        o = TableOpts(h_min, h_max, nnode, du, nval)
        r = TableReport()
        _check(self.lib.lfmm_tables_build(self.h, ctypes.byref(o), ctypes.byref(r)), "lfmm_tables_build")
        return {f: getattr(r, f) for f, _ in TableReport._fields_}

    def tables_gate(self, tol):
        _check(self.lib.lfmm_tables_gate(self.h, float(tol)), "lfmm_tables_gate")

    def tables_bounds(self):
        cnt = ctypes.c_int()
        _check(self.lib.lfmm_tables_bounds(self.h, 0, None, ctypes.byref(cnt)), "lfmm_tables_bounds")
        out = np.zeros(max(cnt.value, 1))
        _check(self.lib.lfmm_tables_bounds(self.h, cnt.value, out.ctypes.data_as(_D), ctypes.byref(cnt)),
               "lfmm_tables_bounds")
        return out[:cnt.value]

    def tables_release(self):
        _check(self.lib.lfmm_tables_release(self.h), "lfmm_tables_release")

    def tables_save(self, path):
        _check(self.lib.lfmm_tables_save(self.h, os.fsencode(path)), "lfmm_tables_save")

    def tables_load(self, path):
        _check(self.lib.lfmm_tables_load(self.h, os.fsencode(path)), "lfmm_tables_load")

    # ---- component entry points ----
    def translation(self, kind, kw, b):
        nc = (self.p + 1) ** 2
        out = np.zeros(2 * nc * nc)
        bb = _f64(b)
        _check(self.lib.lfmm_translation(self.h, int(kind), float(kw), bb.ctypes.data_as(_D),
                                         out.ctypes.data_as(_D)), "lfmm_translation")
        return (out[0::2] + 1j * out[1::2]).reshape(nc, nc)

    def reaction_operator(self, l, a, lp, b, dx, dy, zt, zs):
        nc = (self.p + 1) ** 2
        out = np.zeros(2 * nc * nc)
        _check(self.lib.lfmm_reaction_operator(self.h, l, a, lp, b, float(dx), float(dy), float(zt), float(zs),
                                               out.ctypes.data_as(_D)), "lfmm_reaction_operator")
        return (out[0::2] + 1j * out[1::2]).reshape(nc, nc)

    def densities(self, krho, l, lp):
        kr = np.ascontiguousarray(np.asarray(krho, dtype=np.complex128)).view(np.float64)
        n = len(kr) // 2
        out = np.zeros(8 * n)
        _check(self.lib.lfmm_densities(self.h, n, kr.ctypes.data_as(_D), l, lp, out.ctypes.data_as(_D)),
               "lfmm_densities")
        return (out[0::2] + 1j * out[1::2]).reshape(n, 2, 2)


def eval_batch(plans, xyzs, qs, phis, layers=None, nworkers=8):
    """lfmm_eval_batch over torch device tensors: plans[i] with xyzs[i] (3, n_i) float64,
    qs[i] / phis[i] (n_i,) complex128 (all contiguous, on the GPU).  Returns the
    per-problem status codes; raises on failure."""
    import torch
    m = len(plans)
    if not (len(xyzs) == len(qs) == len(phis) == m) or (layers is not None and len(layers) != m):
        raise LfmmError(1, "eval_batch: one plan, xyz, q and phi (and layer) per problem")
    ns, xp, qp, fp, lp = [], [], [], [], []
    for i in range(m):
        n, p = _xyz_arg(xyzs[i], "xyzs[%d]" % i)
        dev = xyzs[i].device
        ns.append(n)
        xp.append(p)
        qp.append(_dev_arg(qs[i], "qs[%d]" % i, torch.complex128, n, dev))
        fp.append(_dev_arg(phis[i], "phis[%d]" % i, torch.complex128, n, dev))
        if layers is not None:
            lp.append(_dev_arg(layers[i], "layers[%d]" % i, torch.int32, n, dev))
    L = load()
    vp = ctypes.c_void_p
    P = (vp * m)(*[pl.h.value for pl in plans])
    N = (ctypes.c_int64 * m)(*ns)
    X = (vp * m)(*xp)
    Q = (vp * m)(*qp)
    F = (vp * m)(*fp)
    Ly = (vp * m)(*lp) if layers is not None else None
    st = (ctypes.c_int * m)()
    rc = L.lfmm_eval_batch(m, P, N, X, Ly, Q, F, int(nworkers), st)
    _check(rc, "lfmm_eval_batch")
    return list(st)


def batch_prepare(plans, xyzs, layers=None, nworkers=8):
    """lfmm_batch_prepare: lfmm_prepare of every problem (plans[i] with xyzs[i], float64
    (3, n_i) on the GPU) on host worker threads.  Returns the per-problem codes; raises
    on failure."""
    import torch
    m = len(plans)
    if len(xyzs) != m or (layers is not None and len(layers) != m):
        raise LfmmError(1, "batch_prepare: one plan and xyz (and layer) per problem")
    ns, xp, lp = [], [], []
    for i in range(m):
        n, p = _xyz_arg(xyzs[i], "xyzs[%d]" % i)
        ns.append(n)
        xp.append(p)
        if layers is not None:
            lp.append(_dev_arg(layers[i], "layers[%d]" % i, torch.int32, n, xyzs[i].device))
    L = load()
    vp = ctypes.c_void_p
    P = (vp * m)(*[pl.h.value for pl in plans])
    st = (ctypes.c_int * m)()
    for pl in plans:
        pl._prep_n = None
    rc = L.lfmm_batch_prepare(m, P, (ctypes.c_int64 * m)(*ns), (vp * m)(*xp),
                              (vp * m)(*lp) if layers is not None else None, int(nworkers), st)
    _check(rc, "lfmm_batch_prepare")
    for pl, n in zip(plans, ns):
        pl._prep_n = n
    return list(st)


class Batch:
    """lfmm_batch_capture: the prepared problems' lfmm_apply captured into one HIP graph;
    launch() runs it.  The graph reads qs[i] and writes phis[i] (complex128 on the GPU)
    each time it runs; plans and tensors are kept referenced for the batch's lifetime."""

    def __init__(self, plans, qs, phis, nbranch=4):
        import torch
        m = len(plans)
        if not (len(qs) == len(phis) == m):
            raise LfmmError(1, "Batch: one plan, q and phi per problem")
        qp, fp = [], []
        for i in range(m):
            n = getattr(plans[i], "_prep_n", None)
            if n is None:
                raise LfmmError(1, "Batch: plan %d has no prepared positions" % i)
            qp.append(_dev_arg(qs[i], "qs[%d]" % i, torch.complex128, n))
            fp.append(_dev_arg(phis[i], "phis[%d]" % i, torch.complex128, n, qs[i].device))
        self.lib = load()
        vp = ctypes.c_void_p
        self.rep = BatchReport()
        h = vp()
        self._keep = (list(plans), list(qs), list(phis))
        rc = self.lib.lfmm_batch_capture(m, (vp * m)(*[pl.h.value for pl in plans]), (vp * m)(*qp), (vp * m)(*fp),
                                         int(nbranch), ctypes.byref(h), ctypes.byref(self.rep))
        _check(rc, "lfmm_batch_capture")
        self.h = h

    def report(self):
        return {f: getattr(self.rep, f) for f, _ in BatchReport._fields_}

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(self.lib.lfmm_batch_launch(self.h, ctypes.c_void_p(s.cuda_stream)), "lfmm_batch_launch")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.lfmm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward_backward(x, params, t, nin, width, nhidden, nout):
    """One forward and backward pass of the surrogate network's kernels on the GPU:
    x [B, nin], t [B, nout], params packed per layer (W [out][in], then b).  Returns
    (y, grad, loss) with the gradient in the parameters' packing."""
    L = load()
    _F = ctypes.POINTER(ctypes.c_float)
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    params = np.ascontiguousarray(params, dtype=np.float32)
    B = x.shape[0]
    y = np.zeros((B, nout), dtype=np.float32)
    g = np.zeros(params.size, dtype=np.float32)
    loss = ctypes.c_double()
    _check(L.lfmm_mlp_forward_backward(B, nin, width, nhidden, nout, x.ctypes.data_as(_F), params.ctypes.data_as(_F),
                                       t.ctypes.data_as(_F), y.ctypes.data_as(_F), g.ctypes.data_as(_F),
                                       ctypes.byref(loss)), "lfmm_mlp_forward_backward")
    return y, g, loss.value


def exported_symbols_from_header(path=None):
    """Function names declared in include/lfmm.h."""
    import re
    path = path or os.path.join(os.path.dirname(HERE), "include", "lfmm.h")
    text = open(path).read()
    return sorted(set(re.findall(r"\b(lfmm_[a-z_]+)\s*\(", text)))
