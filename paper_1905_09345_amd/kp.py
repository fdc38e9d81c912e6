"""ctypes binding of libkp (include/kp.h): argument marshalling only.

Every step of the K-means iteration runs in the library's HIP kernels; torch
is used here for device memory (the workspace and outputs) and for the
current stream.  If libkp.so has not been built this module raises at load
time instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkp.so")

KP_OK, KP_ERR_INVALID, KP_ERR_NOMEM, KP_ERR_HIP, KP_ERR_STATE, KP_ERR_UNSUPPORTED = range(6)
KP_PREC_FP32, KP_PREC_BF16_RECHECK = 0, 1
PRECISIONS = {"fp32": KP_PREC_FP32, "bf16": KP_PREC_BF16_RECHECK, "bf16_recheck": KP_PREC_BF16_RECHECK}

# Every function kp.h declares; the CPU tests check that the library exports each.
EXPORTS = ("kp_workspace_bytes", "kp_init", "kp_iterate", "kp_assign", "kp_centroids", "kp_stats",
           "kp_stage_times", "kp_iterations", "kp_destroy", "kp_autotune", "kp_autotune_groups", "kp_predict_scratch_bytes", "kp_predict", "kp_predict_noalloc",
           "kp_probe_estimates", "kp_bounds", "kp_strerror", "kp_last_error")


class kp_problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32), ("g", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("points_dev", ctypes.c_void_p),
                ("init_centroids_dev", ctypes.c_void_p), ("seed", ctypes.c_uint64)]


class kp_tuning(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("timing", ctypes.c_int32), ("chunk_depth", ctypes.c_int32),
                ("bound_codes", ctypes.c_int32), ("timing_stages", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("local_filter", ctypes.c_int32), ("plain", ctypes.c_int32)]


# stage indices of kp_tuning.timing_stages
STAGES = ("begin", "bound_filter", "l1_sort", "assign_dense", "group_filter", "assign", "recheck", "update",
          "centroids")


class kp_iter_stats(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("dense", ctypes.c_int32), ("point_filter_fail", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("distances", ctypes.c_int64), ("rechecks", ctypes.c_int64),
                ("moved", ctypes.c_int64), ("max_drift", ctypes.c_double), ("tile_groups", ctypes.c_int64),
                ("closed", ctypes.c_int64), ("row_test", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class kp_stage_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("ms", ctypes.c_double), ("launches", ctypes.c_int64)]


class KPError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, kp_strerror(status), detail))


_lib = None


def lib():
    """The loaded libkp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkp.so is not built (run paper_1905_09345_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, vp = ctypes.POINTER, ctypes.c_void_p
        L.kp_workspace_bytes.argtypes = [P(kp_problem), ctypes.c_int32, P(kp_tuning)]
        L.kp_workspace_bytes.restype = ctypes.c_size_t
        L.kp_init.argtypes = [P(vp), P(kp_problem), ctypes.c_int32, vp, ctypes.c_size_t, vp, P(kp_tuning)]
        L.kp_init.restype = ctypes.c_int
        L.kp_iterate.argtypes = [vp, ctypes.c_int32]
        L.kp_iterate.restype = ctypes.c_int
        L.kp_assign.argtypes = [vp, ctypes.c_int32, vp]
        L.kp_assign.restype = ctypes.c_int
        L.kp_centroids.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.kp_centroids.restype = ctypes.c_int
        L.kp_stats.argtypes = [vp, ctypes.c_int32, P(kp_iter_stats), ctypes.c_int32, P(ctypes.c_int32)]
        L.kp_stats.restype = ctypes.c_int
        L.kp_stage_times.argtypes = [vp, P(kp_stage_time), ctypes.c_int32, P(ctypes.c_int32)]
        L.kp_stage_times.restype = ctypes.c_int
        L.kp_iterations.argtypes = [vp]
        L.kp_iterations.restype = ctypes.c_int32
        L.kp_destroy.argtypes = [vp]
        L.kp_destroy.restype = ctypes.c_int
        L.kp_autotune.argtypes = [P(kp_problem), ctypes.c_int32, vp, ctypes.c_size_t, vp, ctypes.c_int32, P(kp_tuning)]
        L.kp_autotune.restype = ctypes.c_int
        L.kp_autotune_groups.argtypes = [P(kp_problem), ctypes.c_int32, vp, ctypes.c_size_t, vp, ctypes.c_int32,
                                         P(kp_tuning), P(ctypes.c_int32)]
        L.kp_autotune_groups.restype = ctypes.c_int
        L.kp_predict_scratch_bytes.argtypes = [vp, ctypes.c_int32, ctypes.c_int64]
        L.kp_predict_scratch_bytes.restype = ctypes.c_size_t
        L.kp_predict.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64, vp, vp, ctypes.c_size_t]
        L.kp_predict.restype = ctypes.c_int
        L.kp_predict_noalloc.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64, vp]
        L.kp_predict_noalloc.restype = ctypes.c_int
        L.kp_probe_estimates.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64, ctypes.c_int32, vp, vp]
        L.kp_probe_estimates.restype = ctypes.c_int
        L.kp_bounds.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64, vp, vp, vp, vp]
        L.kp_bounds.restype = ctypes.c_int
        L.kp_strerror.argtypes = [ctypes.c_int]
        L.kp_strerror.restype = ctypes.c_char_p
        L.kp_last_error.argtypes = []
        L.kp_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


# ------------------------------------------------------------ same-name calls
def _probs(problems):
    if isinstance(problems, kp_problem):
        problems = [problems]
    arr = (kp_problem * len(problems))(*problems)
    return arr, len(problems)


def kp_workspace_bytes(problems, tuning=None):
    arr, n = _probs(problems)
    return int(lib().kp_workspace_bytes(arr, n, ctypes.byref(tuning) if tuning else None))


def kp_init(problems, workspace_ptr, workspace_bytes, stream=0, tuning=None):
    """Returns the ctx handle (an int)."""
    arr, n = _probs(problems)
    out = ctypes.c_void_p()
    st = lib().kp_init(ctypes.byref(out), arr, n, ctypes.c_void_p(workspace_ptr), workspace_bytes,
                       ctypes.c_void_p(stream), ctypes.byref(tuning) if tuning else None)
    _check(st, "kp_init")
    return out.value


def kp_iterate(ctx, iters):
    _check(lib().kp_iterate(ctypes.c_void_p(ctx), int(iters)), "kp_iterate")


def kp_assign(ctx, problem, labels_ptr):
    _check(lib().kp_assign(ctypes.c_void_p(ctx), int(problem), ctypes.c_void_p(labels_ptr)), "kp_assign")


def kp_predict_scratch_bytes(ctx, problem, nq):
    return int(lib().kp_predict_scratch_bytes(ctypes.c_void_p(ctx), int(problem), int(nq)))


def kp_predict(ctx, problem, queries_ptr, nq, labels_ptr, scratch_ptr, scratch_bytes):
    _check(lib().kp_predict(ctypes.c_void_p(ctx), int(problem), ctypes.c_void_p(queries_ptr), int(nq),
                            ctypes.c_void_p(labels_ptr), ctypes.c_void_p(scratch_ptr), int(scratch_bytes)),
           "kp_predict")


def kp_centroids(ctx, problem, c32_ptr=None, c64_ptr=None):
    _check(lib().kp_centroids(ctypes.c_void_p(ctx), int(problem), ctypes.c_void_p(c32_ptr),
                              ctypes.c_void_p(c64_ptr)), "kp_centroids")


def kp_stats(ctx, problem, cap=1024):
    buf = (kp_iter_stats * max(cap, 1))()
    n = ctypes.c_int32(0)
    _check(lib().kp_stats(ctypes.c_void_p(ctx), int(problem), buf, int(cap), ctypes.byref(n)), "kp_stats")
    return [dict(iter=s.iter, dense=s.dense, point_filter_fail=s.point_filter_fail, pairs=s.pairs,
                 distances=s.distances, rechecks=s.rechecks, moved=s.moved, max_drift=s.max_drift,
                 tile_groups=s.tile_groups, closed=s.closed, row_test=s.row_test)
            for s in buf[:n.value]]


def kp_stage_times(ctx, cap=16):
    buf = (kp_stage_time * cap)()
    n = ctypes.c_int32(0)
    _check(lib().kp_stage_times(ctypes.c_void_p(ctx), buf, int(cap), ctypes.byref(n)), "kp_stage_times")
    return {s.name.decode(): dict(ms=s.ms, launches=s.launches) for s in buf[:n.value]}


def kp_iterations(ctx):
    return int(lib().kp_iterations(ctypes.c_void_p(ctx)))


def kp_destroy(ctx):
    _check(lib().kp_destroy(ctypes.c_void_p(ctx)), "kp_destroy")


def kp_autotune(problems, workspace_ptr, workspace_bytes, stream=0, iters=4):
    """Returns the fastest kp_tuning for these problems (see kp.h)."""
    arr, n = _probs(problems)
    best = kp_tuning()
    _check(lib().kp_autotune(arr, n, ctypes.c_void_p(workspace_ptr), workspace_bytes, ctypes.c_void_p(stream),
                             int(iters), ctypes.byref(best)), "kp_autotune")
    return best


def kp_autotune_groups(problems, workspace_ptr, workspace_bytes, stream=0, iters=4, tuning=None):
    """Returns the fastest g of each problem (see kp.h)."""
    arr, n = _probs(problems)
    out = (ctypes.c_int32 * max(n, 1))()
    tp = ctypes.byref(tuning) if tuning is not None else None
    _check(lib().kp_autotune_groups(arr, n, ctypes.c_void_p(workspace_ptr), workspace_bytes, ctypes.c_void_p(stream),
                                    int(iters), tp, out), "kp_autotune_groups")
    return [int(v) for v in out[:n]]


KP_PREDICT_NOALLOC_MAX_QUERIES = 1 << 22


def kp_predict_noalloc(ctx, problem, queries_ptr, nq, labels_ptr):
    _check(lib().kp_predict_noalloc(ctypes.c_void_p(ctx), int(problem), ctypes.c_void_p(queries_ptr), int(nq),
                                    ctypes.c_void_p(labels_ptr)), "kp_predict_noalloc")


def kp_probe_estimates(ctx, problem, queries_ptr, nq, anchor, est_ptr, eta_ptr):
    _check(lib().kp_probe_estimates(ctypes.c_void_p(ctx), int(problem), ctypes.c_void_p(queries_ptr), int(nq),
                                    int(anchor), ctypes.c_void_p(est_ptr), ctypes.c_void_p(eta_ptr)),
           "kp_probe_estimates")


def kp_bounds(ctx, problem, idx_ptr, np_, ub_ptr, lbp_ptr, lb_ptr, group_ptr=None):
    _check(lib().kp_bounds(ctypes.c_void_p(ctx), int(problem), ctypes.c_void_p(idx_ptr), int(np_),
                           ctypes.c_void_p(ub_ptr), ctypes.c_void_p(lbp_ptr), ctypes.c_void_p(lb_ptr),
                           ctypes.c_void_p(group_ptr)), "kp_bounds")


def kp_strerror(status):
    return lib().kp_strerror(int(status)).decode()


def kp_last_error():
    return lib().kp_last_error().decode()


def _check(status, where):
    if status != KP_OK:
        raise KPError(status, where, kp_last_error())


# --------------------------------------------------------------- convenience
class KMeans:
    """Filtered K-means on one or more problems resident on one GPU.

    problems: a list of (points, init, g) or (points, init, g, precision[, seed])
    where points (n, d) and init (k, d) are contiguous float32 CUDA tensors
    (kept referenced: the library borrows the points).  precision is "fp32"
    or "bf16".  Work is queued on torch's current stream.
    """

    def __init__(self, problems, *, tuning=None, stream=None):
        import torch
        self._torch = torch
        self._keep = []
        descs = []
        for pr in problems:
            X, C0, g = pr[0], pr[1], int(pr[2])
            prec = PRECISIONS[pr[3]] if len(pr) > 3 else KP_PREC_FP32
            seed = int(pr[4]) if len(pr) > 4 else 0
            for T in (X, C0):
                if not (T.is_cuda and T.dtype == torch.float32 and T.is_contiguous() and T.dim() == 2):
                    raise ValueError("points and initial centroids must be contiguous 2-D float32 CUDA tensors")
            if X.shape[1] != C0.shape[1]:
                raise ValueError("points and centroids differ in d")
            self._keep += [X, C0]
            descs.append(kp_problem(n=X.shape[0], d=X.shape[1], k=C0.shape[0], g=g, precision=prec,
                                    points_dev=X.data_ptr(), init_centroids_dev=C0.data_ptr(), seed=seed))
        self.problems = descs
        self.device = problems[0][0].device
        self.tuning = tuning
        nbytes = kp_workspace_bytes(descs, tuning)
        if nbytes == 0:
            raise KPError(KP_ERR_INVALID, "kp_workspace_bytes", kp_last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = kp_init(descs, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream, tuning)

    @staticmethod
    def autotune(problems, iters=4):
        """Tuning for these problems from kp_autotune (same problem tuples as the constructor)."""
        import torch
        descs, keep = [], []
        for pr in problems:
            X, C0, g = pr[0], pr[1], int(pr[2])
            prec = PRECISIONS[pr[3]] if len(pr) > 3 else KP_PREC_FP32
            seed = int(pr[4]) if len(pr) > 4 else 0
            keep += [X, C0]
            descs.append(kp_problem(n=X.shape[0], d=X.shape[1], k=C0.shape[0], g=g, precision=prec,
                                    points_dev=X.data_ptr(), init_centroids_dev=C0.data_ptr(), seed=seed))
        nbytes = kp_workspace_bytes(descs)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=problems[0][0].device)
        stream = torch.cuda.current_stream(problems[0][0].device).cuda_stream
        best = kp_autotune(descs, ws.data_ptr(), nbytes, stream, iters)
        del ws
        return best

    @staticmethod
    def autotune_groups(problems, iters=4, tuning=None):
        """Group count per problem from kp_autotune_groups (same problem tuples
        as the constructor; each problem's own g is one of the candidates)."""
        import torch
        descs, keep = [], []
        for pr in problems:
            X, C0, g = pr[0], pr[1], int(pr[2])
            prec = PRECISIONS[pr[3]] if len(pr) > 3 else KP_PREC_FP32
            seed = int(pr[4]) if len(pr) > 4 else 0
            keep += [X, C0]
            descs.append(kp_problem(n=X.shape[0], d=X.shape[1], k=C0.shape[0], g=g, precision=prec,
                                    points_dev=X.data_ptr(), init_centroids_dev=C0.data_ptr(), seed=seed))
        nbytes = kp_workspace_bytes(descs, tuning)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=problems[0][0].device)
        stream = torch.cuda.current_stream(problems[0][0].device).cuda_stream
        gs = kp_autotune_groups(descs, ws.data_ptr(), nbytes, stream, iters, tuning)
        del ws
        return gs

    def iterate(self, iters=1):
        kp_iterate(self.ctx, iters)

    @property
    def iterations(self):
        return kp_iterations(self.ctx)

    def assign(self, problem=0, out=None):
        p = self.problems[problem]
        if out is None:
            out = self._torch.empty(p.n, dtype=self._torch.int32, device=self.device)
        kp_assign(self.ctx, problem, out.data_ptr())
        return out

    def predict(self, queries, problem=0, out=None):
        """Labels of new points (n_q x d FP32 on the ctx's device) against the
        problem's current centroids (kp_predict); scratch from torch."""
        p = self.problems[problem]
        q = queries.contiguous()
        if q.dtype != self._torch.float32 or q.dim() != 2 or q.shape[1] != p.d or q.device != self.device:
            raise ValueError("queries must be an (n, %d) float32 tensor on %s" % (p.d, self.device))
        nq = q.shape[0]
        if out is None:
            out = self._torch.empty(nq, dtype=self._torch.int32, device=self.device)
        nbytes = kp_predict_scratch_bytes(self.ctx, problem, nq)
        scratch = self._torch.empty(nbytes + 256, dtype=self._torch.uint8, device=self.device)
        base = (scratch.data_ptr() + 255) // 256 * 256
        kp_predict(self.ctx, problem, q.data_ptr(), nq, out.data_ptr(), base, nbytes)
        # the queued work reads both; held until the next call or close
        self._serve_keep = (q, scratch)
        return out

    def probe_estimates(self, queries, problem=0, anchor=-1):
        """(est, eta) of kp_probe_estimates: (n_q, k) FP32 tensors on the ctx's device."""
        p = self.problems[problem]
        q = queries.contiguous()
        if q.dtype != self._torch.float32 or q.dim() != 2 or q.shape[1] != p.d or q.device != self.device:
            raise ValueError("queries must be an (n, %d) float32 tensor on %s" % (p.d, self.device))
        est = self._torch.empty((q.shape[0], p.k), dtype=self._torch.float32, device=self.device)
        eta = self._torch.empty_like(est)
        kp_probe_estimates(self.ctx, problem, q.data_ptr(), q.shape[0], anchor, est.data_ptr(), eta.data_ptr())
        self._torch.cuda.current_stream(self.device).synchronize()
        return est, eta

    def bounds(self, idx, problem=0):
        """(ub, lbp, lb, group) of kp_bounds for the int32 point indices idx."""
        p = self.problems[problem]
        ix = idx.to(device=self.device, dtype=self._torch.int32).contiguous()
        n = ix.shape[0]
        ub = self._torch.empty(n, dtype=self._torch.float32, device=self.device)
        lbp = self._torch.empty_like(ub)
        lb = self._torch.empty((n, p.g), dtype=self._torch.float32, device=self.device)
        grp = self._torch.empty(p.k, dtype=self._torch.int32, device=self.device)
        kp_bounds(self.ctx, problem, ix.data_ptr(), n, ub.data_ptr(), lbp.data_ptr(), lb.data_ptr(), grp.data_ptr())
        self._torch.cuda.current_stream(self.device).synchronize()
        return ub, lbp, lb, grp

    def centroids(self, problem=0):
        p = self.problems[problem]
        c32 = self._torch.empty((p.k, p.d), dtype=self._torch.float32, device=self.device)
        c64 = self._torch.empty((p.k, p.d), dtype=self._torch.float64, device=self.device)
        kp_centroids(self.ctx, problem, c32.data_ptr(), c64.data_ptr())
        return c32, c64

    def stats(self, problem=0):
        return kp_stats(self.ctx, problem)

    def stage_times(self):
        return kp_stage_times(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            kp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
