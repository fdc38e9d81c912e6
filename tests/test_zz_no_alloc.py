"""kp_predict_noalloc: serving with the library's fixed per-device scratch
instead of a caller's buffer, called through the C ABI, checked against
kp_predict (same kernels, so the labels must be identical) and against the
FP64 oracle's near-tie rule.  Two calls in a row, the second with fewer
queries, then a query count beyond the fixed scratch, which must be refused
before any work is queued."""
import ctypes

import numpy as np
import pytest

import datagen
from parity import check_assignment

pytestmark = pytest.mark.gpu


def _noalloc(km, Q, problem=0):
    import torch
    from paper_1905_09345_amd import kp
    q = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    out = torch.full((Q.shape[0],), -1, dtype=torch.int32, device=q.device)
    kp.kp_predict_noalloc(km.ctx, problem, q.data_ptr(), Q.shape[0], out.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _with_scratch(km, Q, problem=0):
    import torch
    return km.predict(torch.from_numpy(np.ascontiguousarray(Q)).cuda(), problem).cpu().numpy()


@pytest.mark.parametrize("precision,d,k,g", [("bf16", 128, 512, 52), ("bf16", 256, 300, 30), ("fp32", 32, 128, 13)])
def test_noalloc_matches_predict(precision, d, k, g):
    import torch
    from paper_1905_09345_amd import KMeans
    rng = np.random.default_rng(d + k)
    X = datagen.gaussian_mixture(rng, 30_011, d, k)
    C0 = datagen.kmeanspp(rng, X, k, sample=5000)
    print("CASE noalloc", precision, d, k, g, flush=True)
    km = KMeans([(torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda(), g, precision)])
    try:
        km.iterate(4)
        c32 = km.centroids()[0].cpu().numpy()
        Q1 = datagen.gaussian_mixture(np.random.default_rng(1), 60_013, d, k)
        Q2 = datagen.gaussian_mixture(np.random.default_rng(2), 7_001, d, k)   # a smaller second call
        a1 = _noalloc(km, Q1)
        a2 = _noalloc(km, Q2)
        np.testing.assert_array_equal(a1, _with_scratch(km, Q1))
        np.testing.assert_array_equal(a2, _with_scratch(km, Q2))
        m1, ok1 = check_assignment(Q1, c32, a1)
        m2, ok2 = check_assignment(Q2, c32, a2)
        assert m1 == ok1 and m2 == ok2
    finally:
        km.close()


def test_noalloc_refuses_more_than_its_scratch():
    import torch
    from paper_1905_09345_amd import KMeans, kp
    rng = np.random.default_rng(5)
    X = datagen.gaussian_mixture(rng, 2_000, 16, 8)
    km = KMeans([(torch.from_numpy(X).cuda(), torch.from_numpy(X[:8].copy()).cuda(), 2, "bf16")])
    try:
        km.iterate(1)
        q = torch.from_numpy(X).cuda()
        out = torch.empty(X.shape[0], dtype=torch.int32, device=q.device)
        with pytest.raises(kp.KPError) as e:
            kp.kp_predict_noalloc(km.ctx, 0, q.data_ptr(), kp.KP_PREDICT_NOALLOC_MAX_QUERIES + 1, out.data_ptr())
        assert e.value.status == kp.KP_ERR_INVALID
        kp.kp_predict_noalloc(km.ctx, 0, q.data_ptr(), 0, out.data_ptr())   # nq = 0: nothing to do
        a = _noalloc(km, X)
        np.testing.assert_array_equal(a, _with_scratch(km, X))
    finally:
        km.close()
