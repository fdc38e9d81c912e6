"""GPU parity of serving (kp_predict): new points assigned to a problem's
current centroids, called through the C ABI, against the FP64 oracle's
nearest centroid under those FP32 centroids.  A query may differ from the
oracle only at a near-tie (the same band as the iteration's assignment)."""
import numpy as np
import pytest

import datagen
import oracle
from parity import check_assignment

pytestmark = pytest.mark.gpu


def _case(name, **kw):
    print("CASE", name, kw, flush=True)


def _train(X, C0, g, precision, iters, problems_extra=()):
    import torch
    from paper_1905_09345_amd import KMeans
    dev = [(torch.from_numpy(np.ascontiguousarray(X)).cuda(), torch.from_numpy(np.ascontiguousarray(C0)).cuda(),
            g, precision, 0)]
    for Xe, Ce, ge, pe in problems_extra:
        dev.append((torch.from_numpy(np.ascontiguousarray(Xe)).cuda(), torch.from_numpy(np.ascontiguousarray(Ce)).cuda(),
                    ge, pe, 0))
    km = KMeans(dev)
    if iters:
        km.iterate(iters)
    return km, dev


def _predict_check(km, Q, problem=0):
    import torch
    lab = km.predict(torch.from_numpy(np.ascontiguousarray(Q)).cuda(), problem).cpu().numpy()
    c32 = km.centroids(problem)[0].cpu().numpy()
    k = c32.shape[0]
    assert lab.shape == (Q.shape[0],)
    assert ((lab >= 0) & (lab < k)).all()
    return check_assignment(Q, c32, lab), lab, c32


@pytest.mark.parametrize("precision,d,k,g", [("bf16", 128, 256, 26), ("bf16", 256, 512, 52), ("bf16", 32, 64, 7),
                                             ("fp32", 32, 256, 26), ("fp32", 8, 16, 2)])
def test_predict_after_training(precision, d, k, g):
    rng = np.random.default_rng(1000 + d + k)
    X = datagen.gaussian_mixture(rng, 20_011, d, k)
    C0 = datagen.kmeanspp(rng, X, k, sample=4000)
    Q = datagen.gaussian_mixture(np.random.default_rng(7 + d), 10_037, d, k)   # ragged last tile
    _case("predict", precision=precision, d=d, k=k, g=g, nq=Q.shape[0])
    km, _ = _train(X, C0, g, precision, 4)
    try:
        (mism, allowed), lab, c32 = _predict_check(km, Q)
        assert mism == allowed
        # the training points themselves get the label of the last assignment
        # step unless the last update moved their nearest centroid
        lab_x = km.predict(__import__("torch").from_numpy(X[:5000]).cuda()).cpu().numpy()
        check_assignment(X[:5000], c32, lab_x)
    finally:
        km.close()


def test_predict_before_training_and_exact_ties():
    """Initial centroids; queries equal to centroids (distance 0), midpoints of
    duplicated centroids (exact ties: lowest original index), a single query
    and an empty call."""
    import torch
    rng = np.random.default_rng(5)
    d, k = 64, 40
    X = datagen.gaussian_mixture(rng, 8_000, d, k)
    C0 = datagen.kmeanspp(rng, X, k, sample=2000)
    C0[7] = C0[3]          # duplicated centroid: ties go to index 3
    _case("predict-ties", d=d, k=k)
    km, _ = _train(X, C0, 5, "bf16", 0)
    try:
        Q = np.concatenate([C0, C0[[3, 3, 3]], X[:50]]).astype(np.float32)
        (mism, allowed), lab, c32 = _predict_check(km, Q)
        assert mism == allowed
        exact = lab[:k]
        assert exact[3] == 3 and exact[7] == 3
        ref, _ = oracle.assign(Q[:k].astype(np.float64), C0.astype(np.float64))
        assert np.array_equal(exact, ref)
        one = km.predict(torch.from_numpy(Q[5:6].copy()).cuda()).cpu().numpy()
        assert one[0] == 5
        empty = km.predict(torch.empty((0, d), dtype=torch.float32).cuda())
        assert empty.numel() == 0
    finally:
        km.close()


def test_predict_batched_problem():
    """Serving from the second problem of a two-problem context."""
    rng = np.random.default_rng(11)
    X0 = datagen.gaussian_mixture(rng, 6_000, 16, 16)
    X1 = datagen.gaussian_mixture(rng, 9_000, 48, 64)
    C00 = datagen.kmeanspp(rng, X0, 16, sample=2000)
    C10 = datagen.kmeanspp(rng, X1, 64, sample=2000)
    _case("predict-batched")
    km, _ = _train(X0, C00, 2, "fp32", 3, problems_extra=[(X1, C10, 7, "bf16")])
    try:
        Q = datagen.gaussian_mixture(np.random.default_rng(12), 3_001, 48, 64)
        (mism, allowed), _, _ = _predict_check(km, Q, problem=1)
        assert mism == allowed
        Q0 = datagen.gaussian_mixture(np.random.default_rng(13), 2_000, 16, 16)
        (mism, allowed), _, _ = _predict_check(km, Q0, problem=0)
        assert mism == allowed
    finally:
        km.close()


def test_predict_argument_errors():
    import torch
    from paper_1905_09345_amd import kp
    rng = np.random.default_rng(3)
    X = datagen.gaussian_mixture(rng, 2_000, 32, 16)
    km, _ = _train(X, X[:16].copy(), 2, "bf16", 1)
    try:
        Q = torch.from_numpy(X[:100]).cuda()
        lab = torch.empty(100, dtype=torch.int32, device="cuda")
        nb = kp.kp_predict_scratch_bytes(km.ctx, 0, 100)
        assert nb >= 256 + 400
        assert kp.kp_predict_scratch_bytes(km.ctx, 1, 100) == 0          # bad problem
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        base = (scratch.data_ptr() + 255) // 256 * 256
        with pytest.raises(RuntimeError):
            kp.kp_predict(km.ctx, 0, Q.data_ptr(), 100, lab.data_ptr(), base, nb - 1)   # short scratch
        with pytest.raises(RuntimeError):
            kp.kp_predict(km.ctx, 0, Q.data_ptr(), 100, lab.data_ptr(), base + 4, nb)   # misaligned scratch
        with pytest.raises(RuntimeError):
            kp.kp_predict(km.ctx, 2, Q.data_ptr(), 100, lab.data_ptr(), base, nb)       # bad problem
        with pytest.raises(RuntimeError):
            kp.kp_predict(km.ctx, 0, Q.data_ptr(), -1, lab.data_ptr(), base, nb)        # negative count
        kp.kp_predict(km.ctx, 0, Q.data_ptr(), 100, lab.data_ptr(), base, nb)
        torch.cuda.synchronize()
        c32 = km.centroids(0)[0].cpu().numpy()
        check_assignment(X[:100], c32, lab.cpu().numpy())
    finally:
        km.close()


def test_predict_c5_shape_two_passes():
    """The C5 recipe (D = 256, Student-t mixture): many queries are uncertain
    under the plain estimate, so the sorted, anchored second pass and the
    FP32 pass both run.  Exact ties (queries equal to a centroid's midpoint
    pair) and far outliers are mixed in."""
    P = datagen.make_config(5, n=90_000)
    k = P.C0.shape[0]
    X, Q = P.X[:60_000], P.X[60_000:]   # queries from the same mixture
    _case("predict-c5", nq=Q.shape[0], k=k, g=P.g)
    km, _ = _train(X, P.C0, P.g, "bf16", 3)
    try:
        c32 = km.centroids()[0].cpu().numpy()
        mid = 0.5 * (c32[:50].astype(np.float64) + c32[50:100].astype(np.float64))
        far = c32[:7] * np.float32(40.0)
        Qx = np.concatenate([Q, mid.astype(np.float32), far, c32[:13]]).astype(np.float32)
        (mism, allowed), lab, _ = _predict_check(km, Qx)
        assert mism == allowed
        # a query equal to a centroid gets that centroid (or an equal one)
        d = ((Qx[-13:, None, :].astype(np.float64) - c32[None].astype(np.float64)) ** 2).sum(2)
        assert (d[np.arange(13), lab[-13:]] == d.min(1)).all()
    finally:
        km.close()


def test_predict_without_anchor_tables():
    """More than 16384 slots: no anchor tables, so serving keeps the plain
    estimate and sends every uncertain query to the FP32 pass."""
    rng = np.random.default_rng(5)
    d, k, g = 16, 17_000, 1000
    X = datagen.gaussian_mixture(rng, 20_000, d, 400)
    C0 = X[rng.choice(X.shape[0], k, replace=False)].copy()
    Q = datagen.gaussian_mixture(np.random.default_rng(6), 5_003, d, 400)
    _case("predict-no-anchor", d=d, k=k, g=g, nq=Q.shape[0])
    km, _ = _train(X, C0, g, "bf16", 2)
    try:
        (mism, allowed), _, _ = _predict_check(km, Q)
        assert mism == allowed
    finally:
        km.close()
