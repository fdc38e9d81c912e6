"""Validity of the filters' bounds, read back after every iteration.

kp_bounds returns, for listed points, the bounds the point-level and
group-level filters will test in the next iteration, brought to the current
centroids.  In FP64 they must satisfy, for a point x assigned to c_a:

    ub(x)       >= d(x, c_a)
    lbp(x)      <= d(x, c_j)  for every j != a
    lb(x, q)    <= d(x, c_j)  for every member j != a of group q

Filtering is exact only if these hold: a bound that is too tight would let a
filter skip the centroid that is actually nearest.
"""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

SLACK = 1e-12   # relative: the FP64 reference distances carry ~1e-16 rounding


def _direct_dist(Xs, C, budget=1 << 25):
    """FP64 direct-form distances (rows of Xs against rows of C), in chunks."""
    s, k, d = Xs.shape[0], C.shape[0], C.shape[1]
    D = np.empty((s, k))
    step = max(1, budget // (k * d))
    for i in range(0, s, step):
        D[i:i + step] = np.sqrt(((Xs[i:i + step, None, :] - C[None, :, :]) ** 2).sum(-1))
    return D


def _check_bounds(X, c32, lab, idx, ub, lbp, lb, grp):
    Xs = X[idx].astype(np.float64)
    C = c32.astype(np.float64)
    D = _direct_dist(Xs, C)   # (s, k)
    a = lab[idx]
    rows = np.arange(len(idx))
    da = D[rows, a]
    assert (ub >= da * (1 - SLACK)).all(), "upper bound below the assigned distance at %d points" % int(
        (ub < da * (1 - SLACK)).sum())
    Do = D.copy()
    Do[rows, a] = np.inf
    assert (lbp <= Do.min(1) * (1 + SLACK) + 1e-30).all(), "point-level lower bound too high"
    g = lb.shape[1]
    for q in range(g):
        members = np.flatnonzero(grp == q)
        if members.size == 0:
            continue
        mq = Do[:, members].min(1)
        bad = lb[:, q] > mq * (1 + SLACK) + 1e-30
        assert not bad.any(), "group %d: lower bound above the nearest member at %d points" % (q, int(bad.sum()))
    # the bounds are useful, not merely valid: most upper bounds are tight
    return float(np.median(ub / np.maximum(da, 1e-30)))


def _run(X, C0, g, precision, iters, sample, tuning=None, seed=0):
    import torch
    from paper_1905_09345_amd import KMeans
    km = KMeans([(torch.from_numpy(np.ascontiguousarray(X)).cuda(),
                  torch.from_numpy(np.ascontiguousarray(C0)).cuda(), g, precision)], tuning=tuning)
    rng = np.random.default_rng(seed)
    tight = []
    try:
        for t in range(1, iters + 1):
            km.iterate(1)
            idx = np.sort(rng.choice(X.shape[0], size=min(sample, X.shape[0]), replace=False)).astype(np.int32)
            ub, lbp, lb, grp = [a.cpu().numpy() for a in km.bounds(torch.from_numpy(idx))]
            lab = km.assign().cpu().numpy()
            c32 = km.centroids()[0].cpu().numpy()
            tight.append(_check_bounds(X, c32, lab, idx, ub.astype(np.float64), lbp.astype(np.float64),
                                       lb.astype(np.float64), grp))
        return tight
    finally:
        km.close()


@pytest.mark.parametrize("codes", [1, 2])
def test_bounds_c3_shape(codes):
    from paper_1905_09345_amd.kp import kp_tuning
    P = datagen.make_config(3, n=60_000)
    print("CASE bounds-c3", codes, flush=True)
    tight = _run(P.X, P.C0, P.g, "bf16", 12, 2048, tuning=kp_tuning(bound_codes=codes))
    print("median ub / d(x, c_a) per iteration", ["%.4f" % v for v in tight], flush=True)
    assert tight[-1] < 1.01


def test_bounds_c5_shape():
    P = datagen.make_config(5, n=40_000)
    print("CASE bounds-c5", flush=True)
    _run(P.X, P.C0, P.g, "bf16", 6, 1024)


@pytest.mark.parametrize("lf", [0, 1])
@pytest.mark.parametrize("g", [1, 3, 40])
def test_bounds_fp32(g, lf):
    """FP32 form, with and without the local filter (whose skipped members
    enter the group bounds and lbp with a lower bound instead of a distance)."""
    from paper_1905_09345_amd.kp import kp_tuning
    rng = np.random.default_rng(g)
    X = datagen.gaussian_mixture(rng, 20_000, 24, 40)
    C0 = datagen.kmeanspp(rng, X, 40)
    print("CASE bounds-fp32", g, lf, flush=True)
    _run(X, C0, g, "fp32", 14, 2048, tuning=kp_tuning(local_filter=lf))


def test_bounds_full_c3_sampled():
    """The full C3 workload (N = 4e6), 4096 sampled points per iteration."""
    P = datagen.make_config(3)
    print("CASE bounds-c3-full", flush=True)
    tight = _run(P.X, P.C0, P.g, "bf16", P.iters, 4096)
    print("median ub / d(x, c_a) per iteration", ["%.4f" % v for v in tight], flush=True)
