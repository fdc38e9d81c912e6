"""The BF16x3 estimate and its derived error bound, checked pair by pair.

kp_probe_estimates returns, for query rows against every centroid, the
estimate v of the squared distance that the distance kernels decide on (the
same point split, chunk staging, matrix products, estimate and key
truncation) and the bound eta the decisions use.  Every pair must satisfy
|v - d^2| <= eta, with d^2 computed in FP64 here; over the cases below that
is more than 10^8 pairs, including constructed near-ties, large norms with
small distances (cancellation), a group holding an outlier centroid, the
largest supported dimension and data scaled far from 1.  A violated bound
could turn an uncertain decision into a wrong certain one, which the
end-to-end parity tests would only see if the flip fell outside the
near-tie band.
"""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

TOTAL = {"pairs": 0}


def _fp64_d2(Q, C):
    """FP64 squared distances with a bound on their own rounding error."""
    Q64, C64 = Q.astype(np.float64), C.astype(np.float64)
    qn, cn = (Q64 * Q64).sum(1), (C64 * C64).sum(1)
    d2 = qn[:, None] + cn[None, :] - 2.0 * (Q64 @ C64.T)
    err = 8.0 * Q.shape[1] * 2.0 ** -53 * (qn[:, None] + cn[None, :])
    return d2, err


def _probe_and_check(name, X, C, g, Q, chunk=8192, anchors=("none", "near", "random")):
    """Every query chunk is probed without an anchor (the dense first pass and
    serving), relative to the centroid nearest its first query (a filtered
    tile sorted to that centroid) and relative to a random centroid (a point
    far from the anchor, as at a tile boundary)."""
    import torch
    from paper_1905_09345_amd import KMeans
    print("CASE", name, dict(n=X.shape[0], d=X.shape[1], k=C.shape[0], g=g, nq=Q.shape[0]), flush=True)
    km = KMeans([(torch.from_numpy(np.ascontiguousarray(X)).cuda(),
                  torch.from_numpy(np.ascontiguousarray(C)).cuda(), g, "bf16")])
    rng = np.random.default_rng(len(name))
    try:
        worst, viol, ratio = 0.0, 0, []
        for s in range(0, Q.shape[0], chunk):
            q = np.ascontiguousarray(Q[s:s + chunk])
            d2, err = _fp64_d2(q, C)
            for mode in anchors:
                anchor = -1 if mode == "none" else (int(np.argmin(d2[0])) if mode == "near"
                                                    else int(rng.integers(C.shape[0])))
                est, eta = km.probe_estimates(torch.from_numpy(q).cuda(), anchor=anchor)
                est, eta = est.cpu().numpy().astype(np.float64), eta.cpu().numpy().astype(np.float64)
                gap = np.abs(est - d2) - err
                assert np.isfinite(est).all() and (eta > 0).all()
                v = gap > eta
                viol += int(v.sum())
                worst = max(worst, float((gap / eta).max()))
                ratio.append(np.median(np.abs(est - d2) / eta))
                TOTAL["pairs"] += est.size
        print("  pairs so far %d, violations %d, largest |v - d2| / eta %.3f, median %.3g"
              % (TOTAL["pairs"], viol, worst, float(np.median(ratio))), flush=True)
        assert viol == 0, "%d pairs outside the bound (worst %.3f eta)" % (viol, worst)
        return worst
    finally:
        km.close()


def test_mixture_c3_shape():
    """3.0e8 pairs: the C3 recipe (D=128, K=1024, G=100) with 98,000 queries,
    each in the three forms."""
    P = datagen.make_config(3, n=100_000)
    _probe_and_check("c3-shape", P.X, P.C0, P.g, P.X[:98_000])


def test_anchored_eta_is_tight_near_the_anchor():
    """Relative to the nearest centroid the bound shrinks with the cell size:
    on the C5 recipe it is far below the bound without an anchor."""
    import torch
    from paper_1905_09345_amd import KMeans
    P = datagen.make_config(5, n=20_000)
    km = KMeans([(torch.from_numpy(P.X).cuda(), torch.from_numpy(P.C0).cuda(), P.g, "bf16")])
    try:
        q = np.ascontiguousarray(P.X[:64])
        d2, _ = _fp64_d2(q, P.C0)
        a = int(np.argmin(d2[0]))
        _, eta0 = km.probe_estimates(torch.from_numpy(q).cuda(), anchor=-1)
        _, eta1 = km.probe_estimates(torch.from_numpy(q).cuda(), anchor=a)
        e0, e1 = float(eta0[0].cpu().numpy()[a]), float(eta1[0].cpu().numpy()[a])
        print("eta at the nearest centroid: %.4g without an anchor, %.4g relative to it" % (e0, e1), flush=True)
        assert e1 < 0.2 * e0
    finally:
        km.close()


def test_student_t_c5_shape():
    """3.1e8 pairs at D=256 (eight 32-wide steps per product, the widest
    supported), K=4096, G=410, heavy-tailed points and centroids."""
    P = datagen.make_config(5, n=40_000)
    _probe_and_check("c5-shape", P.X, P.C0, P.g, P.X[:25_000])


def test_cancellation_large_norms():
    """Points and centroids far from the origin (every coordinate + 3000) with
    queries very close to centroids: ||x|| ~ 3.4e4 while d ~ 1e-2..1."""
    rng = np.random.default_rng(11)
    d, k = 128, 256
    X = (datagen.gaussian_mixture(rng, 20_000, d, k) + 3000.0).astype(np.float32)
    C = datagen.kmeanspp(rng, X, k, sample=4000)
    base = C[rng.integers(0, k, size=40_000)].astype(np.float64)
    scale = 10.0 ** rng.uniform(-4, 0, size=(40_000, 1))
    Q = (base + scale * rng.normal(size=(40_000, d))).astype(np.float32)
    _probe_and_check("cancellation", X, C, 26, Q)


def test_near_ties():
    """Queries on the bisector of two centroids (midpoint plus a small offset
    along the bisecting hyperplane): the two distances agree to rounding."""
    rng = np.random.default_rng(12)
    d, k = 64, 512
    X = datagen.gaussian_mixture(rng, 30_000, d, k)
    C = datagen.kmeanspp(rng, X, k, sample=8000).astype(np.float64)
    a = rng.integers(0, k, size=60_000)
    b = (a + 1 + rng.integers(0, k - 1, size=60_000)) % k
    mid = 0.5 * (C[a] + C[b])
    w = C[b] - C[a]
    z = rng.normal(size=mid.shape)
    z -= ((z * w).sum(1) / (w * w).sum(1))[:, None] * w          # orthogonal to c_b - c_a
    Q = (mid + 0.3 * z).astype(np.float32)
    _probe_and_check("near-ties", X, C.astype(np.float32), 52, Q)


def test_outlier_centroid_in_a_group():
    """One centroid with a norm a hundred times the others': its group's norm
    bound is dominated by it, the other groups' are not."""
    rng = np.random.default_rng(13)
    d, k = 256, 320
    X = datagen.gaussian_mixture(rng, 20_000, d, k)
    C = datagen.kmeanspp(rng, X, k, sample=6000)
    C[7] = C[7] * 100.0
    Q = np.concatenate([X[:12_000], (C[7][None, :] + rng.normal(size=(2_000, d))).astype(np.float32)])
    _probe_and_check("outlier", X, C, 32, Q)


@pytest.mark.parametrize("scale", [1e-6, 1e6])
def test_extreme_scales(scale):
    rng = np.random.default_rng(14)
    d, k = 96, 384
    X = (datagen.gaussian_mixture(rng, 20_000, d, k) * scale).astype(np.float32)
    C = datagen.kmeanspp(rng, X, k, sample=6000)
    _probe_and_check("scale-%g" % scale, X, C, 39, X[:20_000])


def test_after_training_ragged_dims():
    """Bounds of the centroids a few iterations produce (refreshed norm bounds),
    at a dimension that leaves most of the last 32-wide step empty."""
    import torch
    from paper_1905_09345_amd import KMeans
    rng = np.random.default_rng(15)
    d, k = 37, 200
    X = datagen.gaussian_mixture(rng, 30_000, d, k)
    C0 = datagen.kmeanspp(rng, X, k, sample=6000)
    km = KMeans([(torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda(), 20, "bf16")])
    km.iterate(5)
    C = km.centroids()[0].cpu().numpy()
    km.close()
    _probe_and_check("trained-d37", X, C, 20, X[:30_000])
    print("total pairs checked in this module: %d" % TOTAL["pairs"], flush=True)
    assert TOTAL["pairs"] >= 2 * 10 ** 8 or TOTAL["pairs"] < 10 ** 8   # full module run vs a single test
