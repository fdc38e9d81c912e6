"""Step-locked comparison of the GPU library with the FP64 oracle.

At every iteration t the oracle assigns the points with the GPU's own FP32
centroids from iteration t-1 and the two assignments are compared:

  * a point may differ only at a near-tie: with d1 the oracle's nearest FP64
    distance and d2 the FP64 distance to the centroid the GPU chose (both
    against the same centroids), d2 - d1 <= 1e-5 * d1;
  * the GPU's FP64 centroids must equal the FP64 means of the points under
    the GPU's assignment (empty centroids keep their previous value) to
    1e-9 relative -- far inside the required 1e-5 -- and its FP32 centroids
    must be their round-to-nearest FP32 values.
"""
from __future__ import annotations

import numpy as np

import oracle

NEAR_TIE = 1e-5
C64_TOL = 1e-9


def check_assignment(X, c_prev32, labels, idx=None):
    """Returns (mismatches, allowed_mismatches); raises on a mismatch outside the band."""
    Xs = X if idx is None else X[idx]
    lab = labels if idx is None else labels[idx]
    C = c_prev32.astype(np.float64)
    ref, d1sq = oracle.assign(Xs, C)
    d2sq = oracle.dist2_to(Xs, C, lab)
    mism = ref != lab
    d1, d2 = np.sqrt(d1sq), np.sqrt(d2sq)
    ok = (d2 - d1) <= NEAR_TIE * d1
    bad = mism & ~ok
    if bad.any():
        i = int(np.flatnonzero(bad)[0])
        raise AssertionError("assignment differs outside the near-tie band at %d of %d points; first: point %d "
                             "gpu=%d (d=%.9g) oracle=%d (d=%.9g)" % (int(bad.sum()), len(lab), i, int(lab[i]),
                                                                    d2[i], int(ref[i]), d1[i]))
    return int(mism.sum()), int((mism & ok).sum())


def check_centroids(X, labels, c_prev64, c32, c64, scale):
    cref, cnt = oracle.update(X, labels, c_prev64)
    err = np.linalg.norm(c64 - cref, axis=1)
    tol = C64_TOL * np.maximum(np.linalg.norm(cref, axis=1), scale)
    if not (err <= tol).all():
        j = int(np.argmax(err / tol))
        raise AssertionError("FP64 centroid %d off by %.3g (tolerance %.3g)" % (j, err[j], tol[j]))
    if not np.array_equal(c32, c64.astype(np.float32)):
        raise AssertionError("FP32 centroids are not the rounded FP64 centroids")
    return cnt


def rms_norm(X, chunk=1 << 20):
    """sqrt of the mean squared norm of the rows of X (FP64, in chunks)."""
    tot = 0.0
    for s in range(0, X.shape[0], chunk):
        xs = X[s:s + chunk].astype(np.float64)
        tot += float((xs * xs).sum())
    return float(np.sqrt(tot / max(X.shape[0], 1)))


def run_steplocked(X, C0, g, precision, iters, *, seed=0, tuning=None, sample=None, check_every=1,
                   rng_seed=0):
    """Run `iters` GPU iterations one at a time and check each against the oracle.

    sample: when given, the assignment check uses that many seeded random
    points per checked iteration (the centroid check always uses all points).
    Returns a report dict.
    """
    import torch
    from paper_1905_09345_amd import KMeans

    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Cd = torch.from_numpy(np.ascontiguousarray(C0)).cuda()
    km = KMeans([(Xd, Cd, g, precision, seed)], tuning=tuning)
    rng = np.random.default_rng(rng_seed)
    scale = rms_norm(X)
    c32p, c64p = C0.astype(np.float32), C0.astype(np.float64)
    report = dict(mismatch=[], allowed=[], checked=[])
    try:
        for t in range(1, iters + 1):
            km.iterate(1)
            lab = km.assign().cpu().numpy()
            c32, c64 = [a.cpu().numpy() for a in km.centroids()]
            if t % check_every == 0 or t == 1 or t == iters:
                idx = None if sample is None else rng.choice(X.shape[0], size=min(sample, X.shape[0]),
                                                             replace=False)
                m, a = check_assignment(X, c32p, lab, idx)
                report["mismatch"].append(m)
                report["allowed"].append(a)
                report["checked"].append(t)
                check_centroids(X, lab, c64p, c32, c64, scale)
            c32p, c64p = c32, c64
        report["stats"] = km.stats()
        report["labels"] = lab
        report["c64"] = c64
    finally:
        km.close()
    return report


def run_steplocked_batch(problems, iters, *, tuning=None, check_every=1, sample=None, rng_seed=0):
    """Several problems in one ctx (batched launches), each checked step-locked
    against the oracle as in run_steplocked.  problems: list of
    (X, C0, g, precision).  sample: when given, each problem's assignment
    check uses that many seeded random points (its centroid check uses all
    of them).  Returns one report per problem."""
    import torch
    from paper_1905_09345_amd import KMeans

    dev = [(torch.from_numpy(np.ascontiguousarray(X)).cuda(), torch.from_numpy(np.ascontiguousarray(C0)).cuda(),
            g, prec, 0) for X, C0, g, prec in problems]
    km = KMeans(dev, tuning=tuning)
    rng = np.random.default_rng(rng_seed)
    prev = [(C0.astype(np.float32), C0.astype(np.float64)) for _, C0, _, _ in problems]
    scales = [rms_norm(X) for X, _, _, _ in problems]
    reports = [dict(mismatch=[], allowed=[]) for _ in problems]

    def checked(t):
        return t % check_every == 0 or t == 1 or t == iters
    try:
        for t in range(1, iters + 1):
            if t > 1 and checked(t) and not checked(t - 1):
                prev = [tuple(a.cpu().numpy() for a in km.centroids(i)) for i in range(len(problems))]
            km.iterate(1)
            if not checked(t):
                continue
            for i, (X, _, _, _) in enumerate(problems):
                lab = km.assign(i).cpu().numpy()
                c32, c64 = [a.cpu().numpy() for a in km.centroids(i)]
                idx = None
                if sample is not None and sample < X.shape[0]:
                    idx = np.sort(rng.choice(X.shape[0], size=sample, replace=False))
                try:
                    m, a = check_assignment(X, prev[i][0], lab, idx)
                    check_centroids(X, lab, prev[i][1], c32, c64, scales[i])
                except AssertionError as e:
                    raise AssertionError("problem %d, iteration %d: %s" % (i, t, e))
                reports[i]["mismatch"].append(m)
                reports[i]["allowed"].append(a)
                prev[i] = (c32, c64)
        for i in range(len(problems)):
            reports[i]["stats"] = km.stats(i)
    finally:
        km.close()
    return reports
