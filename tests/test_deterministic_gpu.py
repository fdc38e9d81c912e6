"""Deterministic mode (kp_tuning.deterministic = 1): the list of point-filter
failures is built in chunk order and sorted stably, and every centroid
update recomputes the FP64 sums from all points in a fixed order, with no
floating-point atomics.  Two runs must agree bit for bit -- labels, FP32 and
FP64 centroids and the per-iteration statistics -- and each run must still
match the FP64 oracle step by step."""
import numpy as np
import pytest

import datagen
from parity import run_steplocked

pytestmark = pytest.mark.gpu


def _run(X, C0, g, prec, iters, tuning):
    import torch
    from paper_1905_09345_amd import KMeans
    km = KMeans([(torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda(), g, prec)], tuning=tuning)
    try:
        km.iterate(iters)
        lab = km.assign().cpu().numpy()
        c32, c64 = [a.cpu().numpy() for a in km.centroids()]
        st = km.stats()
    finally:
        km.close()
    return lab, c32, c64, st


@pytest.mark.parametrize("case", ["c3", "c5", "fp32", "codes"])
def test_two_runs_bitwise_identical(case):
    from paper_1905_09345_amd.kp import kp_tuning
    t = kp_tuning(deterministic=1)
    if case == "c3":
        P = datagen.make_config(3, n=50_000)
        X, C0, g, prec, T = P.X, P.C0, P.g, "bf16", 10
    elif case == "c5":
        P = datagen.make_config(5, n=40_000)
        X, C0, g, prec, T = P.X, P.C0, P.g, "bf16", 6
    elif case == "fp32":
        P = datagen.make_config(2, n=50_000)
        X, C0, g, prec, T = P.X, P.C0, P.g, "fp32", 12
    else:
        P = datagen.make_config(3, n=50_000)
        X, C0, g, prec, T = P.X, P.C0, P.g, "bf16", 10
        t = kp_tuning(deterministic=1, bound_codes=2)
    print("CASE deterministic", case, flush=True)
    a = _run(X, C0, g, prec, T, t)
    b = _run(X, C0, g, prec, T, t)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1].tobytes() == b[1].tobytes()
    assert a[2].tobytes() == b[2].tobytes()
    assert a[3] == b[3]


@pytest.mark.parametrize("prec,n", [("bf16", 30_011), ("fp32", 20_011)])
def test_deterministic_matches_oracle(prec, n):
    from paper_1905_09345_amd.kp import kp_tuning
    P = datagen.make_config(3 if prec == "bf16" else 2, n=n)
    print("CASE deterministic-parity", prec, flush=True)
    r = run_steplocked(P.X, P.C0, P.g, prec, 8, tuning=kp_tuning(deterministic=1))
    assert len(r["stats"]) == 8


def test_deterministic_zipf_segments():
    """Segments of the fixed-order sums spanning many pieces: a cluster of most
    of the points next to small ones (several thousand points per slot)."""
    from paper_1905_09345_amd.kp import kp_tuning
    rng = np.random.default_rng(3)
    X = np.concatenate([rng.normal(size=(60_000, 16)), rng.normal(size=(3_000, 16)) + 8.0]).astype(np.float32)
    X = X[rng.permutation(X.shape[0])]
    C0 = X[:12].copy()
    print("CASE deterministic-big-segments", flush=True)
    run_steplocked(X, C0, 3, "bf16", 6, tuning=kp_tuning(deterministic=1))
    run_steplocked(X, C0, 3, "fp32", 6, tuning=kp_tuning(deterministic=1))


def _run_calls(X, C0, g, prec, calls, tuning):
    import torch
    from paper_1905_09345_amd import KMeans
    km = KMeans([(torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda(), g, prec)], tuning=tuning)
    try:
        for c in calls:
            km.iterate(c)
        lab = km.assign().cpu().numpy()
        c32, c64 = [a.cpu().numpy() for a in km.centroids()]
        st = km.stats()
    finally:
        km.close()
    return lab, c32, c64, st


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_whole_call_graph_bitwise(prec):
    """use_graph = 2 (every iteration of a kp_iterate call in one graph,
    replayed by a later call of the same length) gives bit for bit what
    per-iteration graphs and plain launches give, in deterministic mode."""
    from paper_1905_09345_amd.kp import kp_tuning
    P = datagen.make_config(3 if prec == "bf16" else 2, n=40_000)
    print("CASE whole-call graph", prec, flush=True)
    calls = [3, 4, 4, 1]   # the third call replays the second's graph
    ref = _run_calls(P.X, P.C0, P.g, prec, calls, kp_tuning(deterministic=1, use_graph=-1))
    for ug in (1, 2):
        got = _run_calls(P.X, P.C0, P.g, prec, calls, kp_tuning(deterministic=1, use_graph=ug))
        np.testing.assert_array_equal(got[0], ref[0])
        assert got[1].tobytes() == ref[1].tobytes()
        assert got[2].tobytes() == ref[2].tobytes()
        assert got[3] == ref[3]
