"""Pins of the FP64 Lloyd oracle against things other than itself (CPU only).

Each check targets a plausible mistake: a dropped coordinate, a wrong sign
or index, a transposed operand, a wrong tie rule or a wrong empty-cluster
rule would each fail at least one of them.
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import datagen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _frac(pair):
    return float(Fraction(int(pair[0]), int(pair[1])))


def test_worked_example_1d():
    """Hand-derived 1-D example, exact to the last bit (tests/golden/worked_1d.json)."""
    g = json.load(open(os.path.join(GOLD, "worked_1d.json")))
    X = np.array(g["X"], np.float32)
    C0 = np.array(g["C0"], np.float64)
    r = oracle.lloyd(X, C0, len(g["iterations"]))
    for t, it in enumerate(g["iterations"]):
        assert r["labels"][t].tolist() == it["labels"], t
        want = np.array([[_frac(c)] for c in it["centroids"]])
        np.testing.assert_allclose(r["centroids"][t], want, rtol=1e-15, atol=0)
        assert r["sse_assign"][t] == pytest.approx(_frac(it["sse_assign"]), rel=1e-14)
        assert r["sse_update"][t] == pytest.approx(_frac(it["sse_update"]), rel=1e-14)


def _enumerate_best_labels(X, C):
    """Lexicographically first labelling minimising sum ||x - c_l||^2 (brute force)."""
    X = X.astype(np.float64)
    n, k = X.shape[0], C.shape[0]
    best, best_lab = None, None
    for lab in itertools.product(range(k), repeat=n):   # lexicographic order
        s = 0.0
        for i, j in enumerate(lab):
            diff = X[i] - C[j]
            s += float(diff @ diff)
        if best is None or s < best:
            best, best_lab = s, lab
    return np.array(best_lab, np.int32), best


def _optimal_sse(X, k):
    """Global optimum of the K-means objective over all labelings (brute force)."""
    X = X.astype(np.float64)
    n = X.shape[0]
    best = np.inf
    for lab in itertools.product(range(k), repeat=n):
        lab = np.array(lab)
        s = 0.0
        for j in range(k):
            m = lab == j
            if m.any():
                s += float(((X[m] - X[m].mean(axis=0)) ** 2).sum())
        best = min(best, s)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_assignment(seed):
    """Assignment step == first minimiser over all K^N labelings; small grids create exact ties."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    k = int(rng.integers(1, 4))
    d = int(rng.integers(1, 4))
    if seed % 3 == 0:   # integer grid: many exact ties
        X = rng.integers(-2, 3, size=(n, d)).astype(np.float32)
        C = rng.integers(-2, 3, size=(k, d)).astype(np.float64)
    else:
        X = rng.normal(size=(n, d)).astype(np.float32)
        C = rng.normal(size=(k, d))
    want, s = _enumerate_best_labels(X, C)
    lab, d1 = oracle.assign(X, C)
    assert lab.tolist() == want.tolist()
    assert d1.sum() == pytest.approx(s, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_objective_bound(seed):
    """Lloyd's final SSE is never below the global optimum found by enumeration."""
    rng = np.random.default_rng(100 + seed)
    n, k, d = 7, 2 + seed % 2, 2
    X = rng.normal(size=(n, d)).astype(np.float32)
    C0 = X[:k].astype(np.float64)
    r = oracle.lloyd(X, C0, 10)
    opt = _optimal_sse(X, k)
    assert r["sse_update"][-1] >= opt - 1e-9


def test_k1_global_mean():
    X = datagen.make_config(2, n=5000).X
    r = oracle.lloyd(X, X[:1].astype(np.float64), 1)
    np.testing.assert_allclose(r["final"][0], X.astype(np.float64).mean(axis=0), rtol=1e-12, atol=1e-12)
    assert (r["labels"][0] == 0).all()


def test_k_equals_n_distinct():
    rng = np.random.default_rng(7)
    X = rng.normal(size=(9, 3)).astype(np.float32)
    r = oracle.lloyd(X, X.astype(np.float64), 3)
    assert r["labels"][-1].tolist() == list(range(9))
    assert r["sse_update"][-1] == 0.0


def test_exact_ties_lowest_index():
    X = np.array([[0.5], [2.0]], np.float32)
    lab, _ = oracle.assign(X, np.array([[0.0], [1.0], [3.0]]))
    assert lab.tolist() == [0, 1]            # 0.5 ties between c0 and c1; 2.0 ties c1 and c2
    lab, _ = oracle.assign(X, np.array([[3.0], [1.0], [0.0]]))
    assert lab.tolist() == [1, 0]            # same ties, reversed order
    X2 = np.array([[0.0, 0.0]], np.float32)  # four centroids at equal distance
    C2 = np.array([[1.0, 0.0], [0.0, -1.0], [-1.0, 0.0], [0.0, 1.0]])
    assert oracle.assign(X2, C2)[0].tolist() == [0]


def test_empty_cluster_keeps_centroid():
    X = np.array([[0.0, 0.0], [0.1, 0.0], [5.0, 5.0]], np.float32)
    C0 = np.array([[0.0, 0.0], [100.0, -100.0], [5.0, 5.0]])
    r = oracle.lloyd(X, C0, 2)
    assert r["labels"][0].tolist() == [0, 0, 2]
    np.testing.assert_array_equal(r["centroids"][0][1], C0[1])
    np.testing.assert_array_equal(r["centroids"][0][0], [float(np.float32(0.1)) / 2, 0.0])


def test_update_counts_and_transposition():
    """Non-square shapes catch a transposed operand; counts sum to n."""
    rng = np.random.default_rng(3)
    X = rng.normal(size=(40, 5)).astype(np.float32)
    C = rng.normal(size=(3, 5))
    lab, _ = oracle.assign(X, C)
    Cn, cnt = oracle.update(X, lab, C)
    assert cnt.sum() == 40
    for j in range(3):
        if cnt[j]:
            np.testing.assert_allclose(Cn[j], X[lab == j].astype(np.float64).mean(axis=0), rtol=1e-13)


def test_sse_monotone():
    P = datagen.make_config(1, n=3000)
    r = oracle.lloyd(P.X, P.C0.astype(np.float64), 12)
    sa, su = r["sse_assign"], r["sse_update"]
    assert (su <= sa * (1 + 1e-12)).all()
    assert (sa[1:] <= su[:-1] * (1 + 1e-12)).all()


def test_permutation_equivariance():
    P = datagen.make_config(2, n=4000)
    C = P.C0.astype(np.float64)
    lab, d1, d2 = oracle.assign(P.X, C, second=True)
    perm = np.random.default_rng(5).permutation(C.shape[0])
    lab_p, d1p = oracle.assign(P.X, C[perm])
    unique = d2 > d1          # points with no exact tie
    inv = np.argsort(perm)
    assert (inv[lab[unique]] == lab_p[unique]).all()
    np.testing.assert_array_equal(d1, d1p)


def test_matches_independent_library_lloyd():
    """An independent Lloyd implementation (scikit-learn, FP64) on well-separated blobs."""
    sk = pytest.importorskip("sklearn.cluster")
    P = datagen.make_config(1, n=4000)
    X64 = P.X.astype(np.float64)
    C0 = P.C0.astype(np.float64)
    T = 15
    r = oracle.lloyd(P.X, C0, T)
    assert (np.bincount(r["labels"][-1], minlength=16) > 0).all()
    km = sk.KMeans(n_clusters=16, init=C0, n_init=1, max_iter=T, tol=0.0, algorithm="lloyd")
    km.fit(X64)
    # scikit-learn reports labels from one more assignment step with its final centers
    np.testing.assert_array_equal(km.labels_, oracle.assign(P.X, r["final"])[0])
    np.testing.assert_allclose(km.cluster_centers_, r["final"], rtol=1e-10, atol=1e-10)


def test_datagen_shapes_and_determinism():
    a = datagen.make_config(2, n=1000)
    b = datagen.make_config(2, n=1000)
    assert a.X.shape == (1000, 32) and a.C0.shape == (256, 32)
    assert a.X.dtype == np.float32 and a.C0.dtype == np.float32
    np.testing.assert_array_equal(a.X, b.X)
    np.testing.assert_array_equal(a.C0, b.C0)
    c1 = datagen.make_config(1)
    np.testing.assert_array_equal(c1.C0, c1.X[:16])


def _exact_d2(x, c):
    """Exact squared distance of an FP32 point to an FP64 centroid (rational arithmetic)."""
    return sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(x, c))


def test_dist2_to_hand_values():
    """dist2_to reads the labelled row: 1-2-2 triangle distances by hand."""
    X = np.array([[1.0, 2.0], [0.0, 0.0]], np.float32)
    C = np.array([[0.0, 0.0], [4.0, 6.0], [1.0, 2.0]])
    np.testing.assert_array_equal(oracle.dist2_to(X, C, np.array([1, 1])), [25.0, 52.0])
    np.testing.assert_array_equal(oracle.dist2_to(X, C, np.array([0, 2])), [5.0, 5.0])
    np.testing.assert_array_equal(oracle.dist2_to(X, C, np.array([2, 0])), [0.0, 0.0])


@pytest.mark.parametrize("seed", range(4))
def test_dist2_to_bruteforce(seed):
    """Every point's distance to an arbitrary (random) labelled centroid equals
    the exact rational value within FP64 rounding; the centroids are far
    apart, so a wrong row, a dropped coordinate or a sign slip is visible."""
    rng = np.random.default_rng(50 + seed)
    n, k, d = 37, 5, 1 + seed * 3
    X = rng.normal(size=(n, d)).astype(np.float32)
    C = rng.normal(size=(k, d)) + 10.0 * np.arange(k)[:, None]
    lab = rng.integers(0, k, size=n).astype(np.int32)
    got = oracle.dist2_to(X, C, lab)
    for i in range(n):
        want = float(_exact_d2(X[i], C[lab[i]]))
        assert got[i] == pytest.approx(want, rel=4 * d * 2.0 ** -53, abs=0), (i, lab[i])


def test_dist2_to_of_assignment_is_dmin_and_second_is_bruteforce():
    """dist2_to under the oracle's own labels returns its nearest distances
    bit for bit, and the second distance of assign() is the second smallest
    of the exact distances (brute force)."""
    rng = np.random.default_rng(9)
    X = rng.normal(size=(60, 4)).astype(np.float32)
    C = rng.normal(size=(7, 4))
    lab, d1, d2 = oracle.assign(X, C, second=True)
    np.testing.assert_array_equal(oracle.dist2_to(X, C, lab), d1)
    for i in range(X.shape[0]):
        ex = sorted(float(_exact_d2(X[i], C[j])) for j in range(C.shape[0]))
        assert d1[i] == pytest.approx(ex[0], rel=1e-14)
        assert d2[i] == pytest.approx(ex[1], rel=1e-14)
    assert (oracle.assign(X, C[:1], second=True)[2] == np.inf).all()   # k = 1: no second


def test_near_tie_check_rejects_a_wrong_label():
    """The parity check (tests/parity.py) accepts the oracle's own labels,
    accepts a swap at an exact tie, and rejects a label that is farther than
    the near-tie band -- a mistake planted on the CPU side."""
    from parity import check_assignment
    X = np.array([[0.5], [3.0], [9.0]], np.float32)
    C = np.array([[0.0], [1.0], [10.0]], np.float32)
    lab, _ = oracle.assign(X, C.astype(np.float64))
    assert check_assignment(X, C, lab) == (0, 0)
    tie = lab.copy()
    tie[0] = 1                                         # 0.5 is equidistant from 0 and 1
    assert check_assignment(X, C, tie) == (1, 1)
    bad = lab.copy()
    bad[1] = 2                                         # 3.0 is 2 from c1 and 7 from c2
    with pytest.raises(AssertionError):
        check_assignment(X, C, bad)
