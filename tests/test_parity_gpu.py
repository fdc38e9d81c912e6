"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle.

Sizes are chosen so that the oracle finishes in seconds while the GPU runs
several tiles and a ragged tail; the full-size workloads are checked on
sampled points (test_fullsize_gpu.py).
"""
import numpy as np
import pytest

import datagen
from parity import run_steplocked

pytestmark = pytest.mark.gpu


def _print_case(name, **kw):
    print("CASE", name, kw, flush=True)


def test_c1_full_fp32():
    P = datagen.make_config(1)
    _print_case("c1", n=P.n)
    r = run_steplocked(P.X, P.C0, P.g, "fp32", P.iters)
    st = r["stats"]
    assert st[0]["dense"] == 1 and len(st) == P.iters
    assert st[-1]["point_filter_fail"] < P.n // 2     # the point-level filter prunes


def test_c2_reduced_fp32():
    P = datagen.make_config(2, n=60_007)
    _print_case("c2-reduced", n=P.n)
    r = run_steplocked(P.X, P.C0, P.g, "fp32", 12)
    st = r["stats"]
    assert st[-1]["distances"] < 0.5 * P.n * P.k


def test_c3_shape_bf16():
    P = datagen.make_config(3, n=30_011)
    _print_case("c3-reduced", n=P.n)
    r = run_steplocked(P.X, P.C0, P.g, "bf16", 6)
    st = r["stats"]
    assert st[0]["dense"] == 1
    # the FP32 recheck runs: the uncertain points of the dense first pass
    assert st[0]["rechecks"] > 0


def test_c5_shape_bf16():
    """The large workload's shape (D=256, K=4096, G=410, Student-t mixture with
    Zipf sizes) at a reduced N: eight 32-wide steps per MFMA tile, seven
    rounds of the group filter."""
    P = datagen.make_config(5, n=40_000)
    _print_case("c5-reduced", n=P.n)
    r = run_steplocked(P.X, P.C0, P.g, "bf16", 4)
    assert r["stats"][-1]["pairs"] < P.n * P.g


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_row_test_in_point_filter(prec):
    """Late in a run many points have every group closed, their own included.
    After an iteration where at least an eighth of the points were such
    points, the point-level filter reads whole bound rows and leaves them out
    of L1.  The run stays step-locked with the oracle, the gate follows that
    rule in every iteration, and it switches on."""
    rng = np.random.default_rng(21)
    X = datagen.gaussian_mixture(rng, 20_011, 24, 40)
    C0 = datagen.kmeanspp(rng, X, 60, sample=4000)
    _print_case("row-test", prec=prec)
    r = run_steplocked(X, C0, 8, prec, 25)
    st = r["stats"]
    n = X.shape[0]
    assert st[0]["row_test"] == 0 and st[0]["closed"] == 0
    for prev, cur in zip(st, st[1:]):
        assert cur["row_test"] == int(8 * prev["closed"] >= n), (prev, cur)
        assert cur["point_filter_fail"] + (cur["closed"] if cur["row_test"] else 0) <= n
    on = [s for s in st if s["row_test"]]
    assert on and sum(s["closed"] for s in on) > 0, [(s["iter"], s["closed"]) for s in st]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_plain_lloyd_mode(prec):
    """kp_tuning.plain (the comparator): every iteration is a dense pass over
    sums recomputed from all points; step-locked with the oracle."""
    from paper_1905_09345_amd.kp import kp_tuning
    rng = np.random.default_rng(33)
    X = datagen.gaussian_mixture(rng, 12_007, 24, 40)
    C0 = datagen.kmeanspp(rng, X, 48, sample=4000)
    _print_case("plain", prec=prec)
    r = run_steplocked(X, C0, 5, prec, 8, tuning=kp_tuning(plain=1))
    assert all(s["dense"] == 1 for s in r["stats"]) and len(r["stats"]) == 8


def test_plain_lloyd_mode_batch():
    from paper_1905_09345_amd.kp import kp_tuning
    from parity import run_steplocked_batch
    probs = []
    for i, (n, d, k) in enumerate([(3_001, 16, 16), (5_003, 32, 64), (2_011, 8, 12)]):
        rng = np.random.default_rng(70 + i)
        X = datagen.gaussian_mixture(rng, n, d, k)
        probs.append((X, datagen.kmeanspp(rng, X, k, sample=2000), int(np.ceil(k / 10)), "fp32"))
    _print_case("plain-batch")
    run_steplocked_batch(probs, 5, tuning=kp_tuning(plain=1))


@pytest.mark.parametrize("case", ["c1", "c2", "groups1", "groups30", "ties"])
def test_fp32_local_filter(case):
    """The FP32 form with the per-centroid local filter on: step-locked with
    the oracle, and it computes fewer distances than the surviving pairs'
    groups hold."""
    from paper_1905_09345_amd.kp import kp_tuning
    t = kp_tuning(local_filter=1)
    if case in ("c1", "c2"):
        P = datagen.make_config(int(case[1]), n=None if case == "c1" else 60_007)
        X, C0, g, iters = P.X, P.C0, P.g, (P.iters if case == "c1" else 12)
    elif case == "ties":
        gr = np.arange(-4, 5, dtype=np.float32)
        X = np.concatenate([np.stack(np.meshgrid(gr, gr, gr), axis=-1).reshape(-1, 3)] * 3).astype(np.float32)
        C0 = np.array([[0.5, 0, 0], [-0.5, 0, 0], [0, 0.5, 0], [0, -0.5, 0], [2, 2, 2], [2, 2, 2],
                       [100, 100, 100], [-3, -3, 3]], np.float32)
        g, iters = 3, 5
    else:
        rng = np.random.default_rng(7)
        X = datagen.gaussian_mixture(rng, 5_000, 24, 30)
        C0 = datagen.kmeanspp(rng, X, 30)
        g, iters = (1 if case == "groups1" else 30), 8
    _print_case("fp32-local-filter", case=case)
    r = run_steplocked(X, C0, g, "fp32", iters, tuning=t)
    if case in ("c1", "c2"):
        st = [s for s in r["stats"] if not s["dense"]]
        assert sum(s["distances"] for s in st) < sum(s["pairs"] for s in st) * (C0.shape[0] / g)


@pytest.mark.parametrize("case", ["d100_g2", "d24_g1_k100", "d100_g2_local_filter", "batch"])
def test_fp32_groups_over_one_staged_batch(case):
    """The FP32 tile kernel copies a visited group's member rows into LDS in
    batches of 1024 floats (10 rows at d = 100, 42 at d = 24).  Groups larger
    than one batch, a partial last batch, the local filter's skips across
    batches and the batched launch stay step-locked with the oracle."""
    from paper_1905_09345_amd.kp import kp_tuning
    from parity import run_steplocked_batch
    shapes = {"d100_g2": (6_007, 100, 64, 2), "d24_g1_k100": (8_009, 24, 100, 1),
              "d100_g2_local_filter": (6_007, 100, 64, 2)}
    tuning = kp_tuning(local_filter=1) if case.endswith("local_filter") else None
    _print_case("fp32-staged", case=case)
    if case == "batch":
        probs = []
        for i, (n, d, k, g) in enumerate([(4_001, 100, 64, 2), (3_001, 24, 100, 1), (2_003, 8, 40, 1)]):
            rng = np.random.default_rng(90 + i)
            X = datagen.gaussian_mixture(rng, n, d, k)
            probs.append((X, datagen.kmeanspp(rng, X, k, sample=2000), g, "fp32"))
        run_steplocked_batch(probs, 6)
        return
    n, d, k, g = shapes[case]
    rng = np.random.default_rng(n + d)
    X = datagen.gaussian_mixture(rng, n, d, k)
    C0 = datagen.kmeanspp(rng, X, k, sample=4000)
    r = run_steplocked(X, C0, g, "fp32", 8, tuning=tuning)
    assert sum(s["distances"] for s in r["stats"] if not s["dense"]) > 0


@pytest.mark.parametrize("d", [16, 32, 64])
def test_bf16_small_dims(d):
    rng = np.random.default_rng(d)
    X = datagen.gaussian_mixture(rng, 9_001, d, 64)
    C0 = datagen.kmeanspp(rng, X, 64, sample=2000)
    _print_case("bf16-d", d=d)
    run_steplocked(X, C0, 7, "bf16", 8)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [5, 13, 37])
def test_ragged_dims(prec, d):
    rng = np.random.default_rng(100 + d)
    X = datagen.gaussian_mixture(rng, 3_333, d, 20)
    C0 = X[:20].copy()
    _print_case("ragged", d=d, prec=prec)
    run_steplocked(X, C0, 4, prec, 6)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("g", [1, 2, 30])
def test_group_extremes(prec, g):
    """G=1 (one group), G=K (every centroid alone) and in between."""
    rng = np.random.default_rng(7)
    X = datagen.gaussian_mixture(rng, 5_000, 24, 30)
    C0 = datagen.kmeanspp(rng, X, 30)
    _print_case("groups", g=g, prec=prec)
    run_steplocked(X, C0, g, prec, 8)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_k1(prec):
    rng = np.random.default_rng(1)
    X = rng.normal(size=(777, 9)).astype(np.float32)
    _print_case("k1", prec=prec)
    r = run_steplocked(X, X[:1].copy(), 1, prec, 3)
    np.testing.assert_allclose(r["c64"][0], X.astype(np.float64).mean(axis=0), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_ties_duplicates_and_empty_clusters(prec):
    """Exact ties (points on a grid, centroids at symmetric positions), duplicated
    centroids and a centroid that never receives a point."""
    g = np.arange(-4, 5, dtype=np.float32)
    X = np.stack(np.meshgrid(g, g, g), axis=-1).reshape(-1, 3)
    X = np.concatenate([X] * 3).astype(np.float32)           # 2187 points with many exact ties
    C0 = np.array([[0.5, 0, 0], [-0.5, 0, 0], [0, 0.5, 0], [0, -0.5, 0],
                   [2, 2, 2], [2, 2, 2],                      # duplicate centroid
                   [100, 100, 100],                           # never used
                   [-3, -3, 3]], np.float32)
    _print_case("ties", prec=prec)
    r = run_steplocked(X, C0, 3, prec, 5)
    assert r["c64"][6].tolist() == [100.0, 100.0, 100.0]


@pytest.mark.parametrize("use_graph", [1, -1, 2])
def test_graph_and_plain_launches(use_graph):
    from paper_1905_09345_amd.kp import kp_tuning
    P = datagen.make_config(1, n=4_097)
    _print_case("graph", use_graph=use_graph)
    run_steplocked(P.X, P.C0, P.g, "fp32", 6, tuning=kp_tuning(use_graph=use_graph))


@pytest.mark.parametrize("case", ["c3", "c5", "long", "d16"])
def test_fp16_bound_codes(case):
    """Group bounds stored as FP16 codes rounded down (looser, never above the
    true bound): the same exact result as the oracle."""
    from paper_1905_09345_amd.kp import kp_tuning
    t = kp_tuning(bound_codes=2)
    _print_case("fp16-codes", case=case)
    if case == "c3":
        P = datagen.make_config(3, n=30_011)
        run_steplocked(P.X, P.C0, P.g, "bf16", 6, tuning=t)
    elif case == "c5":
        P = datagen.make_config(5, n=40_000)
        run_steplocked(P.X, P.C0, P.g, "bf16", 4, tuning=t)
    elif case == "long":
        P = datagen.make_config(2, n=20_011)
        run_steplocked(P.X, P.C0, P.g, "bf16", 45, tuning=t, check_every=3)
    else:
        rng = np.random.default_rng(16)
        X = datagen.gaussian_mixture(rng, 9_001, 16, 64)
        C0 = datagen.kmeanspp(rng, X, 64, sample=2000)
        run_steplocked(X, C0, 7, "bf16", 8, tuning=t)


@pytest.mark.parametrize("scale", [1e-6, 1e6])
def test_fp16_bound_codes_extreme_scales(scale):
    """FP16 bound codes on data scaled far from 1: the code scale follows the
    data (distances land near 2^10), so the bounds stay valid and useful."""
    from paper_1905_09345_amd.kp import kp_tuning
    rng = np.random.default_rng(77)
    X = (datagen.gaussian_mixture(rng, 12_001, 32, 48) * scale).astype(np.float32)
    C0 = datagen.kmeanspp(rng, X, 48, sample=3000)
    _print_case("fp16-codes-scale", scale=scale)
    r = run_steplocked(X, C0, 5, "bf16", 8, tuning=kp_tuning(bound_codes=2))
    assert r["stats"][-1]["pairs"] < 12_001 * 5   # the group filter still prunes


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_long_run(prec):
    """Many iterations: the cumulative drift sums keep growing while bounds stay valid."""
    P = datagen.make_config(2, n=20_011)
    _print_case("long", prec=prec)
    r = run_steplocked(P.X, P.C0, P.g, prec, 45, check_every=3)
    assert len(r["stats"]) == 45


def test_stage_times():
    import torch
    from paper_1905_09345_amd import KMeans
    from paper_1905_09345_amd.kp import kp_tuning
    P = datagen.make_config(3, n=10_000)
    _print_case("timing")
    for use_graph in (1, -1):
        km = KMeans([(torch.from_numpy(P.X).cuda(), torch.from_numpy(P.C0).cuda(), P.g, "bf16")],
                    tuning=kp_tuning(timing=1, use_graph=use_graph))
        km.iterate(4)
        t = km.stage_times()
        km.close()
        assert t["assign_dense"]["launches"] == 1 and t["assign_dense"]["ms"] > 0
        if use_graph == 1:
            assert t["filtered_iter"]["launches"] == 3
        # every stage is timed on its own, inside graph replays as well
        from paper_1905_09345_amd.kp import kp_last_error
        assert "assign" in t, (sorted(t), kp_last_error())
        assert t["assign"]["launches"] == 3 and t["bound_filter"]["launches"] == 3
        assert t["assign"]["ms"] > 0


def test_stage_times_of_selected_stages():
    """kp_tuning.timing_stages: only the selected stages carry events (plus
    the whole replays), and the results are those of an untimed run."""
    import torch
    from paper_1905_09345_amd import KMeans
    from paper_1905_09345_amd.kp import kp_tuning, STAGES
    P = datagen.make_config(3, n=10_000)
    _print_case("timing-mask")
    X, C = torch.from_numpy(P.X).cuda(), torch.from_numpy(P.C0).cuda()
    labels = []
    for use_graph in (1, -1):
        km = KMeans([(X, C, P.g, "bf16")], tuning=kp_tuning(timing=1, use_graph=use_graph,
                                                           timing_stages=1 << STAGES.index("assign")))
        km.iterate(4)
        t = km.stage_times()
        labels.append(km.assign().cpu().numpy())
        km.close()
        assert set(t) <= {"assign", "filtered_iter"}, sorted(t)
        assert t["assign"]["launches"] == 3 and t["assign"]["ms"] > 0
    km = KMeans([(X, C, P.g, "bf16")])
    km.iterate(4)
    ref = km.assign().cpu().numpy()
    km.close()
    for lab in labels:
        assert (lab == ref).all()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [5, 17, 41, 63, 64, 65, 112, 129])
def test_tail_tiles(prec, n):
    """Point counts whose last 64-point tile has empty 16-point blocks."""
    rng = np.random.default_rng(n)
    X = datagen.gaussian_mixture(rng, n, 16, 3)
    C0 = X[:5].copy()
    _print_case("tail", n=n, prec=prec)
    run_steplocked(X, C0, 2, prec, 4)
