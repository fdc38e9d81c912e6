"""Full-size workloads on the GPU, checked on sampled points every iteration.

The assignment check uses 16384 seeded random points per checked iteration
(the oracle computes each one's nearest centroid against the GPU's previous
FP32 centroids); the centroid check uses every point.
"""
import pytest

import datagen
from parity import run_steplocked

pytestmark = pytest.mark.gpu


def test_c2_full_fp32_sampled():
    P = datagen.make_config(2)
    print("CASE c2-full", flush=True)
    r = run_steplocked(P.X, P.C0, P.g, "fp32", P.iters, sample=16384)
    print("mismatches per checked iteration", r["mismatch"], flush=True)


def test_c3_full_bf16_sampled():
    P = datagen.make_config(3)
    print("CASE c3-full", flush=True)
    r = run_steplocked(P.X, P.C0, P.g, "bf16", P.iters, sample=16384, check_every=3)
    print("mismatches per checked iteration", r["mismatch"], flush=True)
    st = r["stats"]
    print("rechecks", [s["rechecks"] for s in st], flush=True)


def test_c5_full_bf16_sampled():
    """The largest single-GPU workload: N = 1.6e7, D = 256, K = 4096, G = 410,
    20 iterations, the regime where many points need the FP32 recheck."""
    P = datagen.make_config(5)
    print("CASE c5-full", flush=True)
    r = run_steplocked(P.X, P.C0, P.g, "bf16", P.iters, sample=16384, check_every=2)
    print("mismatches per checked iteration", r["mismatch"], flush=True)
    st = r["stats"]
    rech = [s["rechecks"] for s in st]
    print("rechecks", rech, flush=True)
    assert len(st) == P.iters and st[0]["dense"] == 1
    assert rech[0] > 0                       # the first (dense) pass leaves uncertain points to the recheck
    assert st[-1]["pairs"] < P.n * P.g       # the group-level filter prunes by the last iteration


def test_c4_batched_512_problems():
    """The batched workload at its real shape: 512 problems (N ~ U{2000..200000},
    D in {16, 32, 64}, K in {16, 64, 256}, G = ceil(K/10)), 25 iterations in
    one context.  Every problem's centroids are checked against the oracle
    at the checked iterations; assignments on 2048 sampled points each."""
    from parity import run_steplocked_batch
    probs = datagen.make_batched(512)
    print("CASE c4-full", len(probs), sum(p.n for p in probs), flush=True)
    reps = run_steplocked_batch([(p.X, p.C0, p.g, p.precision) for p in probs], probs[0].iters,
                                check_every=6, sample=2048)
    assert all(len(r["stats"]) == probs[0].iters for r in reps)
    print("near-tie mismatches", sum(sum(r["mismatch"]) for r in reps), flush=True)
