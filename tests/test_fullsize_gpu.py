"""Full-size workloads on the GPU, checked on sampled points every iteration.

The assignment check uses 16384 seeded random points per iteration (the
oracle computes each one's nearest centroid against the GPU's previous FP32
centroids); the centroid check uses every point.
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
