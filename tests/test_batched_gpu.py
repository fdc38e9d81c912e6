"""GPU parity of the batched form: several independent problems of uneven
N, D, K and precision in one context, every stage launched once for all of
them, each problem checked step-locked against the FP64 oracle."""
import math

import numpy as np
import pytest

import datagen
from parity import run_steplocked_batch

pytestmark = pytest.mark.gpu


def _problem(seed, n, d, k, prec):
    rng = np.random.default_rng(seed)
    X = datagen.gaussian_mixture(rng, n, d, k)
    C0 = datagen.kmeanspp(rng, X, k, sample=min(n, 64 * k))
    return X, C0, int(math.ceil(k / 10)), prec


def test_mixed_batch():
    """Uneven sizes, both precisions, ragged and padded dimensions."""
    specs = [(1, 3_001, 16, 16, "bf16"), (2, 9_017, 32, 64, "bf16"), (3, 20_011, 64, 256, "bf16"),
             (4, 4_099, 37, 20, "bf16"), (5, 7_001, 5, 12, "fp32"), (6, 12_007, 32, 64, "fp32"),
             (7, 150, 16, 16, "bf16"), (8, 65, 8, 3, "fp32")]
    print("CASE batch-mixed", len(specs), flush=True)
    reps = run_steplocked_batch([_problem(*sp) for sp in specs], 8)
    for r in reps:
        assert len(r["stats"]) == 8 and r["stats"][0]["dense"] == 1


@pytest.mark.parametrize("depth", [1, 3])
def test_batch_of_small_problems(depth):
    """Many small problems of the batched workload's shapes."""
    from paper_1905_09345_amd.kp import kp_tuning
    rng = np.random.default_rng(42)
    specs = []
    for p in range(24):
        specs.append((500 + p, int(rng.integers(300, 3000)), int(rng.choice([16, 32, 64])),
                      int(rng.choice([16, 64, 256])), "bf16"))
    print("CASE batch-small", len(specs), depth, flush=True)
    run_steplocked_batch([_problem(*sp) for sp in specs], 6, tuning=kp_tuning(chunk_depth=depth), check_every=2)


def test_batch_fp16_bound_codes():
    """The batched form with its group bounds stored as FP16 codes."""
    from paper_1905_09345_amd.kp import kp_tuning
    specs = [(40 + i, 3_000 + 97 * i, 32 * (1 + i % 4), 48 + 8 * i, "bf16") for i in range(6)]
    print("CASE batch-fp16-codes", specs, flush=True)
    run_steplocked_batch([_problem(*sp) for sp in specs], 6, tuning=kp_tuning(bound_codes=2), check_every=2)


def test_batch_graph_and_timing():
    """Batched iterations replayed from a captured graph, stages timed inside it."""
    import torch
    from paper_1905_09345_amd import KMeans
    from paper_1905_09345_amd.kp import kp_tuning
    probs = [_problem(900 + i, 2_000 + 500 * i, 32, 64, "bf16") for i in range(5)]
    dev = [(torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda(), g, prec) for X, C0, g, prec in probs]
    print("CASE batch-graph", flush=True)
    km = KMeans(dev, tuning=kp_tuning(timing=1, use_graph=1))
    km.iterate(4)
    t = km.stage_times()
    assert t["filtered_iter"]["launches"] == 3 and t["assign"]["launches"] == 3
    for i in range(len(probs)):
        assert len(km.stats(i)) == 4
    km.close()


def test_autotune_then_run():
    """kp_autotune picks one of its candidates; the batch then runs with it and matches the oracle."""
    import torch
    from paper_1905_09345_amd import KMeans
    probs = [_problem(700 + i, 3_000 + 1_000 * i, 16 * (1 + i % 3), 64, "bf16") for i in range(6)]
    dev = [(torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda(), g, prec) for X, C0, g, prec in probs]
    print("CASE autotune", flush=True)
    best = KMeans.autotune(dev, iters=3)
    assert best.chunk_depth in (1, 3) and best.blocks_per_cu in (8, 16, 32) and best.use_graph == 1
    run_steplocked_batch(probs, 5, tuning=best)


def test_autotune_groups_then_run():
    """kp_autotune_groups gives every problem of a (d, k, precision) class the
    same g, one of its candidates (the problem's own g, ceil(k/16), ceil(k/10));
    the batch then runs with those group counts and matches the oracle."""
    import torch
    from paper_1905_09345_amd import KMeans
    from paper_1905_09345_amd.kp import kp_tuning
    specs = [(11, 6_000, 32, 64, "bf16"), (12, 9_000, 32, 64, "bf16"), (13, 12_000, 64, 256, "bf16"),
             (14, 5_000, 16, 16, "bf16"), (15, 7_000, 32, 48, "fp32"), (16, 4_000, 32, 48, "fp32")]
    probs = [_problem(*sp) for sp in specs]
    probs[1] = probs[1][:2] + (3,) + probs[1][3:]   # an own g that differs within its class
    dev = [(torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda(), g, prec) for X, C0, g, prec in probs]
    print("CASE autotune-groups", flush=True)
    tun = kp_tuning(bound_codes=2, blocks_per_cu=16, chunk_depth=1)
    gs = KMeans.autotune_groups(dev, iters=3, tuning=tun)
    assert len(gs) == len(probs)
    for (X, C0, g, prec), gt, sp in zip(probs, gs, specs):
        k = C0.shape[0]
        assert gt in (g, max(1, math.ceil(k / 16)), math.ceil(k / 10)), (sp, g, gt)
    for a, b in ((0, 1), (4, 5)):   # one g per class, unless each kept its own
        own = gs[a] == probs[a][2] and gs[b] == probs[b][2]
        assert gs[a] == gs[b] or own
    tuned = [(X, C0, gt, prec) for (X, C0, _, prec), gt in zip(probs, gs)]
    run_steplocked_batch(tuned, 5, tuning=tun)


def test_batch_whole_call_graph():
    """A batch iterated with use_graph = 2: the calls' iterations run as one
    graph each (the last call replays the previous one's); the final step is
    checked against the oracle."""
    import torch
    from paper_1905_09345_amd import KMeans
    from paper_1905_09345_amd.kp import kp_tuning
    from parity import check_assignment, check_centroids, rms_norm
    specs = [(1, 3000, 16, 16, "bf16"), (2, 2500, 32, 64, "fp32"), (3, 4000, 64, 256, "bf16"),
             (4, 1200, 8, 16, "fp32")]
    probs = [_problem(*sp) for sp in specs]
    print("CASE batch whole-call graph", len(probs), flush=True)
    dev = [(torch.from_numpy(np.ascontiguousarray(X)).cuda(), torch.from_numpy(np.ascontiguousarray(C0)).cuda(),
            g, prec, 0) for X, C0, g, prec in probs]
    km = KMeans(dev, tuning=kp_tuning(use_graph=2))
    try:
        for c in (3, 4, 4):
            km.iterate(c)
        prev = [tuple(a.cpu().numpy() for a in km.centroids(i)) for i in range(len(probs))]
        km.iterate(1)
        assert km.iterations == 12
        for i, (X, _, _, _) in enumerate(probs):
            lab = km.assign(i).cpu().numpy()
            c32, c64 = [a.cpu().numpy() for a in km.centroids(i)]
            check_assignment(X, prev[i][0], lab)
            check_centroids(X, lab, prev[i][1], c32, c64, rms_norm(X))
    finally:
        km.close()
