"""bench.py's host-side models (no GPU): the algorithmic byte counts behind
the roofline figures and the rule that reports measured HBM traffic only
for the kernel source and launch tuning the counters were taken under."""
import hashlib
import json
import os
import types

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _problem(precision, d=128, g=100):
    return types.SimpleNamespace(precision=precision, d=d, g=g)


def test_bound_bytes_follow_the_format():
    bench.TUNING.clear()
    assert bench.bound_layout(_problem("bf16")) == (4, 100)
    bench.TUNING.update(bound_codes=2)
    assert bench.bound_layout(_problem("bf16")) == (2, 100)
    assert bench.bound_layout(_problem("fp32")) == (4, 100)   # FP32 problems keep FP32 bounds
    bench.TUNING.clear()


def test_algorithmic_bytes_per_launch():
    bench.TUNING.clear()
    bench.TUNING.update(bound_codes=2)
    s = dict(point_filter_fail=1000, pairs=3000, rechecks=10)
    P = _problem("bf16", d=128, g=100)
    per_point = 4 * 128 + 16 + 4 + 4 * 4 + 4 + 16 + 12     # row, entry, norm, masks, closed bound, state, update
    assert bench.assign_bytes(P, s) == 1000 * per_point + 3000 * 2 + 10 * 20
    assert bench.gfilter_bytes(P, s) == 1000 * (16 + 2 * 100 + 4 * 4 + 4)
    bench.TUNING.clear()
    assert bench.gfilter_bytes(P, s) == 1000 * (16 + 4 * 100 + 4 * 4 + 4)


def test_traffic_only_for_matching_source_and_tuning(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1905_09345_amd", "csrc", "kp_kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (tmp_path / "paper_1905_09345_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_1905_09345_amd" / "csrc" / "kp_kernels.hip").write_bytes(open(src, "rb").read())
    ent = dict(workload="W", source_sha256=digest, bytes_per_launch=123.0,
               tuning=dict(chunk_depth=1, bound_codes=2))
    (prof / "traffic.json").write_text(json.dumps({"k@depth1": ent,
                                                   "k@depth3": dict(ent, bytes_per_launch=456.0,
                                                                    tuning=dict(chunk_depth=3, bound_codes=2))}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    bench.TUNING.clear()
    bench.TUNING.update(chunk_depth=3, bound_codes=2)
    assert bench.traffic_of("k", "W") == 456.0
    bench.TUNING.update(chunk_depth=1)
    assert bench.traffic_of("k", "W") == 123.0
    bench.TUNING.update(bound_codes=1)          # counters taken under another tuning
    assert bench.traffic_of("k", "W") is None
    bench.TUNING.update(bound_codes=2)
    assert bench.traffic_of("k", "other workload") is None
    (tmp_path / "paper_1905_09345_amd" / "csrc" / "kp_kernels.hip").write_text("changed")
    assert bench.traffic_of("k", "W") is None   # the source has changed since
    bench.TUNING.clear()


def test_batched_plain_lloyd_matches_per_problem_lloyd(monkeypatch):
    """The batched torch comparator (problems of one (D, K) class padded and
    stacked) computes the same Lloyd iterations as each problem alone:
    padding rows take no part, and the labels and sums are per problem."""
    import numpy as np
    import torch
    import bench
    import datagen
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(torch.cuda, "empty_cache", lambda *a, **k: None)
    rng = np.random.default_rng(0)
    Xs, Cs = [], []
    for n, d, k in [(500, 16, 16), (300, 16, 16), (700, 32, 64), (200, 8, 16), (90, 8, 16)]:
        X = datagen.gaussian_mixture(rng, n, d, k).astype(np.float32)
        Xs.append(torch.from_numpy(X))
        Cs.append(torch.from_numpy(X[:k].copy()))
    out = []
    bench.plain_fp32_lloyd_batched(torch, Xs, Cs, iters=2, warmup=1, rows=128, centroids_out=out)

    def lloyd(X, C, T):
        for _ in range(T):
            lab = ((X[:, None, :].double() - C[None].double()) ** 2).sum(2).argmin(1)
            s = torch.zeros_like(C).index_add_(0, lab, X)
            c = torch.bincount(lab, minlength=C.shape[0]).float()
            C = torch.where(c[:, None] > 0, s / c.clamp(min=1)[:, None], C)
        return C
    for X, C, Cb in zip(Xs, Cs, out):
        assert torch.allclose(lloyd(X, C, 3), Cb, rtol=1e-5, atol=1e-5)


def test_fp32_filtered_roofline_counts_direct_form_work():
    """The FP32 form's filtered stage is priced at 3d operations per distance
    computed against the FP32 vector peak, with its HBM bytes beside it."""
    import types
    import bench
    P = types.SimpleNamespace(precision="fp32", d=32, g=26, k=256, n=10 ** 6, meta={"name": "w"})
    st = [dict(dense=1, point_filter_fail=0, pairs=0, distances=0),
          dict(dense=0, point_filter_fail=1000, pairs=3000, distances=20000),
          dict(dense=0, point_filter_fail=3000, pairs=5000, distances=40000)]
    r = bench.roofline_of("assign", dict(ms=2.0, launches=2), P, st)   # 1 ms per launch
    ops = 3 * 32 * 30000
    assert r["bound"] == "alu" and abs(r["achieved"] - ops / 1e-3 / 1e12) < 1e-12
    assert abs(r["frac"] - r["achieved"] / 78.6) < 1e-15
    byts = 2000 * (4 * 32 + 4 * 26 + 48) + 4000 * 8
    assert abs(r["hbm"]["achieved"] - byts / 1e-3 / 1e9) < 1e-9
