"""Benchmark: point-iterations/sec of the filtered K-means path on one MI355X.

One step = one complete K-means run of the workload's T iterations (the
dense first iteration, then T-1 filtered iterations with centroid updates)
from the initial centroids, on inputs already resident in HBM.  Each step
uses its own context, created (with its per-point BF16 shadow) before the
timed region, so every step starts from iteration 1.

value = N * T * steps / seconds.  Printed beside it, on the same JSON line:
  plain_fp32_lloyd  dense FP32 Lloyd on the same GPU (torch FP32 GEMM with
                    TF32 off, argmin, full centroid recompute)
  roofline          the dominant kernel's achieved rate against the MI355X
                    peak, from HIP events the library records around it
  cpu_baseline      the FP64 oracle on the host cores, on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "point-iterations/sec, filtered BF16+recheck vs plain FP32 Lloyd, same GPU"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5, choices=[1, 2, 3, 4, 5],
                    help="headline workload (default 5: the largest single-GPU configuration)")
    ap.add_argument("--secondary", default="2,4",
                    help="comma-separated workloads measured after the headline with --secondary-steps steps "
                         "(default: 2 = plain filtered FP32, 4 = the batched form; empty to skip)")
    ap.add_argument("--secondary-steps", type=int, default=3)
    ap.add_argument("--problems", type=int, default=512, help="problems of the batched workload (config 4)")
    ap.add_argument("--n", type=int, default=None, help="override N (same recipe)")
    ap.add_argument("--no-baseline", action="store_true", help="skip the plain FP32 Lloyd comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU seconds the oracle sample is sized for (it tends to land at about 0.6 of this)")
    ap.add_argument("--stats", action="store_true", help="print per-iteration filter statistics")
    ap.add_argument("--plain", action="store_true",
                    help="plain launches instead of graph replays")
    ap.add_argument("--depth", type=int, default=0, choices=[0, 1, 3],
                    help="centroid chunks in flight per workgroup (0: library default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0,
                    help="workgroups per CU of the grid-stride launches (0: library default)")
    ap.add_argument("--bound-codes", type=int, default=0, choices=[0, 1, 2],
                    help="BF16 mode: 1 = FP32 group bounds, 2 = FP16 codes (0: library default)")
    ap.add_argument("--no-group-autotune", action="store_true",
                    help="skip the extra run at the group counts kp_autotune_groups picks")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip kp_autotune (untimed, before the contexts are made) and use the defaults")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device twice (reference for the HBM byte counters) and exit")
    return ap.parse_args()


def plain_fp32_lloyd_batched(torch, Xs, Cs, iters, warmup=1, rows=1 << 13, centroids_out=None):
    """Dense FP32 Lloyd with torch over many problems at once.  Each problem
    is cut into tiles of `rows` points (only its last tile is padded) and the
    tiles of one (D, K) class are stacked, each with its own problem's
    centroids gathered beside it, so a few batched GEMMs, one argmin and one
    scatter-add serve the whole class per iteration; padding rows take no
    part in the sums.  Returns seconds per iteration of all problems;
    centroids_out (a list), when given, receives every problem's centroids
    after the warmup and timed iterations."""
    torch.backends.cuda.matmul.allow_tf32 = False
    torch.set_float32_matmul_precision("highest")
    dev = Xs[0].device
    classes = {}
    for i, (X, C) in enumerate(zip(Xs, Cs)):
        classes.setdefault((X.shape[1], C.shape[0]), []).append(i)
    state = []
    for (d, k), idx in classes.items():
        tiles = [(j, s) for j, i in enumerate(idx) for s in range(0, Xs[i].shape[0], rows)]
        t = len(tiles)
        Xt = torch.zeros((t, rows, d), dtype=torch.float32, device=dev)
        valid = torch.zeros((t, rows), dtype=torch.bool, device=dev)
        for u, (j, s) in enumerate(tiles):
            part = Xs[idx[j]][s:s + rows]
            Xt[u, :part.shape[0]] = part
            valid[u, :part.shape[0]] = True
        owner = torch.tensor([j for j, _ in tiles], dtype=torch.int64, device=dev)
        C = torch.stack([Cs[i] for i in idx]).contiguous()
        step = max(1, (1 << 28) // (rows * k))               # tiles per GEMM: at most 2^28 distances
        state.append(dict(X=Xt, xn=(Xt * Xt).sum(2), valid=valid, owner=owner,
                          flat_base=(owner * k).unsqueeze(1), Xv=Xt[valid], C=C,
                          b=len(idx), t=t, d=d, k=k, step=step))

    def one():
        for st in state:
            X, C, b, t, d, k = st["X"], st["C"], st["b"], st["t"], st["d"], st["k"]
            cn = (C * C).sum(2)                                   # (b, k)
            Ct = C.transpose(1, 2).contiguous()                   # (b, d, k)
            lab = torch.empty((t, X.shape[1]), dtype=torch.int64, device=dev)
            for s in range(0, t, st["step"]):
                e = min(t, s + st["step"])
                own = st["owner"][s:e]
                D = torch.baddbmm(cn[own].unsqueeze(1), X[s:e], Ct[own], beta=1.0, alpha=-2.0)
                D.add_(st["xn"][s:e].unsqueeze(2))
                lab[s:e] = D.argmin(2)
            flat = (lab + st["flat_base"])[st["valid"]]
            sums = torch.zeros((b * k, d), dtype=torch.float32, device=dev).index_add_(0, flat, st["Xv"])
            cnt = torch.bincount(flat, minlength=b * k).to(torch.float32).view(b, k)
            st["C"] = torch.where(cnt.unsqueeze(2) > 0, sums.view(b, k, d) / cnt.clamp(min=1).unsqueeze(2), C)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        one()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / iters
    if centroids_out is not None:
        got = {}
        for (_, idx), st in zip(classes.items(), state):
            for j, i in enumerate(idx):
                got[i] = st["C"][j]
        centroids_out.extend(got[i] for i in range(len(Xs)))
    del state
    torch.cuda.empty_cache()
    return sec


def plain_fp32_kernels(torch, KMeans, kp_tuning, spec, iters, warmup=1):
    """Plain FP32 Lloyd with this library's hand-written kernels
    (kp_tuning.plain: the FP32 direct-form dense pass and a full centroid
    recompute in every iteration, no filtering) on the same problems; returns
    seconds per iteration, or None where the FP32 form does not apply
    (d > 128)."""
    if any(sp[0].shape[1] > 128 for sp in spec):
        return None
    fp = [(sp[0], sp[1], sp[2], "fp32") for sp in spec]
    km = KMeans(fp, tuning=kp_tuning(plain=1))
    try:
        km.iterate(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        km.iterate(iters)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / iters
    finally:
        km.close()


def plain_fp32_lloyd(torch, Xd, C0d, iters, warmup=1, chunk=1 << 19):
    """Dense FP32 Lloyd with torch on the same GPU; returns seconds per iteration."""
    torch.backends.cuda.matmul.allow_tf32 = False
    torch.set_float32_matmul_precision("highest")
    n, d = Xd.shape
    k = C0d.shape[0]
    xn = (Xd * Xd).sum(1)
    C = C0d.clone()
    lab = torch.empty(n, dtype=torch.int64, device=Xd.device)

    def one():
        nonlocal C
        cn = (C * C).sum(1)
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            D = torch.addmm(cn.unsqueeze(0), Xd[s:e], C.t(), beta=1.0, alpha=-2.0)
            D.add_(xn[s:e].unsqueeze(1))
            lab[s:e] = D.argmin(1)
        sums = torch.zeros((k, d), dtype=torch.float32, device=Xd.device).index_add_(0, lab, Xd)
        cnt = torch.bincount(lab, minlength=k).to(torch.float32)
        C = torch.where(cnt.unsqueeze(1) > 0, sums / cnt.clamp(min=1).unsqueeze(1), C)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        one()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / iters


def serving(torch, km, Xd, nq=1_000_000, reps=5):
    """kp_predict throughput with the context's trained centroids: nq queries
    = training rows plus N(0, 0.05^2) noise (seeded), so they follow the same
    mixture; plain torch FP32 GEMM + argmin on the same queries as the
    comparator.  Queries are resident in HBM; HIP events around the calls."""
    nq = min(nq, Xd.shape[0])
    g = torch.Generator(device=Xd.device).manual_seed(4242)
    Q = (Xd[:nq] + 0.05 * torch.randn(Xd[:nq].shape, generator=g, device=Xd.device)).contiguous()
    out = km.predict(Q)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        km.predict(Q, out=out)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    c32 = km.centroids(0)[0]
    torch.backends.cuda.matmul.allow_tf32 = False
    cn = (c32 * c32).sum(1)
    ct = c32.t().contiguous()
    chunk = 1 << 19

    def plain():
        return torch.cat([torch.argmin(cn[None, :] - 2.0 * (Q[i:i + chunk] @ ct), dim=1)
                          for i in range(0, nq, chunk)])
    ref = plain()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        plain()
    ev1.record()
    torch.cuda.synchronize()
    ms_plain = ev0.elapsed_time(ev1) / reps
    agree = float((ref.to(torch.int32) == out).float().mean().item())
    return dict(queries=nq, ms=ms, value=nq / (ms * 1e-3), unit="queries/s", plain_fp32_ms=ms_plain,
                speedup_vs_plain_fp32=ms_plain / ms, agreement_with_plain_fp32=agree,
                queries_recipe="training rows + N(0, 0.05^2) noise, seeded")


def cpu_model():
    """The host CPU's model name and the threads the oracle uses."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def check_run(KMeans, kp_tuning, spec, tun, T):
    """An untimed run of the same workload stopped after T-1 iterations to
    take the centroids the last assignment step uses, then the last
    iteration: returns (c32 before, c64 before, labels, c32, c64) as numpy
    arrays, and the run's context (kept for serving)."""
    t = kp_tuning(**{f: getattr(tun, f) for f, _ in kp_tuning._fields_})
    t.timing = 0
    t.timing_stages = 0
    km = KMeans(spec, tuning=t)
    if T > 1:
        km.iterate(T - 1)
    c32p, c64p = [a.cpu().numpy() for a in km.centroids()]
    km.iterate(1)
    lab = km.assign().cpu().numpy()
    c32, c64 = [a.cpu().numpy() for a in km.centroids()]
    return (c32p, c64p, lab, c32, c64), km


def cpu_baseline(P, target_s, ref):
    """The FP64 oracle on the host cores: iteration T of the workload (assign
    with the FP32 centroids the GPU's last assignment used, then the update)
    on a bounded sample, the first m points, m sized for about target_s.

    The same oracle outputs state the GPU result's precision: the share of
    the sample whose GPU label differs from the oracle's (a difference is
    allowed only at a near-tie, d(x, c_gpu) - d(x, c_best) <= 1e-5 d(x,
    c_best)), and the largest relative error of the GPU's FP64 centroids
    against the oracle's means of all N points under the GPU's assignment."""
    import oracle
    threads = oracle.threads()
    c32p, c64p, lab, c32, c64 = ref
    C = c32p.astype(np.float64)

    def one_iteration(m):
        t0 = time.perf_counter()
        a, _ = oracle.assign(P.X[:m], C)
        oracle.update(P.X[:m], a, C)
        return max(time.perf_counter() - t0, 1e-6)

    # size the sample from a probe of about a second (a tiny probe is dominated
    # by the thread pool's start and undersizes it)
    probe = min(P.n, 2000)
    dt = one_iteration(probe)
    probe = int(min(P.n, max(probe, probe * 1.0 / dt)))
    dt = one_iteration(probe)
    m = int(min(P.n, max(probe, probe * target_s / dt)))
    t0 = time.perf_counter()
    ref_lab, d1sq = oracle.assign(P.X[:m], C)
    oracle.update(P.X[:m], ref_lab, C)
    el = time.perf_counter() - t0
    cpu = dict(value=m / el, unit="point-iterations/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
               sample="FP64 Lloyd iteration %d (assign + update) over the first %d of %d points, all %d "
                      "centroids, %.1f s" % (P.iters, m, P.n, P.k, el))
    # precision of the GPU's iteration T against those oracle outputs
    mism = ref_lab != lab[:m]
    d2sq = oracle.dist2_to(P.X[:m], C, lab[:m])
    d1, d2 = np.sqrt(d1sq), np.sqrt(d2sq)
    near = (d2 - d1) <= 1e-5 * d1
    cref, _ = oracle.update(P.X, lab, c64p)
    scale = float(np.sqrt((P.X[:m].astype(np.float64) ** 2).sum(axis=1).mean()))
    err = np.linalg.norm(c64 - cref, axis=1) / np.maximum(np.linalg.norm(cref, axis=1), scale)
    prec = dict(iteration=P.iters, sample_points=m, assign_mismatch_rate=float(mism.mean()),
                assign_mismatches=int(mism.sum()), mismatches_outside_near_tie=int((mism & ~near).sum()),
                near_tie_band="d(x,c_gpu) - d(x,c_best) <= 1e-5 d(x,c_best)",
                centroid_rel_err_max=float(err.max()), centroids_checked=int(P.k),
                c32_is_rounded_c64=bool(np.array_equal(c32, c64.astype(np.float32))),
                reference="FP64 oracle: assignment of the sample with the GPU's previous FP32 centroids; "
                          "means of all N points under the GPU's assignment")
    return cpu, prec


def measure_single(args, torch, datagen, KMeans, kp_tuning, config, steps, warmup, *, extras=True):
    """One workload of a single problem: returns the result dict (value,
    roofline, precision, comparators)."""
    t0 = time.perf_counter()
    P = datagen.make_config(config, n=args.n if config == args.config else None)
    log("data: %s n=%d d=%d k=%d g=%d T=%d (%.1f s)" % (P.meta["name"], P.n, P.d, P.k, P.g, P.iters,
                                                           time.perf_counter() - t0))
    prec = "bf16" if P.precision == "bf16" else "fp32"
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(P.X).to(dev)
    C0d = torch.from_numpy(P.C0).to(dev)
    spec = [(Xd, C0d, P.g, prec, P.seed)]
    tun = tuned(args, KMeans, kp_tuning, spec)
    el, agg, timed, dom, st = run_steps(torch, KMeans, kp_tuning, spec, tun, P.iters, steps, warmup)
    value = P.n * P.iters * steps / el
    if args.stats:
        for s in st:
            log("iter %(iter)3d dense=%(dense)d fail=%(point_filter_fail)d pairs=%(pairs)d dist=%(distances)d "
                "rechecks=%(rechecks)d moved=%(moved)d maxdrift=%(max_drift).4g tilegroups=%(tile_groups)d "
                "closed=%(closed)d rowtest=%(row_test)d" % s)
    for nm, a in sorted(agg.items(), key=lambda kv: -kv[1]["ms"]):
        log("stage %-14s %8.3f ms/step over %5.1f launches" % (nm, a["ms"], a["launches"]))
    # the dominant kernel stage, timed inside the timed region
    roofline = roofline_of(dom, timed[dom], P, st)
    others = {}
    for nm in ("assign", "assign_dense", "group_filter", "bound_filter", "recheck"):
        if nm in agg and nm != dom:
            r = roofline_of(nm, agg[nm], P, st)
            others[nm] = {k: r[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac")}
    groups = None
    if not args.no_group_autotune:
        groups = autotuned_groups(args, torch, KMeans, kp_tuning, spec, tun, P.iters, min(steps, 2))
        if "ms_per_step" in groups:
            log("with autotuned groups: %.3f ms/step" % groups["ms_per_step"])
    ref, km = check_run(KMeans, kp_tuning, spec, tun, P.iters)
    serve = None
    if extras:
        serve = serving(torch, km, Xd)
        log("serving: %d queries in %.3f ms (%.3g queries/s), plain FP32 argmin %.3f ms" % (
            serve["queries"], serve["ms"], serve["value"], serve["plain_fp32_ms"]))
    km.close()
    del km
    torch.cuda.empty_cache()
    baseline = None
    if not args.no_baseline:
        # small problems are launch-bound: time more iterations after more warmup
        small = P.n * P.k < 1 << 26
        sec_t = plain_fp32_lloyd(torch, Xd, C0d, iters=30 if small else 3, warmup=5 if small else 1)
        sec_k = plain_fp32_kernels(torch, KMeans, kp_tuning, spec, iters=30 if small else 3,
                                   warmup=5 if small else 1)
        sec = min(sec_t, sec_k) if sec_k else sec_t
        baseline = dict(value=P.n / sec, unit="point-iterations/s", ms_per_iteration=sec * 1e3,
                        ms_per_iteration_torch=sec_t * 1e3,
                        ms_per_iteration_hand_written=sec_k * 1e3 if sec_k else None,
                        impl="the faster of torch FP32 GEMM (TF32 off) + argmin + index_add and this library's "
                             "FP32 direct-form kernels (kp_tuning.plain; d <= 128), every iteration dense, "
                             "full centroid recompute")
        log("plain FP32 Lloyd: %.3f ms/iteration (torch %.3f, hand-written %s)" % (
            sec * 1e3, sec_t * 1e3, "%.3f" % (sec_k * 1e3) if sec_k else "n/a (d > 128)"))
    del Xd, C0d
    torch.cuda.empty_cache()
    cpu, precision = (None, None) if args.no_cpu else cpu_baseline(P, args.cpu_seconds if extras else
                                                                   min(args.cpu_seconds, 8.0), ref)
    if precision:
        log("precision: %d of %d sampled labels differ from the oracle (%d outside the near-tie band); "
            "largest centroid error %.3g" % (precision["assign_mismatches"], precision["sample_points"],
                                             precision["mismatches_outside_near_tie"],
                                             precision["centroid_rel_err_max"]))
    return dict(
        value=value, ms_per_step=el / steps * 1e3, steps=steps, warmup=warmup, dtype="bf16" if prec == "bf16" else "f32",
        config={"workload": P.meta["name"], "n": P.n, "d": P.d, "k": P.k, "g": P.g, "iterations": P.iters,
                "precision": "bf16 MFMA + fp32 recheck + fp64 centroids" if prec == "bf16"
                else "fp32 direct + fp64 centroids", "tuning": dict(TUNING)},
        roofline=roofline, stage_rooflines=others, serving=serve, cpu_baseline=cpu, precision=precision,
        plain_fp32_lloyd=baseline, speedup_vs_plain_fp32_lloyd=(value / baseline["value"]) if baseline else None,
        autotuned_groups=groups,
        stage_ms_per_step={nm: round(a["ms"], 4) for nm, a in agg.items()},
        stage_ms_source="warmup runs with every stage timed" if warmup else "the timed runs",
        filter={"iter_%d" % s["iter"]: [s["point_filter_fail"], s["pairs"], s["rechecks"], s["moved"], s["closed"],
                                        s["row_test"]]
                for s in st if s["iter"] in (1, 2, 3, 5, 10, P.iters)},
        filter_fields=["point_filter_fail (L1)", "pairs", "rechecks", "moved", "closed (every group closed)",
                       "row_test"])


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 2 x %d bytes" % (src.numel() * 4))
        return
    import datagen
    from paper_1905_09345_amd import KMeans
    from paper_1905_09345_amd.kp import kp_tuning
    if args.config == 4:
        res = measure_batched(args, torch, datagen, KMeans, kp_tuning, args.steps, args.warmup)
    else:
        res = measure_single(args, torch, datagen, KMeans, kp_tuning, args.config, args.steps, args.warmup)
    out = {
        "metric": METRIC, "value": res["value"], "unit": "point-iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": res["dtype"],
        "data": "synthetic (seeded mixtures, see datagen)",
    }
    out.update({k: v for k, v in res.items() if k not in ("value", "ms_per_step", "steps", "warmup", "dtype")})
    # the other forms the workload set names, measured in the same process
    # with fewer steps: plain filtered FP32 (C2) and the batched form (C4)
    secondary = {}
    for c in [int(x) for x in args.secondary.split(",") if x.strip()]:
        if c == args.config:
            continue
        TUNING.clear()
        if c == 4:
            r = measure_batched(args, torch, datagen, KMeans, kp_tuning, args.secondary_steps, 1, extras=False)
        else:
            r = measure_single(args, torch, datagen, KMeans, kp_tuning, c, args.secondary_steps, 1, extras=False)
        secondary["C%d" % c] = {k: r[k] for k in ("value", "ms_per_step", "steps", "dtype", "config", "roofline",
                                                  "stage_rooflines", "precision", "plain_fp32_lloyd",
                                                  "speedup_vs_plain_fp32_lloyd", "autotuned_groups",
                                                  "cpu_baseline") if k in r}
        secondary["C%d" % c]["unit"] = "point-iterations/s"
        torch.cuda.empty_cache()
    if secondary:
        out["other_forms"] = secondary
    print(json.dumps(out), flush=True)


def bound_layout(P):
    """Bytes per stored group bound and the bounds a row holds that the
    algorithm needs (g; the padding of the stored rows is not counted): BF16
    problems keep FP32 bounds or FP16 codes (kp_tuning.bound_codes = 2), FP32
    problems FP32 bounds."""
    if P.precision == "bf16":
        return (2 if TUNING.get("bound_codes") == 2 else 4), P.g
    return 4, P.g


def assign_bytes(P, s):
    """Algorithmic HBM bytes of one filtered assignment launch (BF16 mode): per
    entry of L1 its FP32 row, the sorted entry, its norm, its open-group mask
    words and closed-group bound (from the group filter), the new state and the
    update entries; per visited (point, group) pair the new bound; per
    uncertain point its recheck record and list entry."""
    bsz, _ = bound_layout(P)
    per_point = 4 * P.d + 16 + 4 + 4 * ((P.g + 31) // 32) + 4 + 16 + 12
    return s["point_filter_fail"] * per_point + s["pairs"] * bsz + s["rechecks"] * 20


def gfilter_bytes(P, s):
    """Algorithmic HBM bytes of one group-filter launch: per entry of L1 the
    sorted entry, the point's g bounds (FP32 or FP16 codes), and the written
    mask words and closed-group bound."""
    bsz, gs = bound_layout(P)
    return s["point_filter_fail"] * (16 + bsz * gs + 4 * ((P.g + 31) // 32) + 4)


def traffic_of(kernel, workload):
    """Measured HBM bytes per launch from the committed counter summary, if it
    was taken on the kernel source as it is now; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    import hashlib
    src = os.path.join(ROOT, "paper_1905_09345_amd", "csrc", "kp_kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for key, ent in rec.items():   # entries "<kernel>@<tuning>", one per profiled launch tuning
        if key.split("@")[0] != kernel:
            continue
        if ent.get("source_sha256") != digest or ent.get("workload") != workload:
            continue
        if any(TUNING.get(k) != v for k, v in ent.get("tuning", {}).items()):
            continue   # counters taken under another launch tuning
        return ent.get("bytes_per_launch")
    return None


def tuned(args, KMeans, kp_tuning, spec):
    """Launch tuning of the measured runs: kp_autotune's pick unless disabled
    or fixed on the command line; timing on (stage events)."""
    tun = kp_tuning(chunk_depth=args.depth, blocks_per_cu=args.blocks_per_cu, bound_codes=args.bound_codes)
    if not args.no_autotune and not args.depth and not args.blocks_per_cu and not args.bound_codes:
        t0 = time.perf_counter()
        tun = KMeans.autotune(spec, iters=3)
        log("autotune: chunk_depth=%d blocks_per_cu=%d bound_codes=%d (%.1f s)" % (
            tun.chunk_depth, tun.blocks_per_cu, tun.bound_codes, time.perf_counter() - t0))
    tun.timing = 1
    tun.use_graph = -1 if args.plain else 1
    TUNING.update(chunk_depth=tun.chunk_depth, blocks_per_cu=tun.blocks_per_cu, use_graph=tun.use_graph,
                  bound_codes=tun.bound_codes)
    return tun


def run_steps(torch, KMeans, kp_tuning, spec, tun, T, steps, warmup):
    """W warmup runs with events around every stage (the per-stage breakdown,
    untimed), then K timed runs with events around the dominant stage only:
    its launches are what the roofline divides by, and no other stage pays
    for instrumentation inside the timed region.  Every run is a fresh
    context iterated T times; only one context exists at a time, made and
    destroyed outside the timed region, and each run is bracketed by a
    device synchronisation on both sides.  Returns the summed seconds of the
    K runs, the breakdown, the timed runs' stage times, the dominant stage
    and the per-iteration statistics of the last run."""
    from paper_1905_09345_amd.kp import STAGES

    def with_stages(mask):
        t = kp_tuning(**{f: getattr(tun, f) for f, _ in kp_tuning._fields_})
        t.timing_stages = mask
        return t

    def aggregate(stages):
        return {nm: dict(ms=sum(x[nm]["ms"] for x in stages) / len(stages),
                         launches=sum(x[nm]["launches"] for x in stages) / len(stages)) for nm in stages[0]}

    breakdown = None
    mask = 0
    if warmup > 0:
        times = []
        for _ in range(warmup):
            km = KMeans(spec, tuning=with_stages(0))
            km.iterate(T)
            times.append(km.stage_times())
            km.close()
        breakdown = aggregate(times)
        dom = max((nm for nm in breakdown if nm != "filtered_iter"), key=lambda nm: breakdown[nm]["ms"])
        mask = 1 << STAGES.index(dom)
        log("warmup done (stage breakdown; timed runs time %s only)" % dom)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall = gpu_s = 0.0
    times = []
    st = None
    for i in range(steps):
        km = KMeans(spec, tuning=with_stages(mask))
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev0.record()
        km.iterate(T)
        ev1.record()
        torch.cuda.synchronize()
        wall += time.perf_counter() - w0
        gpu_s += ev0.elapsed_time(ev1) / 1e3
        times.append(km.stage_times())
        if i == steps - 1:
            st = km.stats()
        km.close()
    timed = aggregate(times)
    if breakdown is None:
        breakdown = timed
    dom = max((nm for nm in breakdown if nm != "filtered_iter"), key=lambda nm: breakdown[nm]["ms"])
    log("timed: %d steps, %.3f ms/step (events %.3f ms/step)" % (steps, max(wall, gpu_s) / steps * 1e3,
                                                                   gpu_s / steps * 1e3))
    return max(wall, gpu_s), breakdown, timed, dom, st


TUNING = {}


def autotuned_groups(args, torch, KMeans, kp_tuning, spec, tun, T, steps):
    """The same workload with the group counts kp_autotune_groups picks (per
    (D, K) class; the configured g is one of the candidates).  The method's
    result does not depend on g, so this is the configured run's work at the
    group counts the library would choose.  Returns the picked g per class,
    the time per step of `steps` timed runs and the autotuner's own time."""
    t0 = time.perf_counter()
    gs = KMeans.autotune_groups(spec, iters=3, tuning=tun)
    tune_s = time.perf_counter() - t0
    picks = {}
    for sp, g in zip(spec, gs):
        picks.setdefault("d%d_k%d" % (sp[0].shape[1], sp[1].shape[0]), g)
    log("group autotune (%.1f s): %s" % (tune_s, picks))
    res = dict(g=picks, autotune_seconds=tune_s, candidates="per (D, K) class: the configured g, ceil(K/16), ceil(K/10)")
    if all(int(sp[2]) == g for sp, g in zip(spec, gs)):
        res["same_as_configured"] = True   # nothing to measure apart
        return res
    spec2 = [(sp[0], sp[1], g) + tuple(sp[3:]) for sp, g in zip(spec, gs)]
    el, _, _, _, _ = run_steps(torch, KMeans, kp_tuning, spec2, tun, T, steps, 1)
    ntot = sum(sp[0].shape[0] for sp in spec)
    res.update(value=ntot * T * steps / el, ms_per_step=el / steps * 1e3, steps=steps)
    return res


def measure_batched(args, torch, datagen, KMeans, kp_tuning, steps, warmup, extras=True):
    """The batched workload: many independent problems in one context, every
    stage launched once for all of them, one graph replay per iteration."""
    t0 = time.perf_counter()
    probs = datagen.make_batched(args.problems)
    T = probs[0].iters
    ntot = sum(p.n for p in probs)
    log("data: %d problems, sum N=%d, T=%d (%.1f s)" % (len(probs), ntot, T, time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    Xd = [torch.from_numpy(p.X).to(dev) for p in probs]
    Cd = [torch.from_numpy(p.C0).to(dev) for p in probs]
    spec = [(Xd[i], Cd[i], p.g, p.precision, p.seed) for i, p in enumerate(probs)]
    tun = tuned(args, KMeans, kp_tuning, spec)
    el, agg, timed, dom, _ = run_steps(torch, KMeans, kp_tuning, spec, tun, T, steps, warmup)
    value = ntot * T * steps / el
    for nm, a in sorted(agg.items(), key=lambda kv: -kv[1]["ms"]):
        log("stage %-14s %8.3f ms/step over %5.1f launches" % (nm, a["ms"], a["launches"]))
    groups = None
    if not args.no_group_autotune:
        groups = autotuned_groups(args, torch, KMeans, kp_tuning, spec, tun, T, min(steps, 2))
        if "ms_per_step" in groups:
            log("with autotuned groups: %.3f ms/step" % groups["ms_per_step"])
    # statistics and the oracle check come from one more (untimed) run
    t = kp_tuning(**{f: getattr(tun, f) for f, _ in kp_tuning._fields_})
    t.timing = 0
    t.timing_stages = 0
    km = KMeans(spec, tuning=t)
    km.iterate(T - 1)
    ncheck = len(probs) if args.no_cpu else min(len(probs), 64)
    prev = [[a.cpu().numpy() for a in km.centroids(i)] for i in range(ncheck)]
    km.iterate(1)
    refs = [(prev[i][0], prev[i][1], km.assign(i).cpu().numpy()) + tuple(a.cpu().numpy() for a in km.centroids(i))
            for i in range(ncheck)]
    stats = [km.stats(i) for i in range(len(probs))]
    km.close()
    del km
    roofline = None
    if dom == "assign":
        byts = 0.0
        for i, p in enumerate(probs):
            filt = [s for s in stats[i] if not s["dense"]]
            byts += sum(assign_bytes(p, s) for s in filt) / max(len(filt), 1)
        ms = timed[dom]["ms"] / max(timed[dom]["launches"], 1e-9)   # timed inside the timed region
        ach = byts / (ms * 1e-3) / 1e9
        roofline = dict(kernel="kb_blk64 (filtered iteration, all problems)", bound="hbm", achieved=ach,
                        peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                        traffic=traffic_of("kb_blk64_filtered", datagen.CONFIGS[4]["name"]),
                        work_per_launch="%.4g B" % byts, ms_per_launch=ms)
    else:
        roofline = dict(kernel=dom, bound="unknown", achieved=None, peak=None, unit=None, frac=None, traffic=None,
                        ms_per_launch=timed[dom]["ms"] / max(timed[dom]["launches"], 1e-9))
    others = {}
    if "group_filter" in agg and dom != "group_filter" and agg["group_filter"]["launches"] > 0:
        byts = 0.0
        for i, p in enumerate(probs):
            filt = [s for s in stats[i] if not s["dense"]]
            if p.precision == "bf16":
                byts += sum(gfilter_bytes(p, s) for s in filt) / max(len(filt), 1)
        ms = agg["group_filter"]["ms"] / agg["group_filter"]["launches"]
        ach = byts / (ms * 1e-3) / 1e9
        others["group_filter"] = dict(kernel="kb_gfilter (all problems)", bound="hbm", achieved=ach,
                                      peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS)
    torch.cuda.empty_cache()
    baseline = None
    if not args.no_baseline:
        # the stronger of two torch forms: one problem after another, and the
        # problems of each (D, K) class padded and batched
        sec_seq = sum(plain_fp32_lloyd(torch, Xd[i], Cd[i], iters=2, warmup=1) for i in range(len(probs)))
        sec_bat = plain_fp32_lloyd_batched(torch, Xd, Cd, iters=3, warmup=1)
        sec_k = plain_fp32_kernels(torch, KMeans, kp_tuning, spec, iters=3, warmup=1)
        sec = min(x for x in (sec_seq, sec_bat, sec_k) if x)
        baseline = dict(value=ntot / sec, unit="point-iterations/s", ms_per_iteration=sec * 1e3,
                        ms_per_iteration_per_problem=sec_seq * 1e3, ms_per_iteration_batched=sec_bat * 1e3,
                        ms_per_iteration_hand_written=sec_k * 1e3 if sec_k else None,
                        impl="the fastest of torch FP32 GEMM (TF32 off) + argmin + index_add per problem, the same "
                             "batched per (D, K) class over 8192-point tiles, and this library's FP32 direct-form "
                             "kernels on the whole batch (kp_tuning.plain); every iteration dense, full centroid "
                             "recompute")
        log("plain FP32 Lloyd: %.3f ms per iteration of all problems (%.3f one problem at a time, %.3f batched by class, "
            "%s hand-written)" % (sec * 1e3, sec_seq * 1e3, sec_bat * 1e3, "%.3f" % (sec_k * 1e3) if sec_k else "n/a"))
    del Xd, Cd, spec
    torch.cuda.empty_cache()
    cpu = precision = None
    if not args.no_cpu:
        cpu, precision = cpu_baseline_batched(probs, args.cpu_seconds if extras else min(args.cpu_seconds, 8.0),
                                              refs)
        log("precision: %d of %d labels of %d problems differ from the oracle (%d outside the near-tie band); "
            "largest centroid error %.3g" % (precision["assign_mismatches"], precision["sample_points"],
                                             precision["problems_checked"],
                                             precision["mismatches_outside_near_tie"],
                                             precision["centroid_rel_err_max"]))
    return dict(
        value=value, ms_per_step=el / steps * 1e3, steps=steps, warmup=warmup, dtype="bf16",
        config={"workload": "C4 batched, %d problems, N~U{2000..200000}, D in {16,32,64}, K in {16,64,256}, "
                            "G=ceil(K/10)" % len(probs), "problems": len(probs), "sum_n": ntot,
                "iterations": T, "precision": "bf16 MFMA + fp32 recheck + fp64 centroids", "tuning": dict(TUNING)},
        roofline=roofline, stage_rooflines=others, cpu_baseline=cpu, precision=precision,
        plain_fp32_lloyd=baseline, speedup_vs_plain_fp32_lloyd=(value / baseline["value"]) if baseline else None,
        autotuned_groups=groups,
        stage_ms_per_step={nm: round(a["ms"], 4) for nm, a in agg.items()})


def cpu_baseline_batched(probs, target_s, refs):
    """The FP64 oracle on the host cores over the first problems of the batch
    (whole problems, until about target_s has passed): iteration T of each,
    from the FP32 centroids the GPU's last assignment used.  The same oracle
    outputs give the precision of the GPU's result on those problems (as in
    cpu_baseline)."""
    import oracle
    m, npts, mism, outside, worst = 0, 0, 0, 0, 0.0
    el_c = 0.0
    while m < len(refs) and el_c < target_s:
        p = probs[m]
        c32p, c64p, lab, c32, c64 = refs[m]
        C = c32p.astype(np.float64)
        t1 = time.perf_counter()
        ref_lab, d1sq = oracle.assign(p.X, C)
        oracle.update(p.X, ref_lab, C)
        el_c += time.perf_counter() - t1
        bad = ref_lab != lab
        d1, d2 = np.sqrt(d1sq), np.sqrt(oracle.dist2_to(p.X, C, lab))
        mism += int(bad.sum())
        outside += int((bad & ((d2 - d1) > 1e-5 * d1)).sum())
        cref, _ = oracle.update(p.X, lab, c64p)
        scale = float(np.sqrt((p.X.astype(np.float64) ** 2).sum(axis=1).mean()))
        err = np.linalg.norm(c64 - cref, axis=1) / np.maximum(np.linalg.norm(cref, axis=1), scale)
        worst = max(worst, float(err.max()))
        npts += p.n
        m += 1
    cpu = dict(value=npts / el_c, unit="point-iterations/s", cores=oracle.threads(), cpu_model=cpu_model(),
               kind="oracle", sample="FP64 Lloyd iteration %d of each of the first %d of %d problems (%d points), "
                                     "%.1f s" % (probs[0].iters, m, len(probs), npts, el_c))
    prec = dict(iteration=probs[0].iters, problems_checked=m, sample_points=npts,
                assign_mismatch_rate=mism / max(npts, 1), assign_mismatches=mism,
                mismatches_outside_near_tie=outside,
                near_tie_band="d(x,c_gpu) - d(x,c_best) <= 1e-5 d(x,c_best)", centroid_rel_err_max=worst,
                reference="FP64 oracle per problem: assignment with the GPU's previous FP32 centroids; means "
                          "under the GPU's assignment")
    return cpu, prec


def roofline_of(stage, a, P, st):
    """Achieved rate of the dominant stage from its algorithmic work per launch."""
    ms_per_launch = a["ms"] / max(a["launches"], 1e-9)
    wl = P.meta["name"]
    if stage == "assign" and P.precision == "bf16":
        filt = [s for s in st if not s["dense"]]
        byts = sum(assign_bytes(P, s) for s in filt) / max(len(filt), 1)
        ach = byts / (ms_per_launch * 1e-3) / 1e9
        # the method's flops on the same launches: 2d per distance computed
        flops = sum(2.0 * P.d * s["distances"] for s in filt) / max(len(filt), 1)
        tf = flops / (ms_per_launch * 1e-3) / 1e12
        return dict(kernel="k_blk64 (filtered iteration: BF16x3 distances of the open groups)", bound="hbm",
                    achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                    traffic=traffic_of("k_blk64_filtered", wl),
                    work_per_launch="%.4g B (per L1 entry 4d+52+4*ceil(g/32) B, per pair %d B, per recheck 20 B)"
                    % (byts, bound_layout(P)[0]), ms_per_launch=ms_per_launch,
                    mfma_side=dict(achieved=tf, peak=MFMA_BF16_PEAK_TFLOPS, unit="TFLOP/s",
                                   frac=tf / MFMA_BF16_PEAK_TFLOPS,
                                   work_per_launch="2*d*distances = %.4g flop" % flops))
    if stage == "group_filter":
        filt = [s for s in st if not s["dense"]]
        byts = sum(gfilter_bytes(P, s) for s in filt) / max(len(filt), 1)
        ach = byts / (ms_per_launch * 1e-3) / 1e9
        return dict(kernel="k_gfilter", bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=traffic_of("k_gfilter", wl),
                    work_per_launch="%%.4g B (per L1 entry 16+%d*g+4*ceil(g/32)+4 B)" % bound_layout(P)[0] % byts,
                    ms_per_launch=ms_per_launch)
    if stage == "assign":
        # FP32 form: the group test and the direct-form tile kernel.  Work:
        # 3d FP32 operations (subtract, multiply, add) per distance computed,
        # against the vector FMA peak without packed instructions; the HBM
        # bytes (point row, bound row, state and entries per L1 entry, a bound
        # per open pair) are given beside it.
        filt = [s for s in st if not s["dense"]]
        ops = sum(3.0 * P.d * s["distances"] for s in filt) / max(len(filt), 1)
        byts = sum(s["point_filter_fail"] * (4 * P.d + 4 * P.g + 16 + 4 + 16 + 12) + s["pairs"] * 8
                   for s in filt) / max(len(filt), 1)
        ach = ops / (ms_per_launch * 1e-3) / 1e12
        peak = 78.6
        return dict(kernel="k_group_test + k_tile_f32 (filtered iteration, FP32 direct form)", bound="alu",
                    achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    traffic=traffic_of("fp32_filtered", wl),
                    work_per_launch="3*d per distance computed = %.4g FP32 operations" % ops,
                    ms_per_launch=ms_per_launch,
                    hbm=dict(achieved=byts / (ms_per_launch * 1e-3) / 1e9, unit="GB/s",
                             frac=byts / (ms_per_launch * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             work_per_launch="%.4g B (per L1 entry 4d+4g+48 B, per open pair 8 B)" % byts))
    if stage == "assign_dense":
        flops = 2.0 * P.n * P.k * P.d
        ach = flops / (ms_per_launch * 1e-3) / 1e12
        if P.precision == "bf16":
            # the method's 2NKD flops against the BF16 matrix-core peak (the
            # BF16x3 split issues three products per distance: the issue rate
            # is given beside it)
            return dict(kernel="k_blk64 (dense iteration 1, BF16x3)", bound="mfma", achieved=ach,
                        peak=MFMA_BF16_PEAK_TFLOPS, unit="TFLOP/s", frac=ach / MFMA_BF16_PEAK_TFLOPS,
                        traffic=traffic_of("k_blk64_dense", wl),
                        work_per_launch="2*N*K*D = %.4g flop" % flops, ms_per_launch=ms_per_launch,
                        mfma_issue_rate=dict(achieved=3 * ach, unit="TFLOP/s",
                                             work_per_launch="3*2*N*K*D = %.4g flop" % (3 * flops)))
        peak = 78.6   # FP32 vector FMA without packed instructions (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
        return dict(kernel="k_dense_f32 (dense, iteration 1)", bound="alu", achieved=ach, peak=peak,
                    unit="TFLOP/s", frac=ach / peak, traffic=None,
                    work_per_launch="2*N*K*D = %.4g flop" % flops, ms_per_launch=ms_per_launch)
    if stage == "bound_filter":
        # every point's state read, an L1 entry written per point that fails;
        # in iterations with the row test, the bound row of every point that
        # fails ub < lbp (those in L1 and those the row test dropped)
        filt = [s for s in st if not s["dense"]]
        fails = sum(s["point_filter_fail"] for s in filt) / max(len(filt), 1)
        bsz, gs = bound_layout(P)
        rows = sum((s["point_filter_fail"] + s["closed"]) for s in filt if s.get("row_test")) / max(len(filt), 1)
        byts = 16.0 * P.n + 16.0 * fails + bsz * gs * rows
        ach = byts / (ms_per_launch * 1e-3) / 1e9
        return dict(kernel="k_bound_filter", bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=None,
                    work_per_launch="16 B/point x N + 16 B per L1 entry + one bound row per point tested by rows "
                                    "= %.4g B" % byts,
                    ms_per_launch=ms_per_launch)
    return dict(kernel=stage, bound="unknown", achieved=None, peak=None, unit=None, frac=None, traffic=None,
                ms_per_launch=ms_per_launch)


if __name__ == "__main__":
    main()
