"""Seeded synthetic inputs for the filtered K-means path.

This module only draws numbers: Gaussian / Student-t mixtures, uniform noise
and the k-means++ seeding of the initial centroids.  It holds none of the
K-means iteration itself, so both the FP64 oracle and the GPU library take
their inputs from here without sharing any of the method's arithmetic.

The paper evaluates on six UCI datasets that it does not name (Section 2,
"Experiment and Conclusion"); they are not available here.  The mixtures
below stand in for them, with the sizes, dimensionalities and cluster counts
of the five workloads the build is measured on:

  C1  N=10,000     D=8    K=16    G=2    16 isotropic blobs, sigma=0.5,
                                         equal weights, init = first K points
  C2  N=1,000,000  D=32   K=256   G=26   256 blobs, sigma~U[0.3,1.5],
                                         Dirichlet(1) weights, k-means++ init
  C3  N=4,000,000  D=128  K=1024  G=100  1024 blobs as C2 plus 5% uniform
                                         background noise, k-means++ init
  C4  512 problems, N~U{2000..200000}, D in {16,32,64}, K in {16,64,256},
      G=ceil(K/10), per-problem mixtures as C2
  C5  N=16,000,000 D=256  K=4096  G=410  Student-t (nu=3) mixture with
                                         Zipf(1.1) component sizes

Blob centers are uniform in [-10, 10]^D.  Every generator is
numpy.random.Generator(PCG64(seed)); config c uses seed 1000 + c and batched
problem p uses seed 100000 + p, unless the caller passes a seed.  The point
rows are drawn in chunks on a thread pool, each chunk from a child generator
of that seed, so the data do not depend on the number of threads.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "gaussian_mixture", "student_t_mixture", "kmeanspp",
    "make_config", "make_batched", "CONFIGS",
]

CONFIGS = {
    1: dict(name="C1 plain filtered FP32, N=10000 D=8 K=16 G=2", n=10_000, d=8, k=16, g=2, iters=20,
            precision="fp32"),
    2: dict(name="C2 plain filtered FP32, N=1e6 D=32 K=256 G=26", n=1_000_000, d=32, k=256, g=26, iters=30,
            precision="fp32"),
    3: dict(name="C3 precision form BF16+recheck, N=4e6 D=128 K=1024 G=100", n=4_000_000, d=128, k=1024,
            g=100, iters=30, precision="bf16"),
    4: dict(name="C4 batched, 512 problems, BF16+recheck", n=None, d=None, k=None, g=None, iters=25,
            precision="bf16"),
    5: dict(name="C5 large skewed, N=1.6e7 D=256 K=4096 G=410", n=16_000_000, d=256, k=4096, g=410,
            iters=20, precision="bf16"),
}


@dataclass
class Problem:
    """One K-means problem: FP32 points, FP32 initial centroids and its sizes."""
    X: np.ndarray                 # (n, d) float32, row-major
    C0: np.ndarray                # (k, d) float32
    g: int                        # number of centroid groups
    iters: int                    # iterations to run
    precision: str = "fp32"       # "fp32" or "bf16"
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    @property
    def k(self):
        return self.C0.shape[0]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _fill_chunks(rng, n, chunk, body):
    """Run body(child_rng, s, e) over the chunks [s, e) of range(n) on a thread
    pool.  Chunk i draws from its own generator, seeded by child i of one
    SeedSequence that `rng` draws, so the numbers do not depend on the
    thread count or on the order in which chunks finish."""
    starts = list(range(0, n, chunk))
    seqs = np.random.SeedSequence(int(rng.integers(0, 2 ** 63))).spawn(len(starts))

    def run(i):
        s = starts[i]
        body(np.random.Generator(np.random.PCG64(seqs[i])), s, min(n, s + chunk))

    if len(starts) <= 1:
        for i in range(len(starts)):
            run(i)
        return
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(run, range(len(starts))))


def gaussian_mixture(rng, n, d, k, *, sigma=None, sigma_range=(0.3, 1.5), dirichlet=True,
                     noise_frac=0.0, box=10.0, chunk=1 << 18):
    """Isotropic Gaussian mixture with centers uniform in [-box, box]^d.

    sigma: a fixed standard deviation for every component, else each
    component draws its own from U[sigma_range].  dirichlet: component
    weights ~ Dirichlet(1) (else equal weights).  noise_frac: that fraction
    of the n points is replaced by uniform samples in the same box.
    Component labels are i.i.d. categorical.  Returns float32 (n, d).
    """
    centers = rng.uniform(-box, box, size=(k, d))
    sig = np.full(k, float(sigma)) if sigma is not None else rng.uniform(*sigma_range, size=k)
    w = rng.dirichlet(np.ones(k)) if dirichlet else np.full(k, 1.0 / k)
    n_noise = int(round(noise_frac * n))
    n_mix = n - n_noise
    X = np.empty((n, d), dtype=np.float32)
    lab = rng.choice(k, size=n_mix, p=w)

    def body(r, s, e):
        z = r.standard_normal(size=(e - s, d))
        X[s:e] = centers[lab[s:e]] + z * sig[lab[s:e], None]

    _fill_chunks(rng, n_mix, chunk, body)
    if n_noise:
        X[n_mix:] = rng.uniform(-box, box, size=(n_noise, d))
        perm = rng.permutation(n)
        X = X[perm]
    return X


def student_t_mixture(rng, n, d, k, *, nu=3.0, zipf_s=1.1, sigma_range=(0.3, 1.5), box=10.0,
                      chunk=1 << 16, out=None):
    """Multivariate Student-t mixture with Zipf-sized components.

    Component r (1-based) gets a share proportional to r^-zipf_s of the n
    points (largest-remainder rounding), then the points are shuffled.  A
    point of component k is mu_k + s_k * z / sqrt(w / nu) with z ~ N(0, I_d)
    and one w ~ chi-square(nu) shared by all of its coordinates.
    """
    centers = rng.uniform(-box, box, size=(k, d))
    sig = rng.uniform(*sigma_range, size=k)
    share = np.arange(1, k + 1, dtype=np.float64) ** (-zipf_s)
    share /= share.sum()
    raw = share * n
    cnt = np.floor(raw).astype(np.int64)
    rem = n - int(cnt.sum())
    cnt[np.argsort(-(raw - cnt), kind="stable")[:rem]] += 1
    lab = np.repeat(np.arange(k), cnt)
    rng.shuffle(lab)
    X = out if out is not None else np.empty((n, d), dtype=np.float32)

    def body(r, s, e):
        z = r.standard_normal(size=(e - s, d))
        w = r.chisquare(nu, size=(e - s, 1))
        X[s:e] = centers[lab[s:e]] + sig[lab[s:e], None] * z / np.sqrt(w / nu)

    _fill_chunks(rng, n, chunk, body)
    return X


def kmeanspp(rng, X, k, *, sample=None):
    """k-means++ seeding (Arthur & Vassilvitskii 2007), non-greedy, FP64.

    Runs on a seeded uniform subsample of `sample` rows when given (the
    whole X otherwise).  The first center is a uniform draw; each next
    center is drawn with probability proportional to the squared distance
    to the nearest center chosen so far.  Returns float32 (k, d).
    """
    n = X.shape[0]
    if sample is not None and sample < n:
        idx = np.sort(rng.choice(n, size=sample, replace=False))
        S = X[idx].astype(np.float64)
    else:
        S = X.astype(np.float64)
    m = S.shape[0]
    if k > m:
        raise ValueError("k-means++ needs at least k sample points")
    C = np.empty((k, S.shape[1]), dtype=np.float64)
    sn = (S * S).sum(axis=1)

    def d2(c):   # squared distances of the sample to one center (clamped at 0)
        return np.maximum(sn - 2.0 * (S @ c) + c @ c, 0.0)

    C[0] = S[rng.integers(m)]
    best = d2(C[0])
    for j in range(1, k):
        tot = best.sum()
        if tot <= 0.0:
            C[j] = S[rng.integers(m)]
        else:
            u = rng.random() * tot
            c = int(np.searchsorted(np.cumsum(best), u, side="right"))
            C[j] = S[min(c, m - 1)]
        np.minimum(best, d2(C[j]), out=best)
    return C.astype(np.float32)


def make_config(c, *, seed=None, n=None):
    """Inputs of workload C1..C3 or C5 (see module docstring).

    n: an optional smaller point count with the same recipe (parity tests and
    bounded CPU samples use it); the seed stays that of the config.
    """
    if c not in (1, 2, 3, 5):
        raise ValueError("make_config covers C1, C2, C3 and C5; use make_batched for C4")
    spec = CONFIGS[c]
    seed = 1000 + c if seed is None else seed
    rng = _rng(seed)
    n = spec["n"] if n is None else int(n)
    d, k, g = spec["d"], spec["k"], spec["g"]
    if c == 1:
        X = gaussian_mixture(rng, n, d, k, sigma=0.5, dirichlet=False)
        C0 = X[:k].copy()
    elif c == 2:
        X = gaussian_mixture(rng, n, d, k)
        C0 = kmeanspp(rng, X, k, sample=min(n, 64 * k))
    elif c == 3:
        X = gaussian_mixture(rng, n, d, k, noise_frac=0.05)
        C0 = kmeanspp(rng, X, k, sample=min(n, 8 * k))
    else:
        X = student_t_mixture(rng, n, d, k)
        C0 = kmeanspp(rng, X, k, sample=min(n, 4 * k))
    return Problem(X=X, C0=C0, g=g, iters=spec["iters"], precision=spec["precision"], seed=seed,
                   meta=dict(config=c, name=spec["name"]))


def make_batched(count=512, *, first_seed=100000, n_range=(2000, 200000), scale=1.0,
                 precision="bf16", iters=25):
    """The C4 batch: `count` independent problems of uneven N, D and K.

    Problem p uses seed first_seed + p: N ~ U{n_range} (times `scale`, at
    least 2K points), D uniform over {16, 32, 64}, K uniform over
    {16, 64, 256}, G = ceil(K / 10), a Gaussian mixture as in C2 and a
    k-means++ init on a subsample of 8K points.
    """
    out = []
    for p in range(count):
        seed = first_seed + p
        rng = _rng(seed)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int(rng.choice([16, 32, 64]))
        k = int(rng.choice([16, 64, 256]))
        n = max(2 * k, int(round(n * scale)))
        X = gaussian_mixture(rng, n, d, k)
        C0 = kmeanspp(rng, X, k, sample=min(n, 8 * k))
        out.append(Problem(X=X, C0=C0, g=int(math.ceil(k / 10)), iters=iters, precision=precision,
                           seed=seed, meta=dict(config=4, problem=p)))
    return out
