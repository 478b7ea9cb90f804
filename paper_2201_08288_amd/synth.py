"""Seeded synthetic inputs for the k-d tree build.

This module holds only random-input recipes (no step of the tree build).  The
same arrays feed the CPU oracle and the GPU library.  Every array is SoA
float32 of shape (d, n): coordinate c of point i is ``x[c, i]``.

Workload recipes (the paper evaluates on simulated data only, §5):
  uniform24      x = k * 2^-24, k uniform on [0, 2^24)            (24-bit uniform [0,1))
  gmm            equal-weight isotropic Gaussian mixture: means uniform in
                 [-5, 5]^d (fp64), sigma 0.5, rounded to fp32
  student_t_grid Student-t(nu) coordinates rounded to a 2^-10 grid (heavy ties),
                 clamped to |x| < 2^13
  corr_normal    p-variate normal, mean 0, common correlation rho (the §5 study)
  dirichlet_pool rows of cumulative Dirichlet(alpha) weights as uint32 fractions
                 of 2^32 (entry 0 is 0), one row per pool entry
"""
import numpy as np

BASE_SEED = 220108288


def rng_for(seed, *stream):
    return np.random.default_rng([int(seed) & 0xFFFFFFFF, *[int(s) for s in stream]])


def uniform24(n, d, seed=BASE_SEED, stream=0):
    rng = rng_for(seed, 1, stream)
    k = rng.integers(0, 1 << 24, size=(d, n), dtype=np.uint32)
    return (k.astype(np.float32) * np.float32(2.0 ** -24)).astype(np.float32)


def _columns(d, fn, workers=16):
    """Run fn(c) for every column c in parallel threads (numpy's generators
    release the GIL); each column has its own seeded stream."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(workers, d)) as ex:
        list(ex.map(fn, range(d)))


def gmm(n, d, seed=BASE_SEED, stream=0, components=10, box=5.0, sigma=0.5):
    rng = rng_for(seed, 2, stream)
    means = rng.uniform(-box, box, size=(components, d))
    comp = rng.integers(0, components, size=n)
    out = np.empty((d, n), dtype=np.float32)

    def col(c):
        z = rng_for(seed, 2, stream, 1 + c).standard_normal(n, dtype=np.float32).astype(np.float64)
        out[c] = (means[comp, c] + sigma * z).astype(np.float32)

    _columns(d, col)
    return out


def student_t_grid(n, d, seed=BASE_SEED, stream=0, nu=3.0, grid_bits=10, clamp_log2=13):
    out = np.empty((d, n), dtype=np.float32)
    lim = np.float32(2.0 ** clamp_log2 - 2.0 ** -grid_bits)
    scale = np.float32(2.0 ** grid_bits)
    chunk = 1 << 22

    def col(c):
        rng = rng_for(seed, 3, stream, 1 + c)
        for s in range(0, n, chunk):
            m = min(chunk, n - s)
            z = rng.standard_normal(m, dtype=np.float32)
            g = rng.standard_gamma(nu / 2.0, size=m, dtype=np.float32) * np.float32(2.0 / nu)
            x = z / np.sqrt(np.maximum(g, np.float32(1e-30)))
            x = np.rint(x * scale) / scale
            out[c, s:s + m] = np.clip(x, -lim, lim)

    _columns(d, col)
    return out


def corr_normal(n, p=3, rho=0.5, seed=BASE_SEED, stream=0):
    rng = rng_for(seed, 4, stream)
    cov = np.full((p, p), rho) + (1.0 - rho) * np.eye(p)
    L = np.linalg.cholesky(cov)
    z = rng.standard_normal((p, n))
    return (L @ z).astype(np.float32)


def dirichlet_pool(entries, subsets, alpha=0.5, seed=BASE_SEED, stream=0):
    rng = rng_for(seed, 5, stream)
    w = rng.dirichlet(np.full(subsets, alpha), size=entries)
    cum = np.cumsum(w, axis=1)
    pool = np.zeros((entries, subsets), dtype=np.uint32)
    frac = np.floor(cum[:, :-1] * 2.0 ** 32)
    pool[:, 1:] = np.clip(frac, 0, 2.0 ** 32 - 1).astype(np.uint32)
    pool = np.maximum.accumulate(pool, axis=1)
    return pool


def generate(kind, n, d, seed=BASE_SEED, stream=0):
    if kind == "uniform24":
        return uniform24(n, d, seed, stream)
    if kind == "gmm":
        return gmm(n, d, seed, stream)
    if kind == "student_t_grid":
        return student_t_grid(n, d, seed, stream)
    if kind == "corr_normal":
        return corr_normal(n, d, seed=seed, stream=stream)
    raise ValueError(kind)


# The five workloads (sizes, input recipe, tree parameters).
WORKLOADS = {
    "plain_n65536_d3": dict(n=65536, d=3, gen="uniform24", num_subsets=16, key="cyclic",
                            leaf_size=32),
    "scale_n2^24_d8": dict(n=1 << 24, d=8, gen="gmm", num_subsets=256, key="cyclic",
                           leaf_size=64),
    "hard_n2^26_d16": dict(n=1 << 26, d=16, gen="student_t_grid", num_subsets=64,
                           key="maxvar", leaf_size=128, pool_entries=4096, pool_alpha=0.5),
}


def batched_shapes(trees=512, lo_log2=10, hi_log2=20, dims=(2, 3, 8, 32), seed=BASE_SEED):
    """(n_t, d_t) per tree: n log-uniform on [2^lo, 2^hi], d uniform over dims."""
    rng = rng_for(seed, 6, 0)
    ns = np.floor(2.0 ** rng.uniform(lo_log2, hi_log2, size=trees)).astype(np.int64)
    ds = rng.choice(np.array(dims), size=trees)
    return [(int(a), int(b)) for a, b in zip(ns, ds)]


def poisson_requests(count, rate, lo_log2=12, hi_log2=22, dims=(3, 16), seed=BASE_SEED,
                     stream=0):
    """Arrival times (s), n and d per request for the serving workload."""
    rng = rng_for(seed, 7, stream)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    ns = np.floor(2.0 ** rng.uniform(lo_log2, hi_log2, size=count)).astype(np.int64)
    ds = rng.choice(np.array(dims), size=count)
    return [(float(a), int(b), int(c)) for a, b, c in zip(t, ns, ds)]
