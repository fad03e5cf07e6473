"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds random-number and workload generation only (point clouds,
marginal weights, cost matrices for the stored-cost mode, and the block-index
streams the sampler draws).  None of the solver's arithmetic lives here.

Workloads (color-transfer shaped, Sec. 5.1 of the paper uses RGB palette
centroids with histogram weights; the photographs are replaced by seeded
clouds in [0,1]^3):
  * uniform_points(seed, N)          i.i.d. U[0,1]^3, float32
  * mixture_points(seed, N)          8 isotropic Gaussians (sigma 0.08) with
                                     means U[0,1]^3, clipped to [0,1], float32
  * uniform_weights(N)               1/N each, float64
  * dirichlet_weights(seed, N)       Dirichlet(1) draw, float64
  * sqeuclid_cost(X, Y, dtype)       squared Euclidean distances, computed in
                                     float64 and rounded once to dtype
Block-index streams (the uniform sampler's draws, counter-based):
  * philox_uniform_indices(seed, k0, count, m)
      i_k = floor(x_k * m / 2^64) with x_k the k-th 64-bit output of
      Philox4x64-10 (key = (seed, 0)), numpy's counter convention: output k
      is lane k mod 4 of the block at counter 1 + floor(k / 4).
  * philox_uniform_doubles(seed, k0, count)
      u_k = floor(x_k / 2^11) * 2^-53 in [0, 1), same outputs x_k.
  * philox_permutation_indices(seed, p0, npasses, m)
      pass p visits the rows in the order of a stable ascending sort of the
      keys x_{p*m + t}, t = 0..m-1.
"""
import numpy as np

_M64 = (1 << 64) - 1


def uniform_points(seed: int, N: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((N, 3)).astype(np.float32)


def mixture_points(seed: int, N: int, K: int = 8, sigma: float = 0.08) -> np.ndarray:
    rng = np.random.default_rng(seed)
    means = rng.random((K, 3))
    labels = rng.integers(0, K, size=N)
    pts = means[labels] + sigma * rng.standard_normal((N, 3))
    return np.clip(pts, 0.0, 1.0).astype(np.float32)


def uniform_weights(N: int) -> np.ndarray:
    return np.full(N, 1.0 / N, dtype=np.float64)


def dirichlet_weights(seed: int, N: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.dirichlet(np.ones(N)).astype(np.float64)


def sqeuclid_cost(X: np.ndarray, Y: np.ndarray, dtype=np.float32) -> np.ndarray:
    Xd = X.astype(np.float64)
    Yd = Y.astype(np.float64)
    D = (Xd[:, None, 0] - Yd[None, :, 0]) ** 2
    D += (Xd[:, None, 1] - Yd[None, :, 1]) ** 2
    D += (Xd[:, None, 2] - Yd[None, :, 2]) ** 2
    return D.astype(dtype)


def philox_raw(seed: int, k0: int, count: int) -> np.ndarray:
    """64-bit Philox4x64-10 outputs k0 .. k0+count-1 for key (seed, 0)."""
    if count <= 0:
        return np.empty(0, dtype=np.uint64)
    blk0 = k0 // 4
    skip = k0 - 4 * blk0
    bg = np.random.Philox(key=np.array([seed & _M64, 0], dtype=np.uint64),
                          counter=np.array([blk0, 0, 0, 0], dtype=np.uint64))
    raw = bg.random_raw(skip + count)
    return np.asarray(raw[skip:], dtype=np.uint64)


def philox_uniform_indices(seed: int, k0: int, count: int, m: int) -> np.ndarray:
    x = philox_raw(seed, k0, count)
    # floor(x * m / 2^64) via 32-bit halves to stay exact in uint64
    m = np.uint64(m)
    hi = x >> np.uint64(32)
    lo = x & np.uint64(0xFFFFFFFF)
    t = lo * m
    u = hi * m + (t >> np.uint64(32))
    return (u >> np.uint64(32)).astype(np.int32)


def philox_uniform_doubles(seed: int, k0: int, count: int) -> np.ndarray:
    x = philox_raw(seed, k0, count)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def philox_permutation_indices(seed: int, p0: int, npasses: int, m: int) -> np.ndarray:
    out = np.empty(npasses * m, dtype=np.int32)
    for q in range(npasses):
        keys = philox_raw(seed, (p0 + q) * m, m)
        out[q * m:(q + 1) * m] = np.argsort(keys, kind="stable").astype(np.int32)
    return out


def problem_uniform_c1(seed: int = 0, m: int = 256, n: int = 256):
    """m x n uniform RGB points, float64 stored squared-Euclidean cost."""
    X = uniform_points(seed, m)
    Y = uniform_points(seed + 1, n)
    return dict(X=X, Y=Y, C=sqeuclid_cost(X, Y, np.float64),
                a=uniform_weights(m), b=uniform_weights(n))


def problem_mixture(seed: int, m: int, n: int, cost_dtype=np.float32, dirichlet_b: bool = False,
                    with_cost: bool = True):
    X = mixture_points(seed, m)
    Y = mixture_points(seed + 1, n)
    b = dirichlet_weights(seed + 2, n) if dirichlet_b else uniform_weights(n)
    d = dict(X=X, Y=Y, a=uniform_weights(m), b=b)
    if with_cost:
        d["C"] = sqeuclid_cost(X, Y, cost_dtype)
    return d


def batched_sizes(seed: int, count: int, lo: int = 64, hi: int = 4096):
    """count (m, n) pairs, each side log-uniform in [lo, hi], rounded."""
    rng = np.random.default_rng(seed)
    ms = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)
    ns = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)
    return ms, ns


def batched_problem(seed: int, p: int, m: int, n: int, with_cost: bool = False):
    """Problem p of a batch: two mixture palettes, uniform weights."""
    return problem_mixture(seed * 1000003 + 7 * p, m, n, cost_dtype=np.float32, with_cost=with_cost)
