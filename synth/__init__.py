"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays them out.  It holds none of
the sampler's or of CP-ALS's arithmetic (no Gram matrices, no leverage
scores, no normalisation): both the CPU oracle and the GPU path receive the
arrays produced here unchanged.

Conventions
-----------
* Factor matrices are drawn in float64 and rounded to float32; the float32
  values are *the* problem for every precision (the float64 paths upcast
  them exactly).
* Uniforms for the sampler are float64 in the open interval (0, 1), laid out
  ``[J][N][2]``: column 0 drives the eigen-component draw and column 1 the
  row draw of mode ``k`` for sample ``d`` (two inversion draws per mode,
  Section 3.2 of the paper).  They are made from 64-bit words ``x`` as
  ``((x >> 11) + 0.5) * 2**-53`` so that no uniform is exactly 0 or 1.
* Sparse tensors are COO with int32 indices ``[nnz][N]`` and float32 values;
  duplicate coordinates are kept as separate entries (they mean a sum).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "gaussian_factors",
    "uniforms",
    "zipf_indices",
    "sparse_tensor",
    "planted_cp_tensor",
    "CONFIGS",
    "config_seed",
    "uniform_seed",
    "sweep_uniforms",
    "als_problem",
    "batched_problems",
]


def config_seed(config_no: int) -> int:
    """Data seed of workload ``config_no`` (1-based)."""
    return 12584 * 10 + int(config_no)


def uniform_seed(config_no: int) -> int:
    """Seed of the sampler uniforms of workload ``config_no``."""
    return 2301 + int(config_no)


def gaussian_factors(dims, R, seed, heavy_rows_frac=0.0, heavy_row_scale=100.0,
                     heavy_entries_frac=0.0, heavy_entry_scale=10.0):
    """List of float32 factor matrices ``U_j`` of shape ``(dims[j], R)``.

    Entries are i.i.d. N(0, 1).  ``heavy_rows_frac`` scales exactly
    ``round(frac * I_j)`` rows of each factor, chosen uniformly without
    replacement, by ``heavy_row_scale`` (skewed leverage).  ``heavy_entries_frac``
    instead scales a random subset of that fraction of all entries by
    ``heavy_entry_scale`` (the recipe of the paper's least-squares accuracy
    and probability-check experiments, Section 4.2 and Appendix A.13).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for I in dims:
        U = rng.standard_normal((int(I), int(R)))
        if heavy_rows_frac > 0:
            n = int(round(heavy_rows_frac * I))
            rows = rng.choice(int(I), size=n, replace=False)
            U[rows] *= heavy_row_scale
        if heavy_entries_frac > 0:
            n = int(round(heavy_entries_frac * I * R))
            flat = rng.choice(int(I) * int(R), size=n, replace=False)
            U.reshape(-1)[flat] *= heavy_entry_scale
        out.append(np.ascontiguousarray(U.astype(np.float32)))
    return out


def uniforms(J, N, seed):
    """float64 array ``[J][N][2]`` of open-interval uniforms."""
    rng = np.random.Generator(np.random.PCG64(seed))
    words = rng.integers(0, np.iinfo(np.uint64).max, size=(int(J), int(N), 2),
                         dtype=np.uint64, endpoint=True)
    return ((words >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def sweep_uniforms(seed, sweep, N, J):
    """Uniforms of one ALS sweep: float64 ``[N][J][N][2]``, block ``j`` for
    the solve of mode ``j`` (seeded by ``seed + 1000 * sweep + j``)."""
    return np.stack([uniforms(J, N, int(seed) + 1000 * int(sweep) + j) for j in range(int(N))])


def zipf_indices(rng, n, dim, alpha, chunk=1 << 24):
    """``n`` draws of a Zipf(alpha) law truncated to ranks ``1..dim``.

    Truncated Zipf is the Zipf law conditioned on ``k <= dim``; it is drawn
    here by inverting its CDF (same law as rejection on an untruncated
    Zipf sampler, much faster).  Rank ``k`` (1-based) is mapped to index
    ``perm[k-1]`` through a seeded random permutation of ``[0, dim)``, so the
    popular indices are scattered over the mode.
    """
    dim = int(dim)
    # float64 CDF over the ranks; accumulate in blocks to limit memory.
    cdf = np.empty(dim, dtype=np.float64)
    step = 1 << 22
    run = 0.0
    for s in range(0, dim, step):
        k = np.arange(s + 1, min(dim, s + step) + 1, dtype=np.float64)
        w = k ** (-float(alpha))
        c = np.cumsum(w)
        cdf[s:s + len(k)] = run + c
        run += c[-1]
    cdf /= run
    perm = rng.permutation(dim).astype(np.int32)
    out = np.empty(int(n), dtype=np.int32)

    def invert(s, u):
        r = np.searchsorted(cdf, u, side="right")
        np.minimum(r, dim - 1, out=r)
        out[s:s + len(u)] = perm[r]

    # the uniforms are drawn in order; the searches (which release the GIL)
    # run on a few threads, so the result does not depend on the thread count
    nthr = max(1, min(8, os.cpu_count() or 1))
    starts = list(range(0, int(n), chunk))
    with ThreadPoolExecutor(nthr) as ex:
        for b0 in range(0, len(starts), nthr):
            batch = [(s, rng.random(min(chunk, int(n) - s))) for s in starts[b0:b0 + nthr]]
            list(ex.map(lambda su: invert(*su), batch))
    return out


def sparse_tensor(dims, nnz, alpha, seed, sigma=1.0, progress=None):
    """Synthetic sparse tensor: COO ``(idx int32 [nnz][N], val float32 [nnz])``.

    Indices per mode are truncated Zipf(alpha) (see :func:`zipf_indices`),
    values lognormal(0, sigma).  Duplicates are kept.  ``progress(j)`` is
    called after each mode's indices (the draws do not depend on it).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    N = len(dims)
    idx = np.empty((int(nnz), N), dtype=np.int32)
    for j, d in enumerate(dims):
        idx[:, j] = zipf_indices(rng, nnz, d, alpha)
        if progress is not None:
            progress(j)
    val = rng.lognormal(0.0, sigma, size=int(nnz)).astype(np.float32)
    return idx, val


def planted_cp_tensor(dims, R, seed):
    """Dense tensor of exact CP rank ``R`` stored as COO with every entry.

    Returns ``(idx, val, factors)`` where the factors are float64 N(0,1)
    matrices; ``val`` holds the float64 entries ``sum_r prod_k U_k[i_k, r]``
    rounded to float32.  Used only at tiny sizes.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Us = [rng.standard_normal((int(I), int(R))) for I in dims]
    grids = np.meshgrid(*[np.arange(I) for I in dims], indexing="ij")
    idx = np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.int32)
    prod = np.ones((idx.shape[0], R))
    for k, U in enumerate(Us):
        prod *= U[idx[:, k]]
    val = prod.sum(axis=1).astype(np.float32)
    return idx, val, Us


# Synthetic workloads, shaped like the paper's experiments (the FROSTT
# tensors it decomposes are not available; these stand in for them).
CONFIGS = {
    1: dict(name="exact-tiny N=3 I=64 R=8", N=3, dims=(64, 64, 64), R=8, J=4096),
    2: dict(name="sampler N=3 I=2^20 R=32 J=65536 (1% rows x100)", N=3,
            dims=(1 << 20,) * 3, R=32, J=65536, heavy_rows_frac=0.01,
            heavy_row_scale=100.0),
    3: dict(name="sketched CP-ALS 1e6x1e6x1e5 nnz=1e8 R=64 J=65536", N=3,
            dims=(1_000_000, 1_000_000, 100_000), nnz=100_000_000,
            alpha=1.2, R=64, J=65536, sweeps=10),
    4: dict(name="batched 64 samplers J=16384", P=64, J=16384),
    5: dict(name="sketched CP-ALS 2e7^3x1e6 nnz=5e8 R=128 J=131072", N=4,
            dims=(20_000_000, 20_000_000, 20_000_000, 1_000_000),
            nnz=500_000_000, alpha=1.1, R=128, J=131072, sweeps=10),
}


def als_problem(config_no, nnz=None, progress=None):
    """Inputs of a sketched CP-ALS workload: ``(dims, idx, val, U0, R, J,
    sweeps, useed)`` with the COO tensor, the N(0,1) initial factors and
    the uniform seed (pass it to :func:`sweep_uniforms`).  ``nnz`` overrides
    the workload's nonzero count (smaller tests of the same recipe)."""
    cfg = CONFIGS[int(config_no)]
    dims = cfg["dims"]
    n = cfg["nnz"] if nnz is None else int(nnz)
    idx, val = sparse_tensor(dims, n, cfg["alpha"], config_seed(config_no), progress=progress)
    U0 = gaussian_factors(dims, cfg["R"], config_seed(config_no) + 100)
    return dims, idx, val, U0, cfg["R"], cfg["J"], cfg["sweeps"], uniform_seed(config_no)


def batched_problems(P, seed):
    """Heterogeneous sampler problems: N in {3,4,5}, I log-uniform in
    [2^10, 2^22], R in {16,32,64,128}.  Returns a list of (dims, R)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    probs = []
    for _ in range(int(P)):
        N = int(rng.integers(3, 6))
        R = int(rng.choice([16, 32, 64, 128]))
        dims = tuple(int(math.floor(2.0 ** rng.uniform(10, 22))) for _ in range(N))
        probs.append((dims, R))
    return probs
