"""Randomized range-finder initialisation of a CP factor (the initialisation
the paper describes for its sparsest tensor, Section 4.3 / Appendix A.13:
``U_j = mat(T, j) S`` with an i.i.d. Gaussian ``S`` of
``prod_{k != j} I_k`` rows and R columns that is never materialised; only
the rows of ``S`` for fibers that hold entries are generated).

Test infrastructure only (see ``oracle/__init__.py``).

The Gaussian entries come from a counter-based generator so that every
implementation produces the same ``S``:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): 10 rounds of the 4 x 64-bit Philox S-box with
  multipliers 0xD2E7470EE14C6C93 and 0xCA5A826395121157 and Weyl key
  increments 0x9E3779B97F4A7C15 and 0xBB67AE8584CAA73B;
* the row of ``S`` for the fiber with other-mode indices (i_a, i_b, i_c,
  i_d) (increasing mode order, missing ones 0) and the column pair q uses
  counter ``(i_a | i_b << 32, i_c | i_d << 32, q, 0)`` and key
  ``(seed, j)``; of the four outputs, the first two give open-interval
  uniforms ``u = ((x >> 11) + 0.5) 2^-53`` and the Box-Muller transform
  ``sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2)`` gives columns 2q and 2q+1.
"""
from __future__ import annotations

import numpy as np

__all__ = ["philox4x64", "sketch_rows", "range_finder", "philox_uniforms"]

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO = np.uint64(0xFFFFFFFF)
_32 = np.uint64(32)


def _mulhilo(a, b):
    """High and low 64-bit words of the 128-bit product a * b."""
    lo = a * b
    a0, a1 = a & _LO, a >> _32
    b0, b1 = b & _LO, b >> _32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _32) + (p01 & _LO) + (p10 & _LO)
    hi = p11 + (p01 >> _32) + (p10 >> _32) + (mid >> _32)
    return hi, lo


def philox4x64(ctr, key):
    """Philox4x64-10 of counters ``ctr`` (uint64 [..., 4]) under ``key``
    (uint64 [..., 2]); returns uint64 [..., 4]."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.broadcast_to(np.asarray(key, dtype=np.uint64), ctr.shape[:-1] + (2,))
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0, k1 = key[..., 0].copy(), key[..., 1].copy()
    with np.errstate(over="ignore"):
        for _ in range(10):
            h0, l0 = _mulhilo(_M0, c0)
            h1, l1 = _mulhilo(_M1, c2)
            c0, c1, c2, c3 = h1 ^ c1 ^ k0, l1, h0 ^ c3 ^ k1, l0
            k0 = k0 + _W0
            k1 = k1 + _W1
    return np.stack([c0, c1, c2, c3], axis=-1)


def sketch_rows(others, R, seed, j):
    """Rows of S for fibers with other-mode indices ``others`` (int [F, N-1],
    N - 1 <= 4): float64 [F, R]."""
    others = np.asarray(others, dtype=np.uint64)
    F, m = others.shape
    if m > 4:
        raise ValueError("at most four other modes")
    cols = np.zeros((F, 4), dtype=np.uint64)
    cols[:, :m] = others
    w0 = cols[:, 0] | (cols[:, 1] << _32)
    w1 = cols[:, 2] | (cols[:, 3] << _32)
    out = np.empty((F, R))
    for q in range((R + 1) // 2):
        ctr = np.stack([w0, w1, np.full(F, q, dtype=np.uint64), np.zeros(F, dtype=np.uint64)], 1)
        x = philox4x64(ctr, [seed, j])
        u1 = ((x[:, 0] >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
        u2 = ((x[:, 1] >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
        rad = np.sqrt(-2.0 * np.log(u1))
        out[:, 2 * q] = rad * np.cos(2.0 * np.pi * u2)
        if 2 * q + 1 < R:
            out[:, 2 * q + 1] = rad * np.sin(2.0 * np.pi * u2)
    return out


def range_finder(tensor, j, R, seed):
    """``mat(T, j) S`` (I_j x R) over the stored entries (duplicates add)."""
    oth = tensor.others(j)
    fib, inv = np.unique(tensor.idx[:, oth], axis=0, return_inverse=True)
    S = sketch_rows(fib, R, seed, j)
    inv = inv.reshape(-1)
    out = np.zeros((tensor.dims[j], R))
    for r in range(R):
        out[:, r] = np.bincount(tensor.idx[:, j], weights=tensor.val * S[inv, r],
                                minlength=tensor.dims[j])
    return out


def philox_uniforms(J, N, seed, ctr_base=0, ctr2=0):
    """Sampler uniforms generated from (seed, ctr_base): float64 [J][N][2]
    with [d][k][s] from word s of Philox4x64-10 of counter
    (ctr_base + d, k, ctr2, 0) under key (seed, 0); ``ctr2 = sweep * N + j``
    keys the solve of mode j in an ALS sweep."""
    d = np.arange(J, dtype=np.uint64) + np.uint64(ctr_base)
    out = np.empty((J, N, 2))
    for k in range(N):
        ctr = np.stack([d, np.full(J, k, dtype=np.uint64), np.full(J, ctr2, dtype=np.uint64),
                        np.zeros(J, dtype=np.uint64)], 1)
        x = philox4x64(ctr, [seed, 0])
        for s in range(2):
            out[:, k, s] = ((x[:, s] >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    return out
