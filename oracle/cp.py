"""Sketched least squares and CP-ALS (STS-CP) in plain float64.

* :class:`SparseTensor` -- COO tensor with duplicates summed; per mode the
  entries are grouped into mode-``j`` fibers (all entries sharing the other
  modes' indices), the rows of ``mat(T, j)^T`` that a sampled Khatri-Rao
  row selects (Appendix A.9, matricisation; Appendix A.13, the sampled
  spMTTKRP reduces to an SpMM).
* :func:`normal_equations` / :func:`sketched_solve` -- one sampled solve of
  ``min_X || S U_{!=j} X^T - S mat(T, j)^T ||_F`` with the sampling matrix
  ``S`` of Section 2.1 (weights ``1/sqrt(J q_d)``), by the normal equations
  ``U_j = Y M^+`` with ``M = (SA)^T SA`` and ``Y = (SB)^T SA``; then the
  column norms become ``sigma`` and the columns are renormalised
  (the factor update of Algorithm 6).
* :func:`fit` -- ``1 - ||T~ - T||_F / ||T||_F`` (Section 4.3) through
  ``||T~||^2 = sigma^T ((*)_k G_k) sigma`` and ``<T, T~>`` over the nonzeros.
* :func:`cp_als` -- Algorithm 6 with the sampled solve.
* :func:`mttkrp` / :func:`exact_solve` / :func:`exact_als` -- the exact
  least-squares step of Algorithm 6 (no sampling): ``U_j = mat(T, j)
  U_{!=j} ((*)_{k != j} G_k)^+`` with the Khatri-Rao product never formed
  (the sparse MTTKRP over the stored entries), the reference the sampled
  solves approach (Appendix A.13, the exact-ALS column of the accuracy
  table).

The solve method is not fixed by the paper; the reading used is the normal
equations with a float64 eigen-pseudo-inverse (no regularisation).  A column
of zero norm keeps ``sigma = 0`` and stays zero.
"""
from __future__ import annotations

import numpy as np
from scipy import sparse

from .definition import pinv_psd, hadamard_all
from .sampler import KRPSampler

__all__ = ["SparseTensor", "normal_equations", "sketched_solve", "fit",
           "cp_als", "normalize_columns", "sketched_lstsq", "mttkrp", "exact_solve",
           "exact_als"]


class SparseTensor:
    def __init__(self, dims, idx, val):
        self.dims = tuple(int(d) for d in dims)
        self.N = len(self.dims)
        self.idx = np.asarray(idx, dtype=np.int64)
        self.val = np.asarray(val, dtype=np.float64)
        self.nnz = self.val.shape[0]
        self._fib = {}
        # ||T||^2 of the tensor with duplicates summed
        key = self._key(self.idx, list(range(self.N)))
        uk, inv = np.unique(key, return_inverse=True)
        summed = np.bincount(inv.reshape(-1), weights=self.val, minlength=len(uk))
        self.norm2 = float(summed @ summed)

    def _key(self, cols_idx, modes):
        """Mixed-radix key of the columns ``modes`` (int64 when it fits,
        else Python integers)."""
        bits = sum(int(self.dims[m] - 1).bit_length() for m in modes)
        if bits <= 62:
            key = np.zeros(cols_idx.shape[0], dtype=np.int64)
            for c, m in enumerate(modes):
                key = key * self.dims[m] + cols_idx[:, c if cols_idx.shape[1] == len(modes) else m]
            return key
        key = np.zeros(cols_idx.shape[0], dtype=object)
        for c, m in enumerate(modes):
            col = cols_idx[:, c if cols_idx.shape[1] == len(modes) else m]
            key = key * self.dims[m] + col.astype(object)
        return key

    def others(self, j):
        return [k for k in range(self.N) if k != j]

    def fibers(self, j):
        """Entries sorted by the other modes' indices: ``(keys_sorted,
        order)`` where ``order`` permutes the COO entries."""
        if j not in self._fib:
            oth = self.others(j)
            key = self._key(self.idx[:, oth], oth)
            order = np.argsort(key, kind="stable")
            self._fib[j] = (key[order], order)
        return self._fib[j]

    def lookup(self, j, sample_idx):
        """``[lo, hi)`` ranges (into the mode-``j`` sorted order) of the fiber
        selected by each sampled multi-index ``sample_idx[J, N]``."""
        oth = self.others(j)
        keys, _ = self.fibers(j)
        q = self._key(np.asarray(sample_idx)[:, oth], oth)
        lo = np.searchsorted(keys, q, side="left")
        hi = np.searchsorted(keys, q, side="right")
        return lo, hi


def normal_equations(tensor, j, idx, rows, w2):
    """``M = sum_d w_d^2 a_d a_d^T`` and ``Y = sum_d w_d^2 b_d a_d^T`` where
    ``b_d`` is the mode-``j`` fiber of sample ``d`` (a sparse ``I_j`` vector).

    Samples drawn more than once (the same multi-index) select the same row
    ``a_d`` and the same fiber ``b_d``, so their terms of ``Y`` are gathered
    first: each distinct sampled fiber is expanded once with the summed
    weight ``sum w_d^2`` of its samples (the rows of the sampling matrix of
    Section 2.1 are i.i.d. draws; repeated rows add).  This bounds the
    expansion by the number of stored entries.
    """
    rows = np.asarray(rows, dtype=np.float64)
    M = (rows * w2[:, None]).T @ rows
    oth = tensor.others(j)
    idx = np.asarray(idx, dtype=np.int64)
    _, first, inv = np.unique(idx[:, oth], axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    W = np.bincount(inv, weights=w2, minlength=len(first))       # summed w_d^2
    A = rows[first]                                              # a_u, one per fiber
    lo, hi = tensor.lookup(j, idx[first])
    cnt = hi - lo
    _, order = tensor.fibers(j)
    uid = np.repeat(np.arange(len(cnt)), cnt)
    starts = np.repeat(lo - np.concatenate(([0], np.cumsum(cnt)[:-1])), cnt)
    ent = order[starts + np.arange(cnt.sum())]
    # P[i, u] = W_u * sum of x_e over the entries of fiber u with i_j(e) = i
    P = sparse.coo_matrix((W[uid] * tensor.val[ent], (tensor.idx[ent, j], uid)),
                          shape=(tensor.dims[j], len(first))).tocsr()
    Y = np.asarray(P @ A)
    return M, Y


def sketched_lstsq(rows, prob, sb_rows):
    """``argmin_X ||S A X - S B||_F`` from sampled rows ``a_d`` of ``A``,
    their probabilities ``q_d`` and the rows ``b_d`` of ``B`` at the same
    indices (Section 2.1: weights ``w_d = 1/sqrt(J q_d)``), by the normal
    equations ``X = M^+ (SA)^T SB`` with the float64 eigen-pseudo-inverse."""
    rows = np.asarray(rows, dtype=np.float64)
    sb_rows = np.asarray(sb_rows, dtype=np.float64)
    J = rows.shape[0]
    w2 = 1.0 / (J * np.asarray(prob, dtype=np.float64))
    M = (rows * w2[:, None]).T @ rows
    Z = (rows * w2[:, None]).T @ sb_rows
    Mp, _ = pinv_psd(M)
    return Mp @ Z


def normalize_columns(U):
    """Column norms ``sigma`` and the renormalised copy (zero columns stay)."""
    U = np.asarray(U, dtype=np.float64)
    sigma = np.sqrt(np.einsum("ir,ir->r", U, U))
    out = U.copy()
    nz = sigma > 0
    out[:, nz] /= sigma[nz]
    return out, sigma


def sketched_solve(sampler: KRPSampler, tensor: SparseTensor, j, u01):
    """One STS-CP solve for mode ``j``; returns ``(U_j, sigma, draw, M, Y)``.

    The sampler is refreshed with the new ``U_j`` (the factor update of
    Algorithm 6 and Theorem 1.1 part 1)."""
    draw = sampler.draw(j, u01)
    J = draw.prob.shape[0]
    w2 = 1.0 / (J * draw.prob)
    M, Y = normal_equations(tensor, j, draw.idx, draw.rows, w2)
    Mp, _ = pinv_psd(M)
    Unew, sigma = normalize_columns(Y @ Mp)
    sampler.refresh(j, Unew)
    return Unew, sigma, draw, M, Y


def fit(tensor: SparseTensor, Us, sigma, chunk=1 << 20):
    """``1 - ||T~ - T||_F / ||T||_F`` with ``T~ = [sigma; U_1..U_N]``."""
    Us = [np.asarray(U, dtype=np.float64) for U in Us]
    sigma = np.asarray(sigma, dtype=np.float64)
    inner = 0.0
    for s in range(0, tensor.nnz, chunk):
        e = min(tensor.nnz, s + chunk)
        p = np.ones((e - s, sigma.shape[0]))
        for k, U in enumerate(Us):
            p *= U[tensor.idx[s:e, k]]
        inner += float(tensor.val[s:e] @ (p @ sigma))
    G = hadamard_all([U.T @ U for U in Us])
    model2 = float(sigma @ G @ sigma)
    resid2 = max(0.0, tensor.norm2 + model2 - 2.0 * inner)
    return 1.0 - np.sqrt(resid2) / np.sqrt(tensor.norm2)


def cp_als(tensor: SparseTensor, U0, sweeps, u01_of, F=None, factor_dtype=None, progress=None):
    """Algorithm 6 with the sampled solve.  ``U0``: initial factors (their
    columns are normalised here, ``sigma = 1``); ``u01_of(sweep, j)`` gives
    the uniforms of each solve.  Returns ``(Us, sigma, fits)`` with the fit
    after every sweep.

    ``factor_dtype`` (None or a NumPy float type) is the type the factors
    are kept in: each normalised factor is rounded to it, and those rounded
    values are the factors of the problem from then on (trees, draws and
    solves use them in float64).  ``progress(sweep, j)`` is called after
    every solve."""
    def keep(U):
        return U if factor_dtype is None else U.astype(factor_dtype).astype(np.float64)

    Us = [keep(normalize_columns(U)[0]) for U in U0]
    sigma = np.ones(Us[0].shape[1])
    sampler = KRPSampler(Us, F)
    fits = []
    for s in range(sweeps):
        for j in range(tensor.N):
            Uj, sigma, _, _, _ = sketched_solve(sampler, tensor, j, u01_of(s, j))
            Us[j] = keep(Uj)
            if factor_dtype is not None:
                sampler.refresh(j, Us[j])
            if progress is not None:
                progress(s, j)
        fits.append(fit(tensor, Us, sigma))
    return Us, sigma, fits


def mttkrp(tensor: SparseTensor, Us, j, chunk=1 << 20):
    """``mat(T, j) U_{!=j}``: ``Y[i_j(e), :] += x_e prod_{k != j} U_k[i_k(e), :]``
    over every stored entry (duplicates add)."""
    R = next(np.asarray(U).shape[1] for k, U in enumerate(Us) if k != j)
    Y = np.zeros((tensor.dims[j], R))
    for s in range(0, tensor.nnz, chunk):
        e = min(tensor.nnz, s + chunk)
        p = np.ones((e - s, R))
        for k, U in enumerate(Us):
            if k != j:
                p *= np.asarray(U, dtype=np.float64)[tensor.idx[s:e, k]]
        # the sum over entries as a sparse (I_j x chunk) matrix of values
        X = sparse.coo_matrix((tensor.val[s:e], (tensor.idx[s:e, j], np.arange(e - s))),
                              shape=(tensor.dims[j], e - s)).tocsr()
        Y += X @ p
    return Y


def exact_solve(tensor: SparseTensor, Us, j):
    """The exact least-squares update of factor ``j`` (Algorithm 6 without
    sampling): ``U_j = mat(T, j) U_{!=j} M^+`` with ``M = (*)_{k != j}
    U_k^T U_k``; returns ``(U_j normalised, sigma, Y, M)``."""
    G = hadamard_all([np.asarray(U, dtype=np.float64).T @ np.asarray(U, dtype=np.float64)
                      for k, U in enumerate(Us) if k != j])
    Y = mttkrp(tensor, Us, j)
    Mp, _ = pinv_psd(G)
    Unew, sigma = normalize_columns(Y @ Mp)
    return Unew, sigma, Y, G


def exact_als(tensor: SparseTensor, U0, sweeps, factor_dtype=None, progress=None):
    """Algorithm 6 with the exact solve: columns normalised first, factors
    kept in ``factor_dtype`` (as :func:`cp_als`); returns ``(Us, sigma,
    fits)`` with the fit after every sweep."""
    def keep(U):
        return U if factor_dtype is None else U.astype(factor_dtype).astype(np.float64)

    Us = [keep(normalize_columns(U)[0]) for U in U0]
    sigma = np.ones(Us[0].shape[1])
    fits = []
    for s in range(sweeps):
        for j in range(tensor.N):
            Uj, sigma, _, _ = exact_solve(tensor, Us, j)
            Us[j] = keep(Uj)
            if progress is not None:
                progress(s, j)
        fits.append(fit(tensor, Us, sigma))
    return Us, sigma, fits
