"""Definition-level oracle: everything computed straight from the definitions.

Only for tiny inputs (the Khatri-Rao product is materialised).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "khatri_rao",
    "multi_index_rows",
    "pinv_psd",
    "leverage_qr",
    "leverage_svd",
    "leverage_formula",
    "conditional_q",
    "hadamard_all",
]


def khatri_rao(mats):
    """Row-wise materialisation of ``U_1 (.) U_2 (.) ... (.) U_N``.

    Row ``r`` holds the Hadamard product ``U_1[i_1] * ... * U_N[i_N]`` of
    the rows selected by the multi-index ``(i_1, ..., i_N)``, with ``r`` the
    C-order (last index fastest) ravel of that multi-index.  Column ``c`` is
    therefore the Kronecker product of the factors' columns ``c`` (Section 2,
    notation; Appendix A.2, table of matrix products).
    """
    A = np.asarray(mats[0], dtype=np.float64)
    R = A.shape[1]
    for U in mats[1:]:
        U = np.asarray(U, dtype=np.float64)
        A = (A[:, None, :] * U[None, :, :]).reshape(-1, R)
    return A


def multi_index_rows(dims, rows):
    """Multi-indices (C order) of flat KRP row numbers ``rows``."""
    return np.stack(np.unravel_index(np.asarray(rows), tuple(dims)), axis=-1)


def hadamard_all(mats):
    """Elementwise product of equally shaped matrices (empty -> None)."""
    out = None
    for M in mats:
        out = np.array(M, dtype=np.float64) if out is None else out * M
    return out


def pinv_psd(G, tau_scale=None):
    """Pseudo-inverse and numerical rank of a symmetric p.s.d. matrix.

    The paper writes ``M^+`` for the pseudo-inverse (Section 2) without a
    cutoff; the reading used here keeps eigenvalues above
    ``tau = R * 2**-52 * lambda_max`` and inverts them.  The rank is the
    count of kept eigenvalues (equal to trace(G G^+)).
    """
    G = np.asarray(G, dtype=np.float64)
    R = G.shape[0]
    lam, V = np.linalg.eigh((G + G.T) * 0.5)
    lmax = max(float(lam.max()), 0.0)
    tau = (R if tau_scale is None else tau_scale) * 2.0 ** -52 * lmax
    keep = lam > tau
    Vk = V[:, keep]
    return (Vk / lam[keep]) @ Vk.T, int(keep.sum())


def leverage_qr(A):
    """Leverage scores as squared row norms of Q from a reduced QR of ``A``
    (Section 2.1).  Valid for full column rank."""
    Q, _ = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    return np.einsum("ij,ij->i", Q, Q)


def leverage_svd(A, rtol=None):
    """Leverage scores from the left singular vectors of the nonzero singular
    values (rank-revealing form of the same definition)."""
    A = np.asarray(A, dtype=np.float64)
    Uq, s, _ = np.linalg.svd(A, full_matrices=False)
    if rtol is None:
        rtol = max(A.shape) * np.finfo(np.float64).eps
    keep = s > rtol * (s[0] if s.size else 0.0)
    Uq = Uq[:, keep]
    return np.einsum("ij,ij->i", Uq, Uq)


def leverage_formula(A):
    """``l_i = A[i] (A^T A)^+ A[i]^T`` (Section 2.1, leverage definition)."""
    A = np.asarray(A, dtype=np.float64)
    Gp, _ = pinv_psd(A.T @ A)
    return np.einsum("ir,rs,is->i", A, Gp, A)


def conditional_q(h, U, Y):
    """Distribution ``q_{h,U,Y}[s] = <h h^T, U[s]^T U[s], Y> / C`` over the
    rows of ``U`` (Theorem 3.1 and Section 3.1).

    ``<h h^T, U[s]^T U[s], Y>`` is the generalised inner product, i.e.
    ``w Y w^T`` with ``w = U[s] * h``.  Returns ``(q, C)``.
    """
    h = np.asarray(h, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    W = U * h[None, :]
    num = np.einsum("sa,ab,sb->s", W, Y, W)
    C = float(num.sum())
    return num / C, C
