"""Least-squares accuracy of a leverage-score sketch (Section 4.2 and
Appendix A.12), for Khatri-Rao design matrices that are never materialised.

Test infrastructure only (see ``oracle/__init__.py``).

The problem: ``min_x ||A x - b||`` with ``A = U_1 (.) ... (.) U_N`` (rows in
the multi-index order of the U list) and ``b = c_1 (x) ... (x) c_N``.  With
``G_k = U_k^T U_k``:

* ``A^T A = (*)_k G_k`` (the Khatri-Rao Gram identity of Section 3);
* ``A^T b = (*)_k U_k^T c_k`` (column r of A is the Kronecker product of
  the columns r, whose inner product with b factors over the modes);
* ``||b||^2 = prod_k ||c_k||^2``;
* so ``||A x - b||^2 = x^T (A^T A) x - 2 x^T A^T b + ||b||^2`` for any x,
  the optimum is ``x* = (A^T A)^+ A^T b``, and the residual error of an
  approximate solution is ``eps = ||A x - b|| / ||A x* - b|| - 1``.

Distortion (Appendix A.12): with ``A = Q Sigma V^T`` (reduced SVD) and the
sampling matrix S (rows ``w_d e_{t_d}^T``, ``w_d = 1 / sqrt(J q_d)``),
``D = kappa(S Q) - 1`` and ``S Q = (S A) V Sigma^{-1}``, where V and
Sigma come from the eigendecomposition of ``A^T A``.
"""
from __future__ import annotations

import numpy as np

from .definition import hadamard_all, pinv_psd

__all__ = ["KronProblem", "distortion"]


class KronProblem:
    """``A = U_1 (.) ... (.) U_N``, ``b = c_1 (x) ... (x) c_N``."""

    def __init__(self, Us, cs):
        self.U = [np.asarray(U, dtype=np.float64) for U in Us]
        self.c = [np.asarray(c, dtype=np.float64) for c in cs]
        self.G = hadamard_all([U.T @ U for U in self.U])
        self.Atb = hadamard_all([U.T @ c for U, c in zip(self.U, self.c)])
        self.bb = float(np.prod([c @ c for c in self.c]))
        Gp, _ = pinv_psd(self.G)
        self.x_opt = Gp @ self.Atb
        self.r_opt = self.residual(self.x_opt)

    def residual(self, x):
        x = np.asarray(x, dtype=np.float64)
        r2 = float(x @ self.G @ x - 2.0 * x @ self.Atb + self.bb)
        return np.sqrt(max(r2, 0.0))

    def epsilon(self, x):
        return self.residual(x) / self.r_opt - 1.0

    def b_entries(self, idx):
        """``b`` at the rows with multi-indices ``idx [J, N]``."""
        out = np.ones(idx.shape[0])
        for k, c in enumerate(self.c):
            out *= c[idx[:, k]]
        return out

    def rows(self, idx):
        """Rows of ``A`` at the multi-indices ``idx [J, N]``."""
        out = np.ones((idx.shape[0], self.U[0].shape[1]))
        for k, U in enumerate(self.U):
            out *= U[idx[:, k]]
        return out


def distortion(G, rows, prob):
    """``kappa(S Q) - 1`` for the sketch with sampled rows ``rows [J, R]``
    of A (unscaled) and their probabilities ``prob`` (weights
    ``1/sqrt(J q_d)``), given ``G = A^T A``."""
    rows = np.asarray(rows, dtype=np.float64)
    J = rows.shape[0]
    lam, V = np.linalg.eigh((G + G.T) * 0.5)
    keep = lam > G.shape[0] * 2.0 ** -52 * lam.max()
    SA = rows / np.sqrt(J * np.asarray(prob, dtype=np.float64))[:, None]
    SQ = SA @ (V[:, keep] / np.sqrt(lam[keep]))
    s = np.linalg.svd(SQ, compute_uv=False)
    s = s[s > s[0] * 2.0 ** -52 * max(SQ.shape)]
    return s[0] / s[-1] - 1.0
