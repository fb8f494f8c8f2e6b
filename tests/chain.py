"""Checks of one sketched solve on the GPU's own draw (Section 2.1: the
sampled normal equations; the factor update of Algorithm 6).

Given the factors the solve started from, the indices the GPU drew and its
pieces (``CPALS.parts``), every deterministic step after the draw is
recomputed by the float64 oracle and compared step by step, each step fed
with the GPU's result of the step before, so that an error is attributed to
the step that makes it:

* ``q_d = a_d G^+ a_d^T / rank`` from the factor rows (definition),
* ``M = sum_d w_d^2 a_d a_d^T`` and ``Y = (S B)^T S A`` (oracle normal
  equations with the GPU's weights ``w_d^2 = 1 / (J q_d)``),
* ``M^+`` (oracle pseudo-inverse of the GPU's ``M``),
* ``U_j`` and ``sigma`` (the GPU's ``Y`` times the GPU's ``M^+``, columns
  normalised).

Tolerances per precision (relative to the largest entry of the quantity):
float64 and float32 paths form ``a_d``, ``M``, ``Y`` in float64 (float32
factor values multiply exactly), so they differ from the oracle by the
summation order only; the split path stores ``w_d a_d`` in float32, forms
``M`` from three bf16 products (~2^-16 of the products) and ``Y`` with
float32 atomics.  ``q_d`` is formed in float64 from ``G^+`` of the float64
Grams in every precision (error ~1e-16 kappa(G)).
"""
import numpy as np

from oracle import cp as ocp
from oracle import definition as dfn

TOL = {
    #          q       M       Y       U (stored)
    "fp64": (1e-10, 1e-11, 1e-10, 1e-10),
    "fp32": (1e-9, 1e-11, 1e-10, 1e-6),
    "bf16x2": (1e-9, 1e-4, 1e-5, 1e-6),
}


def rows_of(Us, idx, j):
    a = None
    for k, U in enumerate(Us):
        if k == j:
            continue
        r = np.asarray(U, dtype=np.float64)[idx[:, k]]
        a = r if a is None else a * r
    return a


def check_solve(tensor, Us_before, j, parts, U_after, sigma, prec, grams=None, rows=None):
    """Compares one solve's pieces with the oracle; returns the error
    figures (each already asserted against ``TOL``).

    ``tensor``: ``oracle.cp.SparseTensor``; ``Us_before``: host factors the
    solve started from (``Us_before[j]`` unused); ``parts``: host arrays of
    ``CPALS.parts(j)``; ``U_after``, ``sigma``: the GPU's new factor and
    column norms.  ``grams`` (optional) are the float64 Grams of the other
    factors and ``rows`` the sampled rows, when the factors are too large to
    pass whole."""
    tq, tm, ty, tu = TOL[prec]
    idx = parts["idx"].astype(np.int64)
    J = idx.shape[0]
    a = rows_of(Us_before, idx, j) if rows is None else np.asarray(rows, dtype=np.float64)
    oth = [k for k in range(tensor.N) if k != j]
    if grams is None:
        grams = {k: np.asarray(Us_before[k], dtype=np.float64).T @ np.asarray(Us_before[k],
                                                                               dtype=np.float64)
                 for k in oth}
    G = dfn.hadamard_all([grams[k] for k in oth])
    Gp, rank = dfn.pinv_psd(G)
    q = np.einsum("da,ab,db->d", a, Gp, a) / rank
    out = {}
    # a zero row a_d (rows of an updated factor that no sampled fiber
    # touched are zero) has q_d = 0 in any arithmetic; only a walk whose
    # mass rounding swallowed can land there, and it gets weight 0
    zero = ~np.any(a != 0.0, axis=1)
    assert np.all(parts["prob"][zero] == 0.0), "q_d of a zero row"
    out["q"] = float(np.max(np.abs(parts["prob"][~zero] - q[~zero]) / q[~zero]))
    assert out["q"] <= tq, ("q", out["q"])
    out["zero rows"] = int(np.count_nonzero(zero))
    w2 = np.where(parts["prob"] > 0, 1.0 / (J * parts["prob"]), 0.0)
    if "w" in parts:
        # the GPU's weights are 1 / sqrt(J q_d), or 0 for a sample whose
        # walk met a non-positive mass (counted by check_status)
        wg = np.asarray(parts["w"], dtype=np.float64)
        nz = wg > 0
        assert np.all(np.abs(wg[nz] ** 2 - w2[nz]) <= 1e-12 * w2[nz]), "w_d^2 != 1 / (J q_d)"
        out["w0"] = int(np.count_nonzero(~nz & (w2 > 0)))
        w2 = np.where(nz, w2, 0.0)
    M, Y = ocp.normal_equations(tensor, j, idx, a, w2)
    out["M"] = float(np.abs(parts["M"] - M).max() / np.abs(M).max())
    assert out["M"] <= tm, ("M", out["M"])
    Yg = parts["Y"]
    ys = max(np.abs(Y).max(), 1e-300)
    out["Y"] = float(np.abs(Yg - Y).max() / ys)
    assert out["Y"] <= ty, ("Y", out["Y"])
    Mg = parts["M"]
    lam = np.linalg.eigvalsh((Mg + Mg.T) * 0.5)
    kappa = lam[-1] / max(lam[lam > Mg.shape[0] * 2.0 ** -52 * lam[-1]].min(), 1e-300)
    Mp, _ = dfn.pinv_psd(Mg)
    out["Mp"] = float(np.abs(parts["Mp"] - Mp).max() / np.abs(Mp).max())
    out["kappa"] = float(kappa)
    assert out["Mp"] <= max(1e-10, 1e-13 * kappa), ("M+", out["Mp"], kappa)
    Uref, sref = ocp.normalize_columns(Yg @ parts["Mp"])
    out["sigma"] = float(np.max(np.abs(sigma - sref) / np.maximum(sref, 1e-300)))
    assert out["sigma"] <= 1e-10, ("sigma", out["sigma"])
    cmax = np.maximum(np.abs(Uref).max(axis=0), 1e-300)
    out["U"] = float((np.abs(np.asarray(U_after, dtype=np.float64) - Uref) / cmax).max())
    assert out["U"] <= tu, ("U", out["U"])
    return out
