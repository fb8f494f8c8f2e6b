"""Definition-level pins of the oracle (CPU)."""
import numpy as np
import pytest

import synth
from oracle import definition as dfn

from pins import check_thm31_product


def test_khatri_rao_columns_are_kronecker_products():
    # Appendix A.2: column j of A (.) B is A[:, j] (x) B[:, j]
    rng = np.random.default_rng(0)
    A, B, C = rng.standard_normal((3, 4)), rng.standard_normal((5, 4)), rng.standard_normal((2, 4))
    K = dfn.khatri_rao([A, B, C])
    for j in range(4):
        np.testing.assert_array_equal(K[:, j], np.kron(np.kron(A[:, j], B[:, j]), C[:, j]))


def test_gram_of_krp_is_hadamard_of_grams():
    # Section 3: A^T A = (*)_k U_k^T U_k
    Us = synth.gaussian_factors((7, 5, 6), 4, seed=3)
    A = dfn.khatri_rao(Us)
    G = dfn.hadamard_all([U.T.astype(np.float64) @ U for U in Us])
    np.testing.assert_allclose(A.T @ A, G, rtol=1e-12, atol=1e-12 * np.abs(G).max())


def test_pinv_psd_matches_library_pinv():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((20, 6))
    G = X.T @ X
    Gp, r = dfn.pinv_psd(G)
    assert r == 6
    np.testing.assert_allclose(Gp, np.linalg.pinv(G), rtol=1e-10, atol=1e-12)
    X[:, 5] = X[:, 0] + X[:, 1]          # rank 5
    G = X.T @ X
    Gp, r = dfn.pinv_psd(G)
    assert r == 5
    np.testing.assert_allclose(Gp, np.linalg.pinv(G, rcond=1e-12, hermitian=True),
                               rtol=1e-8, atol=1e-10)


def test_leverage_three_definitions_agree_c1():
    # Section 2.1: QR row norms == A (A^T A)^+ A^T diagonal; sum == rank
    cfg = synth.CONFIGS[1]
    Us = synth.gaussian_factors(cfg["dims"], cfg["R"], synth.config_seed(1))
    A = dfn.khatri_rao(Us)
    assert A.shape == (262144, 8)
    l_qr = dfn.leverage_qr(A)
    l_f = dfn.leverage_formula(A)
    l_svd = dfn.leverage_svd(A)
    assert np.max(np.abs(l_qr - l_f) / l_qr) < 1e-10
    assert np.max(np.abs(l_qr - l_svd) / l_qr) < 1e-10
    assert abs(l_qr.sum() - 8) < 1e-9


def test_leverage_rank_deficient_sums_to_rank():
    Us = synth.gaussian_factors((9, 8, 7), 5, seed=4)
    Us = [U.astype(np.float64) for U in Us]
    Us[1][:, 4] = Us[1][:, 3]
    Us[0][:, 4] = Us[0][:, 3]
    Us[2][:, 4] = Us[2][:, 3]            # two identical columns of A
    A = dfn.khatri_rao(Us)
    l_f = dfn.leverage_formula(A)
    l_svd = dfn.leverage_svd(A)
    assert abs(l_svd.sum() - 4) < 1e-9
    np.testing.assert_allclose(l_f, l_svd, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("exclude", [-1, 0, 1, 2])
def test_theorem_31_conditionals_multiply_to_leverage(exclude):
    # Theorem 3.1: p(s_k | s_<k) = q_{h_<k, U_k, G_>k}[s_k]; their product is
    # the leverage distribution of the (excluded) Khatri-Rao product.
    Us = synth.gaussian_factors((6, 5, 7), 3, seed=5, heavy_entries_frac=0.05)
    rng = np.random.default_rng(7)
    multi = np.stack([rng.integers(0, U.shape[0], 40) for U in Us], axis=1)
    assert check_thm31_product(Us, exclude, multi) < 1e-10


def test_two_stage_mixture_identity():
    # Section 3.2: q = sum_u w[u] W[:, u] / ||W[:, u]||_1 and the first-stage
    # distribution equals q_{h, sqrt(Lambda) V^T, G_k}.
    rng = np.random.default_rng(11)
    U = rng.standard_normal((30, 5))
    X = rng.standard_normal((40, 5))
    Ggt = X.T @ X                       # any p.s.d. matrix
    h = rng.standard_normal(5)
    q, C = dfn.conditional_q(h, U, Ggt)
    lam, V = np.linalg.eigh(Ggt)
    W = np.empty((30, 5))
    for u in range(5):
        W[:, u] = ((U * h) @ V[:, u]) ** 2      # <hh^T, U[t]^T U[t], v v^T>
    w = lam * W.sum(axis=0) / C
    mix = (W / W.sum(axis=0)) @ w
    np.testing.assert_allclose(mix, q, rtol=1e-12, atol=1e-15)
    first, _ = dfn.conditional_q(h, np.sqrt(lam)[:, None] * V.T, U.T @ U)
    np.testing.assert_allclose(first, w, rtol=1e-12, atol=1e-15)
    # second stage: q_{h (*) V[:, u], U, [1]} == W[:, u] / ||W[:, u]||_1
    for u in range(5):
        sec, _ = dfn.conditional_q(h * V[:, u], U, np.ones((5, 5)))
        np.testing.assert_allclose(sec, W[:, u] / W[:, u].sum(), rtol=1e-12, atol=1e-15)
