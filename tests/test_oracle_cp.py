"""Pins of the sketched least-squares / CP-ALS oracle (CPU)."""
import numpy as np
import pytest

import synth
from oracle import cp
from oracle import definition as dfn
from oracle import sampler as smp


def _dense(tensor):
    T = np.zeros(tensor.dims)
    np.add.at(T, tuple(tensor.idx.T), tensor.val)
    return T


def _mat_t(T, j):
    """``mat(T, j)^T``: row u = sum_{k != j} i_k prod_{m < k, m != j} I_m
    (Appendix A.9, matricisation), i.e. the first other mode varies fastest."""
    Tm = np.moveaxis(T, j, -1)
    return Tm.reshape(-1, T.shape[j], order="F")


def _u_neq_j(Us, j):
    """``U_{!=j} = U_N (.) ... (.) U_1`` without ``U_j`` (reversed order)."""
    return dfn.khatri_rao([Us[k] for k in reversed(range(len(Us))) if k != j])


def _tiny_tensor(seed=0, dup=True):
    dims = (12, 10, 8)
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    idx = np.stack([g.reshape(-1) for g in grids], axis=1)
    val = rng.lognormal(size=idx.shape[0])
    if dup:                     # duplicates mean a sum
        extra = rng.integers(0, idx.shape[0], 200)
        idx = np.concatenate([idx, idx[extra]])
        val = np.concatenate([val, rng.standard_normal(200)])
    return cp.SparseTensor(dims, idx.astype(np.int32), val.astype(np.float32))


@pytest.mark.parametrize("j", [0, 1, 2])
def test_sketched_normal_equations_equal_explicit_sampling_matrix(j):
    T = _tiny_tensor()
    Ts = _dense(T)
    Us = synth.gaussian_factors(T.dims, 4, seed=21)
    S = smp.KRPSampler(Us)
    u = synth.uniforms(300, 3, 22 + j)
    dr = S.draw(j, u)
    Jn = 300
    w2 = 1.0 / (Jn * dr.prob)
    M, Y = cp.normal_equations(T, j, dr.idx, dr.rows, w2)
    A = _u_neq_j(Us, j)
    B = _mat_t(Ts, j)
    others = [k for k in range(3) if k != j]
    u_row = np.zeros(Jn, dtype=np.int64)
    stride = 1
    for k in others:
        u_row += dr.idx[:, k] * stride
        stride *= T.dims[k]
    Smat = np.zeros((Jn, A.shape[0]))
    Smat[np.arange(Jn), u_row] = 1.0 / np.sqrt(Jn * dr.prob)
    SA, SB = Smat @ A, Smat @ B
    np.testing.assert_allclose(M, SA.T @ SA, rtol=1e-12, atol=1e-12 * np.abs(M).max())
    np.testing.assert_allclose(Y, SB.T @ SA, rtol=1e-11, atol=1e-12 * np.abs(Y).max())


@pytest.mark.parametrize("j", [0, 2])
def test_full_enumeration_gives_the_exact_als_step(j):
    T = _tiny_tensor(1)
    Us = synth.gaussian_factors(T.dims, 4, seed=23)
    A = _u_neq_j(Us, j)
    B = _mat_t(_dense(T), j)
    others = [k for k in range(3) if k != j]
    grids = np.meshgrid(*[np.arange(T.dims[k]) for k in reversed(others)], indexing="ij")
    idx = np.zeros((A.shape[0], 3), dtype=np.int64) - 1
    for g, k in zip(grids, reversed(others)):
        idx[:, k] = g.reshape(-1)
    rows = np.ones((A.shape[0], 4))
    for k in others:
        rows *= Us[k][idx[:, k]]
    M, Y = cp.normal_equations(T, j, idx, rows, np.ones(A.shape[0]))
    Mp, _ = dfn.pinv_psd(M)
    X = Y @ Mp
    Xref = np.linalg.lstsq(A, B, rcond=None)[0].T
    np.testing.assert_allclose(X, Xref, rtol=1e-9, atol=1e-11 * np.abs(Xref).max())


def test_fit_equals_dense_definition():
    T = _tiny_tensor(2)
    Us = synth.gaussian_factors(T.dims, 3, seed=24)
    Us = [cp.normalize_columns(U)[0] for U in Us]
    sigma = np.array([2.0, 0.5, 1.25])
    f = cp.fit(T, Us, sigma)
    That = np.einsum("r,ir,jr,kr->ijk", sigma, *Us)
    Td = _dense(T)
    ref = 1 - np.linalg.norm(That - Td) / np.linalg.norm(Td)
    assert abs(f - ref) < 1e-13


def test_duplicates_are_summed():
    T = _tiny_tensor(3)
    Td = _dense(T)
    assert abs(T.norm2 - (Td ** 2).sum()) < 1e-10 * T.norm2


def test_planted_exact_rank_tensor_is_recovered():
    idx, val, _ = synth.planted_cp_tensor((14, 12, 10), 3, seed=31)
    T = cp.SparseTensor((14, 12, 10), idx, val)
    U0 = synth.gaussian_factors(T.dims, 3, seed=32)
    _, _, fits = cp.cp_als(T, U0, 30, lambda s, j: synth.uniforms(400, 3, 1000 * s + j))
    assert fits[-1] >= 0.999, fits


def test_leverage_sketch_meets_the_residual_guarantee():
    # Theorem 2.1 regime on the least-squares experiment of Section 4.2
    # (Gaussian factors with 1% of entries x10, b = c_1 (x) c_2 (x) c_3)
    Us = synth.gaussian_factors((16, 16, 16), 6, seed=41, heavy_entries_frac=0.01)
    rng = np.random.default_rng(42)
    c = [rng.standard_normal(16) for _ in range(3)]
    A = dfn.khatri_rao(Us)
    b = np.kron(np.kron(c[0], c[1]), c[2])
    x_opt = np.linalg.lstsq(A, b, rcond=None)[0]
    r_opt = np.linalg.norm(A @ x_opt - b)
    S = smp.KRPSampler(Us)
    eps = []
    for t in range(5):
        dr = S.draw(-1, synth.uniforms(1500, 3, 43 + t))
        r = np.ravel_multi_index(dr.idx.T, (16, 16, 16))
        w = 1 / np.sqrt(1500 * dr.prob)
        x = np.linalg.lstsq(A[r] * w[:, None], b[r] * w, rcond=None)[0]
        eps.append(np.linalg.norm(A @ x - b) / r_opt - 1)
    assert np.mean(eps) < 0.05, eps


def test_sketched_lstsq_full_enumeration_is_exact_least_squares():
    """Every row of A once with q = 1/I (so w = 1): the sketched normal
    equations are the exact ones, and X equals the textbook least-squares
    solution; listing every row twice with q = 1/(2I) changes nothing."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((60, 5))
    B = rng.standard_normal((60, 3))
    X = cp.sketched_lstsq(A, np.full(60, 1 / 60), B)
    ref = np.linalg.lstsq(A, B, rcond=None)[0]
    np.testing.assert_allclose(X, ref, rtol=1e-10, atol=1e-12)
    X2 = cp.sketched_lstsq(np.vstack([A, A]), np.full(120, 1 / 120), np.vstack([B, B]))
    np.testing.assert_allclose(X2, ref, rtol=1e-10, atol=1e-12)


def test_sketched_lstsq_weights_follow_the_probabilities():
    """Halving one sample's probability doubles its weight w^2: the result
    equals the exact weighted least-squares solution with those weights."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((40, 4))
    B = rng.standard_normal((40, 2))
    q = rng.uniform(0.5, 1.5, 40)
    q /= q.sum()
    X = cp.sketched_lstsq(A, q, B)
    w = np.sqrt(1.0 / (40 * q))
    ref = np.linalg.lstsq(A * w[:, None], B * w[:, None], rcond=None)[0]
    np.testing.assert_allclose(X, ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("j", [0, 1, 2])
def test_exact_solve_equals_dense_least_squares(j):
    """The exact step without the Khatri-Rao product formed equals the
    dense least-squares solution on the materialised matricisation
    (min_X ||U_{!=j} X^T - mat(T, j)^T||, the definition), normalised."""
    T = _tiny_tensor(4)
    Us = synth.gaussian_factors(T.dims, 4, seed=25 + j)
    Unew, sigma, Y, M = cp.exact_solve(T, Us, j)
    A = _u_neq_j(Us, j)
    B = _mat_t(_dense(T), j)
    Xref = np.linalg.lstsq(A, B, rcond=None)[0].T
    ref, sref = cp.normalize_columns(Xref)
    np.testing.assert_allclose(sigma, sref, rtol=1e-9)
    np.testing.assert_allclose(Unew, ref, rtol=1e-9, atol=1e-11)
    # and the MTTKRP is mat(T, j) times the materialised Khatri-Rao product
    np.testing.assert_allclose(Y, B.T @ A, rtol=1e-12, atol=1e-12 * np.abs(Y).max())


def test_exact_als_recovers_a_planted_tensor_monotonically():
    idx, val, _ = synth.planted_cp_tensor((14, 12, 10), 3, seed=31)
    T = cp.SparseTensor((14, 12, 10), idx, val)
    U0 = synth.gaussian_factors((14, 12, 10), 3, seed=32)
    _, _, fits = cp.exact_als(T, U0, 40)
    assert fits[-1] >= 0.9999
    # an exact step never increases the residual of the problem it solves:
    # the fit after each sweep does not fall
    assert np.all(np.diff(fits) >= -1e-12)
