"""Pins of the least-squares accuracy oracle (Section 4.2, Appendix A.12)
against the materialised problem on tiny inputs."""
import numpy as np

import synth
from oracle import accuracy as acc
from oracle import cp as ocp
from oracle import definition as dfn
from oracle import sampler as smp


def _tiny(N=3, I=12, R=4, seed=5):
    Us = synth.gaussian_factors((I,) * N, R, seed=seed, heavy_entries_frac=0.01)
    rng = np.random.default_rng(seed + 1)
    cs = [rng.standard_normal(I) for _ in range(N)]
    return Us, cs


def test_gram_identities_equal_the_materialised_problem():
    Us, cs = _tiny()
    P = acc.KronProblem(Us, cs)
    A = dfn.khatri_rao(Us)
    b = cs[0]
    for c in cs[1:]:
        b = np.kron(b, c)
    np.testing.assert_allclose(P.G, A.T @ A, rtol=1e-12)
    np.testing.assert_allclose(P.Atb, A.T @ b, rtol=1e-12)
    assert abs(P.bb - b @ b) <= 1e-12 * (b @ b)
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    np.testing.assert_allclose(P.x_opt, x, rtol=1e-9)
    assert abs(P.r_opt - np.linalg.norm(A @ x - b)) <= 1e-10 * np.linalg.norm(b)
    y = x + 0.1
    assert abs(P.residual(y) - np.linalg.norm(A @ y - b)) <= 1e-10 * np.linalg.norm(b)
    assert P.epsilon(x) < 1e-10
    # rows and entries at given multi-indices
    idx = np.array([[1, 2, 3], [0, 0, 11]])
    r = np.ravel_multi_index(idx.T, (12, 12, 12))
    np.testing.assert_allclose(P.rows(idx), A[r], rtol=1e-14)
    np.testing.assert_allclose(P.b_entries(idx), b[r], rtol=1e-14)


def test_distortion_equals_the_condition_number_of_s_q():
    """kappa(S Q) - 1 with Q from a QR of the materialised A (the
    definition) against the Gram route of Appendix A.12."""
    Us, cs = _tiny(N=3, I=10, R=5, seed=8)
    S = smp.KRPSampler(Us)
    dr = S.draw(-1, synth.uniforms(400, 3, 9))
    A = dfn.khatri_rao(Us)
    Q, _ = np.linalg.qr(A)
    r = np.ravel_multi_index(dr.idx.T, (10, 10, 10))
    SQ = Q[r] / np.sqrt(400 * dr.prob)[:, None]
    s = np.linalg.svd(SQ, compute_uv=False)
    ref = s[0] / s[-1] - 1
    got = acc.distortion(A.T @ A, dr.rows, dr.prob)
    assert abs(got - ref) <= 1e-9 * (1 + ref)
    # a sketch that takes every row once with weight 1 has no distortion
    full = np.arange(1000)
    got0 = acc.distortion(A.T @ A, A[full], np.full(1000, 1.0 / 1000))
    assert got0 < 1e-10


def test_leverage_sketch_residual_error_is_small():
    """Theorem 2.1's regime: with J >> R the sketched solution's residual is
    within a few percent of the optimum (and the oracle's sketched solve
    gives the x it is measured on)."""
    Us, cs = _tiny(N=4, I=16, R=6, seed=11)
    P = acc.KronProblem(Us, cs)
    S = smp.KRPSampler(Us)
    eps = []
    for t in range(4):
        dr = S.draw(-1, synth.uniforms(2000, 4, 20 + t))
        x = ocp.sketched_lstsq(dr.rows, dr.prob, P.b_entries(dr.idx)[:, None])[:, 0]
        eps.append(P.epsilon(x))
    assert 0 <= min(eps) and np.mean(eps) < 0.03, eps
