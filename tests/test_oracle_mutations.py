"""Planted mistakes in the oracle must be caught by the pins (CPU only).

Each test breaks the oracle in a plausible way (a dropped term, a wrong
index, a transposed operand, a misread line of the paper) and checks that
one of the pin checks then reports a large error.
"""
import numpy as np

import synth
from oracle import cp
from oracle import definition as dfn
from oracle import sampler as smp

from pins import check_prob_vs_qr, check_two_stage_vs_bruteforce, check_walk_vs_scan


def _problem():
    Us = synth.gaussian_factors((10, 9, 8), 4, seed=77, heavy_entries_frac=0.03)
    u = synth.uniforms(400, 3, 78)
    return Us, u


class _GeqK(smp.KRPSampler):
    """Uses G_{>=k} (includes G_k itself) instead of G_{>k}."""

    def prepare(self, exclude):
        Gp, rank, eig, E = super().prepare(exclude)
        modes = self.modes(exclude)
        for k in modes:
            later = [self.G[m] for m in modes if m >= k]
            Ggt = Gp * dfn.hadamard_all(later)
            lam, V = np.linalg.eigh(Ggt)
            lam = np.maximum(lam, 0)
            eig[k] = (lam, V)
            E[k] = smp.SegmentTree(np.sqrt(lam)[:, None] * V.T, 1)
        return Gp, rank, eig, E


class _EigRowsNotColumns(smp.KRPSampler):
    """Builds E_k over sqrt(Lambda) V (rows of V) instead of sqrt(Lambda) V^T."""

    def prepare(self, exclude):
        Gp, rank, eig, E = super().prepare(exclude)
        for k, (lam, V) in eig.items():
            E[k] = smp.SegmentTree(np.sqrt(lam)[:, None] * V, 1)
        return Gp, rank, eig, E


def test_g_greater_or_equal_k_is_caught():
    Us, u = _problem()
    assert check_two_stage_vs_bruteforce(smp.KRPSampler(Us), Us, -1, u) == 0.0
    assert check_two_stage_vs_bruteforce(_GeqK(Us), Us, -1, u) > 0.05


def test_transposed_eigenvector_matrix_is_caught():
    Us, u = _problem()
    assert check_two_stage_vs_bruteforce(_EigRowsNotColumns(Us), Us, -1, u) > 0.05
    # the probabilities q_d are computed from the chosen rows, so they stay
    # exact; the histogram of the draws is what moves.  Compare the draw's
    # empirical distribution with the true one on many draws.
    S = _EigRowsNotColumns(Us)
    big = synth.uniforms(20000, 3, 79)
    dr = S.draw(-1, big)
    lev = dfn.leverage_qr(dfn.khatri_rao(Us))
    p = lev / lev.sum()
    r = np.ravel_multi_index(dr.idx.T, (10, 9, 8))
    cnt = np.bincount(r, minlength=len(p)) / 20000
    tv = 0.5 * np.abs(cnt - p).sum()
    good = smp.KRPSampler(Us).draw(-1, big)
    rg = np.ravel_multi_index(good.idx.T, (10, 9, 8))
    tv_good = 0.5 * np.abs(np.bincount(rg, minlength=len(p)) / 20000 - p).sum()
    assert tv > 2 * tv_good


def test_leaf_scan_off_by_one_is_caught(monkeypatch):
    orig = smp._row_sample_chunk

    def shifted(tree, H, Y, dvec, scaled=False, vround=False):
        rows, m, sm = orig(tree, H, Y, dvec, scaled, vround)
        return np.minimum(rows + 1, tree.I - 1), m, sm

    monkeypatch.setattr(smp, "_row_sample_chunk", shifted)
    rng = np.random.default_rng(3)
    U = rng.standard_normal((40, 5))
    t = smp.SegmentTree(U, 5)
    H = rng.standard_normal((100, 5))
    d = synth.uniforms(100, 1, 4)[:, 0, 0]
    assert check_walk_vs_scan(t, H, d) > 0.5


def test_walk_without_low_update_is_caught(monkeypatch):
    def no_low(tree, H, Y, dvec, scaled=False, vround=False):
        n, R = H.shape
        HH = H[:, :, None] * H[:, None, :]
        C = np.einsum("dab,ab->d", HH, tree.root)
        x = dvec * C
        pos = np.zeros(n, dtype=np.int64)
        for lev in range(1, tree.D + 1):
            left = 2 * pos
            mL = np.einsum("dab,dab->d", tree.levels[lev][left], HH)
            go_left = (mL >= x) | ((left + 1) >= tree.real(lev))   # "low" dropped
            pos = np.where(go_left, left, left + 1)
        s0 = pos * tree.F
        return np.minimum(s0, tree.I - 1), np.ones(n), np.full(n, np.inf)

    monkeypatch.setattr(smp, "_row_sample_chunk", no_low)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((64, 4))
    t = smp.SegmentTree(U, 4)
    H = rng.standard_normal((100, 4))
    d = synth.uniforms(100, 1, 6)[:, 0, 0]
    assert check_walk_vs_scan(t, H, d) > 0.2


def test_missing_rank_normalisation_is_caught():
    Us, u = _problem()

    class NoRank(smp.KRPSampler):
        def draw(self, exclude, u01):
            dr = super().draw(exclude, u01)
            dr.prob = dr.prob * dr.rank
            return dr

    err, *_ = check_prob_vs_qr(NoRank(Us), Us, -1, u)
    assert err > 1.0


def test_fiber_of_the_wrong_mode_is_caught(monkeypatch):
    # selecting fibers by the modes including j would break (SB)^T SA
    dims = (6, 5, 4)
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    idx = np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.int32)
    val = np.random.default_rng(0).lognormal(size=idx.shape[0]).astype(np.float32)
    T = cp.SparseTensor(dims, idx, val)
    Us = synth.gaussian_factors(dims, 3, seed=5)
    S = smp.KRPSampler(Us)
    dr = S.draw(1, synth.uniforms(200, 3, 6))
    w2 = 1 / (200 * dr.prob)
    _, Y_good = cp.normal_equations(T, 1, dr.idx, dr.rows, w2)
    monkeypatch.setattr(cp.SparseTensor, "others", lambda self, j: [k for k in range(self.N) if k != (j + 1) % self.N])
    T2 = cp.SparseTensor(dims, idx, val)
    try:
        _, Y_bad = cp.normal_equations(T2, 1, np.maximum(dr.idx, 0), dr.rows, w2)
    except Exception:
        return
    assert np.abs(Y_bad - Y_good).max() > 1e-3 * np.abs(Y_good).max()
