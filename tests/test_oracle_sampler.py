"""Method-level pins of the oracle sampler (CPU)."""
import json
import os

import numpy as np
import pytest
from scipy.stats import chisquare

import synth
from oracle import definition as dfn
from oracle import sampler as smp

from pins import check_prob_vs_qr, check_walk_vs_scan, flat_rows, krp_excluding

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _c1():
    cfg = synth.CONFIGS[1]
    Us = synth.gaussian_factors(cfg["dims"], cfg["R"], synth.config_seed(1))
    return cfg, Us


def test_segment_tree_shape_matches_paper_figure():
    g = json.load(open(os.path.join(GOLDEN, "segment_tree_T8_2.json")))
    U = np.eye(8)
    t = smp.SegmentTree(U, g["F"])
    assert t.D == len(g["levels"]) - 1
    for lev, segs in enumerate(g["levels"]):
        assert t.real(lev) == len(segs)
        for p, (a, b) in enumerate(segs):
            # U = I makes node p's Gram the indicator of its rows
            diag = np.diag(t.levels[lev][p])
            rows = np.nonzero(diag)[0] + 1
            assert rows.min() == a and rows.max() == b and len(rows) == b - a + 1


@pytest.mark.parametrize("I,F", [(37, 4), (64, 8), (5, 8), (1, 1), (33, 1), (100, 7)])
def test_every_node_is_the_gram_of_its_rows(I, F):
    rng = np.random.default_rng(I * 100 + F)
    U = rng.standard_normal((I, 3))
    t = smp.SegmentTree(U, F)
    np.testing.assert_allclose(t.root, U.T @ U, rtol=1e-13, atol=1e-12)
    for lev in range(t.D + 1):
        span = F << (t.D - lev)
        for p in range(t.real(lev)):
            seg = U[p * span: min((p + 1) * span, I)]
            np.testing.assert_allclose(t.levels[lev][p], seg.T @ seg, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("F", [1, 2, 3, 8, 64])
def test_tree_walk_equals_linear_scan_of_the_cdf(F):
    # inversion sampling: the walk must land in the same bin as a linear scan
    rng = np.random.default_rng(F)
    U = rng.standard_normal((53, 6))
    U[rng.integers(0, 53, 4)] *= 30
    t = smp.SegmentTree(U, F)
    H = rng.standard_normal((300, 6))
    d = synth.uniforms(300, 1, 99 + F)[:, 0, 0]
    assert check_walk_vs_scan(t, H, d) == 0.0
    # general p.s.d. Y as in the eigen-trees
    X = rng.standard_normal((9, 6))
    assert check_walk_vs_scan(t, H[:60], d[:60], Y=X.T @ X) == 0.0


def test_scalar_and_batched_row_sample_agree():
    rng = np.random.default_rng(5)
    U = rng.standard_normal((77, 5))
    t = smp.SegmentTree(U, 5)
    H = rng.standard_normal((50, 5))
    d = synth.uniforms(50, 1, 3)[:, 0, 0]
    rows, marg, _ = smp.row_sample_batch(t, H, None, d)
    for i in range(50):
        r, m = smp.row_sample(t, H[i], None, d[i])
        assert r == rows[i]
        assert abs(m - marg[i]) <= 1e-15 + 1e-12 * m


@pytest.mark.parametrize("exclude", [-1, 0, 2])
def test_draw_probabilities_equal_qr_leverage_c1(exclude):
    cfg, Us = _c1()
    S = smp.KRPSampler(Us)
    u = synth.uniforms(cfg["J"], 3, synth.uniform_seed(1) + exclude)
    err, dr, p, r = check_prob_vs_qr(S, Us, exclude, u)
    assert err < 1e-10
    np.testing.assert_allclose(S.row_prob(exclude, dr.idx), dr.prob, rtol=1e-12)
    # the returned row is the Hadamard product of the chosen factor rows
    A = krp_excluding(Us, exclude)
    np.testing.assert_allclose(dr.rows, A[r], rtol=1e-13, atol=1e-13)
    assert np.all(dr.idx[:, exclude] == -1) if exclude >= 0 else np.all(dr.idx >= 0)


def test_eigen_trees_reconstruct_g_greater_k():
    cfg, Us = _c1()
    S = smp.KRPSampler(Us)
    Gp, rank, eig, E = S.prepare(-1)
    assert rank == 8
    for k in range(3):
        later = [S.G[m] for m in range(3) if m > k]
        Ggt = Gp * dfn.hadamard_all(later) if later else Gp
        lam, V = eig[k]
        assert np.all(np.diff(lam) >= 0)
        np.testing.assert_allclose(E[k].root, Ggt, rtol=1e-12, atol=1e-12 * np.abs(Ggt).max())
        res = np.abs(Ggt @ V - V * lam).max()
        assert res <= 1e-12 * np.abs(Ggt).max()


def test_indices_do_not_depend_on_leaf_size():
    # the tie rule makes the drawn row a function of the CDF alone
    Us = synth.gaussian_factors((40, 33, 50), 4, seed=8, heavy_entries_frac=0.02)
    u = synth.uniforms(2000, 3, 17)
    ref = smp.KRPSampler(Us, F=4).draw(1, u)
    for F in (1, 3, 16, 64):
        dr = smp.KRPSampler(Us, F=F).draw(1, u)
        ok = (dr.idx == ref.idx).all(axis=1) | (np.minimum(dr.margin, ref.margin) < 1e-12)
        assert ok.all()


def test_rank_one_closed_form():
    # R = 1: A is a single column, leverage ~ prod_k U_k[i_k]^2
    Us = synth.gaussian_factors((9, 11, 7), 1, seed=9)
    S = smp.KRPSampler(Us)
    u = synth.uniforms(500, 3, 4)
    dr = S.draw(-1, u)
    ref = np.ones(500)
    for k, U in enumerate(Us):
        w = U[:, 0].astype(np.float64) ** 2
        ref *= w[dr.idx[:, k]] / w.sum()
    np.testing.assert_allclose(dr.prob, ref, rtol=1e-12)


def test_single_factor_is_plain_leverage():
    U = synth.gaussian_factors((200,), 6, seed=10, heavy_entries_frac=0.02)[0]
    S = smp.KRPSampler([U])
    u = synth.uniforms(400, 1, 5)
    dr = S.draw(-1, u)
    lev = dfn.leverage_qr(U.astype(np.float64))
    np.testing.assert_allclose(dr.prob, lev[dr.idx[:, 0]] / 6, rtol=1e-11)


def test_orthogonal_columns_closed_form():
    # G_k diagonal: l(i) = sum_r prod_k U_k[i_k, r]^2 / G_k[r, r]
    rng = np.random.default_rng(12)
    Us = []
    for I in (10, 12, 9):
        Q, _ = np.linalg.qr(rng.standard_normal((I, 4)))
        Us.append(Q * rng.uniform(0.5, 3.0, 4))
    S = smp.KRPSampler(Us)
    u = synth.uniforms(300, 3, 6)
    for exclude in (-1, 1):
        dr = S.draw(exclude, u)
        modes = [k for k in range(3) if k != exclude]
        lev = np.zeros(300)
        for r in range(4):
            term = np.ones(300)
            for k in modes:
                term *= Us[k][dr.idx[:, k], r] ** 2 / (Us[k][:, r] @ Us[k][:, r])
            lev += term
        np.testing.assert_allclose(dr.prob, lev / 4, rtol=1e-11)


def test_row_permutation_permutes_the_distribution():
    Us = synth.gaussian_factors((15, 13, 11), 3, seed=13)
    perm = np.random.default_rng(0).permutation(13)
    Up = [Us[0], Us[1][perm], Us[2]]
    S, Sp = smp.KRPSampler(Us), smp.KRPSampler(Up)
    idx = np.stack(np.meshgrid(np.arange(15), np.arange(13), np.arange(11),
                               indexing="ij"), -1).reshape(-1, 3)
    q = S.row_prob(-1, idx)
    idxp = idx.copy()
    idxp[:, 1] = np.argsort(perm)[idx[:, 1]]
    np.testing.assert_allclose(Sp.row_prob(-1, idxp), q, rtol=1e-11)


def test_column_scaling_leaves_the_distribution_unchanged():
    Us = synth.gaussian_factors((12, 10, 9), 4, seed=14)
    Ds = [U * np.array([2.0, 0.5, 3.0, 1.5]) for U in Us]
    S, Sd = smp.KRPSampler(Us), smp.KRPSampler(Ds)
    u = synth.uniforms(400, 3, 7)
    dr = Sd.draw(0, u)
    np.testing.assert_allclose(S.row_prob(0, dr.idx), dr.prob, rtol=1e-10)


def _chi2_groups(counts_by_row, p, groups):
    """Chi-square over ``groups`` equal-mass groups of rows sorted by p."""
    order = np.argsort(p)
    cum = np.cumsum(p[order])
    g = np.minimum((cum * groups / cum[-1]).astype(int), groups - 1)
    obs = np.bincount(g, weights=counts_by_row[order], minlength=groups)
    exp = np.bincount(g, weights=p[order], minlength=groups) * counts_by_row.sum()
    return chisquare(obs, exp).pvalue


def test_histograms_chi_square_c1():
    cfg, Us = _c1()
    S = smp.KRPSampler(Us)
    dims = cfg["dims"]
    pvals = []
    for exclude, groups in ((-1, 32), (0, 64)):
        u = synth.uniforms(cfg["J"], 3, synth.uniform_seed(1) + 10 + exclude)
        dr = S.draw(exclude, u)
        A = krp_excluding(Us, exclude)
        lev = dfn.leverage_qr(A)
        p = lev / lev.sum()
        r = flat_rows(dr.idx, dims, exclude)
        cnt = np.bincount(r, minlength=len(p)).astype(np.float64)
        pvals.append(_chi2_groups(cnt, p, groups))
        modes = [k for k in range(3) if k != exclude]
        pm = p.reshape([dims[k] for k in modes])
        for a, k in enumerate(modes):
            marg = pm.sum(axis=tuple(b for b in range(len(modes)) if b != a))
            obs = np.bincount(dr.idx[:, k], minlength=dims[k])
            pvals.append(chisquare(obs, marg * cfg["J"]).pvalue)
    # Bonferroni over the tests, fixed seeds
    assert min(pvals) > 1e-3 / len(pvals), pvals


def test_histogram_full_resolution_small_krp():
    # Appendix A.13 probability check: three 8x8 factors, 1% of entries x10,
    # true distribution vs a histogram of 50,000 draws
    Us = synth.gaussian_factors((8, 8, 8), 8, seed=2023, heavy_entries_frac=0.01)
    S = smp.KRPSampler(Us)
    u = synth.uniforms(50000, 3, 2024)
    dr = S.draw(-1, u)
    lev = dfn.leverage_qr(dfn.khatri_rao(Us))
    p = lev / lev.sum()
    r = flat_rows(dr.idx, (8, 8, 8), -1)
    cnt = np.bincount(r, minlength=512)
    assert chisquare(cnt, p * 50000).pvalue > 1e-3


@pytest.mark.parametrize("exclude", [-1, 1])
def test_two_stage_draw_equals_bruteforce_inversion(exclude):
    from pins import check_two_stage_vs_bruteforce
    Us = synth.gaussian_factors((20, 17, 23), 5, seed=60, heavy_entries_frac=0.02)
    u = synth.uniforms(500, 3, 61 + exclude)
    assert check_two_stage_vs_bruteforce(smp.KRPSampler(Us), Us, exclude, u) == 0.0
    assert check_two_stage_vs_bruteforce(smp.KRPSampler(Us, F=2), Us, exclude, u) == 0.0


class _Perturbed(smp.KRPSampler):
    """Every stored node entry of the factor trees and eigen-trees and every
    eigenvector entry multiplied by (1 + e), |e| <= u (symmetric in the
    node's two indices, as a packed triangle is stored): the rounding a
    storage precision with unit roundoff u applies."""

    def __init__(self, Us, u, seed):
        self.u = u
        self.rng = np.random.default_rng(seed)
        super().__init__(Us)

    def _jitter(self, a):
        e = self.rng.uniform(-self.u, self.u, a.shape)
        if a.ndim == 3:
            e = np.triu(e) + np.swapaxes(np.triu(e, 1), 1, 2)
        return a * (1.0 + e)

    def refresh(self, j, U=None):
        super().refresh(j, U)
        self.Z[j].levels = [self._jitter(lv) for lv in self.Z[j].levels]

    def prepare(self, exclude):
        Gp, rank, eig, E = super().prepare(exclude)
        for k in E:
            E[k].levels = [self._jitter(lv) for lv in E[k].levels]
            lam, V = eig[k]
            eig[k] = (lam, self._jitter(V))
        return Gp, rank, eig, E


@pytest.mark.parametrize("dims,R,heavy", [((300, 200, 100), 16, 0.01), ((777, 260), 64, 0.0),
                                          ((2000, 50, 900), 8, 0.05)])
def test_scaled_margin_bounds_the_effect_of_storage_rounding(dims, R, heavy):
    """A draw changes under a relative rounding of at most u of every stored
    node entry and eigenvector entry only if its scaled margin is at most u
    (the scale is the rounding's effect on the comparison per unit u); at
    u = 1e-5 or 1e-3 draws do change, so the bound is not vacuous."""
    Us = synth.gaussian_factors(dims, R, seed=70 + R, heavy_rows_frac=heavy)
    u01 = synth.uniforms(3000, len(dims), 71)
    ex = 0
    a = smp.KRPSampler(Us).draw(ex, u01, scaled=True)
    changed = 0
    for u, seed in ((2.0 ** -24, 1), (1e-5, 2), (1e-3, 3), (1e-3, 4)):
        b = _Perturbed(Us, u, seed).draw(ex, u01)
        diff = ~(a.idx == b.idx).all(axis=1)
        assert np.all(a.smargin[diff] <= u), (u, a.smargin[diff].max() / u)
        changed += int(diff.sum())
        # the probabilities of unchanged draws move by the rounding only
        same = ~diff
        np.testing.assert_allclose(b.prob[same], a.prob[same], rtol=1e-12)
    assert changed > 0


def test_scaled_margin_effect_of_one_node():
    # a one-level tree walked with h = 1: the only comparison is x against
    # the left leaf's mass, and its effect is 4 sqrt of the squared packed
    # terms of the root (times d) and of the left leaf
    rng = np.random.default_rng(3)
    U = rng.standard_normal((8, 3))
    t = smp.SegmentTree(U, 4)
    H = np.ones((1, 3))
    d = np.array([0.37])
    _, m, sm = smp.row_sample_batch(t, H, None, d, scaled=True)

    def ss(G):
        iu = np.triu_indices(3)
        w = np.where(iu[0] == iu[1], 1.0, 2.0)
        return float(((w * G[iu]) ** 2).sum())

    C = t.root.sum()
    x = d[0] * C
    cut = t.levels[1][0].sum()
    E = 4 * np.sqrt(d[0] ** 2 * ss(t.root) + ss(t.levels[1][0]))
    # the leaf scan also compares within the chosen leaf; the tree level's
    # comparison is one of the candidates for the minimum
    assert sm[0] <= abs(x - cut) / E * (1 + 1e-12)
    r2, m2, sm2 = smp.row_sample_batch(t, H, None, d)
    assert np.all(np.isinf(sm2)) and np.array_equal(m, m2)


def test_degenerate_flags_mark_only_draws_inside_a_cluster():
    """With orthogonal factor columns of equal norms every G_k is a multiple
    of the identity, so every G_{>k} has one eigenvalue cluster and every
    draw is degenerate; with distinct column norms no draw is."""
    rng = np.random.default_rng(9)
    Q = [np.linalg.qr(rng.standard_normal((40, 4)))[0] for _ in range(3)]
    u01 = synth.uniforms(500, 3, 10)
    flat = smp.KRPSampler(Q).draw(-1, u01)
    assert flat.degenerate.all()
    scaled = [q * np.array([1.0, 2.0, 3.0, 4.0]) for q in Q]
    dr = smp.KRPSampler(scaled).draw(-1, u01)
    assert not dr.degenerate.any()


def _tree_err(t, ref):
    """Largest |node - rebuilt node| over every level, relative to the
    largest diagonal of the rebuilt node."""
    worst = 0.0
    for lev in range(ref.D + 1):
        a, b = t.levels[lev], ref.levels[lev]
        assert a.shape == b.shape
        scale = np.abs(np.diagonal(b, axis1=1, axis2=2)).max(axis=1)[:, None, None] + 1e-300
        worst = max(worst, float((np.abs(a - b) / scale).max()))
    return worst


def _updates(I, R, n, seed):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, I, n)
    rows[: 3] = [0, I - 1, I - 1]          # first row, the ragged last leaf, twice
    cols = rng.integers(0, R, n)
    vals = rng.standard_normal(n) * 3.0
    vals[5] = 0.0                          # an entry set to zero
    return rows, cols, vals


@pytest.mark.parametrize("I,R,F", [(103, 5, 5), (64, 8, 1), (1000, 16, 7), (1, 3, 4)])
def test_entry_update_equals_rebuild(I, R, F):
    """Algorithm 5 (Appendix A.7): after single-entry updates every node of
    the tree equals the Gram of its rows recomputed from the updated factor,
    and nodes whose segment does not hold an updated row are untouched."""
    U = synth.gaussian_factors((I,), R, seed=I + R)[0].astype(np.float64)
    t = smp.SegmentTree(U, F)
    before = [lv.copy() for lv in t.levels]
    rows, cols, vals = _updates(I, R, 40, seed=I)
    U2 = U.copy()
    for r, c, v in zip(rows, cols, vals):
        t.update_entry(int(r), int(c), float(v))
        U2[r, c] = v
    assert np.array_equal(t.U, U2)
    assert np.array_equal(U, synth.gaussian_factors((I,), R, seed=I + R)[0])  # caller's copy kept
    ref = smp.SegmentTree(U2, F)
    assert _tree_err(t, ref) <= 1e-12
    touched = set()
    for r in rows:
        pos = int(r) // F
        for lev in range(t.D, -1, -1):
            touched.add((lev, pos))
            pos //= 2
    for lev in range(t.D + 1):
        for p in range(t.real(lev)):
            if (lev, p) not in touched:
                assert np.array_equal(t.levels[lev][p], before[lev][p])


def test_entry_update_draws_equal_a_fresh_sampler():
    Us = synth.gaussian_factors((300, 200, 100), 8, seed=91, heavy_rows_frac=0.01)
    S = smp.KRPSampler(Us)
    Us2 = [U.astype(np.float64).copy() for U in Us]
    for j in range(3):
        rows, cols, vals = _updates(len(Us[j]), 8, 25, seed=92 + j)
        for r, c, v in zip(rows, cols, vals):
            S.update_entry(j, int(r), int(c), float(v))
            Us2[j][r, c] = v
    fresh = smp.KRPSampler(Us2)
    u = synth.uniforms(2000, 3, 93)
    for exclude in (-1, 1):
        a, b = S.draw(exclude, u), fresh.draw(exclude, u)
        diff = ~(a.idx == b.idx).all(axis=1)
        assert np.all(b.margin[diff] <= 1e-10)
        np.testing.assert_allclose(a.prob[~diff], b.prob[~diff], rtol=1e-10)


def test_entry_update_without_the_square_term_is_caught():
    """Planted mistake: dropping Algorithm 5's delta^2 on the diagonal (or
    using the new row for the cross terms) is seen by the rebuild pin."""
    U = synth.gaussian_factors((50,), 6, seed=5)[0].astype(np.float64)

    class NoSquare(smp.SegmentTree):
        def update_entry(self, r, c, value):
            d = float(value) - self.U[r, c]
            super().update_entry(r, c, value)
            pos = r // self.F
            for lev in range(self.D, -1, -1):
                self.levels[lev][pos][c, c] -= d * d
                pos //= 2

    t = NoSquare(U, 6)
    for r, c, v in zip(*_updates(50, 6, 10, seed=6)):
        t.update_entry(int(r), int(c), float(v))
    U2 = t.U
    assert _tree_err(t, smp.SegmentTree(U2, 6)) > 1e-3
