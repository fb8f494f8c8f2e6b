"""GPU parity of the sampler path (tree build, per-draw preparation, descent)
against the float64 oracle, through the C ABI.  Run with ``-m gpu``."""
import numpy as np
import pytest

import synth
from oracle import definition as dfn
from oracle import sampler as osmp
from parity import compare, report

pytestmark = pytest.mark.gpu

TOL_NODE = {"fp64": 1e-12, "fp32": 1e-5, "bf16x2": 1e-5}
# q_d = a G^+ a^T / rank in float64 from the stored factor rows and the
# float64 Grams (exact products of float32 factors for FP32 and the split
# path): only the summation order differs from the oracle
TOL_PROB = {"fp64": 1e-10, "fp32": 1e-9, "bf16x2": 1e-9}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2301_12584_amd as krps
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = krps.Context(0)
    return krps, torch, ctx


def to_dev(torch, ctx, arrs, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    return [torch.from_numpy(np.asarray(a, dtype=np.float64)).to(ctx.device, dt).contiguous()
            for a in arrs]


def stored_nodes(tree):
    """Oracle tree in the library's storage order: root, then per level the
    left children; packed upper triangles (row-major)."""
    iu = np.triu_indices(tree.R)
    out = [tree.root[iu]]
    for lev in range(1, tree.D + 1):
        for p in range(0, tree.real(lev), 2):
            out.append(tree.levels[lev][p][iu])
    return np.array(out)


def node_scale(tree_nodes_packed, R):
    """max |diagonal| of each stored node (bounds every entry of a Gram)."""
    iu = np.triu_indices(R)
    diag = iu[0] == iu[1]
    return np.abs(tree_nodes_packed[:, diag]).max(axis=1)


SHAPES = [((64, 64, 64), 8, 0), ((1000, 333, 77), 16, 0), ((5000, 2049, 700), 32, 0),
          ((3001, 1500), 64, 0), ((777, 260), 128, 0), ((100, 37, 45), 8, 3),
          ((50, 40), 32, 1), ((1, 5, 9), 4, 0), ((10, 20), 48, 100)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
@pytest.mark.parametrize("dims,R,F", SHAPES)
def test_tree_nodes_match_oracle(env, prec, dims, R, F):
    krps, torch, ctx = env
    print(f"tree {prec} dims={dims} R={R} F={F}", flush=True)
    Us = synth.gaussian_factors(dims, R, seed=sum(dims) + R, heavy_rows_frac=0.01)
    S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec, F=F)
    torch.cuda.synchronize()
    for j, U in enumerate(Us):
        t = osmp.SegmentTree(U, F or R)
        ref = stored_nodes(t)
        got = S.tree_nodes(j).cpu().numpy().astype(np.float64)
        assert got.shape == ref.shape
        scale = node_scale(ref, R)[:, None] + 1e-300
        err = np.abs(got - ref) / scale
        assert err.max() <= TOL_NODE[prec], (j, err.max())
        G = S.gram(j).cpu().numpy()
        Gref = U.astype(np.float64).T @ U
        assert np.abs(G - Gref).max() <= TOL_NODE[prec] * np.abs(np.diag(Gref)).max()


PREP = [((64, 50, 70), 8), ((3000, 2500, 2000), 64), ((900, 700, 500), 128)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,R", PREP)
@pytest.mark.parametrize("exclude", [-1, 0, 2])
def test_prep_matches_oracle(env, prec, dims, R, exclude):
    """G^+, rank, eigenvalues, eigenvectors (isolated eigenvalues; the
    projector onto a cluster otherwise) and the eigen-trees with G_k folded
    in, against the oracle's preparation."""
    krps, torch, ctx = env
    print(f"prep {prec} dims={dims} R={R} exclude={exclude}", flush=True)
    Us = synth.gaussian_factors(dims, R, synth.config_seed(1) + R)
    S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec)
    u = torch.from_numpy(synth.uniforms(16, 3, 1)).to(ctx.device)
    S.sample(exclude, u)
    torch.cuda.synchronize()
    parts = {k: (v.cpu() if hasattr(v, "cpu") else v) for k, v in S.draw_parts().items()}
    ref = osmp.KRPSampler(Us)
    Gp, rank, eig, E = ref.prepare(exclude)
    # float32 storage only rounds the eigenvectors and the eigen-tree nodes
    rtol = 1e-10 if prec == "fp64" else 1e-6
    assert parts["rank"] == rank
    assert np.abs(parts["gplus"].numpy() - Gp).max() <= 1e-10 * np.abs(Gp).max()
    iu = np.triu_indices(R)
    for k in ref.modes(exclude):
        lam, V = eig[k]
        assert np.abs(parts["lam"][k].numpy() - lam).max() <= 1e-10 * lam.max()
        Vg = parts["vecs"][k].numpy().astype(np.float64).T     # columns = eigenvectors
        gaps = np.diff(lam)
        iso = np.ones(R, dtype=bool)
        iso[1:] &= gaps > 1e-6 * lam.max()
        iso[:-1] &= gaps > 1e-6 * lam.max()
        dots = np.abs(np.einsum("eu,eu->u", Vg, V))
        assert np.abs(dots[iso] - 1).max() <= (1e-9 if prec == "fp64" else 1e-6)
        # the whole decomposition: sum_u lam_u v_u v_u^T = G_{>k}
        rec = (Vg * lam) @ Vg.T
        ggt = (V * lam) @ V.T
        assert np.abs(rec - ggt).max() <= rtol * 10 * np.abs(ggt).max()
        Eref = [E[k].root * ref.G[k]]
        for lev in range(1, E[k].D + 1):
            for p in range(0, E[k].real(lev), 2):
                Eref.append(E[k].levels[lev][p] * ref.G[k])
        Eref = np.array([m[iu] for m in Eref])
        Eg = parts["etree"][k].numpy().astype(np.float64)
        if iso.all():
            assert np.abs(Eg - Eref).max() <= rtol * 10 * np.abs(Eref).max()
        else:
            assert np.abs(Eg[0] - Eref[0]).max() <= rtol * 10 * np.abs(Eref).max()


def test_pseudo_inverse_routes(env):
    """Full-rank G takes the Cholesky route (Jacobi sweep count 0, rank R);
    a column repeated in every factor makes G singular, which must take the
    eigen route (rank R - 1); both match the oracle's eigendecomposition
    pseudo-inverse."""
    krps, torch, ctx = env
    R = 8
    base = synth.gaussian_factors((64, 50, 70), R, seed=41)
    rep = [U.copy() for U in base]
    for U in rep:
        U[:, 1] = U[:, 0]
    for Us, want_rank, cholesky in ((base, R, True), (rep, R - 1, False)):
        S = krps.Sampler(ctx, to_dev(torch, ctx, Us, "fp64"), precision="fp64")
        S.sample(-1, torch.from_numpy(synth.uniforms(16, 3, 2)).to(ctx.device))
        torch.cuda.synchronize()
        parts = S.draw_parts()
        Gp, rank, _, _ = osmp.KRPSampler(Us).prepare(-1)
        assert parts["rank"] == rank == want_rank
        assert (parts["sweeps"][0] == 0) == cholesky
        Gg = parts["gplus"].cpu().numpy()
        assert np.abs(Gg - Gp).max() <= 1e-9 * np.abs(Gp).max()


def _compare_draw(krps, torch, ctx, Us, prec, exclude, J, useed, F=0):
    S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec, F=F)
    u01 = synth.uniforms(J, len(Us), useed)
    idx, prob, rows = S.sample(exclude, torch.from_numpy(u01).to(ctx.device), rows=True,
                               check_status=True)
    torch.cuda.synchronize()
    # the plain float64 oracle over the same (float32) factors
    ref = osmp.KRPSampler(Us, F=F or None)
    dr = ref.draw(exclude, u01, scaled=prec != "fp64")
    idx = idx.cpu().numpy().astype(np.int64)
    c = compare(idx, dr, prec)
    same = c["same"]
    rel = np.abs(prob.cpu().numpy()[same] - dr.prob[same]) / dr.prob[same]
    return S, idx, prob, rows, dr, c, rel


CASES = [((64, 64, 64), 8, 4096), ((1000, 333, 77), 16, 2048), ((5000, 2049, 700), 32, 2048),
         ((3001, 1500, 64), 64, 1024), ((777, 260), 128, 512), ((129, 1, 33), 8, 512)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,R,J", CASES)
def test_draw_matches_oracle(env, prec, dims, R, J):
    krps, torch, ctx = env
    Us = synth.gaussian_factors(dims, R, seed=3 * R + len(dims), heavy_rows_frac=0.01)
    for exclude in [-1] + list(range(len(dims))) if len(dims) > 1 else [-1]:
        S, idx, prob, rows, dr, c, rel = _compare_draw(krps, torch, ctx, Us, prec,
                                                       exclude, J, 100 + exclude)
        report(f"draw {prec} dims={dims} R={R} exclude={exclude}", c)
        assert c["unexcused"] == 0
        assert c["excusable_frac"] <= 0.03
        assert rel.max() <= TOL_PROB[prec], rel.max()
        same = c["same"]
        r = rows.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(r[same], dr.rows[same], rtol=1e-12 if prec == "fp64" else 1e-7,
                                   atol=1e-300)
        if exclude >= 0:
            assert np.all(idx[:, exclude] == -1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_leaf_size_does_not_change_indices(env, prec):
    krps, torch, ctx = env
    Us = synth.gaussian_factors((900, 1100, 500), 16, seed=5, heavy_rows_frac=0.01)
    u01 = synth.uniforms(2048, 3, 9)
    ud = torch.from_numpy(u01).to(ctx.device)
    for F in (1, 5, 16, 64, 200):
        ref = osmp.KRPSampler(Us, F=F).draw(1, u01, scaled=prec != "fp64")
        S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec, F=F)
        idx, _, _ = S.sample(1, ud)
        c = compare(idx.cpu().numpy(), ref, prec)
        report(f"leaf size {prec} F={F}", c)
        assert c["unexcused"] == 0, F


def test_row_prob_matches_oracle(env):
    krps, torch, ctx = env
    Us = synth.gaussian_factors((70, 50, 60), 8, seed=11)
    for prec in ("fp64", "fp32"):
        S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec)
        rng = np.random.default_rng(0)
        idx = np.stack([rng.integers(0, d, 500) for d in (70, 50, 60)], 1).astype(np.int32)
        for exclude in (-1, 1):
            p = S.row_prob(exclude, torch.from_numpy(idx).to(ctx.device)).cpu().numpy()
            ref = osmp.KRPSampler(Us).row_prob(exclude, idx.astype(np.int64))
            tol = 1e-10 if prec == "fp64" else 1e-5
            assert np.max(np.abs(p - ref) / ref) <= tol


def test_probabilities_equal_exact_leverage_c1(env):
    # GPU q_d against QR leverage of the materialised Khatri-Rao product
    krps, torch, ctx = env
    cfg = synth.CONFIGS[1]
    Us = synth.gaussian_factors(cfg["dims"], cfg["R"], synth.config_seed(1))
    A = dfn.khatri_rao(Us)
    lev = dfn.leverage_qr(A)
    S = krps.Sampler(ctx, to_dev(torch, ctx, Us, "fp64"), precision="fp64")
    u01 = synth.uniforms(cfg["J"], 3, synth.uniform_seed(1))
    idx, prob, _ = S.sample(-1, torch.from_numpy(u01).to(ctx.device))
    idx = idx.cpu().numpy()
    r = np.ravel_multi_index(tuple(idx.T), cfg["dims"])
    p = prob.cpu().numpy()
    assert np.max(np.abs(p - lev[r] / lev.sum()) / (lev[r] / lev.sum())) <= 1e-10


def test_single_factor_and_rank_one(env):
    krps, torch, ctx = env
    U = synth.gaussian_factors((300,), 6, seed=3)
    _, idx, prob, _, dr, c, rel = _compare_draw(krps, torch, ctx, U, "fp64", -1, 512, 4)
    assert c["unexcused"] == 0 and rel.max() <= 1e-10
    Us = synth.gaussian_factors((40, 30, 20), 1, seed=4)
    _, idx, prob, _, dr, c, rel = _compare_draw(krps, torch, ctx, Us, "fp64", 2, 512, 5)
    assert c["unexcused"] == 0 and rel.max() <= 1e-10


def test_zero_product_is_reported(env):
    krps, torch, ctx = env
    Us = synth.gaussian_factors((30, 20), 4, seed=6)
    Us[1][:] = 0
    S = krps.Sampler(ctx, to_dev(torch, ctx, Us, "fp64"), precision="fp64")
    u = torch.from_numpy(synth.uniforms(64, 2, 1)).to(ctx.device)
    with pytest.raises(krps.KrpsError) as e:
        S.sample(-1, u, check_status=True)
    assert e.value.code == -4
    # excluding the zero factor is fine
    S2 = krps.Sampler(ctx, to_dev(torch, ctx, Us, "fp64"), precision="fp64")
    S2.sample(1, u, check_status=True)


@pytest.mark.parametrize("dims,R", [((5000, 2049, 700), 32), ((3001, 1500, 800), 64),
                                    ((900, 777, 500), 128)])
def test_split_precision_draws_equal_float32_draws(env, dims, R):
    """The split path samples from the float32 path's trees (float64
    products of the float32 factors, float32 nodes, float64 G_j), so its
    draws are the float32 sampler's, index for index and bit for bit in
    q_d, and against the plain float64 oracle under the float32 rule."""
    krps, torch, ctx = env
    Us = synth.gaussian_factors(dims, R, seed=99 + R, heavy_rows_frac=0.01)
    S32 = krps.Sampler(ctx, to_dev(torch, ctx, Us, "fp32"), precision="fp32")
    ud = torch.from_numpy(synth.uniforms(4096, len(dims), 7)).to(ctx.device)
    for exclude in (-1, 0):
        _, idx, prob, _, dr, c, rel = _compare_draw(krps, torch, ctx, Us, "bf16x2", exclude,
                                                    4096, 7)
        report(f"bf16x2 dims={dims} R={R} exclude={exclude}", c)
        print(f"  q_d rel err max {rel.max():.2e}", flush=True)
        assert c["unexcused"] == 0
        assert rel.max() <= TOL_PROB["bf16x2"]
        i32, p32, _ = S32.sample(exclude, ud, check_status=True)
        assert np.array_equal(idx, i32.cpu().numpy().astype(np.int64))
        assert np.array_equal(prob.cpu().numpy(), p32.cpu().numpy())


def test_autotune_measures_then_reads_the_cache(tmp_path):
    import torch
    import paper_2301_12584_amd as krps
    ctx = krps.Context(0)
    Us = synth.gaussian_factors((20000, 15000, 9000), 16, seed=77, heavy_rows_frac=0.01)
    Ud = [torch.from_numpy(U).to(ctx.device).contiguous() for U in Us]
    u = torch.from_numpy(synth.uniforms(4096, 3, 78)).to(ctx.device)
    cache = tmp_path / "tune.jsonl"
    t1 = krps.autotune(ctx, Ud, u, "fp32", cache_path=cache)
    assert not t1["from_cache"] and t1["F"] in (8, 16, 32, 64) and t1["lps"] in (8, 16)
    assert t1["team"] == 1
    t2 = krps.autotune(ctx, Ud, u, "fp32", cache_path=cache)
    assert t2["from_cache"]
    assert (t2["F"], t2["lps"], t2["team"]) == (t1["F"], t1["lps"], t1["team"])
    # a later entry of the same key with shapes the library does not offer
    # at R = 16 (written by another version) is skipped
    line = cache.read_text().splitlines()[-1]
    stale = line.replace(f'"lps": {t1["lps"]}', '"lps": 64').replace(f'"team": {t1["team"]}',
                                                                      '"team": 8')
    assert stale != line
    with open(cache, "a") as f:
        f.write(stale + "\n")
    t3 = krps.autotune(ctx, Ud, u, "fp32", cache_path=cache)
    assert t3["from_cache"]
    assert (t3["F"], t3["lps"], t3["team"]) == (t1["F"], t1["lps"], t1["team"])
    # the tuned shape's draws against the float64 oracle
    S1 = krps.Sampler(ctx, Ud, precision="fp32", F=t1["F"], lps=t1["lps"], team=t1["team"])
    for j in range(3):
        S1.refresh(j)       # rebuilt with the tuned team
    i1, p1, _ = S1.sample(-1, u)
    torch.cuda.synchronize()
    dr = osmp.KRPSampler(Us, F=t1["F"]).draw(-1, u.cpu().numpy(), scaled=True)
    c = compare(i1.cpu().numpy(), dr, "fp32")
    report(f"autotuned F={t1['F']} lps={t1['lps']}", c)
    assert c["unexcused"] == 0
    same = c["same"]
    np.testing.assert_allclose(p1.cpu().numpy()[same], dr.prob[same], rtol=TOL_PROB["fp32"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_in_kernel_uniforms_match_the_oracle(prec):
    """Uniforms generated in the walk from (seed, ctr_base) equal the
    oracle's Philox4x64-10 uniforms: the draws match index for index
    (margin rule), and a disjoint counter range gives other draws."""
    import torch
    import paper_2301_12584_amd as krps
    from oracle import sketch as osk
    ctx = krps.Context(0)
    dims, R, J = (5000, 3000, 2000), 16, 4096
    Us = synth.gaussian_factors(dims, R, seed=81, heavy_rows_frac=0.01)
    dt = torch.float64 if prec == "fp64" else torch.float32
    S = krps.Sampler(ctx, [torch.from_numpy(U).to(ctx.device).to(dt).contiguous() for U in Us],
                     precision=prec)
    first = None
    for exclude in (-1, 1):
        idx, p = S.sample_seeded(exclude, J, seed=2026, ctr_base=1000)
        if first is None:
            first = idx
        torch.cuda.synchronize()
        u = osk.philox_uniforms(J, 3, 2026, 1000)
        dr = osmp.KRPSampler(Us).draw(exclude, u, scaled=prec != "fp64")
        c = compare(idx.cpu().numpy(), dr, prec)
        report(f"in-kernel uniforms {prec} exclude={exclude}", c)
        assert c["unexcused"] == 0
        # the same uniforms through the buffer path give the same draws
        i2, p2, _ = S.sample(exclude, torch.from_numpy(u).to(ctx.device))
        torch.cuda.synchronize()
        assert torch.equal(i2, idx) and torch.equal(p2, p)
    other, _ = S.sample_seeded(-1, J, seed=2026, ctr_base=1000 + J)
    torch.cuda.synchronize()
    assert (other != first).any(dim=1).float().mean().item() > 0.5


FILTER_CASES = [((200000, 150000, 9000), 8, 8192), ((60000, 40000, 3000), 16, 8192),
                ((100000, 70000, 5000), 32, 8192), ((30000, 20000), 64, 4096),
                ((12000, 9000), 128, 2048)]


@pytest.mark.parametrize("dims,R,J", FILTER_CASES)
def test_float32_node_copy_gives_the_float64_walk(env, dims, R, J):
    """The float64 walk deciding its deep levels from the float32 node
    copies draws exactly the indices (and so the probabilities) of the walk
    that reads only the float64 nodes, whichever levels are filtered; the
    undecided share that is walked again stays small by default."""
    krps, torch, ctx = env
    Us = synth.gaussian_factors(dims, R, seed=7 * R + 1, heavy_rows_frac=0.01)
    S = krps.Sampler(ctx, to_dev(torch, ctx, Us, "fp64"), precision="fp64")
    D = max(S.tree_info(j).D for j in range(len(dims)))
    u = torch.from_numpy(synth.uniforms(J, len(dims), 4242 + R)).to(ctx.device)
    out = {}
    for top in (100, -1, 0, D // 2):
        S.set_filter(top)
        for exclude in (-1, 0):
            idx, prob, rows = S.sample(exclude, u, rows=True)
            torch.cuda.synchronize()
            assert S.check_status() == 0
            out[top, exclude] = (idx.cpu(), prob.cpu(), rows.cpu(), S.rewalked)
    walks = J * len(dims)
    for exclude in (-1, 0):
        i0, p0, r0, w0 = out[100, exclude]
        assert w0 == 0  # the copy is off
        for top in (-1, 0, D // 2):
            i1, p1, r1, w1 = out[top, exclude]
            print(f"filter R={R} D={D} top={top} exclude={exclude}: re-walked {w1} of "
                  f"{walks} walks", flush=True)
            assert torch.equal(i0, i1), (top, exclude)
            assert torch.equal(p0, p1) and torch.equal(r0, r1)
        assert out[-1, exclude][3] <= 0.02 * walks


def _chi2_equal_mass_groups(counts, p, groups):
    """Chi-square p-value over ``groups`` equal-mass groups of rows sorted
    by their probability (so that every group expects many draws)."""
    from scipy.stats import chisquare
    order = np.argsort(p)
    cum = np.cumsum(p[order])
    g = np.minimum((cum * groups / cum[-1]).astype(int), groups - 1)
    obs = np.bincount(g, weights=counts[order], minlength=groups)
    exp = np.bincount(g, weights=p[order], minlength=groups) * counts.sum()
    return chisquare(obs, exp).pvalue


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
def test_gpu_histograms_match_exact_leverage(env, prec):
    """Large-J histograms of the GPU's own draws (in-kernel uniforms)
    against the exact leverage distribution of the materialised
    Khatri-Rao product (QR leverage, the definition): the exact tiny
    workload over all modes (4,096 equal-mass groups of its 262,144 rows)
    and excluding mode 0 (all 4,096 rows), and the Appendix A.13 check
    (three 8 x 8 factors with 1% of entries x10, all 512 rows)."""
    from scipy.stats import chisquare
    krps, torch, ctx = env
    cfg = synth.CONFIGS[1]
    cases = [(synth.gaussian_factors(cfg["dims"], cfg["R"], synth.config_seed(1)), -1, 4096),
             (synth.gaussian_factors(cfg["dims"], cfg["R"], synth.config_seed(1)), 0, 0),
             (synth.gaussian_factors((8, 8, 8), 8, seed=2023, heavy_entries_frac=0.01), -1, 0)]
    J = 1 << 22
    pvals = []
    for t, (Us, exclude, groups) in enumerate(cases):
        S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec)
        modes = [k for k in range(len(Us)) if k != exclude]
        A = dfn.khatri_rao([Us[k] for k in modes])
        lev = dfn.leverage_qr(A)
        p = lev / lev.sum()
        idx, _ = S.sample_seeded(exclude, J, seed=777 + t)
        torch.cuda.synchronize()
        idx = idx.cpu().numpy().astype(np.int64)
        flat = np.zeros(J, dtype=np.int64)
        for k in modes:            # C order over the drawn modes, last fastest
            flat = flat * len(Us[k]) + idx[:, k]
        cnt = np.bincount(flat, minlength=len(p)).astype(np.float64)
        assert cnt.sum() == J
        pv = (_chi2_equal_mass_groups(cnt, p, groups) if groups
              else chisquare(cnt, p * J).pvalue)
        print(f"chi-square {prec} case {t}: p = {pv:.3g}", flush=True)
        pvals.append(pv)
    # fixed seeds; Bonferroni over the three tests
    assert min(pvals) > 1e-3 / len(pvals), pvals


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
def test_entry_updates_match_a_rebuilt_oracle(env, prec):
    """krps_sampler_update_entries (Algorithm 5): after single-entry updates
    (first row, the ragged last leaf, repeated rows and entries, a zero)
    the factor holds the new values, every stored node and G_j match the
    oracle tree rebuilt from the updated factor, and the draws match the
    oracle's over the updated factors; for float64 the float32 node copy
    follows (walks with and without it agree)."""
    krps, torch, ctx = env
    dims, R = (5003, 1200, 700), 16
    Us = synth.gaussian_factors(dims, R, seed=44, heavy_rows_frac=0.01)
    S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec)
    Us2 = [U.astype(np.float64).copy() for U in Us]
    rng = np.random.default_rng(45)
    for j in (0, 2):
        I = dims[j]
        rows = list(rng.integers(0, I, 60)) + [0, I - 1, I - 1, 7, 7]
        cols = list(rng.integers(0, R, 60)) + [0, R - 1, 3, 5, 5]
        vals = list((rng.standard_normal(60) * 20).astype(np.float32)) + [0.0, 1.5, -2.0, 0.25,
                                                                         -0.5]
        S.update_entries(j, rows, cols, vals)
        for r, c, v in zip(rows, cols, vals):
            Us2[j][r, c] = v
    torch.cuda.synchronize()
    for j in range(3):
        got = S.factors[j].cpu().numpy().astype(np.float64)
        assert np.array_equal(got, Us2[j]), j
        t = osmp.SegmentTree(Us2[j], R)
        ref = stored_nodes(t)
        nodes = S.tree_nodes(j).cpu().numpy().astype(np.float64)
        scale = node_scale(ref, R)[:, None] + 1e-300
        err = float((np.abs(nodes - ref) / scale).max())
        print(f"update {prec} factor {j}: node error {err:.2e}", flush=True)
        assert err <= TOL_NODE[prec] * (1 if prec == "fp64" else 4), (j, err)
        G = S.gram(j).cpu().numpy()
        Gref = Us2[j].T @ Us2[j]
        assert np.abs(G - Gref).max() <= TOL_NODE[prec] * np.abs(np.diag(Gref)).max()
    u01 = synth.uniforms(2048, 3, 46)
    ud = torch.from_numpy(u01).to(ctx.device)
    for exclude in (-1, 1):
        idx, prob, _ = S.sample(exclude, ud, check_status=True)
        dr = osmp.KRPSampler(Us2).draw(exclude, u01, scaled=prec != "fp64")
        c = compare(idx.cpu().numpy(), dr, prec)
        report(f"after updates {prec} exclude={exclude}", c)
        assert c["unexcused"] == 0
        if prec == "fp64":
            S.set_filter(100)
            i2, p2, _ = S.sample(exclude, ud)
            S.set_filter(-1)
            assert torch.equal(idx, i2) and torch.equal(prob, p2)


TUNE_R = [(16, (3000, 2500, 900)), (32, (4000, 1800, 700)), (64, (3000, 1500)),
          (128, (900, 700))]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
@pytest.mark.parametrize("R,dims", TUNE_R)
def test_every_tunable_shape_matches_the_oracle(env, prec, R, dims):
    """Every shape the autotuner can pick -- leaf size, lanes per sample of
    the walk, team width of the tree build -- draws, against the float64
    oracle, under the same parity rules as the default shape, through the
    single-problem walk and through the batched walk (whose shape classes
    follow the samplers' lanes-per-sample choice)."""
    krps, torch, ctx = env
    lib = krps.lib()
    Us = synth.gaussian_factors(dims, R, seed=600 + R, heavy_rows_frac=0.01)
    J = 1024
    u01 = synth.uniforms(J, len(dims), 601 + R)
    ud = torch.from_numpy(u01).to(ctx.device)
    lps_all = {16: (8, 16), 32: (16, 32, 64), 64: (64,), 128: (64,)}[R]
    teams = {16: (1,), 32: (1, 3), 64: (2, 5), 128: (6, 12)}[R]
    samplers, refs = [], []
    for F in (R // 2, 2 * R):
        ref = osmp.KRPSampler(Us, F=F).draw(-1, u01, scaled=prec != "fp64")
        for lps in lps_all:
            for team in teams:
                S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec, F=F,
                                 lps=lps, team=team)
                for j in range(len(dims)):
                    S.refresh(j)
                idx, prob, _ = S.sample(-1, ud)
                c = compare(idx.cpu().numpy(), ref, prec)
                report(f"shape {prec} R={R} F={F} lps={lps} team={team}", c)
                assert c["unexcused"] == 0
                samplers.append(S)
                refs.append((ref, idx))
    # one batch over all of them: the batched walk of each class gives the
    # single-problem walk's indices
    B = krps.Batch(ctx, samplers, [-1] * len(samplers))
    ib, _ = B.sample([ud] * len(samplers))
    torch.cuda.synchronize()
    for (ref, idx), got in zip(refs, ib):
        assert torch.equal(got, idx)
    # a team width the tree build does not have is refused
    assert lib.krps_sampler_set_build(samplers[0].handle, 7) != 0
