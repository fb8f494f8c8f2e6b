"""GPU parity of the sampler path (tree build, per-draw preparation, descent)
against the float64 oracle, through the C ABI.  Run with ``-m gpu``."""
import numpy as np
import pytest

import synth
from oracle import definition as dfn
from oracle import sampler as osmp

pytestmark = pytest.mark.gpu

TOL_NODE = {"fp64": 1e-12, "fp32": 1e-5, "bf16x2": 1e-4}
TOL_PROB = {"fp64": 1e-10, "fp32": 1e-5, "bf16x2": 1e-3}
MARGIN = 1e-6
STORE = {"fp64": None, "fp32": np.float32, "bf16x2": np.float32}


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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("exclude", [-1, 0, 2])
def test_prep_matches_oracle(env, prec, exclude):
    krps, torch, ctx = env
    print(f"prep {prec} exclude={exclude}", flush=True)
    cfg = synth.CONFIGS[1]
    Us = synth.gaussian_factors((64, 50, 70), 8, synth.config_seed(1))
    S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec)
    u = torch.from_numpy(synth.uniforms(16, 3, 1)).to(ctx.device)
    S.sample(exclude, u)
    torch.cuda.synchronize()
    parts = {k: (v.cpu() if hasattr(v, "cpu") else v) for k, v in S.draw_parts().items()}
    ref = osmp.KRPSampler(Us)
    Gp, rank, eig, E, _ = ref.prepare(exclude)
    rtol = 1e-10 if prec == "fp64" else 1e-4
    assert parts["rank"] == rank
    assert np.abs(parts["gplus"].numpy() - Gp).max() <= rtol * np.abs(Gp).max()
    for k in ref.modes(exclude):
        lam, V = eig[k]
        assert np.abs(parts["lam"][k].numpy() - lam).max() <= rtol * lam.max()
        Vg = parts["vecs"][k].numpy().astype(np.float64)     # [u][:]
        # sign-insensitive: |<v_gpu, v_ref>| = 1
        dots = np.abs(np.einsum("ue,eu->u", Vg, V))
        assert np.abs(dots - 1).max() <= (1e-9 if prec == "fp64" else 1e-4)
        iu = np.triu_indices(8)
        Eref = [E[k].root * ref.G[k]]
        for lev in range(1, E[k].D + 1):
            for p in range(0, E[k].real(lev), 2):
                Eref.append(E[k].levels[lev][p] * ref.G[k])
        Eref = np.array([m[iu] for m in Eref])
        Eg = parts["etree"][k].numpy().astype(np.float64)
        assert np.abs(Eg - Eref).max() <= rtol * 10 * np.abs(Eref).max()


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
        Gp, rank, _, _, _ = osmp.KRPSampler(Us).prepare(-1)
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
    # the float32-storage path decides its indices on float32-rounded nodes
    ref = osmp.KRPSampler(Us, F=F or None, store=STORE[prec])
    dr = ref.draw(exclude, u01)
    idx = idx.cpu().numpy().astype(np.int64)
    same = (idx == dr.idx).all(axis=1)
    excused = (dr.margin <= MARGIN) | dr.degenerate
    bad = ~(same | excused)
    rel = np.abs(prob.cpu().numpy()[same] - dr.prob[same]) / dr.prob[same]
    return S, idx, prob, rows, dr, same, bad, rel


CASES = [((64, 64, 64), 8, 4096), ((1000, 333, 77), 16, 2048), ((5000, 2049, 700), 32, 2048),
         ((3001, 1500, 64), 64, 1024), ((777, 260), 128, 512), ((129, 1, 33), 8, 512)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,R,J", CASES)
def test_draw_matches_oracle(env, prec, dims, R, J):
    krps, torch, ctx = env
    Us = synth.gaussian_factors(dims, R, seed=3 * R + len(dims), heavy_rows_frac=0.01)
    for exclude in [-1] + list(range(len(dims))) if len(dims) > 1 else [-1]:
        print(f"draw {prec} dims={dims} R={R} J={J} exclude={exclude}", flush=True)
        S, idx, prob, rows, dr, same, bad, rel = _compare_draw(krps, torch, ctx, Us, prec,
                                                               exclude, J, 100 + exclude)
        assert bad.sum() == 0, (bad.sum(), J)
        assert same.mean() > 0.9
        assert rel.max() <= TOL_PROB[prec], rel.max()
        r = rows.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(r[same], dr.rows[same], rtol=1e-12 if prec == "fp64" else 1e-5,
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
        ref = osmp.KRPSampler(Us, F=F, store=STORE[prec]).draw(1, u01)
        print(f"leaf size {prec} F={F}", flush=True)
        S = krps.Sampler(ctx, to_dev(torch, ctx, Us, prec), precision=prec, F=F)
        idx, _, _ = S.sample(1, ud)
        idx = idx.cpu().numpy().astype(np.int64)
        ok = (idx == ref.idx).all(axis=1) | (ref.margin <= MARGIN)
        assert ok.all(), (F, (~ok).sum())


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
    _, idx, prob, _, dr, same, bad, rel = _compare_draw(krps, torch, ctx, U, "fp64", -1, 512, 4)
    assert bad.sum() == 0 and rel.max() <= 1e-10
    Us = synth.gaussian_factors((40, 30, 20), 1, seed=4)
    _, idx, prob, _, dr, same, bad, rel = _compare_draw(krps, torch, ctx, Us, "fp64", 2, 512, 5)
    assert bad.sum() == 0 and rel.max() <= 1e-10


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


def test_split_precision_reports_mismatch_rate(env):
    krps, torch, ctx = env
    Us = synth.gaussian_factors((5000, 2049, 700), 32, seed=99, heavy_rows_frac=0.01)
    _, idx, prob, _, dr, same, bad, rel = _compare_draw(krps, torch, ctx, Us, "bf16x2", 0, 4096, 7)
    print(f"bf16x2: mismatch {1 - same.mean():.4f}, unexcused {bad.mean():.4f}, "
          f"prob rel err max {rel.max():.2e}", flush=True)
    assert same.mean() > 0.9
    assert rel.max() <= TOL_PROB["bf16x2"]


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
    t2 = krps.autotune(ctx, Ud, u, "fp32", cache_path=cache)
    assert t2["from_cache"] and (t2["F"], t2["lps"]) == (t1["F"], t1["lps"])
    # the tuned shape draws the same indices as the default one
    S0 = krps.Sampler(ctx, Ud, precision="fp32")
    S1 = krps.Sampler(ctx, Ud, precision="fp32", F=t1["F"], lps=t1["lps"])
    i0, p0, _ = S0.sample(-1, u)
    i1, p1, _ = S1.sample(-1, u)
    torch.cuda.synchronize()
    same = (i0 == i1).all(dim=1).cpu().numpy()
    assert same.mean() >= 0.999, same.mean()
    np.testing.assert_allclose(p1.cpu().numpy()[same], p0.cpu().numpy()[same], rtol=1e-5)


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
        dr = osmp.KRPSampler(Us, store=None if prec == "fp64" else np.float32).draw(exclude, u)
        got = idx.cpu().numpy().astype(np.int64)
        same = (got == dr.idx).all(axis=1)
        assert np.all(same | (dr.margin <= 1e-6)), np.sum(~same)
        # the same uniforms through the buffer path give the same draws
        i2, p2, _ = S.sample(exclude, torch.from_numpy(u).to(ctx.device))
        torch.cuda.synchronize()
        assert torch.equal(i2, idx) and torch.equal(p2, p)
    other, _ = S.sample_seeded(-1, J, seed=2026, ctr_base=1000 + J)
    torch.cuda.synchronize()
    assert (other != first).any(dim=1).float().mean().item() > 0.5
