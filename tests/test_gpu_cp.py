"""GPU parity of the sketched least-squares / CP-ALS path against the oracle,
through the C ABI.  Run with ``-m gpu``."""
import numpy as np
import pytest

import synth
from chain import check_solve
from oracle import cp as ocp
from oracle import sampler as osmp
from parity import compare, report

pytestmark = pytest.mark.gpu

# the type the factors are kept in (the problem's values after each solve)
FACTOR = {"fp64": None, "fp32": np.float32, "bf16x2": np.float32}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2301_12584_amd as krps
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return krps, torch, krps.Context(0)


def dev_factors(torch, ctx, Us, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    return [torch.from_numpy(np.asarray(U, dtype=np.float64)).to(ctx.device, dt).contiguous()
            for U in Us]


def dense_coo(dims, seed, dup=200):
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    idx = np.stack([g.reshape(-1) for g in grids], axis=1)
    val = rng.lognormal(size=idx.shape[0])
    extra = rng.integers(0, idx.shape[0], dup)
    idx = np.concatenate([idx, idx[extra]]).astype(np.int32)
    val = np.concatenate([val, rng.standard_normal(dup)]).astype(np.float32)
    return idx, val


def make(krps, torch, ctx, dims, idx, val, Us, prec, J):
    S = krps.Sampler(ctx, dev_factors(torch, ctx, Us, prec), precision=prec)
    T = krps.Tensor(ctx, dims, torch.from_numpy(idx).to(ctx.device),
                    torch.from_numpy(val).to(ctx.device))
    return S, T, krps.CPALS(S, T, J)


@pytest.mark.parametrize("seed", [0, 1])
def test_tensor_norm_with_duplicates(env, seed):
    krps, torch, ctx = env
    dims = (12, 10, 8)
    idx, val = dense_coo(dims, seed)
    T = krps.Tensor(ctx, dims, torch.from_numpy(idx).to(ctx.device),
                    torch.from_numpy(val).to(ctx.device))
    ref = ocp.SparseTensor(dims, idx, val).norm2
    assert abs(T.norm2 - ref) <= 1e-12 * ref
    zidx, zval = synth.sparse_tensor((500, 400, 300), 50_000, 1.2, seed)
    T2 = krps.Tensor(ctx, (500, 400, 300), torch.from_numpy(zidx).to(ctx.device),
                     torch.from_numpy(zval).to(ctx.device))
    ref2 = ocp.SparseTensor((500, 400, 300), zidx, zval).norm2
    assert abs(T2.norm2 - ref2) <= 1e-9 * ref2


def test_duplicates_are_merged_into_stored_entries(env):
    krps, torch, ctx = env
    dims = (12, 10, 8)
    idx, val = dense_coo(dims, 3, dup=500)
    T = krps.Tensor(ctx, dims, torch.from_numpy(idx).to(ctx.device),
                    torch.from_numpy(val).to(ctx.device))
    assert T.stored_entries == len(np.unique(idx, axis=0))
    zidx, zval = synth.sparse_tensor((50, 40, 30), 100_000, 1.2, seed=8)
    T2 = krps.Tensor(ctx, (50, 40, 30), torch.from_numpy(zidx).to(ctx.device),
                     torch.from_numpy(zval).to(ctx.device))
    assert T2.stored_entries == len(np.unique(zidx, axis=0))


def test_hot_rows_hold_the_most_entries(env):
    """The hot rows are the min(512, I_j) rows with the most stored entries,
    in decreasing count (enough entries per workgroup that the counting
    table fills and the global fallback is taken too)."""
    krps, torch, ctx = env
    dims = (200_000, 100_000, 20)
    idx, val = synth.sparse_tensor(dims, 20_000_000, 1.2, seed=12)
    T = krps.Tensor(ctx, dims, torch.from_numpy(idx).to(ctx.device),
                    torch.from_numpy(val).to(ctx.device))
    key = (idx[:, 0].astype(np.int64) * dims[1] + idx[:, 1]) * dims[2] + idx[:, 2]
    key = np.unique(key)
    cols = [key // (dims[1] * dims[2]), (key // dims[2]) % dims[1], key % dims[2]]
    assert T.stored_entries == len(key)
    for j, d in enumerate(dims):
        cnt = np.bincount(cols[j], minlength=d)
        hot = T.hot_rows(j)
        k = min(512, d)
        assert len(hot) == k and len(set(hot)) == k
        kth = np.sort(cnt)[::-1][k - 1]
        assert min(cnt[h] for h in hot) >= kth, (j, sorted(cnt[hot]), kth)
        c = cnt[hot]
        assert np.all(c[:-1] >= c[1:])  # decreasing: a prefix is the hottest rows


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_repeated_samples_share_one_fiber(env, prec):
    """A factor with one dominant row makes most samples repeat a few
    multi-indices; M and Y must still equal the oracle's normal equations
    on the GPU's own draw (each distinct fiber expanded once with the summed
    weight of its samples)."""
    krps, torch, ctx = env
    dims, R, J = (60, 50, 40), 4, 5000
    idx, val = synth.sparse_tensor(dims, 30_000, 1.1, seed=12)
    Us = synth.gaussian_factors(dims, R, seed=13)
    for U in Us:
        U[:2] *= 50.0
    S, T, A = make(krps, torch, ctx, dims, idx, val, Us, prec, J)
    for k in range(3):
        A.normalize(k)
    Un = [S.factors[k].cpu().numpy().astype(np.float64) for k in range(3)]
    j = 1
    u01 = synth.uniforms(J, 3, 77)
    A.solve(j, torch.from_numpy(u01).to(ctx.device))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in A.parts(j).items()}
    oth = [k for k in range(3) if k != j]
    n_distinct = len(np.unique(got["idx"][:, oth], axis=0))
    assert n_distinct < J // 4, n_distinct          # the draw really repeats
    Tor = ocp.SparseTensor(dims, idx, val)
    w2 = 1.0 / (J * got["prob"])
    rows = np.ones((J, R))
    for k in oth:
        rows *= Un[k][got["idx"][:, k]]
    M2, Y2 = ocp.normal_equations(Tor, j, got["idx"].astype(np.int64), rows, w2)
    tol = 1e-11 if prec == "fp64" else 1e-6
    assert np.abs(got["M"] - M2).max() <= tol * np.abs(M2).max()
    assert np.abs(got["Y"] - Y2).max() <= tol * np.abs(Y2).max()


@pytest.mark.parametrize("prec", ["fp64", "bf16x2"])
def test_solve_touches_exactly_the_reached_rows(env, prec):
    """On a sparse tensor the solve lists exactly the rows of mode j that
    the sampled fibers' entries reach (increasing, each once); Y matches the
    oracle's normal equations on them and every other row of U_j is 0."""
    krps, torch, ctx = env
    dims, R, J, j = (5000, 40, 30), 8, 50, 0
    idx, val = synth.sparse_tensor(dims, 20_000, 1.2, seed=31)
    Us = synth.gaussian_factors(dims, R, seed=32)
    S, T, A = make(krps, torch, ctx, dims, idx, val, Us, prec, J)
    for k in range(3):
        A.normalize(k)
    A.solve(j, torch.from_numpy(synth.uniforms(J, 3, 33)).to(ctx.device))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in A.parts(j).items()}
    rows_got = got["yrows"].astype(np.int64)
    fibers = {}
    for e in np.unique(idx, axis=0):
        fibers.setdefault((int(e[1]), int(e[2])), set()).add(int(e[0]))
    want = set()
    for d in range(J):
        want |= fibers.get((int(got["idx"][d, 1]), int(got["idx"][d, 2])), set())
    assert 0 < len(want) < dims[j] // 2
    assert np.all(np.diff(rows_got) > 0)
    assert set(rows_got.tolist()) == want
    Un = [ocp.normalize_columns(U)[0] for U in Us]
    rows = Un[1][got["idx"][:, 1]] * Un[2][got["idx"][:, 2]]
    M2, Y2 = ocp.normal_equations(ocp.SparseTensor(dims, idx, val), j,
                                  got["idx"].astype(np.int64), rows, 1.0 / (J * got["prob"]))
    assert np.abs(got["Y"] - Y2).max() <= 1e-5 * np.abs(Y2).max()
    U = S.factors[j].cpu().numpy()
    off = np.setdiff1d(np.arange(dims[j]), rows_got)
    assert np.all(U[off] == 0) and np.abs(U[rows_got]).max() > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
@pytest.mark.parametrize("j", [0, 1, 2])
def test_one_solve_matches_oracle(env, prec, j):
    """One solve on a dense 12 x 10 x 8 tensor with duplicates: the drawn
    indices against the oracle's draw (parity rules), every step after the
    draw against the oracle on the GPU's own draw, and for float64 the whole
    solve against the oracle's solve."""
    krps, torch, ctx = env
    dims, R, J = (12, 10, 8), 4, 300
    idx, val = dense_coo(dims, 5)
    Us = synth.gaussian_factors(dims, R, seed=21)
    S, T, A = make(krps, torch, ctx, dims, idx, val, Us, prec, J)
    for k in range(3):
        A.normalize(k)
    before = [U.cpu().numpy().astype(np.float64) for U in S.factors]
    u01 = synth.uniforms(J, 3, 40 + j)
    A.solve(j, torch.from_numpy(u01).to(ctx.device))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in A.parts(j).items()}
    Ugpu = S.factors[j].cpu().numpy().astype(np.float64)
    sig = A.sigma.cpu().numpy()
    Tor = ocp.SparseTensor(dims, idx, val)
    dr = osmp.KRPSampler(before).draw(j, u01, scaled=prec != "fp64")
    c = compare(got["idx"], dr, prec)
    report(f"solve {prec} j={j}", c)
    assert c["unexcused"] == 0
    errs = check_solve(Tor, before, j, got, Ugpu, sig, prec)
    print(f"solve {prec} j={j}: " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()),
          flush=True)
    if prec == "fp64":
        # the oracle's own solve from the same factors and uniforms
        Uref, sref, dr2, Mref, Yref = ocp.sketched_solve(osmp.KRPSampler(before), Tor, j, u01)
        assert (got["idx"].astype(np.int64) == dr2.idx).all()
        np.testing.assert_allclose(got["M"], Mref, rtol=1e-11, atol=1e-12 * np.abs(Mref).max())
        np.testing.assert_allclose(got["Y"], Yref, rtol=1e-10, atol=1e-11 * np.abs(Yref).max())
        np.testing.assert_allclose(sig, sref, rtol=1e-9)
        np.testing.assert_allclose(Ugpu, Uref, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_seeded_solve_and_sweep_match_the_oracle_uniforms(env, prec):
    """krps_sketched_solve_seeded / krps_als_sweep_seeded generate the walk's
    uniforms in the kernel (Philox4x64-10, counter word 2 = sweep N + j):
    they equal the buffer path fed with the oracle's Philox uniforms, and a
    captured seeded sweep replayed for two sweep numbers equals the eager
    seeded sweeps."""
    from oracle import sketch as osk
    krps, torch, ctx = env
    dims, R, J = (300, 200, 100), 8, 2048
    idx, val = synth.sparse_tensor(dims, 20_000, 1.2, seed=52)
    U0 = synth.gaussian_factors(dims, R, seed=53)
    seed, base = 77, 1 << 40

    def fresh():
        S, T, A = make(krps, torch, ctx, dims, idx, val, U0, prec, J)
        for k in range(3):
            A.normalize(k)
        return S, T, A

    # one solve: seeded against the buffer path with the oracle's uniforms
    S1, T1, A1 = fresh()
    S2, T2, A2 = fresh()
    A1.solve_seeded(1, seed, base, 3)
    u = osk.philox_uniforms(J, 3, seed, base, ctr2=3 * 3 + 1)
    A2.solve(1, torch.from_numpy(u).to(ctx.device))
    torch.cuda.synchronize()
    assert torch.equal(A1.parts(1)["idx"], A2.parts(1)["idx"])
    assert torch.equal(A1.parts(1)["prob"], A2.parts(1)["prob"])
    dr = osmp.KRPSampler([U.cpu().numpy() for U in S2.factors]).draw(1, u,
                                                                      scaled=prec != "fp64")
    # (S2's factor 1 is the new one; the draw used the others, unchanged)
    c = compare(A2.parts(1)["idx"].cpu().numpy(), dr, prec)
    report(f"seeded solve {prec}", c)
    assert c["unexcused"] == 0
    if prec != "fp64":
        return
    # eager seeded sweeps 0 and 1 against graph replays of one captured graph
    # (float64: the SpMM's atomic order moves only the last bits)
    S1, T1, A1 = fresh()
    S2, T2, A2 = fresh()
    for sw in (0, 1):
        A1.sweep_seeded(seed, base, sw, use_graph=False)
        A2.sweep_seeded(seed, base, sw, use_graph=True)
        torch.cuda.synchronize()
        _ = (S2.factors[0] * 2).sum().item()   # eager work between replays
        for k in range(3):
            assert torch.allclose(S1.factors[k], S2.factors[k], rtol=1e-10, atol=1e-12), (sw, k)
    # and sweep 1 differs from sweep 0's uniforms: the draws of the last
    # solve of sweep 1 equal the buffer path with ctr2 = 1 * 3 + 2
    u = osk.philox_uniforms(J, 3, seed, base, ctr2=1 * 3 + 2)
    S3, T3, A3 = fresh()
    A3.sweep_seeded(seed, base, 0)
    A3.solve_seeded(0, seed, base, 1)
    A3.solve_seeded(1, seed, base, 1)
    A3.solve(2, torch.from_numpy(u).to(ctx.device))
    torch.cuda.synchronize()
    assert torch.equal(A3.parts(2)["idx"], A1.parts(2)["idx"])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
@pytest.mark.parametrize("R", [3, 8, 12, 128])
def test_fit_matches_oracle(env, prec, R):
    """R = 3: lane-per-column teams; R = 8, 12, 128: 16-byte row loads
    (R = 12 leaves a partial last vector team pass for float64)."""
    krps, torch, ctx = env
    dims = (12, 10, 8)
    idx, val = dense_coo(dims, 9)
    Us = synth.gaussian_factors(dims, R, seed=22)
    S, T, A = make(krps, torch, ctx, dims, idx, val, Us, prec, 64)
    for k in range(3):
        A.normalize(k)
    sig = np.linspace(0.5, 2.0, R)
    A.sigma.copy_(torch.from_numpy(sig))
    f = A.fit()
    Un = [ocp.normalize_columns(U)[0] for U in Us]
    ref = ocp.fit(ocp.SparseTensor(dims, idx, val), Un, sig)
    assert abs(f - ref) <= (1e-12 if prec == "fp64" else 1e-6)


def _sweep_uniforms(seed, sweep, N, J):
    return np.stack([synth.uniforms(J, N, seed + 1000 * sweep + j) for j in range(N)])


def _run_als(krps, torch, ctx, dims, idx, val, Us, prec, J, sweeps, seed, use_graph=False):
    S, T, A = make(krps, torch, ctx, dims, idx, val, Us, prec, J)
    for k in range(len(dims)):
        A.normalize(k)
    A.sigma.fill_(1.0)
    fits = []
    for s in range(sweeps):
        u = torch.from_numpy(_sweep_uniforms(seed, s, len(dims), J)).to(ctx.device)
        A.sweep(u, use_graph=use_graph)
        fits.append(A.fit())
    return fits, S, A


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_planted_tensor_als_matches_oracle(env, prec):
    krps, torch, ctx = env
    dims, R, J = (14, 12, 10), 3, 400
    idx, val, _ = synth.planted_cp_tensor(dims, R, seed=31)
    U0 = synth.gaussian_factors(dims, R, seed=32)
    fits, _, _ = _run_als(krps, torch, ctx, dims, idx, val, U0, prec, J, 20, 500)
    Tor = ocp.SparseTensor(dims, idx, val)
    _, _, ref = ocp.cp_als(Tor, U0, 20, lambda s, j: _sweep_uniforms(500, s, 3, J)[j],
                           factor_dtype=FACTOR[prec])
    print(prec, "fits", fits[-3:], "oracle", ref[-3:], flush=True)
    assert fits[-1] >= 0.999
    assert np.max(np.abs(np.array(fits) - np.array(ref))) <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
def test_zipf_tensor_als_matches_oracle(env, prec):
    """Four sweeps on a 2e5-entry Zipf tensor.  Float64: the whole trajectory
    against the oracle's run with the same uniforms (the draws agree).
    Float32 and the split path: every solve checked step by step on the
    GPU's own draw, sampled indices against the oracle's draw from the same
    factors, and each fit against the oracle's fit of the GPU's factors; the
    trajectory of the oracle's own run is printed beside (its draws part
    from the GPU's where a comparison lies within rounding of its cut,
    after which the two runs are different sketches)."""
    krps, torch, ctx = env
    dims, R, J = (3000, 2000, 500), 16, 4096
    sweeps = 4
    idx, val = synth.sparse_tensor(dims, 200_000, 1.2, seed=44)
    U0 = synth.gaussian_factors(dims, R, seed=45)
    Tor = ocp.SparseTensor(dims, idx, val)
    _, _, ref = ocp.cp_als(Tor, U0, sweeps, lambda s, j: _sweep_uniforms(700, s, 3, J)[j],
                           factor_dtype=FACTOR[prec])
    if prec == "fp64":
        fits, _, _ = _run_als(krps, torch, ctx, dims, idx, val, U0, prec, J, sweeps, 700)
        diff = np.max(np.abs(np.array(fits) - np.array(ref)))
        print(f"{prec}: fits {np.round(fits, 6)} oracle {np.round(ref, 6)} max diff {diff:.2e}",
              flush=True)
        assert diff <= 1e-4
        return
    S, T, A = make(krps, torch, ctx, dims, idx, val, U0, prec, J)
    for k in range(3):
        A.normalize(k)
    A.sigma.fill_(1.0)
    fits = []
    for s in range(sweeps):
        u = _sweep_uniforms(700, s, 3, J)
        for j in range(3):
            before = [U.cpu().numpy().astype(np.float64) for U in S.factors]
            A.solve(j, torch.from_numpy(u[j]).to(ctx.device))
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in A.parts(j).items()}
            errs = check_solve(Tor, before, j, got, S.factors[j].cpu().numpy(),
                               A.sigma.cpu().numpy(), prec)
            dr = osmp.KRPSampler(before).draw(j, u[j][:512], scaled=True)
            c = compare(got["idx"][:512], dr, prec)
            assert c["unexcused"] == 0, (s, j)
            print(f"{prec} sweep {s} solve {j}: " +
                  " ".join(f"{k} {v:.1e}" for k, v in errs.items()) +
                  f"; draws differing {c['mismatch']}/512", flush=True)
        fits.append(A.fit())
        fref = ocp.fit(Tor, [U.cpu().numpy() for U in S.factors], A.sigma.cpu().numpy())
        assert abs(fits[-1] - fref) <= 1e-10
    print(f"{prec}: fits {np.round(fits, 6)}; the oracle's own run {np.round(ref, 6)}",
          flush=True)


def test_matrix_case_two_modes(env):
    krps, torch, ctx = env
    dims, R, J = (40, 30), 5, 500
    rng = np.random.default_rng(3)
    idx = np.stack([rng.integers(0, 40, 600), rng.integers(0, 30, 600)], 1).astype(np.int32)
    val = rng.standard_normal(600).astype(np.float32)
    U0 = synth.gaussian_factors(dims, R, seed=4)
    fits, _, _ = _run_als(krps, torch, ctx, dims, idx, val, U0, "fp64", J, 3, 900)
    _, _, ref = ocp.cp_als(ocp.SparseTensor(dims, idx, val), U0, 3,
                           lambda s, j: _sweep_uniforms(900, s, 2, J)[j])
    assert np.max(np.abs(np.array(fits) - np.array(ref))) <= 1e-6


def test_graph_replays_equal_eager_sweeps(env):
    krps, torch, ctx = env
    dims, R, J = (300, 200, 100), 8, 2048
    idx, val = synth.sparse_tensor(dims, 20_000, 1.2, seed=50)
    U0 = synth.gaussian_factors(dims, R, seed=51)
    S, T, A = make(krps, torch, ctx, dims, idx, val, U0, "fp64", J)
    for k in range(3):
        A.normalize(k)
    start = [U.clone() for U in S.factors]
    u = torch.from_numpy(_sweep_uniforms(60, 0, 3, J)).to(ctx.device)

    def restore():
        for k, U in enumerate(S.factors):
            U.copy_(start[k])
            S.refresh(k)
        torch.cuda.synchronize()

    A.sweep(u, use_graph=False)
    torch.cuda.synchronize()
    eager = [U.clone() for U in S.factors]
    eager_sig = A.sigma.clone()
    for rep in range(3):
        restore()
        A.sweep(u, use_graph=True)
        torch.cuda.synchronize()
        for k in range(3):
            assert torch.allclose(S.factors[k], eager[k], rtol=1e-10, atol=1e-12), (rep, k)
        assert torch.allclose(A.sigma, eager_sig, rtol=1e-10)
        # eager work between replays
        _ = (S.factors[0] * 2).sum().item()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_generic_sketched_lstsq_matches_oracle(env, prec):
    """krps_sketched_lstsq on leverage-sampled rows of a dense A (drawn by
    the sampler over A itself, N = 1) and the rows of B at those indices."""
    krps, torch, ctx = env
    rng = np.random.default_rng(11)
    I, R, n, J = 3000, 24, 7, 5000
    A = synth.gaussian_factors((I,), R, seed=12, heavy_rows_frac=0.02)[0]
    B = rng.standard_normal((I, n)).astype(np.float32)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Ad = torch.from_numpy(A).to(ctx.device).to(dt).contiguous()
    S = krps.Sampler(ctx, [Ad], precision=prec)
    u = torch.from_numpy(synth.uniforms(J, 1, 13)).to(ctx.device)
    idx, prob, _ = S.sample(-1, u)
    rows = Ad[idx[:, 0].long()]
    sb = torch.from_numpy(B).to(ctx.device).to(dt)[idx[:, 0].long()]
    X = krps.sketched_lstsq(ctx, rows, prob, sb).cpu().numpy()
    ref = ocp.sketched_lstsq(rows.cpu().numpy(), prob.cpu().numpy(), sb.cpu().numpy())
    np.testing.assert_allclose(X, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())
    # and close to the exact solution (a leverage sketch with J >> R)
    exact = np.linalg.lstsq(A.astype(np.float64), B.astype(np.float64), rcond=None)[0]
    res = np.linalg.norm(A @ X - B) / np.linalg.norm(A @ exact - B)
    assert res < 1.05, res


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("R", [8, 70])
def test_range_finder_init_matches_oracle(env, prec, R):
    """U_j = mat(T, j) S with the generated sketch, normalised: against the
    oracle's sketch (same Philox counters) on a Zipf tensor with duplicates."""
    from oracle import sketch as osk
    krps, torch, ctx = env
    dims = (300, 200, 100)
    idx, val = synth.sparse_tensor(dims, 20_000, 1.2, seed=71)
    Us = synth.gaussian_factors(dims, R, seed=72)
    S, T, A = make(krps, torch, ctx, dims, idx, val, Us, prec, 256)
    Tor = ocp.SparseTensor(dims, idx, val)
    for j in range(3):
        A.init_range_finder(j, seed=12345)
        torch.cuda.synchronize()
        got = S.factors[j].cpu().numpy().astype(np.float64)
        sig = A.sigma.cpu().numpy()
        ref, rsig = ocp.normalize_columns(osk.range_finder(Tor, j, R, 12345))
        # float32 storage: the factor is rounded before its norms are taken
        tol = 1e-10 if prec == "fp64" else 1e-6
        np.testing.assert_allclose(sig, rsig, rtol=tol)
        np.testing.assert_allclose(got, ref, rtol=tol, atol=tol * np.abs(ref).max())
        # the tree was rebuilt: its root is the Gram of the new factor
        np.testing.assert_allclose(S.gram(j).cpu().numpy(), got.T @ got, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
def test_deterministic_solves_repeat_bit_for_bit(env, prec):
    """krps_sampler_set_deterministic: two independent runs of three sweeps
    (eager and replayed from a graph) on a 2e5-entry Zipf tensor give
    bit-identical factors, sigma and fits, and every solve still matches
    the oracle step by step on the GPU's own draw (the fixed-point Y is as
    accurate as the float64 one)."""
    krps, torch, ctx = env
    dims, R, J = (3000, 2000, 500), 16, 4096
    # the workload of test_zipf_tensor_als_matches_oracle, same uniforms
    idx, val = synth.sparse_tensor(dims, 200_000, 1.2, seed=44)
    U0 = synth.gaussian_factors(dims, R, seed=45)
    Tor = ocp.SparseTensor(dims, idx, val)
    runs = []
    for use_graph in (False, True):
        S, T, A = make(krps, torch, ctx, dims, idx, val, U0, prec, J)
        S.set_deterministic(True)
        for k in range(3):
            A.normalize(k)
        A.sigma.fill_(1.0)
        fits = []
        for s in range(3):
            u = _sweep_uniforms(700, s, 3, J)
            if use_graph:
                A.sweep(torch.from_numpy(u).to(ctx.device), use_graph=True)
            else:
                for j in range(3):
                    before = [U.cpu().numpy().astype(np.float64) for U in S.factors]
                    A.solve(j, torch.from_numpy(u[j]).to(ctx.device))
                    torch.cuda.synchronize()
                    got = {k: v.cpu().numpy() for k, v in A.parts(j).items()}
                    errs = check_solve(Tor, before, j, got, S.factors[j].cpu().numpy(),
                                       A.sigma.cpu().numpy(), prec)
                    print(f"deterministic {prec} sweep {s} solve {j}: " +
                          " ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
            fits.append(A.fit())
        torch.cuda.synchronize()
        runs.append(([U.cpu().clone() for U in S.factors], A.sigma.cpu().clone(), fits))
        assert S.check_status() == 0
    (f0, s0, fit0), (f1, s1, fit1) = runs
    for a, b in zip(f0, f1):
        assert torch.equal(a, b)
    assert torch.equal(s0, s1) and fit0 == fit1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_warm_started_preparations_match_the_oracle(env, prec):
    """The solves of a sweep start each eigendecomposition of G_{>k} from
    the last solve's eigenvectors of the same exclusion and mode: after
    every solve of three sweeps the preparation (eigenvalues, isolated
    eigenvectors, the whole decomposition, G^+) matches the oracle's from
    the factors the solve started from, and the warm-started solves need
    fewer Jacobi sweeps than the first, cold ones."""
    krps, torch, ctx = env
    dims, R, J = (3000, 2000, 500), 16, 4096
    idx, val = synth.sparse_tensor(dims, 200_000, 1.2, seed=44)
    U0 = synth.gaussian_factors(dims, R, seed=45)
    S, T, A = make(krps, torch, ctx, dims, idx, val, U0, prec, J)
    for k in range(3):
        A.normalize(k)
    A.sigma.fill_(1.0)
    sweeps_used = []
    for s in range(3):
        u = _sweep_uniforms(700, s, 3, J)
        for j in range(3):
            before = [U.cpu().numpy().astype(np.float64) for U in S.factors]
            A.solve(j, torch.from_numpy(u[j]).to(ctx.device))
            torch.cuda.synchronize()
            parts = A.draw_parts()
            Gp, rank, eig, _ = osmp.KRPSampler(before).prepare(j)
            assert parts["rank"] == rank
            gp = parts["gplus"].cpu().numpy()
            assert np.abs(gp - Gp).max() <= 1e-9 * np.abs(Gp).max()
            for st, k in enumerate(m for m in range(3) if m != j):
                lam, V = eig[k]
                lg = parts["lam"][k].cpu().numpy()
                assert np.abs(lg - lam).max() <= 1e-10 * lam.max(), (s, j, k)
                Vg = parts["vecs"][k].cpu().numpy().astype(np.float64).T
                gaps = np.diff(lam)
                iso = np.ones(R, dtype=bool)
                iso[1:] &= gaps > 1e-6 * lam.max()
                iso[:-1] &= gaps > 1e-6 * lam.max()
                dots = np.abs(np.einsum("eu,eu->u", Vg, V))
                assert np.abs(dots[iso] - 1).max() <= (1e-9 if prec == "fp64" else 1e-6)
                rec = (Vg * lg) @ Vg.T
                ref = (V * lam) @ V.T
                assert np.abs(rec - ref).max() <= (1e-9 if prec == "fp64" else 1e-5) * \
                    np.abs(ref).max()
                sweeps_used.append((s, parts["sweeps"][1 + st]))
    cold = [n for s, n in sweeps_used if s == 0]
    warm = [n for s, n in sweeps_used if s > 0]
    print(f"{prec}: Jacobi sweeps, first sweep's solves {cold}, later {warm}", flush=True)
    assert np.mean(warm) < np.mean(cold)
