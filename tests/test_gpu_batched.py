"""GPU tests of the batched draw (many samplers, one persistent walk launch
per storage type) through the C ABI.  Run with ``-m gpu``."""
import numpy as np
import pytest

import synth
from oracle import sampler as osmp
from parity import compare, report

pytestmark = pytest.mark.gpu

TOL_PROB = {"fp64": 1e-10, "fp32": 1e-9, "bf16x2": 1e-9}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2301_12584_amd as krps
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return krps, torch, krps.Context(0)


# (dims, R, precision, exclude): every shape class of the walk, I < F,
# N = 1, R = 1, mixed precisions in one batch
PROBLEMS = [
    ((300, 200, 100), 8, "fp32", -1),
    ((64, 64, 64), 16, "fp64", 0),
    ((5000, 40, 3000), 32, "fp32", 1),
    ((700, 900), 48, "bf16x2", -1),
    ((20, 3000, 500, 100), 64, "fp32", 2),
    ((1000, 600, 80), 100, "fp64", -1),
    ((400, 300, 200), 128, "fp32", 0),
    ((50,), 5, "fp64", -1),
    ((30, 10), 1, "fp32", -1),
    ((7, 9, 11, 5, 3), 12, "fp32", 4),
]


def make(krps, torch, ctx, dims, R, prec, seed):
    Us = synth.gaussian_factors(dims, R, seed, heavy_rows_frac=0.02)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Ud = [torch.from_numpy(U).to(ctx.device).to(dt).contiguous() for U in Us]
    return Us, krps.Sampler(ctx, Ud, precision=prec)


def test_batched_equals_one_call_per_problem(env):
    krps, torch, ctx = env
    samplers, excl, unis, Us_all = [], [], [], []
    Js = [3000, 2000, 4096, 1000, 777, 1500, 512, 900, 300, 2048]
    for p, (dims, R, prec, ex) in enumerate(PROBLEMS):
        Us, S = make(krps, torch, ctx, dims, R, prec, 900 + p)
        samplers.append(S)
        excl.append(ex)
        Us_all.append(Us)
        unis.append(torch.from_numpy(synth.uniforms(Js[p], len(dims), 950 + p)).to(ctx.device))
    print("batched: P =", len(samplers), flush=True)
    idx_b, prob_b = krps.sample_batched(ctx, samplers, excl, unis)
    torch.cuda.synchronize()
    for p, S in enumerate(samplers):
        print("single", p, PROBLEMS[p], flush=True)
        idx_s, prob_s, _ = S.sample(excl[p], unis[p])
        torch.cuda.synchronize()
        assert torch.equal(idx_b[p], idx_s), p
        assert torch.equal(prob_b[p], prob_s), p


@pytest.mark.parametrize("p", [0, 2, 4, 6])
def test_batched_matches_oracle(env, p):
    krps, torch, ctx = env
    sel = [p, (p + 3) % len(PROBLEMS), (p + 5) % len(PROBLEMS)]
    samplers, excl, unis, Us_all, u_host = [], [], [], [], []
    for q in sel:
        dims, R, prec, ex = PROBLEMS[q]
        Us, S = make(krps, torch, ctx, dims, R, prec, 900 + q)
        samplers.append(S)
        excl.append(ex)
        Us_all.append(Us)
        u = synth.uniforms(1024, len(dims), 970 + q)
        u_host.append(u)
        unis.append(torch.from_numpy(u).to(ctx.device))
    idx_b, prob_b = krps.sample_batched(ctx, samplers, excl, unis)
    torch.cuda.synchronize()
    for i, q in enumerate(sel):
        dims, R, prec, ex = PROBLEMS[q]
        dr = osmp.KRPSampler(Us_all[i]).draw(ex, u_host[i], scaled=prec != "fp64")
        c = compare(idx_b[i].cpu().numpy(), dr, prec)
        report(f"batched problem {q} {prec} dims={dims} R={R}", c)
        same = c["same"]
        pr = prob_b[i].cpu().numpy()
        rel = np.abs(pr[same] - dr.prob[same]) / dr.prob[same]
        assert rel.max() <= TOL_PROB[prec], rel.max()
        assert c["unexcused"] == 0


def test_batched_seeded_equals_per_problem_seeded_draws(env):
    """krps_sample_batched_seeded: every problem's walk generates its
    uniforms from its own (seed, ctr_base); the result equals one
    krps_sample_seeded call per problem and matches the oracle's draw with
    the oracle's Philox uniforms."""
    from oracle import sketch as osk
    krps, torch, ctx = env
    sel = [0, 2, 5, 9]
    samplers, excl, Us_all = [], [], []
    for q in sel:
        dims, R, prec, ex = PROBLEMS[q]
        Us, S = make(krps, torch, ctx, dims, R, prec, 900 + q)
        samplers.append(S)
        excl.append(ex)
        Us_all.append(Us)
    J = [1500, 800, 1024, 700]
    seeds = [11, 12, 13, 11]
    bases = [0, 5000, 77, 10 ** 12]
    batch = krps.Batch(ctx, samplers, excl)
    idx_b, prob_b = batch.sample_seeded(J, seeds, bases)
    torch.cuda.synchronize()
    for i, S in enumerate(samplers):
        ri, rp = S.sample_seeded(excl[i], J[i], seeds[i], bases[i])
        torch.cuda.synchronize()
        assert torch.equal(idx_b[i], ri), i
        assert torch.equal(prob_b[i], rp), i
    dims, R, prec, ex = PROBLEMS[sel[1]]
    u = osk.philox_uniforms(J[1], len(dims), seeds[1], bases[1])
    dr = osmp.KRPSampler(Us_all[1]).draw(ex, u, scaled=True)
    c = compare(idx_b[1].cpu().numpy(), dr, prec)
    report("batched seeded vs oracle", c)
    assert c["unexcused"] == 0


def test_batched_empty_problem_and_no_prob(env):
    krps, torch, ctx = env
    _, S1 = make(krps, torch, ctx, (100, 80, 60), 8, "fp32", 1)
    _, S2 = make(krps, torch, ctx, (90, 70), 16, "fp32", 2)
    u1 = torch.from_numpy(synth.uniforms(0, 3, 1)).to(ctx.device)
    u2 = torch.from_numpy(synth.uniforms(640, 2, 2)).to(ctx.device)
    idx, prob = krps.sample_batched(ctx, [S1, S2], [-1, 0], [u1, u2], with_prob=False)
    torch.cuda.synchronize()
    assert idx[0].shape == (0, 3) and prob[1] is None
    ref, _, _ = S2.sample(0, u2)
    assert torch.equal(idx[1], ref)
    # a second batched call reuses the context's staging buffer
    idx2, _ = krps.sample_batched(ctx, [S2], [0], [u2])
    torch.cuda.synchronize()
    assert torch.equal(idx2[0], ref)


def test_one_sampler_all_exclusions_prepare_then_draw(env):
    """The same sampler listed once per exclusion; the walk is drawn twice
    after one preparation and equals one krps_sample per exclusion."""
    krps, torch, ctx = env
    _, S = make(krps, torch, ctx, (4000, 3000, 2000), 32, "fp32", 5)
    J = 4096
    unis = [torch.from_numpy(synth.uniforms(J, 3, 60 + k)).to(ctx.device) for k in range(3)]
    batch = krps.Batch(ctx, [S, S, S], [0, 1, 2])
    batch.prepare()
    idx = [torch.empty((J, 3), dtype=torch.int32, device=ctx.device) for _ in range(3)]
    prob = [torch.empty(J, dtype=torch.float64, device=ctx.device) for _ in range(3)]
    for rep in range(2):
        batch.draw(unis, idx, prob)
        torch.cuda.synchronize()
        for k in range(3):
            ref_i, ref_p, _ = S.sample(k, unis[k])
            torch.cuda.synchronize()
            assert torch.equal(idx[k], ref_i), (rep, k)
            assert torch.equal(prob[k], ref_p), (rep, k)
