"""Parity at the full workload sizes, in the launch configuration the
benchmark times, on sampled outputs the oracle computes one by one and on
properties that hold at any size.  Run with ``-m gpu``."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import sampler as osmp

pytestmark = pytest.mark.gpu

MARGIN = 1e-6
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2301_12584_amd as krps
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return krps, torch, krps.Context(0)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sampler_at_scale_sampled_against_oracle(env, prec):
    """N = 3 factors of 2^20 x 32 (1% rows x100), J = 65,536 per excluded
    mode, the three exclusions prepared and walked as one batch."""
    krps, torch, ctx = env
    cfg = synth.CONFIGS[2]
    dims, R, J, N = cfg["dims"], cfg["R"], cfg["J"], cfg["N"]
    print(f"sampler at scale {prec}", flush=True)
    Us = synth.gaussian_factors(dims, R, synth.config_seed(2),
                                heavy_rows_frac=cfg["heavy_rows_frac"],
                                heavy_row_scale=cfg["heavy_row_scale"])
    u01 = [synth.uniforms(J, N, synth.uniform_seed(2) + k) for k in range(N)]
    dt = torch.float64 if prec == "fp64" else torch.float32
    S = krps.Sampler(ctx, [torch.from_numpy(U).to(ctx.device).to(dt).contiguous() for U in Us],
                     precision=prec)
    batch = krps.Batch(ctx, [S] * N, list(range(N)))
    ud = [torch.from_numpy(u).to(ctx.device) for u in u01]
    idx_l, prob_l = batch.sample(ud)
    torch.cuda.synchronize()
    orc = osmp.KRPSampler(Us, store=None if prec == "fp64" else np.float32)
    rng = np.random.default_rng(5)
    for k in range(N):
        idx = idx_l[k].cpu().numpy().astype(np.int64)
        prob = prob_l[k].cpu().numpy()
        # properties over all J draws
        assert (idx[:, k] == -1).all()
        for m in range(N):
            if m != k:
                assert idx[:, m].min() >= 0 and idx[:, m].max() < dims[m]
        assert np.all(prob > 0) and np.all(np.isfinite(prob))
        rp = S.row_prob(k, idx_l[k]).cpu().numpy()
        np.testing.assert_allclose(prob, rp, rtol=1e-12)
        # sampled draws against the oracle
        sel = np.sort(rng.choice(J, 192, replace=False))
        dr = orc.draw(k, u01[k][sel])
        same = (idx[sel] == dr.idx).all(axis=1)
        assert np.all(same | (dr.margin <= MARGIN)), (k, np.sum(~same))
        tol = 1e-10 if prec == "fp64" else 1e-5
        np.testing.assert_allclose(prob[sel][same], dr.prob[same], rtol=tol)


def test_batched_samplers_at_scale(env):
    """The 64-sampler workload (N in {3,4,5}, I log-uniform [2^10, 2^22],
    R in {16,32,64,128}, J = 16,384 each): one batched call equals one call
    per problem for every problem, and sampled draws of the problems with
    the smallest factors match the oracle."""
    krps, torch, ctx = env
    probs = synth.batched_problems(64, synth.config_seed(4))
    J = synth.CONFIGS[4]["J"]
    g = torch.Generator(device=ctx.device)
    g.manual_seed(synth.config_seed(4))
    samplers, unis, facs = [], [], []
    for p, (dims, R) in enumerate(probs):
        Ud = [torch.randn((I, R), generator=g, device=ctx.device, dtype=torch.float32)
              for I in dims]
        facs.append(Ud)
        samplers.append(krps.Sampler(ctx, Ud, precision="fp32"))
        unis.append(torch.from_numpy(synth.uniforms(J, len(dims), synth.uniform_seed(4) + p))
                    .to(ctx.device))
    print("batched at scale: samplers built", flush=True)
    batch = krps.Batch(ctx, samplers, [-1] * len(probs))
    idx_b, prob_b = batch.sample(unis)
    torch.cuda.synchronize()
    for p, S in enumerate(samplers):
        ri, rp, _ = S.sample(-1, unis[p])
        torch.cuda.synchronize()
        assert torch.equal(idx_b[p], ri), p
        assert torch.equal(prob_b[p], rp), p
    small = sorted(range(len(probs)), key=lambda p: sum(probs[p][0]) * probs[p][1] ** 2)[:3]
    rng = np.random.default_rng(6)
    for p in small:
        Us = [U.cpu().numpy() for U in facs[p]]
        orc = osmp.KRPSampler(Us, store=np.float32)
        sel = np.sort(rng.choice(J, 128, replace=False))
        u = unis[p].cpu().numpy()[sel]
        dr = orc.draw(-1, u)
        got = idx_b[p].cpu().numpy().astype(np.int64)[sel]
        same = (got == dr.idx).all(axis=1)
        assert np.all(same | (dr.margin <= MARGIN)), (p, np.sum(~same))
        np.testing.assert_allclose(prob_b[p].cpu().numpy()[sel][same], dr.prob[same], rtol=1e-5)
    del samplers, facs, batch
    torch.cuda.empty_cache()


def _golden(store):
    path = os.path.join(GOLDEN, f"als_fits_c3_{store}.json")
    return json.load(open(path)) if os.path.exists(path) else None


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
def test_sketched_cp_als_at_scale_against_oracle_fits(env, prec):
    """The sketched CP-ALS workload (1e6 x 1e6 x 1e5, 1e8 Zipf(1.2)
    entries, R = 64, J = 65,536, 10 sweeps, graph replay) against the
    fits the float64 oracle stored for the same inputs and uniforms."""
    krps, torch, ctx = env
    ref = _golden("f64" if prec == "fp64" else "f32")
    if ref is None:
        pytest.skip("oracle fits of the 1e8-entry workload not stored")
    dims, idx, val, U0, R, J, sweeps, useed = synth.als_problem(3)
    assert ref["nnz"] == len(val) and ref["sweeps"] == sweeps
    T = krps.Tensor(ctx, dims, torch.from_numpy(idx).to(ctx.device),
                    torch.from_numpy(val).to(ctx.device))
    del idx, val
    dt = torch.float64 if prec == "fp64" else torch.float32
    S = krps.Sampler(ctx, [torch.from_numpy(U).to(ctx.device).to(dt).contiguous() for U in U0],
                     precision=prec)
    A = krps.CPALS(S, T, J)
    for k in range(3):
        A.normalize(k)
    A.sigma.fill_(1.0)
    ubuf = torch.empty((3, J, 3, 2), dtype=torch.float64, device=ctx.device)
    fits = []
    for s in range(sweeps):
        ubuf.copy_(torch.from_numpy(synth.sweep_uniforms(useed, s, 3, J)))
        A.sweep(ubuf, use_graph=True)
        fits.append(A.fit())
    diff = np.abs(np.array(fits) - np.array(ref["fits"]))
    print(f"{prec}: fits {np.round(fits, 6)} oracle {np.round(ref['fits'], 6)} "
          f"max diff {diff.max():.2e}", flush=True)
    # The early sweeps are sensitive.  At the random start G and every
    # G_{>k} are close to the identity (eigenvalue gaps ~1e-5 relative), so
    # their eigenvectors inside near-degenerate clusters are fixed only up to
    # a rotation that any rounding difference changes.  The first stage of
    # the draw picks an eigencomponent (Section 3.2), so two correct
    # implementations draw from the same distribution but realise different
    # sketches from the same uniforms (measured: 152 of 65,536 draws of the
    # very first solve differ between two GPU pseudo-inverse routes whose
    # G^+ agree to 1e-13).  The fits then differ by sketch noise, large at
    # the first sweeps (the fit after one sweep ranges over 0.63-0.78
    # between sketches) and damped by the later ones: the last sweep is held
    # to 1e-4 (1e-3 for the split Grams) and every sweep from the third on to
    # 3e-4 (2e-3).
    last, every = (1e-3, 2e-3) if prec == "bf16x2" else (1e-4, 3e-4)
    assert diff[-1] <= last
    assert diff[2:].max() <= every
