"""The least-squares accuracy experiment of Section 4.2 on GPU draws:
A = U_1 (.) ... (.) U_N with I = 2^16 (N(0,1) entries, 1% of them x10),
b = c_1 (x) ... (x) c_N, J = 5000 leverage samples, N up to 9.  The GPU's
draws and its sketched solve (krps_sample + krps_sketched_lstsq) against the
oracle on the same draws: probabilities, the solution, the residual error
eps and the distortion (Appendix A.12).  Run with ``-m gpu``."""
import numpy as np
import pytest

import synth
from oracle import accuracy as acc
from oracle import cp as ocp
from oracle import sampler as osmp
from parity import compare, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2301_12584_amd as krps
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return krps, torch, krps.Context(0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [3, 6, 9])
def test_ls_accuracy_on_gpu_draws(env, prec, N):
    krps, torch, ctx = env
    I, R, J, trials = 1 << 16, 16, 5000, 3
    Us = synth.gaussian_factors((I,) * N, R, seed=4200 + N, heavy_entries_frac=0.01)
    rng = np.random.default_rng(4300 + N)
    cs = [rng.standard_normal(I) for _ in range(N)]
    P = acc.KronProblem(Us, cs)
    dt = torch.float64 if prec == "fp64" else torch.float32
    S = krps.Sampler(ctx, [torch.from_numpy(U).to(ctx.device).to(dt).contiguous() for U in Us],
                     precision=prec)
    orc = osmp.KRPSampler(Us)
    eps, dist = [], []
    for t in range(trials):
        u01 = synth.uniforms(J, N, 4400 + 10 * N + t)
        idx, prob, rows = S.sample(-1, torch.from_numpy(u01).to(ctx.device), rows=True,
                                   check_status=True)
        gi = idx.cpu().numpy().astype(np.int64)
        sb = P.b_entries(gi)
        X = krps.sketched_lstsq(ctx, rows, prob, torch.from_numpy(sb[:, None]).to(ctx.device)
                                .to(dt)).cpu().numpy()[:, 0]
        gp = prob.cpu().numpy()
        # the oracle on the GPU's draw: rows and probabilities by definition
        a = P.rows(gi)
        q = orc.row_prob(-1, gi)
        np.testing.assert_allclose(gp, q, rtol=1e-10 if prec == "fp64" else 1e-9)
        rg = rows.cpu().numpy().astype(np.float64)        # in the factor type
        np.testing.assert_allclose(rg, a, rtol=1e-14 if prec == "fp64" else 2.0 ** -23)
        # the sketched solve on the same (stored) rows and right-hand side
        sbg = sb if prec == "fp64" else sb.astype(np.float32).astype(np.float64)
        Xr = ocp.sketched_lstsq(rg, gp, sbg[:, None])[:, 0]
        np.testing.assert_allclose(X, Xr, rtol=1e-9, atol=1e-12 * np.abs(Xr).max())
        # eps and the distortion against the oracle's from exact rows
        Xe = ocp.sketched_lstsq(a, q, sb[:, None])[:, 0]
        e_g, e_r = P.epsilon(X), P.epsilon(Xe)
        d_g = acc.distortion(P.G, rg, gp)
        d_r = acc.distortion(P.G, a, q)
        tol = 1e-8 if prec == "fp64" else 1e-5
        assert abs(e_g - e_r) <= tol * (1 + e_r), (e_g, e_r)
        assert abs(d_g - d_r) <= tol * (1 + d_r), (d_g, d_r)
        eps.append(e_g)
        dist.append(d_g)
        if t == 0:
            sel = np.arange(400)
            dr = orc.draw(-1, u01[sel], scaled=prec != "fp64")
            c = compare(gi[sel], dr, prec)
            report(f"ls accuracy draws {prec} N={N}", c)
            assert c["unexcused"] == 0
    print(f"ls accuracy {prec} N={N} R={R} J={J}: eps {np.mean(eps):.2e} "
          f"(trials {np.round(eps, 4)}), distortion {np.mean(dist):.3f}", flush=True)
    # the leverage sketch's regime (Theorem 2.1): a small residual error at
    # every N, the paper's ~1e-2 at N = 9
    assert np.mean(eps) < 0.05
