"""Checks that pin the oracle to what the paper and the mathematics fix.

Each ``check_*`` returns an error figure (0 when exact) so that the same
check serves the pin tests (figure must be tiny) and the planted-mistake
tests (a deliberately broken oracle must make some figure large).
"""
from __future__ import annotations

import numpy as np

from oracle import definition as dfn
from oracle import sampler as smp


def krp_excluding(Us, exclude):
    return dfn.khatri_rao([U for k, U in enumerate(Us) if k != exclude])


def flat_rows(idx, dims, exclude):
    modes = [k for k in range(len(dims)) if k != exclude]
    return np.ravel_multi_index(tuple(idx[:, k] for k in modes),
                                tuple(dims[k] for k in modes))


def check_prob_vs_qr(sampler, Us, exclude, u01):
    """Max relative error of the draw's ``q_d`` against QR leverage / rank."""
    dims = [U.shape[0] for U in Us]
    A = krp_excluding(Us, exclude)
    lev = dfn.leverage_qr(A)
    p = lev / lev.sum()
    dr = sampler.draw(exclude, u01)
    r = flat_rows(dr.idx, dims, exclude)
    return float(np.max(np.abs(dr.prob - p[r]) / p[r])), dr, p, r


def check_walk_vs_scan(tree, H, dvec, Y=None):
    """Fraction of draws whose tree walk disagrees with a linear scan of the
    full distribution (draws with margin <= 1e-12 excused)."""
    rows, margin, _ = smp.row_sample_batch(tree, H, Y, dvec)
    U = tree.U
    bad = 0
    for d in range(H.shape[0]):
        q, _ = dfn.conditional_q(H[d], U, np.ones((U.shape[1],) * 2) if Y is None else Y)
        cdf = np.cumsum(q)
        ref = int(np.searchsorted(cdf, dvec[d], side="left"))
        ref = min(ref, U.shape[0] - 1)
        if ref != rows[d] and margin[d] > 1e-12:
            bad += 1
    return bad / H.shape[0]


def check_thm31_product(Us, exclude, multi):
    """Max relative error between the product of the conditionals of
    Theorem 3.1 and the QR leverage score / rank, over multi-indices."""
    N = len(Us)
    R = Us[0].shape[1]
    modes = [k for k in range(N) if k != exclude]
    G = dfn.hadamard_all([Us[k].T.astype(np.float64) @ Us[k] for k in modes])
    Gp, rank = dfn.pinv_psd(G)
    A = krp_excluding(Us, exclude)
    lev = dfn.leverage_qr(A)
    dims = [U.shape[0] for U in Us]
    worst = 0.0
    for m in multi:
        h = np.ones(R)
        prob = 1.0
        for k in modes:
            later = [Us[x].T.astype(np.float64) @ Us[x] for x in modes if x > k]
            Ggt = Gp * dfn.hadamard_all(later) if later else Gp
            q, _ = dfn.conditional_q(h, Us[k], Ggt)
            prob *= q[m[k]]
            h = h * Us[k][m[k]]
        r = flat_rows(np.asarray([m]), dims, exclude)[0]
        ref = lev[r] / lev.sum()
        worst = max(worst, abs(prob - ref) / ref)
    return worst


def check_two_stage_vs_bruteforce(sampler, Us, exclude, u01, excuse=1e-9):
    """Fraction of draws whose multi-index differs from a brute-force
    two-stage inversion with the same uniforms.

    The brute force follows Section 3.2 with full distributions and no
    trees: stage 1 draws ``u`` from ``q_{h, sqrt(Lambda) V^T, G_k}`` (first
    stage distribution), stage 2 draws ``t`` from ``q_{h (*) V[:,u], U_k, [1]}``
    (second stage), each by a linear scan of its CDF (first bin whose
    cumulative sum reaches the uniform).  Draws whose uniform lies within
    ``excuse`` of a CDF edge are excused.
    """
    N = len(Us)
    R = Us[0].shape[1]
    modes = [k for k in range(N) if k != exclude]
    Gs = [U.T.astype(np.float64) @ U for U in Us]
    G = dfn.hadamard_all([Gs[k] for k in modes])
    Gp, _ = dfn.pinv_psd(G)
    eig = {}
    for k in modes:
        later = [Gs[m] for m in modes if m > k]
        Ggt = Gp * dfn.hadamard_all(later) if later else Gp
        lam, V = np.linalg.eigh((Ggt + Ggt.T) * 0.5)
        eig[k] = (np.maximum(lam, 0.0), V)
    dr = sampler.draw(exclude, u01)
    ones = np.ones((R, R))
    bad = 0
    J = u01.shape[0]
    for d in range(J):
        h = np.ones(R)
        ok = True
        close = False
        for k in modes:
            lam, V = eig[k]
            w, _ = dfn.conditional_q(h, np.sqrt(lam)[:, None] * V.T, Gs[k])
            cw = np.cumsum(w)
            u = min(int(np.searchsorted(cw, u01[d, k, 0], side="left")), R - 1)
            close |= np.min(np.abs(cw - u01[d, k, 0])) <= excuse
            q2, _ = dfn.conditional_q(h * V[:, u], Us[k], ones)
            c2 = np.cumsum(q2)
            t = min(int(np.searchsorted(c2, u01[d, k, 1], side="left")), len(q2) - 1)
            close |= np.min(np.abs(c2 - u01[d, k, 1])) <= excuse
            if t != dr.idx[d, k]:
                ok = False
                break
            h = h * Us[k][t]
        if not ok and not close:
            bad += 1
    return bad / J
