"""Method-level oracle: the exact Khatri-Rao leverage sampler step by step.

Follows the paper's construction in its own order and notation:

* :class:`SegmentTree` -- ``BuildSampler(U, F, Y)`` (Appendix A.5,
  Algorithm 3): a full, complete binary tree over ``ceil(I/F)`` leaves, each
  node ``v`` caching the partial Gram matrix ``G^v = sum_{i in S(v)} U[i]^T U[i]``
  (Section 3.1, partial Gram equation).
* :func:`row_sample` / :func:`row_sample_batch` -- ``RowSample(h)``
  (Appendix A.5, Algorithm 4): inversion sampling by a root-to-leaf walk,
  branching left iff ``low + m(L(c)) >= d``, then a linear scan of the leaf.
* :class:`KRPSampler` -- ``ConstructKRPSampler`` / ``KRPSample``
  (Section 3.2, Algorithms 1 and 2): the per-factor trees ``Z_j`` with
  ``F = R`` and ``Y = [1]``, then per draw the eigen-trees ``E_k`` over
  ``sqrt(Lambda_k) V_k^T`` with ``F = 1`` and ``Y = G_k`` and the two-stage
  draw of each mode.

Readings of the paper used here (where it is silent or garbled):

* The tree is padded to ``2^D`` leaves, ``D = ceil(log2(ceil(I/F)))``; pad
  nodes have zero mass and are never visited.  Left children hold the lower
  row indices (Section 3.1, segment-tree figure).
* The normalisation by ``C`` is applied to the target instead of the node
  masses: the walk compares ``x = d * C`` with unnormalised masses.
* Leaf scan: the row picked is ``S_0(c) + i`` for the smallest 0-based ``i``
  with ``low + sum_{m <= i} q~[m] >= x`` (ties go to the lower bin).
* Rounding guards: a negative computed node mass counts as 0; if the right
  subtree's implied mass ``high - cut`` is not positive, or the right child
  does not exist, the walk goes left; if the leaf scan never reaches ``x``
  the last row of the leaf with positive mass is taken (else the last row).
* ``G_{>k} = G^+ (*) prod_{m > k, m != j} G_m`` (the index of the printed
  Algorithm 2 collides with the loop variable; this is the definition in
  Section 3, equation for ``G_{>k}``).  Eigenvalues are sorted ascending and
  negative ones (rounding) are clamped to 0.  The modes ``k != j`` are drawn
  in increasing order.
* Sample probability ``q_d = a_d G^+ a_d^T / rank(G)`` with ``a_d`` the
  sampled Khatri-Rao row (Section 2.1, leverage definition; the scores sum
  to the rank).
"""
from __future__ import annotations

import math

import numpy as np

from .definition import pinv_psd, hadamard_all

__all__ = ["SegmentTree", "row_sample", "row_sample_batch", "KRPSampler", "Draw"]


class SegmentTree:
    """``T_{I,F}`` with partial Gram matrices at every node (Algorithm 3).

    ``levels[l]`` is an array ``[real_l, R, R]`` of the real (non-pad) nodes
    of level ``l``; level 0 is the root and level ``D`` the leaves.  The
    node at level ``l`` and position ``p`` covers the rows of leaves
    ``[p * 2^(D-l), (p+1) * 2^(D-l))``.
    """

    def __init__(self, U, F):
        U = np.asarray(U, dtype=np.float64)
        self.U = U
        self.I, self.R = U.shape
        self.F = int(F)
        if self.I < 1 or self.F < 1:
            raise ValueError("need I >= 1 and F >= 1")
        self.L = -(-self.I // self.F)
        self.D = int(math.ceil(math.log2(self.L))) if self.L > 1 else 0
        D, L, F, R = self.D, self.L, self.F, self.R
        # leaves: G^v = U[S(v)]^T U[S(v)]
        pad = np.zeros((L * F, R))
        pad[: self.I] = U
        blocks = pad.reshape(L, F, R)
        levels = [None] * (D + 1)
        levels[D] = np.matmul(blocks.transpose(0, 2, 1), blocks)
        # internal nodes, level by level from the one above the leaves
        for lev in range(D - 1, -1, -1):
            child = levels[lev + 1]
            n = self.real(lev)
            G = np.zeros((n, R, R))
            G += child[0::2][:n]
            right = child[1::2]
            G[: right.shape[0]] += right
            levels[lev] = G
        self.levels = levels

    def real(self, lev):
        """Number of real nodes at level ``lev``."""
        return -(-self.L // (1 << (self.D - lev)))

    @property
    def root(self):
        return self.levels[0][0]

    def segment(self, c):
        """Rows ``[S_0, S_1)`` of leaf ``c``."""
        s0 = c * self.F
        return s0, min(s0 + self.F, self.I)


def _gen_inner(h, G, Y):
    """``<h h^T, G, Y>`` for one vector ``h`` (``Y`` None means all ones)."""
    M = G if Y is None else G * Y
    return float(h @ M @ h)


def row_sample(tree, h, Y, d):
    """``RowSample(h)`` of Algorithm 4 for one uniform ``d`` in (0, 1).

    Returns ``(row, min_margin)`` where the margin of a comparison is
    ``|x - cut| / C``.
    """
    h = np.asarray(h, dtype=np.float64)
    C = _gen_inner(h, tree.root, Y)
    x = d * C
    low, high = 0.0, C
    pos = 0
    margin = math.inf
    for lev in range(1, tree.D + 1):
        left = 2 * pos
        mL = max(_gen_inner(h, tree.levels[lev][left], Y), 0.0)
        cut = low + mL
        margin = min(margin, abs(x - cut) / C)
        right_exists = left + 1 < tree.real(lev)
        if cut >= x or not right_exists or high - cut <= 0.0:
            pos, high = left, cut
        else:
            pos, low = left + 1, cut
    s0, s1 = tree.segment(pos)
    W = tree.U[s0:s1] * h[None, :]
    if Y is None:
        qt = (W.sum(axis=1)) ** 2
    else:
        qt = np.einsum("ia,ab,ib->i", W, Y, W)
    acc = low
    chosen = None
    for i, qi in enumerate(qt):
        acc += qi
        margin = min(margin, abs(x - acc) / C)
        if chosen is None and acc >= x:
            chosen = i
    if chosen is None:
        pos_rows = np.nonzero(qt > 0)[0]
        chosen = int(pos_rows[-1]) if pos_rows.size else (s1 - s0 - 1)
    return s0 + chosen, margin


def row_sample_batch(tree, H, Y, dvec, chunk=None):
    """Algorithm 4 for many independent samples at once (the samples march
    level by level, as in the batch-synchronous strategy of Appendix A.10).

    ``H``: ``[J, R]`` history vectors, ``dvec``: ``[J]`` uniforms.  Returns
    ``(rows [J] int64, min_margin [J])``.
    """
    H = np.asarray(H, dtype=np.float64)
    J, R = H.shape
    rows = np.empty(J, dtype=np.int64)
    margins = np.empty(J)
    if chunk is None:
        chunk = max(64, (1 << 23) // (R * R))
    for s in range(0, J, chunk):
        e = min(J, s + chunk)
        rows[s:e], margins[s:e] = _row_sample_chunk(tree, H[s:e], Y, dvec[s:e])
    return rows, margins


def _masses(Gs, HH):
    # <h h^T, G> for a batch: sum over (a, b) of (h_a h_b Y_ab) G_ab
    return np.einsum("dab,dab->d", Gs, HH)


def _row_sample_chunk(tree, H, Y, dvec):
    n, R = H.shape
    HH = H[:, :, None] * H[:, None, :]
    if Y is not None:
        HH = HH * Y[None]
    C = _masses(np.broadcast_to(tree.root, (n, R, R)), HH)
    x = dvec * C
    low = np.zeros(n)
    high = C.copy()
    pos = np.zeros(n, dtype=np.int64)
    margin = np.full(n, np.inf)
    for lev in range(1, tree.D + 1):
        left = 2 * pos
        mL = np.maximum(_masses(tree.levels[lev][left], HH), 0.0)
        cut = low + mL
        margin = np.minimum(margin, np.abs(x - cut) / C)
        right_exists = (left + 1) < tree.real(lev)
        go_left = (cut >= x) | (~right_exists) | (high - cut <= 0.0)
        pos = np.where(go_left, left, left + 1)
        high = np.where(go_left, cut, high)
        low = np.where(go_left, low, cut)
    F = tree.F
    s0 = pos * F
    if F == 1:
        # a one-row leaf: the scan can only return that row, and its right
        # edge is a boundary already compared above
        return s0, margin
    offs = np.arange(F)
    ridx = s0[:, None] + offs[None, :]
    valid = ridx < tree.I
    Wr = tree.U[np.minimum(ridx, tree.I - 1)] * H[:, None, :]
    if Y is None:
        qt = Wr.sum(axis=2) ** 2
    else:
        qt = np.einsum("dia,ab,dib->di", Wr, Y, Wr)
    qt = np.where(valid, qt, 0.0)
    acc = low[:, None] + np.cumsum(qt, axis=1)
    margin = np.minimum(margin, np.where(valid, np.abs(x[:, None] - acc) / C[:, None],
                                         np.inf).min(axis=1))
    hit = (acc >= x[:, None]) & valid
    any_hit = hit.any(axis=1)
    first = np.argmax(hit, axis=1)
    posm = (qt > 0) & valid
    last_pos = F - 1 - np.argmax(posm[:, ::-1], axis=1)
    last_valid = np.minimum(tree.I - s0, F) - 1
    fallback = np.where(posm.any(axis=1), last_pos, last_valid)
    chosen = np.where(any_hit, first, fallback)
    return s0 + chosen, margin


def _round(a, dtype):
    return np.asarray(a).astype(dtype).astype(np.float64)


class Draw:
    """Result of one ``KRPSample`` call."""

    def __init__(self, idx, rows, prob, margin, rank, Gp, eig, degenerate):
        self.idx = idx            # [J, N] int64, -1 in the excluded column
        self.rows = rows          # [J, R] sampled KRP rows a_d (float64)
        self.prob = prob          # [J] q_d = a_d G^+ a_d^T / rank
        self.margin = margin      # [J] smallest |x - cut| / C along the draw
        self.rank = rank
        self.Gp = Gp              # pseudo-inverse of G = (*)_{k != j} G_k
        self.eig = eig            # {k: (lam ascending, V)} of G_{>k}
        self.degenerate = degenerate  # some G_{>k} has a near-degenerate gap


class KRPSampler:
    """``ConstructKRPSampler`` (Algorithm 1) and ``KRPSample`` (Algorithm 2).

    ``F`` is the leaf size of the factor trees ``Z_j`` (the paper uses
    ``F = R``; any positive ``F`` gives the same rows under the tie rule).

    ``store`` (None or a NumPy float type) takes the integer decisions in a
    storage precision: the cached partial Gram matrices, the eigen-tree
    nodes ``P^v (*) G_k`` and the eigenvectors are rounded to ``store``
    before the walks, while every operation stays float64.  With
    ``np.float32`` this is the precision in which a float32-storage
    implementation decides its indices, so both sides compare the same
    decision.
    """

    def __init__(self, Us, F=None, store=None):
        self.U = [np.asarray(U, dtype=np.float64) for U in Us]
        self.N = len(self.U)
        self.R = self.U[0].shape[1]
        self.F = self.R if F is None else int(F)
        self.store = store
        self.Z = [None] * self.N
        self.G = [None] * self.N
        for j in range(self.N):
            self.refresh(j)

    def refresh(self, j, U=None):
        """Rebuild ``Z_j`` and ``G_j`` after ``U_j`` changed (Theorem 1.1,
        part 1: a full-factor update costs a rebuild)."""
        if U is not None:
            self.U[j] = np.asarray(U, dtype=np.float64)
        self.Z[j] = SegmentTree(self.U[j], self.F)
        if self.store is not None:
            self.Z[j].levels = [_round(lv, self.store) for lv in self.Z[j].levels]
        self.G[j] = self.U[j].T @ self.U[j]

    def modes(self, exclude):
        return [k for k in range(self.N) if k != exclude]

    def prepare(self, exclude):
        """The set-up part of Algorithm 2 (before its per-sample loop): ``G``, ``G^+``, every ``G_{>k}`` and its
        eigendecomposition, and the trees ``E_k``."""
        modes = self.modes(exclude)
        G = hadamard_all([self.G[k] for k in modes])
        Gp, rank = pinv_psd(G)
        eig, E, degenerate = {}, {}, False
        for k in modes:
            later = [self.G[m] for m in modes if m > k]
            Ggt = Gp * hadamard_all(later) if later else Gp.copy()
            lam, V = np.linalg.eigh((Ggt + Ggt.T) * 0.5)
            lam = np.maximum(lam, 0.0)
            lmax = lam[-1] if lam.size else 0.0
            tau = self.R * 2.0 ** -52 * lmax
            gaps = np.diff(lam)
            big = (lam[1:] > tau)
            if np.any(gaps[big] < 1e-8 * lmax):
                degenerate = True
            eig[k] = (lam, V)
            B = np.sqrt(lam)[:, None] * V.T          # rows sqrt(lam_u) V[:, u]^T
            E[k] = SegmentTree(B, 1)
            if self.store is not None:
                # node masses <h h^T, P^v, G_k> = h^T (P^v (*) G_k) h with the
                # Hadamard product stored in the storage precision
                E[k].levels = [_round(lv * self.G[k], self.store) for lv in E[k].levels]
                E[k].folded = True
        return Gp, rank, eig, E, degenerate

    def draw(self, exclude, u01):
        """``KRPSample(j, J)`` with the uniforms ``u01[J][N][2]`` given.

        Column 0 of ``u01[d, k]`` drives the draw of ``u_k`` from ``E_k``
        (Section 3.2, first-stage distribution), column 1 the draw of
        ``t_k`` from ``Z_k`` (second-stage distribution).
        """
        u01 = np.asarray(u01, dtype=np.float64)
        J = u01.shape[0]
        modes = self.modes(exclude)
        Gp, rank, eig, E, degenerate = self.prepare(exclude)
        h = np.ones((J, self.R))
        idx = np.full((J, self.N), -1, dtype=np.int64)
        margin = np.full(J, np.inf)
        for k in modes:
            lam, V = eig[k]
            folded = getattr(E[k], "folded", False)
            u, m1 = row_sample_batch(E[k], h, None if folded else self.G[k], u01[:, k, 0])
            Vs = V if self.store is None else _round(V, self.store)
            ht = h * Vs[:, u].T
            t, m2 = row_sample_batch(self.Z[k], ht, None, u01[:, k, 1])
            h = h * self.U[k][t]
            idx[:, k] = t
            margin = np.minimum(margin, np.minimum(m1, m2))
        prob = np.einsum("da,ab,db->d", h, Gp, h) / rank
        return Draw(idx, h, prob, margin, rank, Gp, eig, degenerate)

    def row_prob(self, exclude, idx):
        """``q`` of given multi-indices (``[M, N]``, excluded column ignored)."""
        modes = self.modes(exclude)
        G = hadamard_all([self.G[k] for k in modes])
        Gp, rank = pinv_psd(G)
        a = np.ones((idx.shape[0], self.R))
        for k in modes:
            a = a * self.U[k][idx[:, k]]
        return np.einsum("da,ab,db->d", a, Gp, a) / rank
