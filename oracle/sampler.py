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

    def update_entry(self, r, c, value):
        """``UpdateSampler`` (Appendix A.7, Algorithm 5): ``U[r, c] := value``.

        With ``u`` the old row ``U[r, :]`` and ``delta = value - u[c]``, the
        leaf holding row ``r`` gets ``delta u`` added to its row ``c`` and to
        its column ``c``, and ``delta^2`` more at ``(c, c)``; then each
        ancestor, up to the root, is set to the sum of its two children."""
        if not getattr(self, "_own_u", False):
            self.U = self.U.copy()
            self._own_u = True
        u = self.U[r].copy()
        delta = float(value) - u[c]
        pos = r // self.F
        G = self.levels[self.D][pos]
        G[c, :] += delta * u
        G[:, c] += delta * u
        G[c, c] += delta * delta
        self.U[r, c] = value
        for lev in range(self.D - 1, -1, -1):
            pos //= 2
            child = self.levels[lev + 1]
            s = child[2 * pos].copy()
            if 2 * pos + 1 < child.shape[0]:
                s += child[2 * pos + 1]
            self.levels[lev][pos] = s


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


def row_sample_batch(tree, H, Y, dvec, chunk=None, scaled=False, vround=False):
    """Algorithm 4 for many independent samples at once (the samples march
    level by level, as in the batch-synchronous strategy of Appendix A.10).

    ``H``: ``[J, R]`` history vectors, ``dvec``: ``[J]`` uniforms.  Returns
    ``(rows [J] int64, min_margin [J], min_scaled_margin [J])``.

    The margin of a comparison is ``|x - cut| / C``.  The scaled margin
    (``scaled=True``; ``inf`` otherwise) is ``|x - cut| / E`` with ``E`` the
    effect on ``x - cut`` of storing every node entry, and, with ``vround``,
    every entry of the eigenvector that multiplies the history, with a
    relative rounding of at most 1 (so a rounding ``u`` moves the comparison
    by about ``u E``):

    * node entries: the packed terms ``t = h_a h_b Y_ab G_ab`` of every node
      whose mass enters ``x = d C`` (the root, times ``d``) or the cut (the
      nodes summed into ``low`` and the left child) are rounded
      independently, so their effect is a sum of independent terms of
      standard deviation ``|t| / sqrt(3)``; ``E`` takes 4 times the square
      root of the sum of squares (about seven standard deviations);
    * eigenvector entries (``vround``): one rounding per entry ``a`` of the
      history moves every mass ``h^T G h`` by ``2 sum_a e_a h_a (G h)_a``,
      so ``E`` adds ``2 sum_a |h_a (d G_root h - sum_{nodes in the cut} G h)_a|``
      (the same rounding of ``h`` moves ``x`` and the cut together); the
      rows scanned in a leaf are exact, so the leaf scan adds its rows' terms
      here only.
    """
    H = np.asarray(H, dtype=np.float64)
    J, R = H.shape
    rows = np.empty(J, dtype=np.int64)
    margins = np.empty(J)
    smargins = np.empty(J)
    if chunk is None:
        chunk = max(64, (1 << 23) // (R * R))
    for s in range(0, J, chunk):
        e = min(J, s + chunk)
        rows[s:e], margins[s:e], smargins[s:e] = _row_sample_chunk(tree, H[s:e], Y, dvec[s:e],
                                                                   scaled, vround)
    return rows, margins, smargins


def _masses(Gs, HH):
    # <h h^T, G> for a batch: sum over (a, b) of (h_a h_b Y_ab) G_ab
    return np.einsum("dab,dab->d", Gs, HH)


def _node_ss(Gs, HH):
    """Sum of squares of the packed terms of each node: the upper triangle
    stores (a, b) once, so an off-diagonal pair counts as one term 2 t_ab."""
    T2 = (Gs * HH) ** 2
    return 2.0 * T2.sum(axis=(1, 2)) - np.einsum("daa->d", T2)


def _row_sample_chunk(tree, H, Y, dvec, scaled=False, vround=False):
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
    smargin = np.full(n, np.inf)
    if scaled:
        root = np.broadcast_to(tree.root, (n, R, R))
        ss_x = dvec ** 2 * _node_ss(root, HH)
        ss_low = np.zeros(n)
        g_x = dvec[:, None] * (root @ H[:, :, None])[:, :, 0]   # d G_root h
        g_low = np.zeros((n, R))

    def effect(ss, g):
        e = 4.0 * np.sqrt(ss)
        if vround:
            e = e + 2.0 * np.abs(H * g).sum(axis=1)
        return e

    for lev in range(1, tree.D + 1):
        left = 2 * pos
        GL = tree.levels[lev][left]
        mL = np.maximum(_masses(GL, HH), 0.0)
        cut = low + mL
        margin = np.minimum(margin, np.abs(x - cut) / C)
        right_exists = (left + 1) < tree.real(lev)
        go_left = (cut >= x) | (~right_exists) | (high - cut <= 0.0)
        if scaled:
            ss_L = _node_ss(GL, HH)
            g_L = (GL @ H[:, :, None])[:, :, 0]
            E = effect(ss_x + ss_low + ss_L, g_x - g_low - g_L)
            smargin = np.minimum(smargin, np.where(right_exists, np.abs(x - cut) / E, np.inf))
            ss_low = np.where(go_left, ss_low, ss_low + ss_L)
            g_low = np.where(go_left[:, None], g_low, g_low + g_L)
        pos = np.where(go_left, left, left + 1)
        high = np.where(go_left, cut, high)
        low = np.where(go_left, low, cut)
    F = tree.F
    s0 = pos * F
    if F == 1:
        # a one-row leaf: the scan can only return that row, and its right
        # edge is a boundary already compared above
        return s0, margin, smargin
    offs = np.arange(F)
    ridx = s0[:, None] + offs[None, :]
    valid = ridx < tree.I
    Ur = tree.U[np.minimum(ridx, tree.I - 1)]
    Wr = Ur * H[:, None, :]
    if Y is None:
        qt = Wr.sum(axis=2) ** 2
    else:
        qt = np.einsum("dia,ab,dib->di", Wr, Y, Wr)
    qt = np.where(valid, qt, 0.0)
    acc = low[:, None] + np.cumsum(qt, axis=1)
    margin = np.minimum(margin, np.where(valid, np.abs(x[:, None] - acc) / C[:, None],
                                         np.inf).min(axis=1))
    if scaled:
        if Y is None:
            # row i's mass (U_i . h)^2 with G = U_i^T U_i: (G h)_a = U_ia (U_i . h)
            gr = Ur * np.where(valid, Wr.sum(axis=2), 0.0)[:, :, None]
        else:
            # G_ab = U_ia Y_ab U_ib: (G h)_a = U_ia (Y w)_a with w = U_i * h
            gr = Ur * np.einsum("dib,ab->dia", Wr, Y)
        gcum = np.cumsum(gr, axis=1)                      # sum over the scanned rows
        gtot = (g_x - g_low)[:, None, :] - gcum
        E = 4.0 * np.sqrt(ss_x + ss_low)[:, None] * np.ones((1, F))
        if vround:
            E = E + 2.0 * np.abs(H[:, None, :] * gtot).sum(axis=2)
        # the last row's right edge is the leaf's, compared above
        inner = valid & (offs[None, :] < np.minimum(tree.I - s0, F)[:, None] - 1)
        smargin = np.minimum(smargin, np.where(inner, np.abs(x[:, None] - acc) / E,
                                               np.inf).min(axis=1))
    hit = (acc >= x[:, None]) & valid
    any_hit = hit.any(axis=1)
    first = np.argmax(hit, axis=1)
    posm = (qt > 0) & valid
    last_pos = F - 1 - np.argmax(posm[:, ::-1], axis=1)
    last_valid = np.minimum(tree.I - s0, F) - 1
    fallback = np.where(posm.any(axis=1), last_pos, last_valid)
    chosen = np.where(any_hit, first, fallback)
    return s0 + chosen, margin, smargin


class Draw:
    """Result of one ``KRPSample`` call."""

    def __init__(self, idx, rows, prob, margin, smargin, rank, Gp, eig, degenerate):
        self.idx = idx            # [J, N] int64, -1 in the excluded column
        self.rows = rows          # [J, R] sampled KRP rows a_d (float64)
        self.prob = prob          # [J] q_d = a_d G^+ a_d^T / rank
        self.margin = margin      # [J] smallest |x - cut| / C along the draw
        self.smargin = smargin    # [J] smallest scaled margin (row_sample_batch), or inf
        self.rank = rank
        self.Gp = Gp              # pseudo-inverse of G = (*)_{k != j} G_k
        self.eig = eig            # {k: (lam ascending, V)} of G_{>k}
        self.degenerate = degenerate  # [J] the draw met a near-degenerate eigenspace


def _path_boundaries(u, L):
    """Leaf boundaries that the walk to leaf ``u`` of a tree over ``L``
    leaves (padded to ``2^D``) compares against: at each level the boundary
    between the left and the right child of the node on the path, where the
    right child exists.  Returns ``[J, D]`` boundary indices (``-1``: none)."""
    D = int(math.ceil(math.log2(L))) if L > 1 else 0
    out = np.full((u.shape[0], max(D, 1)), -1, dtype=np.int64)
    for lev in range(1, D + 1):
        parent = u >> (D - lev + 1)
        b = (2 * parent + 1) << (D - lev)
        out[:, lev - 1] = np.where(b < L, b, -1)
    return out


class KRPSampler:
    """``ConstructKRPSampler`` (Algorithm 1) and ``KRPSample`` (Algorithm 2).

    ``F`` is the leaf size of the factor trees ``Z_j`` (the paper uses
    ``F = R``; any positive ``F`` gives the same rows under the tie rule).
    Everything is float64.
    """

    def __init__(self, Us, F=None):
        self.U = [np.asarray(U, dtype=np.float64) for U in Us]
        self.N = len(self.U)
        self.R = self.U[0].shape[1]
        self.F = self.R if F is None else int(F)
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
        self.G[j] = self.U[j].T @ self.U[j]

    def update_entry(self, j, r, c, value):
        """``UpdateSampler(j, r, c, value)`` (Appendix A.7, Algorithm 5):
        ``U_j[r, c] := value`` with the path of ``Z_j`` from the leaf of row
        ``r`` to the root updated; ``G_j`` is that root."""
        self.Z[j].update_entry(r, c, value)
        self.U[j] = self.Z[j].U
        self.G[j] = self.Z[j].root.copy()

    def modes(self, exclude):
        return [k for k in range(self.N) if k != exclude]

    def prepare(self, exclude):
        """The set-up part of Algorithm 2 (before its per-sample loop): ``G``,
        ``G^+``, every ``G_{>k}`` and its eigendecomposition, and the trees
        ``E_k``."""
        modes = self.modes(exclude)
        G = hadamard_all([self.G[k] for k in modes])
        Gp, rank = pinv_psd(G)
        eig, E = {}, {}
        for k in modes:
            later = [self.G[m] for m in modes if m > k]
            Ggt = Gp * hadamard_all(later) if later else Gp.copy()
            lam, V = np.linalg.eigh((Ggt + Ggt.T) * 0.5)
            lam = np.maximum(lam, 0.0)
            eig[k] = (lam, V)
            B = np.sqrt(lam)[:, None] * V.T          # rows sqrt(lam_u) V[:, u]^T
            E[k] = SegmentTree(B, 1)
        return Gp, rank, eig, E

    def degenerate_boundaries(self, lam, gap_tol):
        """``flag[b]`` for the boundary between eigenvalues ``b - 1`` and
        ``b`` (ascending): the gap is below ``gap_tol * lambda_max`` and
        ``lambda_b`` lies above the pseudo-inverse cut.  Inside such a
        cluster the eigenvectors are fixed only up to a rotation, so the
        masses of subtrees that split it depend on the basis (every basis
        gives the same distribution)."""
        lmax = lam[-1] if lam.size else 0.0
        tau = self.R * 2.0 ** -52 * lmax
        flag = np.zeros(lam.size + 1, dtype=bool)
        flag[1:-1] = (np.diff(lam) < gap_tol * lmax) & (lam[1:] > tau)
        return flag

    def draw(self, exclude, u01, scaled=False, gap_tol=1e-8):
        """``KRPSample(j, J)`` with the uniforms ``u01[J][N][2]`` given.

        Column 0 of ``u01[d, k]`` drives the draw of ``u_k`` from ``E_k``
        (Section 3.2, first-stage distribution), column 1 the draw of
        ``t_k`` from ``Z_k`` (second-stage distribution).  A draw is marked
        degenerate when, in some mode, its first-stage walk compared against
        a boundary inside a near-degenerate eigenvalue cluster of ``G_{>k}``
        or picked a component of such a cluster (see
        :meth:`degenerate_boundaries`).
        """
        u01 = np.asarray(u01, dtype=np.float64)
        J = u01.shape[0]
        modes = self.modes(exclude)
        Gp, rank, eig, E = self.prepare(exclude)
        h = np.ones((J, self.R))
        idx = np.full((J, self.N), -1, dtype=np.int64)
        margin = np.full(J, np.inf)
        smargin = np.full(J, np.inf)
        degenerate = np.zeros(J, dtype=bool)
        for k in modes:
            lam, V = eig[k]
            u, m1, s1 = row_sample_batch(E[k], h, self.G[k], u01[:, k, 0], scaled=scaled)
            flag = self.degenerate_boundaries(lam, gap_tol)
            b = _path_boundaries(u, self.R)
            degenerate |= np.where(b >= 0, flag[np.maximum(b, 0)], False).any(axis=1)
            degenerate |= flag[u] | flag[u + 1]
            ht = h * V[:, u].T
            t, m2, s2 = row_sample_batch(self.Z[k], ht, None, u01[:, k, 1], scaled=scaled,
                                         vround=True)
            h = h * self.U[k][t]
            idx[:, k] = t
            margin = np.minimum(margin, np.minimum(m1, m2))
            smargin = np.minimum(smargin, np.minimum(s1, s2))
        prob = np.einsum("da,ab,db->d", h, Gp, h) / rank
        return Draw(idx, h, prob, margin, smargin, rank, Gp, eig, degenerate)

    def row_prob(self, exclude, idx):
        """``q`` of given multi-indices (``[M, N]``, excluded column ignored)."""
        modes = self.modes(exclude)
        G = hadamard_all([self.G[k] for k in modes])
        Gp, rank = pinv_psd(G)
        a = np.ones((idx.shape[0], self.R))
        for k in modes:
            a = a * self.U[k][idx[:, k]]
        return np.einsum("da,ab,db->d", a, Gp, a) / rank
