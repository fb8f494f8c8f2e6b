"""Index parity between the GPU walk and the float64 oracle.

The GPU and the oracle draw with the same uniforms, so their indices must
agree except where the two computations may legitimately decide a
comparison differently.  A draw is excused when

* it met a near-degenerate eigenvalue cluster of some ``G_{>k}``
  (``Draw.degenerate``: inside a cluster the eigenvectors are fixed only up
  to a rotation, which changes the first-stage masses; every basis gives the
  same distribution), or
* float64 path: some comparison lies within ``FP64_MARGIN`` of ``C``
  (``|x - cut| / C``; the two sides sum the same float64 terms in another
  order), or
* float32 path: some comparison's scaled margin (``Draw.smargin``) is at
  most ``FP32_SCALED = u = 2^-24``.  The walk reads every node entry and
  eigenvector entry rounded once to float32 (relative error at most ``u``;
  the nodes are float64 sums rounded once when stored); the scaled margin
  divides the gap ``|x - cut|`` by the effect of such roundings on it
  (oracle/sampler.py, ``row_sample_batch``: seven standard deviations of
  the independent node roundings plus the first-order bound of the
  eigenvector roundings), pinned on the CPU by
  ``test_scaled_margin_bounds_the_effect_of_storage_rounding``.

The split path samples from the float32 path's trees (float64 products of
the float32 factors, float32 nodes), so it is held to the float32 rule.
"""
import numpy as np

U32 = 2.0 ** -24
FP64_MARGIN = 1e-10
FP32_SCALED = U32


def compare(gpu_idx, dr, prec):
    """Splits the draws into same / excused / unexcused for ``prec``."""
    gpu_idx = np.asarray(gpu_idx).astype(np.int64)
    same = (gpu_idx == dr.idx).all(axis=1)
    if prec == "fp64":
        near = dr.margin <= FP64_MARGIN
    else:
        near = dr.smargin <= FP32_SCALED
    excusable = near | dr.degenerate
    diff = ~same
    out = {
        "n": int(same.size),
        "same": same,
        "mismatch": int(diff.sum()),
        "excusable_frac": float(excusable.mean()) if same.size else 0.0,
        "unexcused": int((diff & ~excusable).sum()),
        "needed_smargin": float(dr.smargin[diff & ~dr.degenerate].max())
        if (diff & ~dr.degenerate).any() else 0.0,
        "needed_margin": float(dr.margin[diff & ~dr.degenerate].max())
        if (diff & ~dr.degenerate).any() else 0.0,
    }
    return out


def report(tag, c):
    print(f"{tag}: {c['n']} draws, {c['mismatch']} differ, {c['unexcused']} unexcused, "
          f"excusable {100 * c['excusable_frac']:.2f}%, largest margin needed "
          f"{c['needed_margin']:.2e} (scaled {c['needed_smargin']:.2e})", flush=True)
