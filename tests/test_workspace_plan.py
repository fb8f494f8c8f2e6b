"""Workspace planning of the library, checked on the host (no GPU): for the
workload shapes, every region of every workspace (sampler, per-draw, solve,
tensor, batched, least squares) starts after the previous one and is at
least as large as the largest extent its kernels touch (the tree builder's
ping-pong buffers replayed from its launch geometry, the walk's reads past
a node's end), and the scratch of the fit and of the factor normalisation
lies below every piece of the solve layout, so those calls leave the last
solve's pieces intact."""
import ctypes

import pytest

SHAPES = [
    # (dims, R, F, nnz, J)
    ((1 << 20,) * 3, 32, 0, 1 << 20, 65536),                        # sampler at scale
    ((1_000_000, 1_000_000, 100_000), 64, 0, 100_000_000, 65536),   # sketched CP-ALS
    ((20_000_000,) * 3 + (1_000_000,), 128, 0, 500_000_000, 131072),  # large CP-ALS
    ((3_649_799, 1545, 23371, 240127, 3900), 32, 0, 10_000, 16384),  # a batched problem
    ((1, 5, 9), 4, 0, 7, 3),                                         # I < F, tiny
    ((777, 260), 128, 0, 100, 512),
    ((10, 20), 48, 100, 50, 1),
    ((64,) * 9, 8, 0, 1000, 5000),                                   # N = 9
]


@pytest.fixture(scope="module")
def krps():
    import paper_2301_12584_amd as k
    k.lib()
    return k


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x2"])
@pytest.mark.parametrize("dims,R,F,nnz,J", SHAPES)
def test_regions_are_ordered_and_large_enough(krps, prec, dims, R, F, nnz, J):
    regions = krps.workspace_regions(dims, R, F, prec, nnz=nnz, J=J)
    by_ws = {}
    for r in regions:
        by_ws.setdefault(r["workspace"], []).append(r)
    assert sorted(by_ws) == [0, 1, 2, 3, 4, 5]
    for ws, rs in by_ws.items():
        end = 0
        for r in rs:
            assert r["offset"] >= end, (ws, r["name"])
            assert r["need"] <= r["bytes"], (ws, r["name"], r["need"], r["bytes"])
            end = r["offset"] + r["bytes"]
    # the sampler and least-squares size queries cover every region
    n = len(dims)
    arr = (ctypes.c_int64 * n)(*dims)
    sz = ctypes.c_size_t()
    krps.check(krps.lib().krps_sampler_workspace_bytes(n, arr, R, F, krps.PRECISION[prec],
                                                       ctypes.byref(sz)))
    last = by_ws[0][-1]
    assert last["offset"] + last["bytes"] == sz.value
    krps.check(krps.lib().krps_lstsq_workspace_bytes(R, J, 1, ctypes.byref(sz)))
    last = by_ws[5][-1]
    assert last["offset"] + last["bytes"] == sz.value
    krps.check(krps.lib().krps_tensor_workspace_bytes(n, arr, nnz, ctypes.byref(sz)))
    last = by_ws[3][-1]
    assert last["offset"] + last["bytes"] == sz.value
    # fit / normalisation scratch below every piece of the solve layout
    solve = {r["name"]: r for r in by_ws[2]}
    head = ["fit partials", "fit result", "norm partials",
            "norm sigma", "sweep counter"]
    pieces = ["draw", "idx", "prob", "w", "rows", "M", "M+", "Y", "Y rows", "Y row count"]
    top = max(solve[h]["offset"] + solve[h]["bytes"] for h in head)
    assert all(solve[p]["offset"] >= top for p in pieces)


def test_tree_scratch_extent_grows_with_the_leaves(krps):
    """The replayed extent is the run tops plus the first up-sweep output,
    and it is reached by every leaf count (no slack hides an overflow)."""
    for I in (1, 2, 3, 31, 32, 33, 1000, 4097, 65537):
        for R in (8, 32, 64, 128):
            rs = krps.workspace_regions((I,), R, 1, "fp64", nnz=1, J=1)
            sc = [r for r in rs if r["workspace"] == 0 and r["name"] == "build scratch"][0]
            assert 0 < sc["need"] <= sc["bytes"]


def test_invalid_shapes_are_rejected(krps):
    with pytest.raises(krps.KrpsError):
        krps.workspace_regions((10, 10), 129)
    with pytest.raises(krps.KrpsError):
        krps.workspace_regions((10,) * 11, 4)
