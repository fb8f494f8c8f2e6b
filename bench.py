"""Benchmark of the exact Khatri-Rao leverage sampler (and, when built, the
sketched CP-ALS sweep) on one MI355X.

Workload of the headline number: N = 3 factors of 2^20 x 32 (float32,
N(0,1) with 1% of the rows scaled by 100), J = 65,536 samples drawn from
the Khatri-Rao product of the other two factors for each excluded mode
k in {0, 1, 2}.  One step = rebuild the three segment trees + prepare and
draw the three exclusions (with the probability of every sample).

Prints one JSON line (see README / DESIGN for the fields).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "KRP leverage samples/s + ALS sweep s at fit +-1e-4: BF16-split vs FP64"
HBM_PEAK_GBS = 8000.0
F64_VALU_PEAK_TFS = 78.6
COUNTERS = os.path.join(ROOT, "profiles", "descent_c2_fp32_counters.json")
DESCENT_SRC = os.path.join(ROOT, "paper_2301_12584_amd", "csrc", "descent.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--precisions", default="fp32,fp64,bf16x2")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def unique_descent_bytes(idx, exclude, dims, R, F, elem, J, N):
    """Algorithmic bytes of one draw: every stored node, leaf block and
    eigen-tree a walk must read at least once (unique over samples), plus
    the uniforms read and the indices / probabilities written."""
    import numpy as np
    tri = R * (R + 1) // 2
    total = 0
    for m in range(N):
        if m == exclude:
            continue
        I = dims[m]
        L = -(-I // F)
        D = int(np.ceil(np.log2(L))) if L > 1 else 0
        t = idx[:, m].astype(np.int64)
        c = t // F
        total += tri * elem                                 # root
        for lev in range(1, D + 1):
            total += len(np.unique(c >> (D - lev + 1))) * tri * elem
        leaves = np.unique(c)
        rows = np.minimum((leaves + 1) * F, I) - leaves * F
        total += int(rows.sum()) * R * elem                 # leaf rows
        DE = int(np.ceil(np.log2(R))) if R > 1 else 0
        total += (R * 2) * tri * elem + R * R * elem        # eigen-tree (<= 2R nodes) + vectors
    total += J * N * 2 * 8 + J * N * 4 + J * 8 + tri * 8   # uniforms, idx, prob, G^+
    return total


def descent_flops(dims, R, F, exclude, J, N):
    import numpy as np
    tri = R * (R + 1) // 2
    fl = 0
    for m in range(N):
        if m == exclude:
            continue
        L = -(-dims[m] // F)
        D = int(np.ceil(np.log2(L))) if L > 1 else 0
        DE = int(np.ceil(np.log2(R))) if R > 1 else 0
        fl += 2 * tri * (DE + 1 + D + 1) + 2 * F * R + 2 * R
    fl += 2 * tri
    return fl * J


def counters_for(src_sha):
    try:
        c = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    if c.get("descent_src_sha256") != src_sha:
        return None
    return c


def run_sampler(torch, krps, ctx, Us, u01_dev, prec, steps, warmup, J):
    import numpy as np
    dt = torch.float64 if prec == "fp64" else torch.float32
    Ud = [torch.from_numpy(U).to(ctx.device).to(dt).contiguous() for U in Us]
    S = krps.Sampler(ctx, Ud, precision=prec)
    N = len(Us)
    idx = [torch.empty((J, N), dtype=torch.int32, device=ctx.device) for _ in range(N)]
    prob = [torch.empty(J, dtype=torch.float64, device=ctx.device) for _ in range(N)]
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    marks = []

    def step(record):
        b0, b1 = ev(), ev()
        if record:
            b0.record()
        for j in range(N):
            S.refresh(j)
        if record:
            b1.record()
        dmarks = []
        for k in range(N):
            S.prepare(k)
            e0, e1 = ev(), ev()
            if record:
                e0.record()
            S.draw(k, u01_dev[k], idx[k], prob[k])
            if record:
                e1.record()
                dmarks.append((e0, e1))
        if record:
            marks.append(((b0, b1), dmarks))

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0, t1 = ev(), ev()
    t0.record()
    for _ in range(steps):
        step(True)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    build_ms = float(np.mean([b0.elapsed_time(b1) for (b0, b1), _ in marks]))
    desc_ms = [float(np.mean([d[k][0].elapsed_time(d[k][1]) for _, d in marks])) for k in range(N)]
    out = dict(ms_per_step=ms, samples_per_s=N * J / (ms / 1e3), build_ms=build_ms,
               descent_ms=desc_ms, idx=[i.cpu().numpy() for i in idx])
    del S
    return out


def cpu_baseline(Us, u01, J_full, budget_s=20.0):
    """The oracle (float64 NumPy) on the host: tree build of the three
    factors plus a bounded number of draws per exclusion, scaled to one
    full step."""
    import numpy as np
    from oracle import sampler as osmp
    N = len(Us)
    t0 = time.perf_counter()
    S = osmp.KRPSampler(Us)
    t_build = time.perf_counter() - t0
    Jc = 2048
    t0 = time.perf_counter()
    done = 0
    for k in range(N):
        S.draw(k, u01[k][:Jc])
        done += Jc
        if time.perf_counter() - t0 > budget_s:
            break
    t_draw = (time.perf_counter() - t0) / done
    step_s = t_build + N * J_full * t_draw
    return {"value": N * J_full / step_s, "unit": "samples/s",
            "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": f"float64 NumPy oracle on the full factors: tree build of the 3 factors "
                      f"({t_build:.2f} s) + {done} draws ({Jc} per exclusion, "
                      f"{t_draw * 1e6:.1f} us/draw), scaled to one step of 3 x {J_full} draws"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2301_12584_amd as krps
    import synth

    if args.calib_copy:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": n * 4, "calib_copy_bytes_written": n * 4,
                          "launches": 5}))
        return

    cfg = synth.CONFIGS[2]
    dims, R, J, N = cfg["dims"], cfg["R"], cfg["J"], cfg["N"]
    Us = synth.gaussian_factors(dims, R, synth.config_seed(2),
                                heavy_rows_frac=cfg["heavy_rows_frac"],
                                heavy_row_scale=cfg["heavy_row_scale"])
    u01 = [synth.uniforms(J, N, synth.uniform_seed(2) + k) for k in range(N)]
    ctx = krps.Context(0)
    u01_dev = [torch.from_numpy(u).to(ctx.device) for u in u01]

    results = {}
    for prec in args.precisions.split(","):
        results[prec] = run_sampler(torch, krps, ctx, Us, u01_dev, prec, args.steps,
                                    args.warmup, J)
        print(f"# {prec}: {results[prec]['samples_per_s'] / 1e6:.2f} M samples/s, "
              f"step {results[prec]['ms_per_step']:.3f} ms, build {results[prec]['build_ms']:.3f} ms, "
              f"descent {['%.3f' % x for x in results[prec]['descent_ms']]} ms", file=sys.stderr,
              flush=True)

    head = "fp32" if "fp32" in results else list(results)[0]
    r = results[head]
    elem = 8 if head == "fp64" else 4
    # roofline of the dominant kernel: the descent of exclusion 0
    ub = unique_descent_bytes(r["idx"][0], 0, dims, R, R, elem, J, N)
    fl = descent_flops(dims, R, R, 0, J, N)
    t = r["descent_ms"][0] / 1e3
    sha = hashlib.sha256(open(DESCENT_SRC, "rb").read()).hexdigest()
    cnt = counters_for(sha)
    traffic = None
    if cnt is not None:
        traffic = cnt.get("hbm_bytes_per_launch")
    roof = {"bound": "hbm", "achieved": ub / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ub / t / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "descent_kernel (exclusion 0)", "algorithmic_bytes": ub,
            "launch_ms": r["descent_ms"][0],
            "valu_f64_frac": fl / t / 1e12 / F64_VALU_PEAK_TFS, "flops": fl}

    line = {
        "metric": METRIC, "value": r["samples_per_s"], "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if head != "fp64" else "f64",
        "data": "synthetic (seeded N(0,1) factors, 1% rows x100; host uniforms)",
        "config": {"workload": "sampler N=3, I=2^20, R=32, J=65536 per excluded mode k=0,1,2",
                   "N": N, "I": dims[0], "R": R, "J": J, "leaf_size": R,
                   "precision": head, "arith": "f64 walk over f32-stored trees"},
        "roofline": roof,
        "precisions": {p: {"samples_per_s": v["samples_per_s"], "ms_per_step": v["ms_per_step"],
                           "build_ms": v["build_ms"], "descent_ms": v["descent_ms"]}
                       for p, v in results.items()},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(Us, u01, J)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line))


if __name__ == "__main__":
    main()
