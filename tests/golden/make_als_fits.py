"""Writes the oracle's per-sweep fits of a sketched CP-ALS workload to
``als_fits_c<config>_<f64|f32>.json`` beside this script (``f32``: the
factors are kept rounded to float32 after every solve, as a float32-storage
implementation keeps them; all arithmetic is float64).

Runs the float64 oracle only (``oracle.cp.cp_als``, Algorithm 6 with the
sampled solve) on the seeded inputs of ``synth.als_problem``; the GPU tests
and the benchmark compare their fits with the stored values.  Slow: the
sketched CP-ALS workload with 1e8 nonzeros takes tens of minutes on a
few cores.

usage: python tests/golden/make_als_fits.py CONFIG {f64,f32} [NNZ]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import cp as ocp  # noqa: E402


def main():
    config = int(sys.argv[1])
    store_name = sys.argv[2]
    nnz = int(float(sys.argv[3])) if len(sys.argv) > 3 else None
    factor_dtype = {"f64": None, "f32": np.float32}[store_name]
    t0 = time.time()
    dims, idx, val, U0, R, J, sweeps, useed = synth.als_problem(config, nnz)
    T = ocp.SparseTensor(dims, idx, val)
    N = len(dims)
    print(f"inputs {time.time() - t0:.1f} s", flush=True)

    def u01_of(s, j):
        return synth.uniforms(J, N, useed + 1000 * s + j)

    def progress(s, j):
        print(f"sweep {s} solve {j} {time.time() - t0:.1f} s", flush=True)

    _, sigma, fits = ocp.cp_als(T, U0, sweeps, u01_of, factor_dtype=factor_dtype,
                                progress=progress)
    out = {"config": config, "store": store_name, "dims": list(dims), "nnz": int(T.nnz),
           "R": R, "J": J, "sweeps": sweeps, "uniform_seed": useed, "fits": fits,
           "norm2": T.norm2, "seconds": time.time() - t0,
           "writer": "tests/golden/make_als_fits.py (float64 oracle, oracle.cp.cp_als)"}
    tag = f"_nnz{nnz}" if nnz is not None else ""
    path = os.path.join(HERE, f"als_fits_c{config}{tag}_{store_name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, fits, flush=True)


if __name__ == "__main__":
    main()
