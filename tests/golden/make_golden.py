#!/usr/bin/env python3
"""Write tests/golden/<workload>_oracle.npz: the FP64 oracle's trajectory on a full-size
workload, for the GPU end-to-end parity tests:

* ``paper_4x4`` -- F=513, T=625, four 4-mic subarrays, N=5, K=16; 100 iterations
  (about 4 minutes on 8 cores);
* ``table2`` -- the shape of the paper's Table II: F=2049, T=157, three 4-mic subarrays,
  N=3, K=16; 50 iterations (about a minute on 8 cores);
* ``paper_16`` -- the recording of ``paper_4x4`` separated with one 16-mic block (the
  conventional method, L = 1); 100 iterations.

Only ``oracle/`` and the seeded input generator are called; the inputs are rounded to the
storage precision of the FP32 path first.  Stored: the cost (13) at a few iteration counts
and 8192 entries of the separated source images (Wiener filter per subarray) after the last
iteration, at positions drawn from a fixed seed, and the final state (Q, g, W, H) in FP64, from
which the tests form the oracle's separated images over every bin.  Run from the repository root:
    python tests/golden/make_golden.py paper_4x4
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dfmnmf as D  # noqa: E402
from paper_2605_19388_amd import synth  # noqa: E402

CHECKPOINTS = {"paper_4x4": (0, 1, 2, 5, 10, 20, 50, 100), "table2": (0, 1, 2, 5, 10, 20, 50),
               "paper_16": (0, 1, 2, 5, 10, 20, 50, 100)}
SAMPLES = 8192
SAMPLE_SEED = 4242


def main(name):
    w = synth.make(name)
    # The inputs exactly as the FP32 path receives them (complex64 / float32), held in FP64.
    c64 = lambda a: np.asarray(a).astype(np.complex64).astype(np.complex128)  # noqa: E731
    r32 = lambda a: np.asarray(a).astype(np.float32).astype(np.float64)  # noqa: E731
    X, mics = c64(w["X"]), w["mics"]
    N, F, T, M = w["N"], w["F"], w["T"], w["M"]
    state = (c64(w["Q"]), r32(w["g"]), r32(w["W"]), r32(w["H"]))
    costs = {}
    done = 0
    for target in CHECKPOINTS[name]:
        if target > done:
            state = D.iterate(X, *state, mics, target - done)
            done = target
        costs[target] = D.nll(X, *state, mics)
        print(f"iteration {target}: cost {costs[target]:.12e}", flush=True)
    S = D.separate(X, *state, mics)
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    idx = np.stack([rng.integers(0, N, SAMPLES), rng.integers(0, F, SAMPLES),
                    rng.integers(0, T, SAMPLES), rng.integers(0, M, SAMPLES)]).astype(np.int32)
    vals = S[idx[0], idx[1], idx[2], idx[3]]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.npz")
    np.savez_compressed(out, checkpoints=np.array(CHECKPOINTS[name], dtype=np.int32),
                        costs=np.array([costs[c] for c in CHECKPOINTS[name]]), sample_index=idx, sample_values=vals,
                        source_norms=np.sqrt((np.abs(S) ** 2).sum(axis=(1, 2, 3))),
                        final_iteration=np.int32(done), Q=state[0], g=state[1], W=state[2], H=state[3])
    print("wrote", out)


if __name__ == "__main__":
    if len(sys.argv) != 2 or sys.argv[1] not in CHECKPOINTS:
        sys.exit(f"usage: make_golden.py {{{'|'.join(CHECKPOINTS)}}}")
    main(sys.argv[1])
