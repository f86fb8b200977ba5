"""Writes stored oracle waveforms for the full-size parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded workload generator; no value here
comes from the HIP path.  Usage:  python tests/golden/make_golden.py single-shower
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1001_5341_amd import workloads as W  # noqa: E402
from paper_1001_5341_amd.workloads import workload_digest  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main(name: str):
    w = W.workload_by_name(name)
    t0 = time.time()
    wave = oracle.run(w)
    wall = time.time() - t0
    path = os.path.join(HERE, f"{name}_oracle.npz")
    np.savez_compressed(path, waveforms=wave.astype(np.float32), digest=workload_digest(w),
                        wall_s=wall, threads=os.environ.get("OMP_NUM_THREADS", "all"))
    print(json.dumps({"written": path, "wall_s": wall, "shape": list(wave.shape),
                      "cell_updates_per_s": w.n_cells * w.n_steps / wall}))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "single-shower")
