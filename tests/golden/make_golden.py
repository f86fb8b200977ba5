"""Writes stored oracle waveforms for the full-size parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded workload generator; no value here
comes from the HIP path.  Usage:
    python tests/golden/make_golden.py single-shower   # 256x256x2048, 4000 steps
    python tests/golden/make_golden.py adjoint         # 128x128x1024, 3000 steps: w*, dL/dq
    python tests/golden/make_golden.py batch           # sampled members of the 32-shower batch
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


# members of the 32-shower batch whose waveforms are stored: all 32, smallest first (about 3 h
# of the host oracle on 8 threads; the file is rewritten after each member)
BATCH_SAMPLE = (24, 20, 19, 26, 15, 6, 12, 5, 28, 31, 25, 29, 3, 23, 27, 7, 2, 30, 13, 16, 17, 22, 14, 18,
                4, 21, 10, 1, 8, 11, 0, 9)


def adjoint_golden():
    """Target waveforms w* = A q* and the FP64 adjoint gradient of L = sum (A q - w*)^2 at the
    perturbed profile q, for the differentiation workload."""
    w, q_target = W.adjoint_problem()
    t0 = time.time()
    w_star = oracle.run(w, q_bins=q_target)
    w_q = oracle.run(w)
    grad = oracle.adjoint(w, 2.0 * (w_q - w_star))
    wall = time.time() - t0
    path = os.path.join(HERE, "adjoint_oracle.npz")
    np.savez_compressed(path, w_star=w_star.astype(np.float32), w_q=w_q.astype(np.float32),
                        dl_dq=grad, q_target=q_target, digest=workload_digest(w), wall_s=wall)
    print(json.dumps({"written": path, "wall_s": wall, "grad_norm": float(np.linalg.norm(grad))}))


def batch_golden():
    ws = W.batch_showers()
    out = {}
    t0 = time.time()
    path = os.path.join(HERE, "batch_oracle.npz")
    # members this script stored before, for the same workload (same digest), are kept
    old = dict(np.load(path)) if os.path.exists(path) else {}
    done = []
    for m in BATCH_SAMPLE:
        if f"member{m}" in old and str(old[f"digest{m}"]) == workload_digest(ws[m]):
            out[f"member{m}"], out[f"digest{m}"] = old[f"member{m}"], old[f"digest{m}"]
        else:
            out[f"member{m}"] = oracle.run(ws[m]).astype(np.float32)
            out[f"digest{m}"] = workload_digest(ws[m])
        done.append(m)
        # rewritten after every member, so that an interrupted run leaves a consistent file
        np.savez_compressed(path, members=np.array(done), wall_s=time.time() - t0, **out)
        print(json.dumps({"member": m, "name": ws[m].name, "elapsed_s": time.time() - t0}), flush=True)
    print(json.dumps({"written": path}))


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "single-shower"
    if what == "adjoint":
        adjoint_golden()
    elif what == "batch":
        batch_golden()
    else:
        main(what)
