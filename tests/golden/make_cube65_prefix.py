"""Writes tests/golden/cube65_prefix.npz: the first 10 frames of the FP64
oracle rollout of the 65^3 tet cube in the benchmarked configuration (greedy
coloring in smallest-last order, 100 iterations per frame, per-tet E
log-uniform in [1e4, 1e6] Pa, bottom face pinned), as the positions of 4096
free vertices drawn with a fixed seed after every frame, with each frame's
bounding-box diagonal.

Calls only the oracle (and the seeded input generator).  Run:
    python tests/golden/make_cube65_prefix.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O                                   # noqa: E402
from paper_2403_06321_amd import workloads as W      # noqa: E402

FRAMES = 10
SAMPLES = 4096


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    O.set_threads(threads)
    w = W.config_large_cube(frames=FRAMES, coloring="smallest_last")
    free = np.flatnonzero(w.pinned == 0)
    idx = np.sort(np.random.default_rng(65).choice(free, SAMPLES, replace=False))
    m = O.Model.from_workload(w)
    x, v, vp = w.x0.copy(), w.v0.copy(), w.v0.copy()
    xs, diag = [], []
    t0 = time.time()
    for f in range(FRAMES):
        x, v, vp, _ = O.step(m, w.params, x, v, vp, w.tet_E)
        xs.append(x[idx].copy())
        diag.append(float(np.linalg.norm(x.max(0) - x.min(0))))
        print(f"frame {f} done at {time.time() - t0:.1f} s", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube65_prefix.npz")
    np.savez_compressed(out, idx=idx.astype(np.int64), x=np.stack(xs), diag=np.array(diag),
                        n_iters=np.int64(w.params.n_iters), colors=np.int64(m.n_colors))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
