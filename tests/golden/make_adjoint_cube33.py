"""Writes tests/golden/adjoint_cube33.npz: the FP64 oracle gradient of the
differentiable workload (33^3 tet cube, 30 frames x 20 iterations, loss =
squared distance of the final centroid to the seeded target) with respect to
the per-tet Young's modulus and the initial velocity field.

Calls only the oracle (and the seeded input generator).  Stored in float32
(the comparison tolerance is 1e-3 relative L2).  Run:
    python tests/golden/make_adjoint_cube33.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O                                   # noqa: E402
from paper_2403_06321_amd import workloads as W      # noqa: E402


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    O.set_threads(threads)
    w = W.config_differentiable()
    m = O.Model.from_workload(w)
    t0 = time.time()
    x, v, vp, states = O.rollout(m, w.params, w.x0, w.v0, w.tet_E, w.frames)
    c = x.mean(0)
    loss = float(((c - w.target) ** 2).sum())
    print(f"forward {time.time() - t0:.1f} s, loss {loss:.9e}", flush=True)
    gx = np.tile(2.0 * (c - w.target) / w.n_verts, (w.n_verts, 1))
    gv = np.zeros_like(gx)
    gvp = np.zeros_like(gx)
    gE = np.zeros(w.n_tets)
    for f in reversed(range(w.frames)):
        xt, vt, vpt = states[f]
        gx, gv, gvp, gE = O.step_backward(m, w.params, xt, vt, vpt, w.tet_E, gx, gv, gvp, gE)
        print(f"backward frame {f} done at {time.time() - t0:.1f} s", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_cube33.npz")
    np.savez_compressed(out, loss=np.float64(loss), g_E=gE.astype(np.float32),
                        g_v0=(gv + gvp).astype(np.float32), g_x0=gx.astype(np.float32),
                        x_final=x.astype(np.float32))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
