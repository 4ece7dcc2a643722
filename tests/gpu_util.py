"""Helpers shared by the GPU tests: run the HIP library and the FP64 oracle on
the same seeded inputs and compare per step."""
import dataclasses
import sys

import numpy as np

import oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_rollout(w, frames, params=None, launch_mode=0, cfg=None, topo=None, autotune=False):
    import torch
    from paper_2403_06321_amd.api import Topology
    p = params or w.params
    t = topo or Topology.from_workload(w)
    if cfg:
        t.launch_config = cfg
    dev = torch.device("cuda", 0)
    x = torch.tensor(w.x0, dtype=torch.float32, device=dev).contiguous()
    v = torch.tensor(w.v0, dtype=torch.float32, device=dev).contiguous()
    vp = v.clone()
    E = torch.tensor(w.tet_E, dtype=torch.float32, device=dev).contiguous()
    if autotune:
        t.autotune(x, v, vp, E, p, launch_mode)
    xs, vs = [], []
    for _ in range(frames):
        t.step(x, v, vp, E, p, launch_mode)
        xs.append(x.double().cpu().numpy())
        vs.append(v.double().cpu().numpy())
    torch.cuda.synchronize()
    t.check()
    return xs, vs, t


def oracle_rollout(w, frames, params=None, threads=None):
    p = params or w.params
    if threads:
        O.set_threads(threads)
    m = O.Model.from_workload(w)
    x, v = w.x0.copy(), w.v0.copy()
    vp = v.copy()
    xs, vs = [], []
    for _ in range(frames):
        x, v, vp, _ = O.step(m, p, x, v, vp, w.tet_E)
        xs.append(x.copy())
        vs.append(v.copy())
    return xs, vs


def oracle_states(w, frames, params=None, threads=None):
    """Oracle states (x, v, v_prev) before each frame, plus the final one."""
    p = params or w.params
    if threads:
        O.set_threads(threads)
    m = O.Model.from_workload(w)
    x, v = w.x0.copy(), w.v0.copy()
    vp = v.copy()
    out = [(x.copy(), v.copy(), vp.copy())]
    for _ in range(frames):
        x, v, vp, _ = O.step(m, p, x, v, vp, w.tet_E)
        out.append((x.copy(), v.copy(), vp.copy()))
    return out


def resync_errors(w, states, params=None, launch_mode=0):
    """Per-step bbox-relative errors of every vertex: the GPU takes each frame
    from the oracle's state (rounded to FP32).  Returns a list of arrays."""
    import torch
    from paper_2403_06321_amd.api import Topology
    p = params or w.params
    t = Topology.from_workload(w)
    dev = torch.device("cuda", 0)
    E = torch.tensor(w.tet_E, dtype=torch.float32, device=dev).contiguous()
    out = []
    for f in range(len(states) - 1):
        x, v, vp = (torch.tensor(a, dtype=torch.float32, device=dev).contiguous() for a in states[f])
        t.step(x, v, vp, E, p, launch_mode)
        xg = x.double().cpu().numpy()
        assert np.all(np.isfinite(xg)), f"frame {f}: non-finite"
        xo = states[f + 1][0]
        out.append(np.linalg.norm(xg - xo, axis=1) / bbox_diag(xo))
    t.check()
    return out


def resync_parity(w, states, params=None, launch_mode=0, tol=1e-5, label="", cfg=None):
    """Per-step parity: the GPU takes every frame from the oracle's state
    (rounded to FP32) and its one-step result is compared with the oracle's."""
    import torch
    from paper_2403_06321_amd.api import Topology
    p = params or w.params
    t = Topology.from_workload(w)
    if cfg:
        t.launch_config = cfg
    dev = torch.device("cuda", 0)
    E = torch.tensor(w.tet_E, dtype=torch.float32, device=dev).contiguous()
    worst = 0.0
    for f in range(len(states) - 1):
        x, v, vp = (torch.tensor(a, dtype=torch.float32, device=dev).contiguous() for a in states[f])
        t.step(x, v, vp, E, p, launch_mode)
        xg = x.double().cpu().numpy()
        assert np.all(np.isfinite(xg)), f"{label} frame {f}: non-finite"
        e = max_err_per_mesh(w, xg, states[f + 1][0]).max()
        worst = max(worst, e)
        assert e <= tol, f"{label} frame {f}: per-step bbox-relative error {e:.3e} > {tol:.1e}"
    t.check()
    say(f"{label}: worst per-step bbox-relative error {worst:.3e}")
    return worst


def bbox_diag(x):
    return float(np.linalg.norm(x.max(0) - x.min(0)))


def max_err_per_mesh(w, xg, xo):
    """max_i |x_gpu - x_oracle| / bbox diagonal of the oracle's mesh, per mesh."""
    vo, _ = w.offsets()
    out = []
    for k in range(len(vo) - 1):
        a, b = int(vo[k]), int(vo[k + 1])
        d = np.linalg.norm(xg[a:b] - xo[a:b], axis=1).max()
        out.append(d / bbox_diag(xo[a:b]))
    return np.array(out)


def assert_parity(w, xs_g, xs_o, tol=1e-5, label=""):
    worst = 0.0
    for f, (xg, xo) in enumerate(zip(xs_g, xs_o)):
        assert np.all(np.isfinite(xg)), f"{label} frame {f}: non-finite GPU positions"
        e = max_err_per_mesh(w, xg, xo).max()
        worst = max(worst, e)
        assert e <= tol, f"{label} frame {f}: bbox-relative error {e:.3e} > {tol:.1e}"
    say(f"{label}: worst bbox-relative error {worst:.3e}")
    return worst


def replace(p, **kw):
    return dataclasses.replace(p, **kw)
