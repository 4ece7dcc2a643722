"""vbd_step_static, the step that allocates nothing (its state buffers live
in the library's fixed per-device scratch), against vbd_step on the same
inputs: identical results on two calls in a row, the second on a smaller
topology, in the plain and the persistent launch modes, with and without
Chebyshev acceleration; limits and unsupported modes rejected."""
import dataclasses

import numpy as np
import pytest

from paper_2403_06321_amd import _native as N
from paper_2403_06321_amd import workloads as W
from gpu_util import say

pytestmark = pytest.mark.gpu


def _state(w, dev):
    import torch
    x = torch.tensor(w.x0, dtype=torch.float32, device=dev).contiguous()
    v = torch.tensor(w.v0, dtype=torch.float32, device=dev).contiguous()
    E = torch.tensor(w.tet_E, dtype=torch.float32, device=dev).contiguous()
    return x, v, v.clone(), E


def _run_both(w, params, mode, frames):
    """(x, v) after `frames` steps through vbd_step and through
    vbd_step_static, each on its own copy of the same inputs."""
    import torch
    from paper_2403_06321_amd.api import Topology
    dev = torch.device("cuda", 0)
    t = Topology.from_workload(w)
    out = []
    for static in (False, True):
        x, v, vp, E = _state(w, dev)
        for _ in range(frames):
            (t.step_static if static else t.step)(x, v, vp, E, params, mode)
        torch.cuda.synchronize()
        t.check()
        out.append((x.cpu().numpy(), v.cpu().numpy(), vp.cpu().numpy()))
    return out


@pytest.mark.parametrize("mode", [N.LAUNCH_PLAIN, N.LAUNCH_PERSISTENT])
@pytest.mark.parametrize("cheb", [0.0, 0.9])
def test_static_step_matches_step_on_two_calls(mode, cheb):
    """First a 17^3 cube (4913 vertices), then a 6^3 cube (216 vertices) in
    the scratch the first one left: both equal vbd_step bit for bit."""
    for n, seed in ((17, 11), (6, 12)):
        w = W.tet_cube(n, seed, E_range=(1e4, 1e6), n_iters=10, frames=3)
        w = dataclasses.replace(w, v0=np.random.default_rng(seed).uniform(-0.5, 0.5, (len(w.x0), 3))
                                * (w.pinned[:, None] == 0))
        p = dataclasses.replace(w.params, cheb_rho=cheb)
        (xa, va, pa), (xb, vb, pb) = _run_both(w, p, mode, w.frames)
        say(f"static step {n}^3 mode {mode} rho {cheb}: max |dx| {np.abs(xa - xb).max():.1e}")
        assert np.all(np.isfinite(xa))
        assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(pa, pb)


def test_static_step_springs_and_analytic_contacts():
    """The 32^2 cloth (springs, sphere and ground contacts) for two frames,
    after the larger cubes above have used the scratch."""
    w = W.config_cloth_coarse(32, frames=12)
    (xa, va, _), (xb, vb, _) = _run_both(w, w.params, N.LAUNCH_PLAIN, w.frames)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_static_step_limits_and_unsupported_modes():
    import torch
    from paper_2403_06321_amd.api import Topology
    dev = torch.device("cuda", 0)
    w = W.tet_cube(5, 1, n_iters=2)
    t = Topology.from_workload(w)
    x, v, vp, E = _state(w, dev)
    for mode in (N.LAUNCH_GRAPH, N.LAUNCH_PERSISTENT_GRAPH):
        with pytest.raises(N.VBDError) as ei:
            t.step_static(x, v, vp, E, w.params, mode)
        assert ei.value.status == -6
    # 1.3M particles: 48 B of state each fit in 96 MiB, 80 B (acceleration) do not
    n = 1_300_000
    c = W.single_particle_chain(n, length=1e-3)
    tc = Topology.from_workload(c)
    xc = torch.tensor(c.x0, dtype=torch.float32, device=dev).contiguous()
    vc = torch.zeros_like(xc)
    p = dataclasses.replace(c.params, n_iters=1)
    with pytest.raises(N.VBDError) as ei:
        tc.step_static(xc, vc, vc.clone(), None, dataclasses.replace(p, cheb_rho=0.5))
    assert ei.value.status == -1 and "static scratch" in str(ei.value)
    tc.step_static(xc, vc, vc.clone(), None, p)
    torch.cuda.synchronize()
    tc.check()
    assert bool(torch.isfinite(xc).all())
