"""Pins of the oracle's reverse mode (adjoint of the unrolled color sweeps).

The expected values come from (a) the complex-step directional derivative of
the oracle's forward rollout (Squire & Trapp 1998: Im f(x + i e d)/e, exact to
rounding for analytic code) and (b) FP64 central differences.  The adjoint
must satisfy <J d, w> = <d, J^T w> (dot-product test).
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2403_06321_amd import workloads as W


def _setup(n=3, frames=3, iters=4, seed=0):
    w = W.tet_cube(n, seed, E_range=(1e4, 1e6))
    m = O.Model.from_workload(w)
    rng = np.random.default_rng(seed + 100)
    v0 = rng.normal(scale=0.5, size=w.x0.shape) * (1 - w.pinned[:, None])
    p = dataclasses.replace(w.params, n_iters=iters)
    return w, m, p, v0, frames


def _rollout_cs(m, p, x0, v0, E, frames):
    x, v = x0.astype(np.complex128), v0.astype(np.complex128)
    vp = v.copy()   # v^{-1} := v^0 (tied)
    for _ in range(frames):
        x, v, vp = O.step_cs(m, p, x, v, vp, E)
    return x, v


def _rollout(m, p, x0, v0, E, frames):
    x, v, vp, states = O.rollout(m, p, x0, v0, E, frames)
    return x, v, states


def _adjoint(m, p, states, E, wx, wv):
    gx, gv, gvp = wx.copy(), wv.copy(), np.zeros_like(wx)
    gE = np.zeros(E.shape[0])
    for (xt, vt, vpt) in reversed(states):
        gx, gv, gvp, gE = O.step_backward(m, p, xt, vt, vpt, E, gx, gv, gvp, gE)
    return gx, gv + gvp, gE   # v^{-1} tied to v^0


def test_complex_step_matches_real_forward_and_central_differences():
    w, m, p, v0, frames = _setup()
    rng = np.random.default_rng(1)
    dx = rng.normal(size=w.x0.shape) * (1 - w.pinned[:, None]) * 1e-3
    dv = rng.normal(size=w.x0.shape) * (1 - w.pinned[:, None])
    dE = rng.normal(size=w.n_tets) * w.tet_E
    xr, vr, _ = _rollout(m, p, w.x0, v0, w.tet_E, frames)
    eps = 1e-30
    xc, vc = _rollout_cs(m, p, w.x0 + 1j * eps * dx, v0 + 1j * eps * dv, w.tet_E + 1j * eps * dE, frames)
    assert np.abs(xc.real - xr).max() <= 1e-15
    tan_cs = xc.imag / eps
    h = 1e-5
    xp, _, _ = _rollout(m, p, w.x0 + h * dx, v0 + h * dv, w.tet_E + h * dE, frames)
    xm, _, _ = _rollout(m, p, w.x0 - h * dx, v0 - h * dv, w.tet_E - h * dE, frames)
    tan_fd = (xp - xm) / (2 * h)
    assert np.abs(tan_cs - tan_fd).max() <= 1e-6 * np.abs(tan_cs).max()


@pytest.mark.parametrize("seed,n,frames,iters", [(0, 3, 3, 4), (1, 4, 2, 3)])
def test_adjoint_dot_product(seed, n, frames, iters):
    w, m, p, v0, frames = _setup(n=n, frames=frames, iters=iters, seed=seed)
    rng = np.random.default_rng(seed + 7)
    wx = rng.normal(size=w.x0.shape)
    wv = rng.normal(size=w.x0.shape)
    _, _, states = _rollout(m, p, w.x0, v0, w.tet_E, frames)
    gx, gv, gE = _adjoint(m, p, states, w.tet_E, wx, wv)
    for trial in range(3):
        dx = rng.normal(size=w.x0.shape) * 1e-3
        dv = rng.normal(size=w.x0.shape)
        dE = rng.normal(size=w.n_tets) * w.tet_E
        eps = 1e-30
        xc, vc = _rollout_cs(m, p, w.x0 + 1j * eps * dx, v0 + 1j * eps * dv,
                             w.tet_E + 1j * eps * dE, frames)
        lhs = np.sum(xc.imag / eps * wx) + np.sum(vc.imag / eps * wv)
        rhs = np.sum(dx * gx) + np.sum(dv * gv) + np.sum(dE * gE)
        assert rhs == pytest.approx(lhs, rel=1e-10)


def test_adjoint_centroid_loss_vs_central_differences():
    """Loss of the differentiable workload (squared distance of the final
    centroid to a target) on a small cube: gradient w.r.t. sampled E_t and
    v0 entries against FP64 central differences."""
    w, m, p, v0, frames = _setup(n=3, frames=3, iters=5, seed=2)
    target = w.x0.mean(0) + np.array([0.2, -0.1, 0.3])
    nv = w.n_verts

    def loss(x0, v0_, E):
        x, _, _ = _rollout(m, p, x0, v0_, E, frames)
        d = x.mean(0) - target
        return d @ d

    x, _, states = _rollout(m, p, w.x0, v0, w.tet_E, frames)
    d = x.mean(0) - target
    wx = np.tile(2 * d / nv, (nv, 1))
    gx, gv, gE = _adjoint(m, p, states, w.tet_E, wx, np.zeros_like(wx))
    rng = np.random.default_rng(0)
    for t in rng.choice(w.n_tets, 5, replace=False):
        hE = 1e-4 * w.tet_E[t]
        Ep = w.tet_E.copy(); Ep[t] += hE
        Em = w.tet_E.copy(); Em[t] -= hE
        fd = (loss(w.x0, v0, Ep) - loss(w.x0, v0, Em)) / (2 * hE)
        assert gE[t] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(gE).max())
    free = np.flatnonzero(w.pinned == 0)
    for i in rng.choice(free, 4, replace=False):
        for a in range(3):
            hv = 1e-4
            vp_ = v0.copy(); vp_[i, a] += hv
            vm_ = v0.copy(); vm_[i, a] -= hv
            fd = (loss(w.x0, vp_, w.tet_E) - loss(w.x0, vm_, w.tet_E)) / (2 * hv)
            assert gv[i, a] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(gv).max())


def test_backward_rejects_unsupported_elements():
    w = W.single_particle_chain(3)
    m = O.Model.from_workload(w)
    with pytest.raises(ValueError):
        O.step_backward(m, w.params, w.x0, w.v0, w.v0, np.zeros(0), w.x0, w.v0, w.v0)
