"""Hand-written adjoint on the GPU against the CPU FP64 oracle adjoint and finite differences.

Tolerances.  One adjoint pass on identical inputs: both sides evaluate the same
expression with relative rounding, bar 1e-11 per conserved component (max-norm).
Through several steps the two forward recomputations differ by rounding
(~1e-16 relative), and the adjoint of the entropic relaxation depends on its
input through grad omega, which is bounded but has a derivative of size 1/|d|
(omega(f) is Lipschitz, not smooth, at equilibrium).  Nodes where d is tiny
(extrema of smooth data) therefore amplify that rounding by ~1/|d|: the bar
there is 1e-10 in the normwise L2 sense and 1e-9 in max-norm.  Measured on an
MI355X (the tests print them): Euler and 2D shallow water 1.6e-13 .. 1.1e-12 (L2)
and 2.0e-13 .. 1.3e-12 (max); the 1D cases, whose smooth data hold more nodes with
tiny d, 1.4e-11 .. 2.8e-11 (L2) and 6.5e-11 .. 1.5e-10 (max).
"""
import numpy as np
import pytest

from gpu_common import componentwise_error, off_equilibrium, oracle_system, to_gpu, to_host
from oracle.adjoint import adjoint_run, misfit_gradient, relax_adjoint
from oracle.scheme import Relaxer
from oracle.systems import equilibrium
from paper_2403_13406_amd import workloads as W
from test_gpu_parity import initial_u, small, solver_for

pytestmark = pytest.mark.gpu
ADJ_RTOL = 1e-11
MULTI_STEP_L2 = 1e-10


@pytest.mark.parametrize("name", ["burgers1d", "sw1d", "euler2d", "sw2d", "burgers2d", "advection2d"])
@pytest.mark.parametrize("relax", ["fixed", "entropic"])
def test_relax_adjoint_pass(name, relax):
    w = small(name)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    h = off_equilibrium(lat, sys, w.V, initial_u(w), shift=3)
    gbar = np.random.default_rng(30).standard_normal(h.shape)
    s = solver_for(w, relax)
    out = to_gpu(gbar)
    s.relax_adjoint(to_gpu(h), out)
    assert s.sync() == 0
    want = relax_adjoint(lat, sys, w.V, h, gbar, relax, 2.0)
    err = componentwise_error(to_host(out), want)
    assert max(err) <= ADJ_RTOL, err


@pytest.mark.parametrize("name,nsteps,ck", [("euler2d", 2, 1), ("sw1d", 3, 2), ("burgers1d", 4, 3), ("sw2d", 2, 5)])
def test_adjoint_through_steps(name, nsteps, ck):
    """eslb_adjoint (checkpointing + recomputation) equals the oracle's taped reverse sweep."""
    w = small(name)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = initial_u(w)
    s = solver_for(w, "entropic")
    f0 = s.init_equilibrium(to_gpu(u))
    fbarT = np.random.default_rng(31).standard_normal(f0.shape)
    fb = to_gpu(fbarT)
    s.adjoint(f0, nsteps, ck, fb)
    assert s.sync() == 0
    assert s.offsets == [0] * s.q
    want = adjoint_run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, u), nsteps, fbarT)
    got = to_host(fb)
    err = componentwise_error(got, want)
    l2s = [np.linalg.norm(got[:, m] - want[:, m]) / np.linalg.norm(want[:, m]) for m in range(want.shape[1])]
    print("%s, %d steps: max-norm %.2e, L2 %.2e" % (name, nsteps, max(err), max(l2s)))
    assert max(err) <= 1e-9, err
    for m, l2 in enumerate(l2s):
        assert l2 <= MULTI_STEP_L2, (m, l2)


def test_full_size_adjoint_sampled():
    """The Euler 1024^2 adjoint workload in the benchmark's configuration (checkpoint every 50, taped
    workspace), one step: sampled cotangents of f0 against the oracle's reverse sweep on a 161 x 161
    periodic window around each node (the cotangent at a node depends on the final cotangent within
    36 cells and on f0 within 72, so the window centre is exact); one window straddles the wrap."""
    w = W.euler2d_adjoint()
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = w.initial_state()
    s = solver_for(w, "entropic")
    f0 = s.init_equilibrium(to_gpu(u))
    fbarT = np.random.default_rng(33).standard_normal(f0.shape)
    fb = to_gpu(fbarT)
    s.adjoint(f0, 1, w.extra["ckpt_every"], fb, tape=True)
    assert s.sync() == 0
    got = to_host(fb)
    R = 80
    for cy, cx in [(3, 1020), (517, 290)]:
        ys = (np.arange(-R, R + 1) + cy) % w.ny
        xs = (np.arange(-R, R + 1) + cx) % w.nx
        fw = fbarT[:, :, ys][:, :, :, xs]
        want = adjoint_run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, u[:, ys][:, :, xs]), 1, fw)
        for m in range(want.shape[1]):
            scale = np.max(np.abs(want[:, m]))
            assert np.max(np.abs(got[:, m, cy, cx] - want[:, m, R, R])) <= 1e-9 * scale


def test_checkpoint_interval_does_not_change_the_result():
    """Recomputation is deterministic, so any checkpoint interval gives the same bits."""
    w = small("euler2d")
    u = initial_u(w)
    s = solver_for(w, "entropic")
    f0 = s.init_equilibrium(to_gpu(u))
    fbarT = to_gpu(np.random.default_rng(32).standard_normal(f0.shape))
    outs = []
    for ck in (1, 2, 5, 50):
        fb = fbarT.clone()
        s.adjoint(f0, 5, ck, fb)
        s.sync()
        outs.append(to_host(fb))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("name,scheme,nsteps,ck", [("euler2d", 1, 5, 2), ("sw2d", 2, 3, 2), ("euler2d", 3, 3, 5),
                                                    ("sw1d", 1, 4, 4)])
def test_taped_and_recomputing_workspaces(name, scheme, nsteps, ck):
    """With the taped workspace (one recomputation per segment) eslb_adjoint gives the
    bits of the minimal workspace (per-step recomputation); both match the oracle's
    reverse sweep, for Scheme I and the projected Schemes II and III."""
    import torch
    w = small(name)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = initial_u(w)
    s = solver_for(w, "entropic", scheme=scheme)
    f0 = s.init_equilibrium(to_gpu(u))
    fbarT = np.random.default_rng(33).standard_normal(f0.shape)
    nmin, ntape = s.adjoint_workspace_bytes(nsteps, ck), s.adjoint_tape_bytes(nsteps, ck)
    outs = []
    for nb in (nmin, ntape):
        fb = to_gpu(fbarT)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        s.adjoint(f0, nsteps, ck, fb, work=work)
        assert s.sync() == 0
        outs.append(to_host(fb))
    assert np.array_equal(outs[0], outs[1])
    want = adjoint_run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, u), nsteps, fbarT,
                       scheme=scheme)
    err = componentwise_error(outs[1], want)
    l2s = [np.linalg.norm(outs[1][:, m] - want[:, m]) / np.linalg.norm(want[:, m]) for m in range(want.shape[1])]
    print("%s, scheme %d, %d steps: max-norm %.2e, L2 %.2e" % (name, scheme, nsteps, max(err), max(l2s)))
    assert max(err) <= 1e-9, err
    for m, l2 in enumerate(l2s):
        assert l2 <= MULTI_STEP_L2, (m, l2)


@pytest.mark.parametrize("nsteps,ck", [(5, 2), (4, 4), (3, 7)])
def test_adjoint_from_forward_checkpoints(nsteps, ck):
    """eslb_step_checkpointed + eslb_adjoint_checkpointed: the forward state of
    eslb_step and the cotangent bits of eslb_adjoint, with either workspace."""
    import torch
    w = small("euler2d")
    s = solver_for(w, "entropic")
    f0 = s.init_equilibrium(to_gpu(initial_u(w)))
    fbarT = to_gpu(np.random.default_rng(34).standard_normal(f0.shape))
    want = fbarT.clone()
    s.adjoint(f0, nsteps, ck, want)
    f_plain = f0.clone()
    s.step(f_plain, nsteps)
    s.offsets = [0] * s.q
    f = f0.clone()
    ckpt = s.step_checkpointed(f, nsteps, ck)
    off = s.offsets
    assert s.sync() == 0
    assert torch.equal(f, f_plain)
    s.offsets = [0] * s.q
    cb = s.checkpoint_bytes(nsteps, ck)
    assert ckpt.numel() * 8 == cb
    for nb in (s.adjoint_workspace_bytes(nsteps, ck) - cb, s.adjoint_tape_bytes(nsteps, ck) - cb):
        fb = fbarT.clone()
        s.adjoint_checkpointed(ckpt, nsteps, ck, fb, work=torch.empty(nb, dtype=torch.uint8, device="cuda"))
        assert s.sync() == 0
        assert s.offsets == [0] * s.q
        assert torch.equal(fb, want)
    assert off != [0] * s.q  # the run moved the offsets (they were restored above)


def test_autograd_misfit_gradient_against_oracle_and_finite_differences():
    """dL/dU0 for L = 1/2 |U(T) - U_target|^2 through the torch.autograd.Function."""
    import torch

    from paper_2403_13406_amd.autograd import time_loop
    w = W.euler2d(40, ny=36, nsteps=3, amp=0.01)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u0 = w.initial_state()
    ut = W.euler2d(40, ny=36, nsteps=3, amp=0.01, seed=1).initial_state()
    s = solver_for(w, "entropic")
    x = to_gpu(u0).requires_grad_(True)
    uT = time_loop(x, s, w.nsteps, ckpt_every=2)
    L = 0.5 * torch.sum((uT - to_gpu(ut)) ** 2)
    L.backward()
    g = to_host(x.grad)
    Lo, go = misfit_gradient(Relaxer(lat, sys, w.V, "entropic"), u0, ut, w.nsteps)
    assert abs(float(L) - Lo) <= 1e-12 * Lo
    assert max(componentwise_error(g[None], go[None])) <= 1e-9
    for m in range(go.shape[0]):
        assert np.linalg.norm(g[m] - go[m]) / np.linalg.norm(go[m]) <= MULTI_STEP_L2
    rng = np.random.default_rng(2)

    def loss(uu):
        with torch.no_grad():
            return float(0.5 * torch.sum((time_loop(to_gpu(uu), s, w.nsteps) - to_gpu(ut)) ** 2))

    for _ in range(4):
        dl = rng.standard_normal(u0.shape)
        e = 1e-6
        fd = (loss(u0 + e * dl) - loss(u0 - e * dl)) / (2 * e)
        assert abs(fd - float(np.sum(g * dl))) <= 1e-7 * abs(fd)


def test_adjoint_workspace_and_checkpoint_errors():
    """Workspaces below the minimum are rejected by eslb_adjoint and eslb_adjoint_checkpointed."""
    import ctypes

    import torch

    from paper_2403_13406_amd import _lib as L
    w = small("euler2d")
    s = solver_for(w, "entropic")
    f0 = s.init_equilibrium(to_gpu(initial_u(w)))
    fb = torch.zeros_like(f0)
    need = s.adjoint_workspace_bytes(4, 2)
    work = torch.empty(need - 8, dtype=torch.uint8, device="cuda")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    assert s.lib.eslb_adjoint(s.ctx, ptr(f0), 4, 2, ptr(fb), ptr(work), work.numel()) == L.ERR_INVALID_ARG
    ckpt = torch.empty(s.checkpoint_bytes(4, 2) // 8, dtype=torch.float64, device="cuda")
    w2 = torch.empty(need - s.checkpoint_bytes(4, 2) - 8, dtype=torch.uint8, device="cuda")
    assert s.lib.eslb_adjoint_checkpointed(s.ctx, ptr(ckpt), 4, 2, ptr(fb), ptr(w2), w2.numel()) == L.ERR_INVALID_ARG
    assert s.lib.eslb_step_checkpointed(s.ctx, ptr(f0), 4, 0, ptr(ckpt)) == L.ERR_INVALID_ARG


def test_adjoint_through_a_fallback_node():
    """A node whose entropic root falls back (omega = 1) contributes no grad-omega term; the recorded
    lambda marks it (NaN) for the adjoint passes.  Single pass (no record) and a whole step (records)
    against the oracle's adjoint."""
    import torch

    from paper_2403_13406_amd import Solver
    lat, sys = oracle_system("D1Q2", "burgers", (1.0,))
    f0 = equilibrium(lat, sys, 1.0, 0.2 + 0.05 * np.sin(2 * np.pi * np.arange(16) / 16)[None, None, :])
    f0[0, 0, 0, 3] -= 0.4
    f0[1, 0, 0, 3] += 0.4
    gbar = np.random.default_rng(35).standard_normal(f0.shape)
    s = Solver("D1Q2", "burgers", 16, 1, V=1.0, relax="entropic", param=(1.0,))
    out = to_gpu(gbar)
    s.relax_adjoint(to_gpu(f0), out)
    with pytest.warns(RuntimeWarning):
        s.sync()
    want = relax_adjoint(lat, sys, 1.0, f0, gbar, "entropic", 2.0)
    assert max(componentwise_error(to_host(out), want)) <= ADJ_RTOL
    s.reset_counters()
    fb = to_gpu(gbar)
    s.offsets = [0] * s.q
    s.adjoint(to_gpu(f0), 1, 1, fb, tape=True)
    with pytest.warns(RuntimeWarning):
        s.sync()
    want = adjoint_run(Relaxer(lat, sys, 1.0, "entropic"), f0, 1, gbar)
    assert max(componentwise_error(to_host(fb), want)) <= 1e-9
