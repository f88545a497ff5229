"""Python binding of one eslb context (see include/eslb.h).

PyTorch only provides device memory and the stream; every step of the time loop
runs in libeslb's HIP kernels.  States are float64 CUDA tensors of shape
(q, M, ny, nx) (plane k*M + m, x fastest); conserved moments are (M, ny, nx).
"""
import ctypes
import warnings

from . import _lib as L

LATTICES = {"D1Q2": L.D1Q2, "D2Q4": L.D2Q4}
SYSTEMS = {"advection": L.ADVECTION, "burgers": L.BURGERS, "shallow_water": L.SHALLOW_WATER, "euler": L.EULER}
RELAX = {"fixed": L.OMEGA_FIXED, "entropic": L.OMEGA_ENTROPIC}


class EslbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("eslb error %d (%s): %s" % (code, L.load().eslb_status_string(code).decode(), msg))
        self.code = code


def _check(lib, ctx, rc):
    if rc < 0:
        raise EslbError(rc, lib.eslb_last_error(ctx).decode())
    if rc > 0:
        warnings.warn(lib.eslb_status_string(rc).decode(), RuntimeWarning, stacklevel=3)
    return rc


def make_problem(lattice, system, nx, ny=1, V=1.0, dx=None, kappa=1, relax="entropic", omega=2.0,
                 scheme=1, param=(0.0, 0.0, 0.0, 0.0)):
    p = L.Problem()
    p.lattice = LATTICES[lattice]
    p.system = SYSTEMS[system]
    p.nx, p.ny = int(nx), int(ny)
    p.kappa = int(kappa)
    p.relax = RELAX[relax]
    p.scheme = int(scheme)
    p.reserved = 0
    p.V = float(V)
    p.dx = float(dx if dx is not None else (1.0 / nx if nx > 0 else 0.0))
    p.omega = float(omega)
    prm = list(param) + [0.0] * (4 - len(param))
    for i in range(4):
        p.param[i] = float(prm[i])
    return p


class Solver:
    """One problem on one device stream (eslb_create .. eslb_destroy)."""

    def __init__(self, lattice, system, nx, ny=1, V=1.0, dx=None, kappa=1, relax="entropic", omega=2.0,
                 scheme=1, param=(0.0,), stream=None, fused="auto"):
        """fused: policy of the fused D1Q2 step ("auto": where it is the faster path,
        True: always, False: never); a workspace of one state is attached when the
        policy takes it."""
        import torch
        self.lib = L.load()
        self.problem = make_problem(lattice, system, nx, ny, V, dx, kappa, relax, omega, scheme, param)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        ctx = ctypes.c_void_p()
        rc = self.lib.eslb_create(ctypes.byref(self.problem), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(ctx))
        if rc < 0:
            raise EslbError(rc, self.lib.eslb_last_error(None).decode())
        self.ctx = ctx
        M, q = ctypes.c_int32(), ctypes.c_int32()
        self.lib.eslb_dims(ctx, ctypes.byref(M), ctypes.byref(q))
        self.M, self.q = M.value, q.value
        self.nx, self.ny = int(nx), int(ny)
        self.step_work = None
        self.set_fused(fused)

    def set_fused(self, policy="auto"):
        """Fusion policy ("auto", True, False) and the workspace it needs; True when eslb_step
        now takes the fused kernel."""
        import torch
        code = {"auto": L.FUSE_AUTO, True: L.FUSE_ALWAYS, False: L.FUSE_OFF}[policy]
        _check(self.lib, self.ctx, self.lib.eslb_set_fusion(self.ctx, code))
        avail = ctypes.c_int32()
        self.lib.eslb_fused_step_available(self.ctx, ctypes.byref(avail))
        if avail.value:
            if self.step_work is None:
                self.step_work = torch.empty(self.state_shape, dtype=torch.float64, device="cuda")
            _check(self.lib, self.ctx, self.lib.eslb_set_step_workspace(
                self.ctx, ctypes.c_void_p(self.step_work.data_ptr()), self.step_work.numel() * 8))
            return True
        _check(self.lib, self.ctx, self.lib.eslb_set_step_workspace(self.ctx, None, 0))
        self.step_work = None
        return False

    # -- lifetime
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.eslb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers
    def _ptr(self, t, shape):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected a contiguous float64 CUDA tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(t.shape)))
        return ctypes.c_void_p(t.data_ptr())

    @property
    def state_shape(self):
        return (self.q, self.M, self.ny, self.nx)

    @property
    def moment_shape(self):
        return (self.M, self.ny, self.nx)

    def empty_state(self):
        import torch
        return torch.empty(self.state_shape, dtype=torch.float64, device="cuda")

    # -- scalar queries
    def dt(self):
        v = ctypes.c_double()
        _check(self.lib, self.ctx, self.lib.eslb_dt(self.ctx, ctypes.byref(v)))
        return v.value

    def steps_for_time(self, T):
        n = ctypes.c_int64()
        rc = self.lib.eslb_steps_for_time(self.ctx, float(T), ctypes.byref(n))
        if rc < 0:
            _check(self.lib, self.ctx, rc)
        return n.value

    # -- the time loop
    def init_equilibrium(self, u, f=None):
        f = self.empty_state() if f is None else f
        _check(self.lib, self.ctx, self.lib.eslb_init_equilibrium(self.ctx, self._ptr(u, self.moment_shape),
                                                                   self._ptr(f, self.state_shape)))
        return f

    def step(self, f, nsteps=1):
        _check(self.lib, self.ctx, self.lib.eslb_step(self.ctx, self._ptr(f, self.state_shape), int(nsteps)))
        return f

    def transport(self, cells):
        _check(self.lib, self.ctx, self.lib.eslb_transport(self.ctx, int(cells)))

    def relax(self, f):
        _check(self.lib, self.ctx, self.lib.eslb_relax(self.ctx, self._ptr(f, self.state_shape)))
        return f

    def project(self, f):
        _check(self.lib, self.ctx, self.lib.eslb_project(self.ctx, self._ptr(f, self.state_shape)))
        return f

    def moments(self, f, u=None):
        import torch
        u = torch.empty(self.moment_shape, dtype=torch.float64, device="cuda") if u is None else u
        _check(self.lib, self.ctx, self.lib.eslb_moments(self.ctx, self._ptr(f, self.state_shape),
                                                         self._ptr(u, self.moment_shape)))
        return u

    def gather(self, f, out=None):
        out = self.empty_state() if out is None else out
        _check(self.lib, self.ctx, self.lib.eslb_gather(self.ctx, self._ptr(f, self.state_shape),
                                                        self._ptr(out, self.state_shape)))
        return out

    @property
    def offsets(self):
        arr = (ctypes.c_int64 * self.q)()
        _check(self.lib, self.ctx, self.lib.eslb_get_offsets(self.ctx, arr))
        return list(arr)

    @offsets.setter
    def offsets(self, vals):
        arr = (ctypes.c_int64 * self.q)(*[int(v) for v in vals])
        _check(self.lib, self.ctx, self.lib.eslb_set_offsets(self.ctx, arr))

    # -- status
    def set_stats(self, on=True):
        _check(self.lib, self.ctx, self.lib.eslb_set_stats(self.ctx, 1 if on else 0))

    def reset_counters(self):
        _check(self.lib, self.ctx, self.lib.eslb_reset_counters(self.ctx))

    def sync(self):
        return _check(self.lib, self.ctx, self.lib.eslb_sync_status(self.ctx))

    def diagnostics(self, f):
        d = L.Diag()
        rc = self.lib.eslb_diagnostics(self.ctx, self._ptr(f, self.state_shape), ctypes.byref(d))
        _check(self.lib, self.ctx, rc)
        return {"status": rc, "mass": list(d.mass)[:self.M], "micro_entropy": d.micro_entropy,
                "macro_entropy": d.macro_entropy, "omega_min": d.omega_min, "omega_max": d.omega_max,
                "n_fallback": d.n_fallback, "n_outside": d.n_outside, "n_inadmissible": d.n_inadmissible,
                "n_nan": d.n_nan}

    def diagnostics_sums(self, f, out):
        """eslb_diagnostics_noalloc: mass[M], micro and macro entropy into the float64 CUDA
        tensor out (M + 2 values), asynchronously, with no allocation in the library."""
        _check(self.lib, self.ctx, self.lib.eslb_diagnostics_noalloc(self.ctx, self._ptr(f, self.state_shape),
                                                                     self._ptr(out, (self.M + 2,))))
        return out

    # -- adjoint
    def relax_adjoint(self, h, gbar):
        _check(self.lib, self.ctx, self.lib.eslb_relax_adjoint(self.ctx, self._ptr(h, self.state_shape),
                                                               self._ptr(gbar, self.state_shape)))
        return gbar

    def moments_adjoint(self, ubar, fbar=None):
        fbar = self.empty_state() if fbar is None else fbar
        _check(self.lib, self.ctx, self.lib.eslb_moments_adjoint(self.ctx, self._ptr(ubar, self.moment_shape),
                                                                 self._ptr(fbar, self.state_shape)))
        return fbar

    def init_adjoint(self, u, fbar, ubar=None):
        import torch
        ubar = torch.empty(self.moment_shape, dtype=torch.float64, device="cuda") if ubar is None else ubar
        _check(self.lib, self.ctx, self.lib.eslb_init_adjoint(self.ctx, self._ptr(u, self.moment_shape),
                                                              self._ptr(fbar, self.state_shape),
                                                              self._ptr(ubar, self.moment_shape)))
        return ubar

    def adjoint_workspace_bytes(self, nsteps, ckpt_every):
        b = ctypes.c_size_t()
        _check(self.lib, self.ctx, self.lib.eslb_adjoint_workspace_bytes(self.ctx, int(nsteps), int(ckpt_every),
                                                                         ctypes.byref(b)))
        return b.value

    def adjoint_tape_bytes(self, nsteps, ckpt_every):
        b = ctypes.c_size_t()
        _check(self.lib, self.ctx, self.lib.eslb_adjoint_tape_bytes(self.ctx, int(nsteps), int(ckpt_every),
                                                                    ctypes.byref(b)))
        return b.value

    def checkpoint_bytes(self, nsteps, ckpt_every):
        b = ctypes.c_size_t()
        _check(self.lib, self.ctx, self.lib.eslb_checkpoint_bytes(self.ctx, int(nsteps), int(ckpt_every),
                                                                  ctypes.byref(b)))
        return b.value

    def step_checkpointed(self, f, nsteps, ckpt_every, ckpt=None):
        """nsteps steps on f, keeping the state every ckpt_every steps (returns the checkpoints)."""
        import torch
        nseg = -(-int(nsteps) // int(ckpt_every))
        if ckpt is None:
            ckpt = torch.empty((max(nseg, 1),) + self.state_shape, dtype=torch.float64, device="cuda")
        if ckpt.dtype != torch.float64 or not ckpt.is_cuda or not ckpt.is_contiguous() or \
                ckpt.numel() * 8 < self.checkpoint_bytes(nsteps, ckpt_every):
            raise ValueError("checkpoint buffer too small")
        _check(self.lib, self.ctx, self.lib.eslb_step_checkpointed(self.ctx, self._ptr(f, self.state_shape),
                                                                   int(nsteps), int(ckpt_every),
                                                                   ctypes.c_void_p(ckpt.data_ptr())))
        return ckpt

    def adjoint_checkpointed(self, ckpt, nsteps, ckpt_every, fbar, work=None, tape="auto"):
        """Solver.adjoint from the checkpoints of step_checkpointed (offsets as at its start)."""
        import torch
        cb = self.checkpoint_bytes(nsteps, ckpt_every)
        if ckpt.dtype != torch.float64 or not ckpt.is_cuda or not ckpt.is_contiguous() or ckpt.numel() * 8 < cb:
            raise ValueError("checkpoint buffer too small")
        nb = self.adjoint_workspace_bytes(nsteps, ckpt_every) - cb
        if work is None:
            nt = self.adjoint_tape_bytes(nsteps, ckpt_every) - cb
            if tape is True or (tape == "auto" and nt <= torch.cuda.mem_get_info()[0] // 2):
                nb = max(nb, nt)
            work = torch.empty(max(nb, 8), dtype=torch.uint8, device="cuda")
        _check(self.lib, self.ctx, self.lib.eslb_adjoint_checkpointed(
            self.ctx, ctypes.c_void_p(ckpt.data_ptr()), int(nsteps), int(ckpt_every),
            self._ptr(fbar, self.state_shape), ctypes.c_void_p(work.data_ptr()), work.numel()))
        return fbar

    def adjoint(self, f0, nsteps, ckpt_every, fbar, work=None, tape="auto"):
        """fbar (logical, cotangent of the state after nsteps) -> cotangent of f0, in place.

        work=None allocates the workspace: the taped size (each step recomputed once
        instead of twice) when tape is True, or when tape is "auto" and it takes at
        most half of the free device memory; otherwise the minimal size."""
        import torch
        nb = self.adjoint_workspace_bytes(nsteps, ckpt_every)
        if work is None:
            nt = self.adjoint_tape_bytes(nsteps, ckpt_every)
            if tape is True or (tape == "auto" and nt <= torch.cuda.mem_get_info()[0] // 2):
                nb = max(nb, nt)
            work = torch.empty(max(nb, 8), dtype=torch.uint8, device="cuda")
        _check(self.lib, self.ctx, self.lib.eslb_adjoint(self.ctx, self._ptr(f0, self.state_shape), int(nsteps),
                                                         int(ckpt_every), self._ptr(fbar, self.state_shape),
                                                         ctypes.c_void_p(work.data_ptr()), work.numel()))
        return fbar
