"""Python face of libshk: a Grid owns a torch-allocated workspace and calls
the C ABI with raw device pointers on torch's current HIP stream.  Argument
marshalling only -- every step of the computation runs in the HIP kernels.
"""
import ctypes

import torch

from ._lib import GridDesc, check, lib

F64, F32, MIXED = 0, 1, 2
TRANSMISSIVE, REFLECTIVE, INFLOW, PERIODIC = 0, 1, 2, 3
_PREC = {"f64": F64, "f32": F32, "mixed": MIXED, F64: F64, F32: F32, MIXED: MIXED}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Grid:
    """A uniform grid with its physics, boundary rules and workspace."""

    def __init__(self, nx, ny=1, ndim=2, nbatch=1, domain=(0.0, 1.0, 0.0, 1.0), prec="f64", gamma=1.4,
                 cfl=0.5, weno_eps=1e-6, viscous=False, mu=0.0, prandtl=0.72, nu_art=0.0,
                 bc=(TRANSMISSIVE,) * 4, inflow=(1.0, 0.0, 0.0, 1.0), ibm=False, adjoint=False,
                 flux_net=False, weno_char=False, device="cuda"):
        self._args = dict(nx=nx, ny=ny, ndim=ndim, nbatch=nbatch, domain=domain, prec=prec, gamma=gamma, cfl=cfl,
                          weno_eps=weno_eps, viscous=viscous, mu=mu, prandtl=prandtl, nu_art=nu_art, bc=bc,
                          inflow=inflow, ibm=ibm, adjoint=adjoint, flux_net=flux_net, weno_char=weno_char,
                          device=device)
        d = GridDesc()
        d.ndim, d.nx, d.ny, d.nbatch = ndim, nx, (1 if ndim == 1 else ny), nbatch
        d.x0, d.x1 = domain[0], domain[1]
        d.y0, d.y1 = (domain[2], domain[3]) if ndim == 2 else (0.0, 1.0)
        d.prec = _PREC[prec]
        d.gamma, d.cfl, d.weno_eps = gamma, cfl, weno_eps
        d.viscous, d.mu, d.prandtl, d.nu_art = int(viscous), mu, prandtl, nu_art
        for k in range(4):
            d.bc[k] = bc[k]
            d.inflow_prim[k] = inflow[k]
        d.ibm, d.adjoint, d.flux_net = int(ibm), int(adjoint), int(flux_net)
        d.weno_char = int(weno_char)
        self.desc = d
        self.device = torch.device(device)
        self.dtype = torch.float64 if d.prec == F64 else torch.float32
        self.nvar = 3 if ndim == 1 else 4
        self.shape = (nbatch, self.nvar, d.ny, nx)
        nbytes = lib().shk_workspace_bytes(ctypes.byref(d))
        if nbytes == 0:
            raise ValueError("invalid grid description")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        h = ctypes.c_void_p()
        check(lib().shk_init_grid(ctypes.byref(d), _ptr(self._ws), nbytes, _stream(), ctypes.byref(h)),
              None, "init_grid")
        self.handle = h
        self.phi = None
        self.wall = 0
        self.net = None
        self.version = 0  # bumped by a new level set or network (see replica)
        self._replica = None
        self.nface = (nx + 1) * d.ny + nx * (d.ny + 1)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            lib().shk_destroy(h)
            self.handle = None

    # -- helpers
    def _sync_stream(self):
        check(lib().shk_set_stream(self.handle, _stream()), self.handle, "set_stream")

    def _check_state(self, U):
        if not (U.is_cuda and U.dtype == self.dtype and U.is_contiguous() and U.numel() == self._numel()):
            raise ValueError(f"state must be a contiguous {self.dtype} CUDA tensor with {self._numel()} elements")

    def _check_tape(self, tape):
        if not (tape.is_cuda and tape.dtype == torch.float64 and tape.is_contiguous()
                and tuple(tape.shape) == (3,) + tuple(self.shape)):
            raise ValueError("tape must be a contiguous float64 CUDA tensor of shape (3,) + grid state shape")

    def _numel(self):
        b, v, ny, nx = self.shape
        return b * v * ny * nx

    def empty_state(self):
        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    # -- ABI calls
    def prim_to_cons(self, W):
        W = W.to(device=self.device, dtype=self.dtype).contiguous().reshape(self.shape)
        U = self.empty_state()
        self._sync_stream()
        check(lib().shk_prim_to_cons(self.handle, _ptr(W), _ptr(U)), self.handle, "prim_to_cons")
        return U

    def prim_to_cons_vjp(self, W, U_bar, W_bar=None, param_bar=None):
        """Reverse mode of prim_to_cons: W_bar += (dU/dW)^T U_bar and
        param_bar[:, 0] += (dU/dgamma) . U_bar (each may be None).  Returns
        (W_bar, param_bar)."""
        W = W.to(device=self.device, dtype=torch.float64).contiguous().reshape(self.shape)
        U_bar = U_bar.to(device=self.device, dtype=torch.float64).contiguous().reshape(self.shape)
        self._sync_stream()
        check(lib().shk_prim_to_cons_vjp(self.handle, _ptr(W), _ptr(U_bar), _ptr(W_bar), _ptr(param_bar)),
              self.handle, "prim_to_cons_vjp")
        return W_bar, param_bar

    def set_levelset(self, phi, wall=0):
        self.version += 1
        if phi is None:
            check(lib().shk_set_ib_levelset(self.handle, None, 0), self.handle, "set_ib_levelset")
            self.phi = None
            return 0
        phi = phi.to(device=self.device, dtype=torch.float64).contiguous()
        if phi.numel() != self.desc.nx * self.desc.ny:
            raise ValueError("level set must have ny*nx entries")
        self.phi = phi  # the table is built from it; keep it alive
        self.wall = int(wall)
        self._sync_stream()
        check(lib().shk_set_ib_levelset(self.handle, _ptr(phi), int(wall)), self.handle, "set_ib_levelset")
        n = ctypes.c_int()
        check(lib().shk_ib_ghost_count(self.handle, ctypes.byref(n)), self.handle, "ib_ghost_count")
        return n.value

    def classes(self):
        c = torch.empty((self.desc.ny, self.desc.nx), dtype=torch.uint8, device=self.device)
        self._sync_stream()
        check(lib().shk_ib_classes(self.handle, _ptr(c)), self.handle, "ib_classes")
        return c

    def ib_fill(self, U):
        """Refill the immersed-boundary ghost cells of U in place."""
        self._check_state(U)
        self._sync_stream()
        check(lib().shk_ib_fill(self.handle, _ptr(U)), self.handle, "ib_fill")
        return U

    def rhs(self, U, out=None):
        """L(U) of the semi-discrete scheme; U is not modified."""
        self._check_state(U)
        out = self.empty_state() if out is None else out
        self._sync_stream()
        check(lib().shk_rhs(self.handle, _ptr(U), _ptr(out)), self.handle, "rhs")
        return out

    def step(self, U, dt=None, dt_out=None):
        """One SSP-RK3 step in place; dt: None (automatic CFL step), a float
        or a CUDA float64 tensor of nbatch entries."""
        self._check_state(U)
        if dt is not None and not torch.is_tensor(dt):
            dt = torch.full((self.shape[0],), float(dt), dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(lib().shk_rk3_step(self.handle, _ptr(U), _ptr(dt), _ptr(dt_out)), self.handle, "rk3_step")
        return U

    # -- learned flux correction
    def set_flux_net(self, net):
        """Attach a learn.FluxNet (its device buffers must stay alive) or None."""
        self.version += 1
        if net is None:
            check(lib().shk_set_flux_net(self.handle, None, None, None, 0.0, 0), self.handle, "set_flux_net")
            self.net = None
            return
        norm = (ctypes.c_double * 8)(*net.mean, *net.inv_std)
        check(lib().shk_set_flux_net(self.handle, _ptr(net.w), _ptr(net.bias), norm, float(net.out_scale), 1),
              self.handle, "set_flux_net")
        self.net = net

    def set_flux_cnn(self, net):
        """Attach a learn.FluxCnn (the convolutional correction; grid created
        with flux_net=2) or None."""
        self.version += 1
        if net is None:
            check(lib().shk_set_flux_cnn(self.handle, None, None, None, 0.0, 0), self.handle, "set_flux_cnn")
            self.net = None
            return
        norm = (ctypes.c_double * 8)(*net.mean, *net.inv_std)
        check(lib().shk_set_flux_cnn(self.handle, _ptr(net.w), _ptr(net.bias), norm, float(net.out_scale), 1),
              self.handle, "set_flux_cnn")
        self.net = net

    def flux_cnn_eval(self, U):
        self._check_state(U)
        dF = torch.empty((self.shape[0], self.nface, 4), dtype=torch.float32, device=self.device)
        self._sync_stream()
        check(lib().shk_flux_cnn_eval(self.handle, _ptr(U), _ptr(dF)), self.handle, "flux_cnn_eval")
        return dF

    def flux_cnn_vjp(self, U, lam, grad=None):
        self._check_state(U)
        self._check_state(lam)
        dX = torch.empty((self.shape[0], self.nface, 6, 4), dtype=torch.float32, device=self.device)
        self._sync_stream()
        check(lib().shk_flux_cnn_vjp(self.handle, _ptr(U), _ptr(lam), _ptr(dX), _ptr(grad)), self.handle,
              "flux_cnn_vjp")
        return dX

    def flux_cnn_images(self, U):
        """The network's input images (x-faces [ny][wx], transposed y-faces
        [nx][wy], 4 channels) as float tensors per batch member."""
        self._check_state(U)
        n = ctypes.c_int()
        check(lib().shk_flux_cnn_images(self.handle, None, None, ctypes.byref(n)), self.handle, "flux_cnn_images")
        out = torch.empty((self.shape[0], n.value, 4), dtype=torch.float32, device=self.device)
        self._sync_stream()
        check(lib().shk_flux_cnn_images(self.handle, _ptr(U), _ptr(out), ctypes.byref(n)), self.handle,
              "flux_cnn_images")
        d = self.desc
        wx = d.nx if d.bc[0] == PERIODIC else d.nx + 1
        wy = d.ny if d.bc[2] == PERIODIC else d.ny + 1
        n0 = d.ny * wx
        return out[:, :n0].reshape(-1, d.ny, wx, 4), out[:, n0:].reshape(-1, d.nx, wy, 4)

    def set_flux_net_grad(self, grad):
        check(lib().shk_set_flux_net_grad(self.handle, _ptr(grad)), self.handle, "set_flux_net_grad")

    def flux_net_eval(self, U):
        self._check_state(U)
        dF = torch.empty((self.shape[0], self.nface, 4), dtype=torch.float32, device=self.device)
        self._sync_stream()
        check(lib().shk_flux_net_eval(self.handle, _ptr(U), _ptr(dF)), self.handle, "flux_net_eval")
        return dF

    def flux_net_vjp(self, U, lam, grad=None):
        self._check_state(U)
        self._check_state(lam)
        dX = torch.empty((self.shape[0], self.nface, 6, 4), dtype=torch.float32, device=self.device)
        self._sync_stream()
        check(lib().shk_flux_net_vjp(self.handle, _ptr(U), _ptr(lam), _ptr(dX), _ptr(grad)), self.handle,
              "flux_net_vjp")
        return dX

    def param_bar(self):
        """Zeroed accumulator for (gamma, inflow rho, u, v, p) derivatives."""
        return torch.zeros((self.shape[0], 5), dtype=torch.float64, device=self.device)

    def rhs_adjoint(self, U, dUdt_bar, U_bar, param_bar=None):
        """U_bar += (d rhs/dU)^T dUdt_bar; param_bar += parameter derivatives."""
        for t in (U, dUdt_bar, U_bar):
            self._check_state(t)
        self._sync_stream()
        check(lib().shk_rhs_adjoint(self.handle, _ptr(U), _ptr(dUdt_bar), _ptr(U_bar), _ptr(param_bar)),
              self.handle, "rhs_adjoint")
        return U_bar

    def step_adjoint(self, U_n, dt, U_bar, param_bar=None):
        """U_bar (adjoint after the step) -> adjoint of U_n, in place."""
        self._check_state(U_n)
        self._check_state(U_bar)
        if not torch.is_tensor(dt):
            dt = torch.full((self.shape[0],), float(dt), dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(lib().shk_rk3_step_adjoint(self.handle, _ptr(U_n), _ptr(dt), _ptr(U_bar), _ptr(param_bar)),
              self.handle, "rk3_step_adjoint")
        return U_bar

    def empty_tape(self):
        """Buffer for the three recorded stage-start states of one step."""
        return torch.empty((3,) + tuple(self.shape), dtype=torch.float64, device=self.device)

    def step_record(self, U, tape, dt=None, dt_out=None):
        """One RK3 step in place (as step) that also records U^n, U1, U2
        (after the immersed-boundary refill) into tape for step_adjoint_tape."""
        self._check_state(U)
        self._check_tape(tape)
        if dt is not None and not torch.is_tensor(dt):
            dt = torch.full((self.shape[0],), float(dt), dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(lib().shk_rk3_step_record(self.handle, _ptr(U), _ptr(dt), _ptr(dt_out), _ptr(tape)),
              self.handle, "rk3_step_record")
        return U

    def step_adjoint_tape(self, tape, dt, U_bar, param_bar=None):
        """U_bar (adjoint after a recorded step) -> adjoint of its U^n, in place."""
        self._check_state(U_bar)
        self._check_tape(tape)
        if not torch.is_tensor(dt):
            dt = torch.full((self.shape[0],), float(dt), dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(lib().shk_rk3_step_adjoint_tape(self.handle, _ptr(tape), _ptr(dt), _ptr(U_bar), _ptr(param_bar)),
              self.handle, "rk3_step_adjoint_tape")
        return U_bar

    def _check_tapes(self, tapes, nsteps):
        if not (tapes.is_cuda and tapes.dtype == torch.float64 and tapes.is_contiguous()
                and tuple(tapes.shape[1:]) == (3,) + tuple(self.shape) and tapes.shape[0] >= nsteps):
            raise ValueError("tapes must be a contiguous float64 CUDA tensor of shape (>= nsteps, 3) + grid state shape")

    def _dt_tensor(self, dt):
        if not torch.is_tensor(dt):
            dt = torch.full((self.shape[0],), float(dt), dtype=torch.float64, device=self.device)
        return dt

    def steps_record(self, U, tapes, nsteps, dt):
        """nsteps fixed-dt RK3 steps in place, recording step k into tapes[k]
        (one library call for all of them)."""
        self._check_state(U)
        self._check_tapes(tapes, nsteps)
        dt = self._dt_tensor(dt)
        self._sync_stream()
        check(lib().shk_rk3_steps_record(self.handle, _ptr(U), int(nsteps), _ptr(dt), _ptr(tapes)),
              self.handle, "rk3_steps_record")
        return U

    def steps_adjoint_tape(self, tapes, nsteps, dt, U_bar, param_bar=None):
        """Reverse of nsteps recorded steps (last first), in place on U_bar."""
        self._check_state(U_bar)
        self._check_tapes(tapes, nsteps)
        dt = self._dt_tensor(dt)
        self._sync_stream()
        check(lib().shk_rk3_steps_adjoint_tape(self.handle, _ptr(tapes), int(nsteps), _ptr(dt), _ptr(U_bar),
                                               _ptr(param_bar)), self.handle, "rk3_steps_adjoint_tape")
        return U_bar

    def set_params(self, gamma, inflow=None):
        """New gamma (and inflow primitive state) for the calls that follow."""
        arr = None if inflow is None else (ctypes.c_double * 4)(*[float(x) for x in inflow])
        check(lib().shk_set_params(self.handle, float(gamma), arr), self.handle, "set_params")
        self.desc.gamma = float(gamma)
        if inflow is not None:
            for k in range(4):
                self.desc.inflow_prim[k] = float(inflow[k])

    def replica(self):
        """A second grid with this one's description, immersed boundary,
        physical parameters and network, but its own workspace and HIP stream
        (default priority): fixed-step replays issued on it run concurrently
        with this grid's work.  Cached: rebuilt after a new level set or
        network, given this grid's gamma and inflow state on every call."""
        d = self.desc
        gamma, inflow = d.gamma, tuple(d.inflow_prim[k] for k in range(4))
        r = self._replica
        if r is not None and r[0] == self.version:
            g = r[1]
            if g.desc.gamma != gamma or tuple(g.desc.inflow_prim[k] for k in range(4)) != inflow:
                g.set_params(gamma, inflow)
            return g, r[2]
        args = dict(self._args, gamma=gamma, inflow=inflow)
        side = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(side):
            g = Grid(**args)
            if self.phi is not None:
                g.set_levelset(self.phi, self.wall)
            if self.net is not None:
                (g.set_flux_cnn if getattr(self.net, "kind", "mlp") == "cnn" else g.set_flux_net)(self.net)
        side.synchronize()
        self._replica = (self.version, g, side)
        return g, side

    def replay_buffers(self, nsteps):
        """Two tape buffers of nsteps recorded steps and a work state for
        replays on the replica, kept for later backward passes (no
        allocation, and no deferred frees across streams, per pass)."""
        shape = (nsteps, 3) + tuple(self.shape)
        b = getattr(self, "_replay_bufs", None)
        if b is None or tuple(b[0][0].shape) != shape:
            self._replay_bufs = None
            tapes = [torch.empty(shape, dtype=torch.float64, device=self.device) for _ in range(2)]
            self._replay_bufs = (tapes, torch.empty(self.shape, dtype=torch.float64, device=self.device))
        return self._replay_bufs

    def set_time(self, t0, t_end):
        self._sync_stream()
        check(lib().shk_set_time(self.handle, float(t0), float(t_end)), self.handle, "set_time")

    def get_time(self, b=0):
        t, done, steps = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
        self._sync_stream()
        check(lib().shk_get_time(self.handle, b, ctypes.byref(t), ctypes.byref(done), ctypes.byref(steps)),
              self.handle, "get_time")
        return t.value, bool(done.value), steps.value

    def advance(self, U, t_end, t0=0.0, max_steps=10 ** 7, chunk=64):
        """Automatic-step RK3 from t0 until every batch member reaches t_end
        (steps after the end are no-ops on the device).  Returns the device
        (t, steps) of batch member 0."""
        self.set_time(t0, t_end)
        issued = 0
        while issued < max_steps:
            n = min(chunk, max_steps - issued)
            for _ in range(n):
                self.step(U)
            issued += n
            done = all(self.get_time(b)[1] for b in range(self.shape[0]))
            if done:
                break
        t, _, steps = self.get_time(0)
        return t, steps

    def profile(self, enable=True):
        check(lib().shk_profile(self.handle, int(enable)), self.handle, "profile")

    def profile_read(self):
        """{kernel class: (total ms, launches)} for cfl, stage1..3, ghost_fill."""
        ms, cnt = (ctypes.c_double * 5)(), (ctypes.c_int * 5)()
        check(lib().shk_profile_read(self.handle, ms, cnt), self.handle, "profile_read")
        names = ("cfl", "stage1", "stage2", "stage3", "ghost_fill")
        return {n: (ms[k], cnt[k]) for k, n in enumerate(names)}

    def poll_faults(self):
        f, n = ctypes.c_uint32(), ctypes.c_uint64()
        self._sync_stream()
        check(lib().shk_poll_faults(self.handle, ctypes.byref(f), ctypes.byref(n)), self.handle, "poll_faults")
        return f.value, n.value


def normal_shock_state(mach, gamma=1.4, rho1=1.4, p1=1.0):
    """(rho2, u2, p2) behind a Mach-`mach` shock into gas at rest, with the
    derivatives with respect to mach and gamma (host computation in libshk)."""
    out, dM, dg = (ctypes.c_double * 3)(), (ctypes.c_double * 3)(), (ctypes.c_double * 3)()
    check(lib().shk_normal_shock_state(mach, gamma, rho1, p1, out, dM, dg), None, "normal_shock_state")
    return list(out), list(dM), list(dg)
