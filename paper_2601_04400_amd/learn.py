"""Learned flux correction: parameters, training on solver-generated data,
and evaluation against the uncorrected solver.

Section 2 trains the neural flux on low-resolution runs against block-
averaged high-resolution data with an unrolled m-step mean-squared loss and
Adam, the gradients flowing back through the solver steps.  Here every piece
runs in the library's kernels: fine runs and the 4x4 restriction generate the
data, the coarse solver with the correction is unrolled m steps, the loss
terms seed the adjoint, shk_rk3_step_adjoint (with the network's reverse
pass) accumulates the parameter gradient, and shk_adam updates the FP32
master parameters, which shk_flux_net_pack turns into the bf16 device form.
The Python code only sequences calls and owns memory.
"""
import ctypes
import math
import time

import numpy as np
import torch

from . import inputs
from ._lib import check, lib
from .solver import Grid

NP = 10180
NW, NB = 11264, 208
# Fixed input normalisation from the sampling ranges of the training initial
# states (rho, p ~ U[0.1, 1.5]; u, v ~ U[-1, 1]) and the output scale.
DEFAULT_MEAN = (0.8, 0.0, 0.0, 0.8)
DEFAULT_STD = (0.4, 0.58, 0.58, 0.4)
DEFAULT_OUT_SCALE = 0.1


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def init_theta(seed=0, zero_output=False):
    """He-style random initial parameters in theta order (FP32, host)."""
    g = np.random.default_rng(seed)
    parts = []
    for nout, nin in ((64, 24), (64, 64), (64, 64), (4, 64)):
        W = g.normal(size=(nout, nin)) * math.sqrt(2.0 / nin)
        if nout == 4:
            W = W * (0.0 if zero_output else 0.1)
        parts += [W.ravel(), np.zeros(nout)]
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == NP
    return theta


class FluxNet:
    """FP32 master parameters with Adam state and the bf16 device form."""

    kind = "mlp"

    def __init__(self, theta, mean=DEFAULT_MEAN, inv_std=None, out_scale=DEFAULT_OUT_SCALE, device="cuda"):
        self.theta = torch.as_tensor(np.asarray(theta, dtype=np.float32)).to(device).contiguous()
        assert self.theta.numel() == NP
        self.mean = tuple(float(x) for x in mean)
        self.inv_std = tuple(float(x) for x in (inv_std or [1.0 / s for s in DEFAULT_STD]))
        self.out_scale = float(out_scale)
        self.w = torch.empty(NW, dtype=torch.int16, device=device)
        self.bias = torch.empty(NB, dtype=torch.float32, device=device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.step_count = 0
        self.pack()

    def pack(self):
        check(lib().shk_flux_net_pack(_p(self.theta), _p(self.w), _p(self.bias), _stream()), None, "flux_net_pack")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        check(lib().shk_adam(_p(self.theta), _p(self.grad), _p(self.m), _p(self.v), NP, lr, beta1, beta2, eps,
                             self.step_count, _stream()), None, "adam")
        self.pack()


CNN_NP, CNN_NW, CNN_NB = 6388, 18432, 64
# Fixed normalisation of the convolutional network's conservative inputs
# (rho, rho u_n, rho u_t, E) from the sampling ranges of the training states.
CNN_MEAN = (0.8, 0.0, 0.0, 2.2)
CNN_STD = (0.4, 0.6, 0.6, 1.2)


def init_cnn_theta(seed=0, zero_output=False):
    """He-style random parameters of the convolutional correction in theta
    order (W1, b1, W2, b2, W3, b3; W[out][3][3][in]), FP32, host."""
    g = np.random.default_rng(seed)
    parts = []
    for cout, cin in ((16, 4), (32, 16), (4, 32)):
        W = g.normal(size=(cout, 3, 3, cin)) * math.sqrt(2.0 / (9 * cin))
        if cout == 4:
            W = W * (0.0 if zero_output else 0.1)
        parts += [W.ravel(), np.zeros(cout)]
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == CNN_NP
    return theta


class FluxCnn:
    """The convolutional correction (section 2's 2D form): FP32 master
    parameters with Adam state and the bf16 device form."""

    kind = "cnn"

    def __init__(self, theta, mean=CNN_MEAN, inv_std=None, out_scale=DEFAULT_OUT_SCALE, device="cuda"):
        self.theta = torch.as_tensor(np.asarray(theta, dtype=np.float32)).to(device).contiguous()
        assert self.theta.numel() == CNN_NP
        self.mean = tuple(float(x) for x in mean)
        self.inv_std = tuple(float(x) for x in (inv_std or [1.0 / s for s in CNN_STD]))
        self.out_scale = float(out_scale)
        self.w = torch.empty(CNN_NW, dtype=torch.int16, device=device)
        self.bias = torch.empty(CNN_NB, dtype=torch.float32, device=device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.step_count = 0
        self.pack()

    def pack(self):
        check(lib().shk_flux_cnn_pack(_p(self.theta), _p(self.w), _p(self.bias), _stream()), None, "flux_cnn_pack")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        check(lib().shk_adam(_p(self.theta), _p(self.grad), _p(self.m), _p(self.v), CNN_NP, lr, beta1, beta2, eps,
                             self.step_count, _stream()), None, "adam")
        self.pack()


def net_kind(net):
    """desc.flux_net of a grid that can carry this network."""
    return 2 if getattr(net, "kind", "mlp") == "cnn" else 1


def attach(g, net):
    """Set (or clear, net None) the correction of grid g."""
    if g.desc.flux_net == 2:
        g.set_flux_cnn(net)
    else:
        g.set_flux_net(net)


def restrict(fine, factor):
    """Block average (device doubles [nb][nv][ny][nx]) by factor."""
    nb, nv, ny, nx = fine.shape
    out = torch.empty((nb, nv, ny // factor, nx // factor), dtype=torch.float64, device=fine.device)
    check(lib().shk_restrict(_p(fine), _p(out), nx, ny, factor, nv, nb, _stream()), None, "restrict")
    return out


def mse_accumulate(U, T, G, scale, loss, part):
    """loss[b] += ||U_b - T_b||^2 / N; G_b += scale * dloss/dU_b."""
    nb = U.shape[0]
    per = U[0].numel()
    check(lib().shk_mse(_p(U), _p(T), _p(G), float(scale), per, nb, _p(part), _p(loss), _stream()), None, "mse")


def riemann_batch(seeds, n, device="cuda", ny=None):
    """Primitive fields of random four-quadrant problems (one per seed) on
    n x ny cells of [0, 1] x [0, ny / n], quadrants split at the centre."""
    ny = ny or n
    dom = (0.0, 1.0, 0.0, ny / n)
    W = np.stack([inputs.riemann2d_prim(n, ny, states=S, split=(0.5, 0.5 * ny / n), domain=dom)
                  for S in inputs.riemann_batch_states(seeds)])
    return torch.from_numpy(W).to(device)


def sod_rows_prim(nx, rows):
    """Sod's shock tube along x on [0, 1] as `rows` identical rows of a 2D
    grid (primitive variables, batch of one)."""
    W1 = inputs.sod_prim(nx)  # (rho, u, p) x 1 x nx
    W = np.zeros((1, 4, rows, nx))
    W[0, 0], W[0, 1], W[0, 3] = W1[0, 0], W1[1, 0], W1[2, 0]
    return W


class Dataset:
    """Coarse (restricted) snapshots of fine runs: snaps[k] = d(U_fine(k dt_c)).

    case "riemann": random four-quadrant problems (one per seed) on nc x ny
    coarse cells (ny = nc unless given) against factor times finer,
    transmissive boundaries, coarse step cfl_frac x the CFL step of each
    initial coarse state.
    case "sod" (the 1D problem of section 3; seeds ignored): Sod's shock tube
    with nc cells against nc * factor, as `rows` identical rows of a 2D grid
    (transmissive boundaries make every y-face of a column see one stencil,
    so the y-flux differences -- with or without the correction -- vanish
    exactly and each row evolves as the 1D problem); coarse step t_end / nsnap.
    case "cylinder" (section 3's learned flux for the moving shock and the
    cylinder; seeds ignored): the restricted shock-cylinder set-up (Mach-5
    shock, slip wall) on nc x ny coarse cells (ny = nc / 2 unless given)
    against factor times finer, both with the immersed boundary, to t_end;
    the coarse step is t_end / nsnap with nsnap the least count whose step
    is at most cfl_frac x the CFL step of the initial coarse state (the
    nsnap argument is not used).
    """

    def __init__(self, seeds, nc=128, factor=4, nsnap=24, cfl_frac=0.5, device="cuda", keep_fine_ic=False,
                 case="riemann", rows=4, t_end=0.25, ny=None):
        self.case = case
        self.grid_kw = {}
        self.phi = None
        phi_f = None
        if case == "riemann":
            nb = len(seeds)
            nxc, nyc = nc, ny or nc
            W = riemann_batch(seeds, nc * factor, device, ny=nyc * factor)
            self.domain = (0.0, 1.0, 0.0, nyc / nc)
        elif case == "sod":
            nb, nxc, nyc = 1, nc, rows
            W = torch.from_numpy(sod_rows_prim(nc * factor, rows * factor)).to(device)
            self.domain = (0.0, 1.0, 0.0, rows / nc)
        elif case == "cylinder":
            from .infer import restricted_cylinder
            nb, nxc, nyc = 1, nc, ny or nc // 2
            fine = restricted_cylinder(nxc * factor, nyc * factor)
            W = torch.from_numpy(fine["W"]).to(device)
            self.domain = fine["domain"]
            self.grid_kw = dict(bc=fine["bc"], inflow=fine["inflow"], ibm=True)
            self.phi = torch.from_numpy(restricted_cylinder(nxc, nyc)["phi"])
            phi_f = torch.from_numpy(fine["phi"])
        else:
            raise ValueError("case must be 'riemann', 'sod' or 'cylinder'")
        self.nx, self.ny = nxc, nyc
        gf = Grid(nxc * factor, nyc * factor, nbatch=nb, domain=self.domain, device=device, **self.grid_kw)
        if phi_f is not None:
            gf.set_levelset(phi_f, wall=0)
        Uf = gf.prim_to_cons(W)
        self.fine_ic = Uf.clone() if keep_fine_ic else None
        self.factor = factor
        gc = self.grid(nb, device=device)
        U0c = restrict(Uf, factor)
        if case == "riemann":
            # coarse step: a fraction of the CFL step of the initial coarse state
            d = torch.zeros(nb, dtype=torch.float64, device=device)
            gc.set_time(0.0, 1e30)
            gc.step(U0c.clone(), dt_out=d)
            self.dt_c = (cfl_frac * d).contiguous()
        elif case == "cylinder":
            d = torch.zeros(1, dtype=torch.float64, device=device)
            gc.set_time(0.0, 1e30)
            gc.step(U0c.clone(), dt_out=d)
            nsnap = int(math.ceil(t_end / (cfl_frac * float(d[0]))))
            self.dt_c = torch.full((1,), t_end / nsnap, dtype=torch.float64, device=device)
        else:
            self.dt_c = torch.full((1,), t_end / nsnap, dtype=torch.float64, device=device)
        dt_f = (self.dt_c / factor).contiguous()
        snaps = [U0c]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsnap):
            for _ in range(factor):
                gf.step(Uf, dt_f)
            snaps.append(restrict(Uf, factor))
        torch.cuda.synchronize()
        self.fine_ms_per_coarse_step = (time.perf_counter() - t0) * 1e3 / max(nsnap, 1)
        self.snaps = torch.stack(snaps)  # [nsnap+1][nb][4][ny][nx]
        self.nc, self.nb, self.nsnap = nc, nb, nsnap
        torch.cuda.synchronize()

    def grid(self, nb=None, **kw):
        """A coarse grid of this data set's geometry (boundaries, and the body
        of the cylinder case)."""
        g = Grid(self.nx, self.ny, nbatch=nb or self.nb, domain=self.domain, **self.grid_kw, **kw)
        if self.phi is not None:
            g.set_levelset(self.phi, wall=0)
        return g


def train(net, data, iters=400, m=4, lr=1e-3, lr_late=1e-4, switch=None, log_every=50, log=None, last=None,
          stats=None):
    """Unrolled m-step training: loss = 1/m sum_s ||U^{n+s} - T^{n+s}||^2
    (mean over entries, summed over the batch), gradient by the adjoint.
    Windows cycle over the start snapshots 0 .. last - m (last: the final
    snapshot used, default the data set's last).  An iteration whose
    gradient is not finite (a rollout that left the physical states) makes
    no update; stats, if a dict, receives their count as "skipped"."""
    nb = data.nb
    last = data.nsnap if last is None else last
    g = data.grid(adjoint=True, flux_net=net_kind(net), device=data.snaps.device)
    attach(g, net)
    g.set_flux_net_grad(net.grad)
    part = torch.empty(nb * 256, dtype=torch.float64, device=data.snaps.device)
    tapes = torch.empty((m, 3) + tuple(g.shape), dtype=torch.float64, device=data.snaps.device)
    history = []
    skipped = 0
    switch = switch if switch is not None else int(0.875 * iters)
    for it in range(iters):
        k = it % (last - m + 1)
        U = data.snaps[k].clone()
        states = [None]
        for s in range(m):
            g.step_record(U, tapes[s], data.dt_c)
            states.append(U.clone())
        loss = torch.zeros(nb, dtype=torch.float64, device=U.device)
        net.grad.zero_()
        Ub = torch.zeros_like(U)
        for s in range(m, 0, -1):
            mse_accumulate(states[s], data.snaps[k + s], Ub, 1.0 / m, loss, part)
            g.step_adjoint_tape(tapes[s - 1], data.dt_c, Ub, None)
        if bool(torch.isfinite(net.grad).all()):
            net.adam(lr if it < switch else lr_late)
        else:
            skipped += 1  # a rollout left the physical states: no update from it
        L = float(loss.sum()) / m if (log is not None and (it % log_every == 0 or it == iters - 1)) else None
        if L is not None:
            history.append((it, k, L))
            log(f"iter {it} start {k} loss {L:.6e}")
    g.set_flux_net_grad(None)
    if skipped and log is not None:
        log(f"{skipped} of {iters} iterations skipped (non-finite gradient)")
    if stats is not None:
        stats["skipped"] = skipped
    return history


def dataset_loss(net, data, m=4, last=None):
    """Unrolled m-step loss summed over every start index 0 .. last - m of
    the data set (net = None: the uncorrected solver)."""
    nb = data.nb
    last = data.nsnap if last is None else last
    g = data.grid(flux_net=net_kind(net), device=data.snaps.device)
    attach(g, net)
    part = torch.empty(nb * 256, dtype=torch.float64, device=data.snaps.device)
    loss = torch.zeros(nb, dtype=torch.float64, device=data.snaps.device)
    for k in range(last - m + 1):
        U = data.snaps[k].clone()
        for s in range(1, m + 1):
            g.step(U, data.dt_c)
            mse_accumulate(U, data.snaps[k + s], None, 1.0, loss, part)
    return float(loss.sum()) / m


def evaluate(net, seeds, nc=128, factor=4, nsteps=24, cfl_frac=0.5, device="cuda", ny=None):
    """Held-out error of the coarse solver with and without the correction
    against the restricted fine solution after nsteps coarse steps (mean
    squared error over all conserved entries -- the training metric -- and
    mean absolute error), with the time per coarse step of each and of the
    finer solvers (half spacing, and the fine reference itself)."""
    data = Dataset(seeds, nc=nc, factor=factor, nsnap=nsteps, cfl_frac=cfl_frac, device=device,
                   keep_fine_ic=True, ny=ny)
    target = data.snaps[-1]

    def errs(U):
        d = U - target
        return {"mse": float((d * d).mean()), "l1_error": float(d.abs().mean())}
    out = {f"plain_{nc * factor}": {"mse": 0.0, "l1_error": 0.0, "ms_per_step": data.fine_ms_per_coarse_step,
                                    "note": "the reference itself (restricted fine solution)"}}
    if factor >= 4:
        nm = nc * 2
        gm = Grid(nm, nm * data.ny // nc, nbatch=len(seeds), domain=data.domain, device=device)
        Um = restrict(data.fine_ic, factor // 2)
        dtm = (data.dt_c / 2).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2 * nsteps):
            gm.step(Um, dtm)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"plain_{nm}"] = dict(errs(restrict(Um, 2)), ms_per_step=el * 1e3 / nsteps)
    marks = sorted({max(1, nsteps // 3), max(1, 2 * nsteps // 3), nsteps})
    for name, use in (("plain", False), ("learned", True)):
        g = data.grid(len(seeds), flux_net=net_kind(net), device=device)
        attach(g, net if use else None)
        U = data.snaps[0].clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            g.step(U, data.dt_c)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # error along the rollout (a second, untimed pass)
        U = data.snaps[0].clone()
        horizon = {}
        for s in range(1, nsteps + 1):
            g.step(U, data.dt_c)
            if s in marks:
                d = U - data.snaps[s]
                horizon[s] = float((d * d).mean())
        out[f"{name}_{nc}"] = dict(errs(U), ms_per_step=el * 1e3 / nsteps, mse_after_steps=horizon)
    out["learned"] = out[f"learned_{nc}"]
    out["plain"] = out[f"plain_{nc}"]
    return out


def evaluate_sod(net, data, marks):
    """Error of the coarse Sod solver with and without the correction against
    the restricted fine solution at the given snapshot indices (mean squared
    error over the conserved entries and mean absolute density error), with
    the time per coarse step."""
    out = {}
    for name, use in (("plain", False), ("learned", True)):
        g = data.grid(flux_net=net_kind(net), device=data.snaps.device)
        attach(g, net if use else None)
        U = data.snaps[0].clone()
        errs = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(1, max(marks) + 1):
            g.step(U, data.dt_c)
            if s in marks:
                d = U - data.snaps[s]
                errs[s] = {"mse": float((d * d).mean()), "rho_l1": float(d[:, 0].abs().mean())}
        torch.cuda.synchronize()
        out[name] = {"errors": errs, "ms_per_step": (time.perf_counter() - t0) * 1e3 / max(marks)}
    return out


def cnn_norm_from(data, centre=None):
    """Input normalisation of the convolutional correction from a data set's
    coarse snapshots: inverse standard deviation of rho and E, and of the two
    momenta taken together (the normal and tangential channels of x- and
    y-faces share the statistics, as the faces share the network); centred
    on the snapshots' mean, or on `centre` (conservative rho, m_n, m_t, E)
    if given.  The zero padding of the 3x3 layers at non-periodic edges
    stands for the centre state."""
    S = data.snaps  # [snapshot][member][4][ny][nx]
    r, E = S[:, :, 0], S[:, :, 3]
    m = torch.cat([S[:, :, 1].flatten(), S[:, :, 2].flatten()])
    mean = (float(r.mean()), float(m.mean()), float(m.mean()), float(E.mean()))
    if centre is not None:
        mean = tuple(float(x) for x in centre)
    std = (float(r.std()), float(m.std()), float(m.std()), float(E.std()))
    return mean, [1.0 / x for x in std]


def evaluate_cylinder(net, data, times=(0.18, 0.2), x_line=0.29, gamma=1.4):
    """Error of the coarse cylinder run with and without the correction
    against the restricted fine solution at the given times: mean squared
    error over the coarse fluid cells, and the density, velocity and pressure
    profiles along the column through x = x_line (mean absolute error over
    its fluid cells, relative to the reference profile's largest magnitude),
    with the time per coarse step."""
    dt = float(data.dt_c[0])
    marks = {t: min(data.nsnap, int(round(t / dt))) for t in times}
    g0 = data.grid(device=data.snaps.device)
    fluid = g0.classes() == 0
    x0, x1 = data.domain[0], data.domain[1]
    col = min(data.nx - 1, int((x_line - x0) / ((x1 - x0) / data.nx)))
    cf = fluid[:, col]

    def prim(U):
        r = U[0]
        u, v = U[1] / r, U[2] / r
        return {"rho": r, "u": u, "v": v, "p": (gamma - 1.0) * (U[3] - 0.5 * r * (u * u + v * v))}
    out = {"line_x": x0 + (col + 0.5) * (x1 - x0) / data.nx, "steps": marks, "dt": dt}
    for name, use in (("plain", False), ("learned", True)):
        g = data.grid(flux_net=net_kind(net), device=data.snaps.device)
        attach(g, net if use else None)
        g.step(data.snaps[0].clone(), data.dt_c)  # untimed: first-use costs
        U = data.snaps[0].clone()
        res = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(1, max(marks.values()) + 1):
            g.step(U, data.dt_c)
            for t, k in marks.items():
                if s == k:
                    T = data.snaps[k][0]
                    d = U[0] - T
                    pu, pt = prim(U[0][:, :, col]), prim(T[:, :, col])
                    line = {}
                    for q in pu:
                        ref = pt[q][cf]
                        line[q] = float((pu[q][cf] - ref).abs().mean() / ref.abs().max())
                    res[str(t)] = {"mse_fluid": float((d[:, fluid] ** 2).mean()), "line_rel_l1": line}
        torch.cuda.synchronize()
        out[name] = {"errors": res, "ms_per_step": (time.perf_counter() - t0) * 1e3 / max(marks.values())}
    return out


def main_cylinder(a):
    """Section 3's learned flux for the moving shock and the cylinder: the
    convolutional correction on 128 x 64 against 256 x 128 restricted 2 x 2,
    trained up to t = 0.2 with the paper's rates (1e-4, then 1e-5), and the
    density, velocity and pressure along x = 0.29 at t = 0.18 and 0.2."""
    import json
    t0 = time.perf_counter()
    data = Dataset(None, nc=a.nc_cyl, factor=2, case="cylinder", t_end=0.2, cfl_frac=a.cfl_frac_cyl)
    print(f"data: cylinder {data.nx}x{data.ny} vs {2 * data.nx}x{2 * data.ny}, {data.nsnap} coarse steps "
          f"to t = 0.2, {time.perf_counter() - t0:.1f} s", flush=True)
    centre = None
    if a.norm_cyl == "ambient":
        from .infer import PRE
        gm1 = 1.4 - 1.0  # the set-up runs at the grids' default gamma
        r, u, v, p = PRE
        centre = (r, r * u, r * v, p / gm1 + 0.5 * r * (u * u + v * v))
    mean, inv = cnn_norm_from(data, centre)
    net = FluxCnn(init_cnn_theta(0, zero_output=True), mean, inv, out_scale=a.out_scale_cyl)
    before = dataset_loss(net, data, m=a.m_cyl)
    t1 = time.perf_counter()
    stats = {}
    hist = train(net, data, iters=a.iters_cyl, m=a.m_cyl, lr=a.lr_cyl, lr_late=a.lr_late_cyl,
                 switch=a.switch_cyl, log_every=250, log=lambda s: print(s, flush=True), stats=stats)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    after = dataset_loss(net, data, m=a.m_cyl)
    ev = evaluate_cylinder(net, data)
    res = {"case": "cylinder", "coarse": [data.nx, data.ny], "fine": [2 * data.nx, 2 * data.ny],
           "coarse_steps": data.nsnap, "unroll_m": a.m_cyl, "iters": a.iters_cyl, "lr": [a.lr_cyl, a.lr_late_cyl],
           "lr_switch": a.switch_cyl, "norm": a.norm_cyl, "norm_mean": mean, "norm_inv_std": inv, "out_scale": a.out_scale_cyl,
           "train_seconds": round(train_s, 2), "train_ms_per_iter": round(train_s * 1e3 / a.iters_cyl, 3),
           "iters_skipped": stats["skipped"], "training_loss_before": before, "training_loss_after": after,
           "eval": ev, "history": hist}
    print(json.dumps({k: v for k, v in res.items() if k != "history"}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


def main_sod(a):
    """Section 3's 1D learned flux: Sod's shock tube with N = 500 cells
    against N = 1000 restricted, trained on t <= 0.2 and evaluated to 0.25."""
    import json
    t0 = time.perf_counter()
    n_eval = a.nsnap_sod
    n_train = int(round(n_eval * 0.2 / 0.25))
    data = Dataset(None, nc=a.nc_sod, factor=2, nsnap=n_eval, case="sod", rows=4, t_end=0.25)
    print(f"data: Sod {a.nc_sod} vs {2 * a.nc_sod} cells, {n_eval} coarse steps to t = 0.25, "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    net = FluxNet(init_theta(0, zero_output=True))
    before = dataset_loss(net, data, m=a.m_sod, last=n_train)
    t1 = time.perf_counter()
    hist = train(net, data, iters=a.iters_sod, m=a.m_sod, lr=a.lr, lr_late=a.lr_late, log_every=100,
                 log=lambda s: print(s, flush=True), last=n_train)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    after = dataset_loss(net, data, m=a.m_sod, last=n_train)
    ev = evaluate_sod(net, data, [n_train // 2, n_train, n_eval])
    res = {"case": "sod", "coarse": a.nc_sod, "fine": 2 * a.nc_sod, "steps_train": n_train, "steps_eval": n_eval,
           "unroll_m": a.m_sod, "iters": a.iters_sod, "train_seconds": round(train_s, 2),
           "train_ms_per_iter": round(train_s * 1e3 / a.iters_sod, 3), "training_loss_before": before,
           "training_loss_after": after, "eval": ev, "history": hist}
    print(json.dumps({k: v for k, v in res.items() if k != "history"}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train and evaluate the learned flux correction")
    ap.add_argument("--train-seeds", type=int, default=64)
    ap.add_argument("--heldout", type=int, default=16)
    ap.add_argument("--nc", type=int, default=128)
    ap.add_argument("--factor", type=int, default=4)
    ap.add_argument("--nsnap", type=int, default=24)
    ap.add_argument("--m", type=int, default=16)
    ap.add_argument("--iters", type=int, default=400)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-late", type=float, default=1e-4)
    ap.add_argument("--out", default=None)
    ap.add_argument("--case", choices=("riemann", "sod", "cylinder"), default="riemann")
    ap.add_argument("--net", choices=("mlp", "cnn"), default="mlp")
    ap.add_argument("--ny", type=int, default=None, help="coarse rows (default: nc)")
    ap.add_argument("--nc-sod", type=int, default=500)
    ap.add_argument("--nsnap-sod", type=int, default=625)
    ap.add_argument("--m-sod", type=int, default=64)
    ap.add_argument("--iters-sod", type=int, default=1000)
    ap.add_argument("--nc-cyl", type=int, default=128)
    ap.add_argument("--cfl-frac-cyl", type=float, default=0.5)
    ap.add_argument("--m-cyl", type=int, default=32)
    ap.add_argument("--iters-cyl", type=int, default=5000)
    ap.add_argument("--switch-cyl", type=int, default=3500)
    ap.add_argument("--lr-cyl", type=float, default=1e-4)
    ap.add_argument("--lr-late-cyl", type=float, default=1e-5)
    ap.add_argument("--out-scale-cyl", type=float, default=0.1)
    ap.add_argument("--norm-cyl", choices=("data", "ambient"), default="ambient",
                    help="centre of the input normalisation: the data mean or the gas at rest ahead of the shock")
    a = ap.parse_args()
    if a.case == "sod":
        return main_sod(a)
    if a.case == "cylinder":
        return main_cylinder(a)
    t0 = time.perf_counter()
    data = Dataset(list(range(a.train_seeds)), nc=a.nc, factor=a.factor, nsnap=a.nsnap, ny=a.ny)
    print(f"data: {a.train_seeds} problems, {a.nsnap} coarse snapshots, {time.perf_counter() - t0:.1f} s", flush=True)
    net = FluxCnn(init_cnn_theta(0, zero_output=True)) if a.net == "cnn" else FluxNet(init_theta(0, zero_output=True))
    before = dataset_loss(net, data, m=a.m)
    t1 = time.perf_counter()
    hist = train(net, data, iters=a.iters, m=a.m, lr=a.lr, lr_late=a.lr_late, log_every=50,
                 log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    after = dataset_loss(net, data, m=a.m)
    ev = evaluate(net, list(range(1000, 1000 + a.heldout)), nc=a.nc, factor=a.factor, nsteps=a.nsnap, ny=a.ny)
    res = {"net": a.net, "train_problems": a.train_seeds, "heldout_problems": a.heldout, "coarse": a.nc,
           "coarse_rows": data.ny, "fine": a.nc * a.factor, "unroll_m": a.m, "iters": a.iters, "train_seconds": round(train_s, 2),
           "train_ms_per_iter": round(train_s * 1e3 / a.iters, 3), "training_loss_before": before,
           "training_loss_after": after, "heldout": ev, "history": hist}
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
