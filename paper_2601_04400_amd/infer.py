"""Reverse learning of physical parameters through the differentiable solver.

Section 3 infers physical parameters from flow-field data by differentiating
the whole solver run: the solver runs from the initial state with the current
parameter, the loss compares the density with the target data, and the
gradient -- through every RK3 step (the hand-written adjoint,
`adjoint.rollout`) and through the initial and boundary states' dependence on
the parameter -- drives Adam.  The target data come from this solver run with
the target parameter (no external data).

Cases:

* gamma on the restricted shock-cylinder domain: [0, 1.5] x [0, 1] (the lower
  half of the section 3 set-up up to x = 1.5, cylinder of radius 0.25
  centred on the top edge at x = 0.6), a Mach-5 shock at x = 0.3 with the
  section 3 states, inflow of the post-shock state on the left, outflow on
  the right, reflective bottom and top (the top is the symmetry plane
  through the cylinder's centre), slip wall; warm-up-then-cosine learning
  rate;
* gamma from Sod shock-tube data (section 3, constant learning rate 0.1):
  the tube runs along x as identical rows of a 2D grid with transmissive
  boundaries -- every y-face of a column then sees one stencil, the y-flux
  differences vanish exactly and each row evolves as the 1D problem;
* the shock Mach number on the restricted shock-cylinder domain: the
  post-shock state (initial data behind the shock and the inflow boundary)
  follows from the normal-shock relations, so the gradient adds the
  adjoint of the initial state over the post-shock cells and the inflow
  partials, both chained through d(post-shock state)/dMach.
"""
import math
import time

import numpy as np
import torch

from . import inputs
from .adjoint import rollout
from .solver import Grid, normal_shock_state

PRE = (1.4, 0.0, 0.0, 1.0)  # gas at rest ahead of the section 3 shock


def warm_cosine(it, iters, peak, end, warm):
    """Learning rate: linear warm-up to `peak` over `warm` iterations, then a
    cosine decay to `end` at the last iteration."""
    if it < warm:
        return peak * (it + 1) / warm
    x = (it - warm) / max(1, iters - 1 - warm)
    return end + 0.5 * (peak - end) * (1.0 + math.cos(math.pi * x))


def restricted_cylinder(nx=128, ny=64, post=(7.0, 4.0, 0.0, 29.0)):
    dom = (0.0, 1.5, 0.0, 1.0)
    W = inputs.shock_prim(nx, ny, dom, 0.3, post, PRE)
    phi = inputs.circle_phi(nx, ny, dom, (0.6, 1.0), 0.25)
    return dict(W=W, phi=phi, domain=dom, bc=(2, 0, 1, 1), inflow=post)


def sod_rows(nx=200, ny=4):
    """Sod's shock tube on [0, 1] along x as ny identical rows (dy = dx)."""
    W1 = inputs.sod_prim(nx)  # (rho, u, p) x 1 x nx
    W = np.zeros((4, ny, nx))
    W[0], W[1], W[3] = W1[0, 0], W1[1, 0], W1[2, 0]
    return dict(W=W, phi=None, domain=(0.0, 1.0, 0.0, ny / nx), bc=(0, 0, 0, 0), inflow=(1.0, 0.0, 0.0, 1.0))


class ReverseFit:
    """Adam on one scalar parameter p through the differentiable solver;
    loss = mean over fluid cells of (rho - rho_target)^2 after nsteps fixed
    steps.  Subclasses give initial_state(p) (which also sets the grid's
    physical parameters) and chain(p, U0_bar, param_bar) = the part of dLoss/dp
    that enters through the initial state and the solver parameters."""

    lower, upper = 1.05, None  # the search range (the fixed step is stable up to upper)

    def _setup(self, sc, gamma, nsteps, every, dt, device):
        self.sc, self.nsteps, self.every = sc, nsteps, every
        nx, ny = sc["W"].shape[2], sc["W"].shape[1]
        self.g = Grid(nx, ny, domain=sc["domain"], bc=sc["bc"], inflow=sc["inflow"], gamma=gamma,
                      ibm=sc["phi"] is not None, adjoint=True, device=device)
        if sc["phi"] is not None:
            self.g.set_levelset(torch.from_numpy(sc["phi"]), wall=0)
            self.fluid = torch.from_numpy(sc["phi"] >= 0.0).to(device)
        else:
            self.fluid = torch.ones((ny, nx), dtype=torch.bool, device=device)
        self.W0 = torch.from_numpy(sc["W"]).to(device)
        self.dt = torch.full((1,), float(dt), dtype=torch.float64, device=device)

    def cfl_step(self, U):
        """The automatic (CFL 0.5) step of state U."""
        d = torch.zeros(1, dtype=torch.float64, device=U.device)
        self.g.set_time(0.0, 1e30)
        self.g.step(U.clone(), dt_out=d)
        return float(d.cpu()[0])

    def density_after(self, p):
        U = self.initial_state(p)
        for _ in range(self.nsteps):
            self.g.step(U, self.dt)
        return U[0, 0]

    def loss(self, p):
        d = (self.density_after(p) - self.target)[self.fluid]
        return float((d * d).mean())

    def loss_and_grad(self, p):
        """Loss and dLoss/dp: the adjoint through the steps plus the initial
        and boundary states' dependence on p."""
        U0 = self.initial_state(p).requires_grad_(True)
        d = self.g.desc
        params = torch.tensor([[d.gamma, *[d.inflow_prim[k] for k in range(4)]]], dtype=torch.float64,
                              device=U0.device, requires_grad=True)
        U = rollout(self.g, U0, params, self.nsteps, self.dt, self.every)
        r = (U[0, 0] - self.target)[self.fluid]
        loss = (r * r).mean()
        loss.backward()
        return float(loss.detach()), self.chain(p, U0.grad[0], params.grad[0])

    def fit(self, p0, iters=100, peak=0.05, end=1e-4, warm=5, b1=0.8, b2=0.9, lr=None, log=None):
        """Adam on p; the learning rate is `lr` if given, else the warm-cosine
        schedule (peak, end, warm).  Returns [(iteration, p, loss, lr)], the
        last entry the final parameter and its loss."""
        p, m, v = p0, 0.0, 0.0
        eps = 1e-8
        hist = []
        for it in range(iters):
            loss, grad = self.loss_and_grad(p)
            rate = lr if lr is not None else warm_cosine(it, iters, peak, end, warm)
            m = b1 * m + (1 - b1) * grad
            v = b2 * v + (1 - b2) * grad * grad
            mh, vh = m / (1 - b1 ** (it + 1)), v / (1 - b2 ** (it + 1))
            hist.append((it, p, loss, rate))
            if log is not None:
                log(f"iter {it} {self.name} {p:.6f} loss {loss:.6e} lr {rate:.3e}")
            p = min(self.upper, max(self.lower, p - rate * mh / (math.sqrt(vh) + eps)))
        hist.append((iters, p, self.loss_and_grad(p)[0], 0.0))
        return hist


class GammaFit(ReverseFit):
    """gamma from density data: case "cylinder" (restricted shock-cylinder,
    nx x ny, nsteps fixed steps of cfl_frac x the CFL step of the stiffest
    initial state, gamma 2.5) or "sod" (Sod rows, nsteps steps to t_end)."""

    name = "gamma"

    def __init__(self, nx=128, ny=64, gamma_target=2.0, nsteps=60, every=20, cfl_frac=0.6, case="cylinder",
                 t_end=0.2, device="cuda"):
        self.upper = max(gamma_target, 2.5)
        if case == "cylinder":
            sc = restricted_cylinder(nx, ny)
            self._setup(sc, gamma_target, nsteps, every, 1.0, device)
            self.dt.fill_(cfl_frac * self.cfl_step(self.initial_state(self.upper)))
        elif case == "sod":
            # fixed step landing on t_end; nsteps must keep the CFL number
            # below 0.5 for every gamma tried (200 cells: 250 steps to t = 0.2
            # give CFL <= 0.4 for wave speeds up to 2.5)
            self._setup(sod_rows(nx, ny), gamma_target, nsteps, every, t_end / nsteps, device)
        else:
            raise ValueError("case must be 'cylinder' or 'sod'")
        self.case = case
        self.target = self.density_after(gamma_target).detach()

    def initial_state(self, gamma):
        # E = p/(gamma - 1) + rho |u|^2 / 2: the initial state depends on gamma
        self.g.set_params(gamma)
        return self.g.prim_to_cons(self.W0)

    def chain(self, gamma, U0_bar, pb):
        # the initial state's dependence on gamma (through its energy), by the
        # library's reverse mode of the primitive-to-conservative conversion
        g_bar = self.g.param_bar()
        self.g.prim_to_cons_vjp(self.W0, U0_bar, None, g_bar)
        return float(pb[0]) + float(g_bar[0, 0])


class MachFit(ReverseFit):
    """The shock Mach number on the restricted shock-cylinder domain (gamma
    fixed): post-shock state from the normal-shock relations into PRE; the
    fixed step is cfl_frac x the CFL step of the Mach-6 initial state."""

    name = "mach"

    def __init__(self, nx=128, ny=64, mach_target=5.0, gamma=1.4, nsteps=60, every=20, cfl_frac=0.6,
                 device="cuda"):
        self.gamma = gamma
        sc = restricted_cylinder(nx, ny, self.post(mach_target)[0])
        self._setup(sc, gamma, nsteps, every, 1.0, device)
        self.x_post = torch.from_numpy(inputs.centres(nx, *sc["domain"][:2]) < 0.3).to(device)
        self.upper = max(mach_target, 6.0)
        self.dt.fill_(cfl_frac * self.cfl_step(self.initial_state(self.upper)))
        self.target = self.density_after(mach_target).detach()

    def post(self, mach):
        w, dM, _ = normal_shock_state(mach, self.gamma, PRE[0], PRE[3])
        return (w[0], w[1], 0.0, w[2]), dM

    def initial_state(self, mach):
        post, _ = self.post(mach)
        self.g.set_params(self.gamma, post)
        W = self.W0.clone()
        for k in range(4):
            W[k][:, self.x_post] = post[k]
        self.W = W
        return self.g.prim_to_cons(W)

    def chain(self, mach, U0_bar, pb):
        # primitive adjoint of the initial state (the library's reverse mode
        # of the conversion), summed over the post-shock cells, and the
        # inflow partials: both times d(post-shock state)/dMach
        _, (dr, du, dp) = self.post(mach)
        W_bar = torch.zeros_like(self.W)
        self.g.prim_to_cons_vjp(self.W, U0_bar, W_bar, None)
        post_bar = [float(W_bar[k][:, self.x_post].sum()) for k in range(4)]
        return ((post_bar[0] + float(pb[1])) * dr + (post_bar[1] + float(pb[2])) * du
                + (post_bar[3] + float(pb[4])) * dp)


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="recover a physical parameter by reverse-mode differentiation "
                                             "through the solver")
    ap.add_argument("--case", choices=("cylinder-gamma", "sod-gamma", "cylinder-mach"), default="cylinder-gamma")
    ap.add_argument("--nx", type=int, default=None)
    ap.add_argument("--ny", type=int, default=None)
    ap.add_argument("--target", type=float, default=None)
    ap.add_argument("--start", type=float, default=None)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    t0 = time.perf_counter()
    if a.case == "cylinder-gamma":
        fit = GammaFit(a.nx or 128, a.ny or 64, gamma_target=a.target or 2.0, nsteps=a.steps or 60)
        kw = dict(iters=a.iters or 100)
        start = a.start or 1.4
    elif a.case == "sod-gamma":
        fit = GammaFit(a.nx or 200, a.ny or 4, gamma_target=a.target or 1.4, nsteps=a.steps or 250, every=25,
                       case="sod")
        kw = dict(iters=a.iters or 100, lr=0.1, b1=0.9, b2=0.999)
        start = a.start or 1.2
    else:
        fit = MachFit(a.nx or 128, a.ny or 64, mach_target=a.target or 5.0, nsteps=a.steps or 60)
        kw = dict(iters=a.iters or 100, peak=0.2, end=1e-4)
        start = a.start or 4.0
    hist = fit.fit(start, log=lambda s: print(s, flush=True), **kw)
    res = {"case": a.case, "target": fit_target(a, fit), "start": start, "final": hist[-1][1],
           "final_loss": hist[-1][2], "seconds": round(time.perf_counter() - t0, 2), "history": hist}
    print(json.dumps({k: v for k, v in res.items() if k != "history"}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


def fit_target(a, fit):
    if a.target is not None:
        return a.target
    return {"cylinder-gamma": 2.0, "sod-gamma": 1.4, "cylinder-mach": 5.0}[a.case]


if __name__ == "__main__":
    main()
