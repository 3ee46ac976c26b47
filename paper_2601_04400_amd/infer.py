"""Reverse learning of a physical parameter through the differentiable solver.

Section 3 recovers the ratio of specific heats from density fields on a
restricted part of the shock-cylinder domain: the solver runs from the
initial state with the current gamma, the loss compares the density with the
target data, and the gradient with respect to gamma -- through every RK3
step (the hand-written adjoint, `adjoint.rollout`) and through the initial
state's energy -- drives an optimizer with a warm-up-then-cosine learning-rate
schedule.  Here the target data come from this solver run with the target
gamma (no external data).

Domain: [0, 1.5] x [0, 1] (the lower half of the section 3 set-up up to
x = 1.5, cylinder of radius 0.25 centred on the top edge at x = 0.6), a
Mach-5 shock at x = 0.3 with the section 3 states, inflow of the left state on
the left, outflow on the right, reflective bottom and top (the top is the
symmetry plane through the cylinder's centre), slip wall.
"""
import math
import time

import numpy as np
import torch

from . import inputs
from .adjoint import rollout
from .solver import Grid


def warm_cosine(it, iters, peak, end, warm):
    """Learning rate: linear warm-up to `peak` over `warm` iterations, then a
    cosine decay to `end` at the last iteration."""
    if it < warm:
        return peak * (it + 1) / warm
    x = (it - warm) / max(1, iters - 1 - warm)
    return end + 0.5 * (peak - end) * (1.0 + math.cos(math.pi * x))


def restricted_cylinder(nx=128, ny=64):
    dom = (0.0, 1.5, 0.0, 1.0)
    post, pre = (7.0, 4.0, 0.0, 29.0), (1.4, 0.0, 0.0, 1.0)
    W = inputs.shock_prim(nx, ny, dom, 0.3, post, pre)
    phi = inputs.circle_phi(nx, ny, dom, (0.6, 1.0), 0.25)
    return dict(W=W, phi=phi, domain=dom, bc=(2, 0, 1, 1), inflow=post)


class GammaFit:
    """Fit gamma so that the density after `nsteps` fixed steps matches the
    target run's; loss = mean over fluid cells of (rho - rho_target)^2."""

    def __init__(self, nx=128, ny=64, gamma_target=2.0, nsteps=60, every=20, cfl_frac=0.6, device="cuda"):
        sc = restricted_cylinder(nx, ny)
        self.sc, self.nsteps, self.every = sc, nsteps, every
        self.g = Grid(nx, ny, domain=sc["domain"], bc=sc["bc"], inflow=sc["inflow"], gamma=gamma_target,
                      ibm=True, adjoint=True, device=device)
        self.g.set_levelset(torch.from_numpy(sc["phi"]), wall=0)
        self.fluid = torch.from_numpy(sc["phi"] >= 0.0).to(device)
        self.W0 = torch.from_numpy(sc["W"]).to(device)
        # one fixed step for every gamma tried: a fraction of the CFL step of
        # the stiffest initial state (largest gamma of the search range)
        d = torch.zeros(1, dtype=torch.float64, device=device)
        self.g.set_params(max(gamma_target, 2.5))
        U = self.g.prim_to_cons(self.W0)
        self.g.set_time(0.0, 1e30)
        self.g.step(U.clone(), dt_out=d)
        self.dt = torch.full((1,), cfl_frac * float(d.cpu()[0]), dtype=torch.float64, device=device)
        self.target = self.density_after(gamma_target).detach()

    def initial_state(self, gamma):
        # E = p/(gamma - 1) + rho |u|^2 / 2: the initial state depends on gamma
        self.g.set_params(gamma)
        return self.g.prim_to_cons(self.W0)

    def density_after(self, gamma):
        U = self.initial_state(gamma)
        for _ in range(self.nsteps):
            self.g.step(U, self.dt)
        return U[0, 0]

    def loss_and_grad(self, gamma):
        """Loss and dLoss/dgamma (adjoint through the steps plus the initial
        state's dependence on gamma)."""
        U0 = self.initial_state(gamma).requires_grad_(True)
        params = torch.tensor([[gamma, *self.sc["inflow"]]], dtype=torch.float64, device=U0.device,
                              requires_grad=True)
        U = rollout(self.g, U0, params, self.nsteps, self.dt, self.every)
        d = (U[0, 0] - self.target)[self.fluid]
        loss = (d * d).mean()
        loss.backward()
        W = self.W0
        dE_dgamma = -W[3] / (gamma - 1.0) ** 2
        g_init = float((U0.grad[0, 3] * dE_dgamma).sum())
        return float(loss.detach()), float(params.grad[0, 0]) + g_init

    def fit(self, gamma0=1.4, iters=100, peak=0.05, end=1e-4, warm=5, b1=0.8, b2=0.9, log=None):
        """Adam on gamma with the warm-cosine schedule; returns the history
        [(iteration, gamma, loss, lr)].  The moment decays are shorter than
        Adam's usual (0.9, 0.999): with one parameter and a loss that falls
        by orders of magnitude, a long second-moment memory makes the steps
        after an overshoot too small to come back."""
        gamma, m, v = gamma0, 0.0, 0.0
        eps = 1e-8
        hist = []
        for it in range(iters):
            loss, grad = self.loss_and_grad(gamma)
            lr = warm_cosine(it, iters, peak, end, warm)
            m = b1 * m + (1 - b1) * grad
            v = b2 * v + (1 - b2) * grad * grad
            mh, vh = m / (1 - b1 ** (it + 1)), v / (1 - b2 ** (it + 1))
            hist.append((it, gamma, loss, lr))
            if log is not None:
                log(f"iter {it} gamma {gamma:.6f} loss {loss:.6e} lr {lr:.3e}")
            gamma = max(1.05, gamma - lr * mh / (math.sqrt(vh) + eps))
        hist.append((iters, gamma, self.loss_and_grad(gamma)[0], 0.0))
        return hist


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="recover gamma by reverse-mode differentiation through the solver")
    ap.add_argument("--nx", type=int, default=128)
    ap.add_argument("--ny", type=int, default=64)
    ap.add_argument("--target", type=float, default=2.0)
    ap.add_argument("--start", type=float, default=1.4)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    t0 = time.perf_counter()
    fit = GammaFit(a.nx, a.ny, gamma_target=a.target, nsteps=a.steps)
    hist = fit.fit(gamma0=a.start, iters=a.iters, log=lambda s: print(s, flush=True))
    res = {"target": a.target, "start": a.start, "final_gamma": hist[-1][1], "final_loss": hist[-1][2],
           "seconds": round(time.perf_counter() - t0, 2), "history": hist}
    print(json.dumps({k: v for k, v in res.items() if k != "history"}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
