"""Seeded synthetic inputs shared by the GPU path and its tests.

This module only draws numbers and lays out fields: primitive states
(rho, u, v, p) as cell-centred planes, signed-distance level sets and seeds.
It holds none of the solver's arithmetic (no equation of state, no flux, no
reconstruction), so either side converts primitives to conservative variables
with its own code.

Layout: primitive planes [nvar][ny][nx], x fastest; nvar = 3 in 1D
(rho, u, p) and 4 in 2D (rho, u, v, p).
"""
import numpy as np


def centres(n, lo, hi):
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h


def sod_prim(n=200, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), xd=0.5):
    """Sod shock tube on [0,1] (section 3 initial data): point values at the
    cell centres, left state for x < xd."""
    x = centres(n, 0.0, 1.0)
    W = np.empty((3, 1, n))
    for k in range(3):
        W[k, 0] = np.where(x < xd, left[k], right[k])
    return W


def quadrant_states(seed_states=1, seed_perturb=0, rho=(0.5, 1.5), p=(0.3, 1.5), vel=(-0.5, 0.5),
                    perturb=0.05):
    """Four piecewise-constant quadrant states (rho, u, v, p), ordered
    (x<xc,y<yc), (x>=xc,y<yc), (x<xc,y>=yc), (x>=xc,y>=yc).  Base states are
    drawn from `seed_states`; every nonzero component is then scaled by
    (1 + U[-perturb, perturb]) drawn from `seed_perturb`."""
    g = np.random.default_rng(seed_states)
    S = np.empty((4, 4))
    S[:, 0] = g.uniform(*rho, size=4)
    S[:, 1] = g.uniform(*vel, size=4)
    S[:, 2] = g.uniform(*vel, size=4)
    S[:, 3] = g.uniform(*p, size=4)
    h = np.random.default_rng(seed_perturb)
    S = S * (1.0 + h.uniform(-perturb, perturb, size=S.shape))
    return S


def riemann2d_prim(nx=512, ny=512, states=None, split=(0.5, 0.5), domain=(0.0, 1.0, 0.0, 1.0)):
    """2D four-quadrant Riemann problem on `domain`, quadrants split at `split`."""
    if states is None:
        states = quadrant_states()
    x = centres(nx, domain[0], domain[1])
    y = centres(ny, domain[2], domain[3])
    right = (x >= split[0])[None, :]
    top = (y >= split[1])[:, None]
    q = right.astype(int) + 2 * top.astype(int)
    W = np.empty((4, ny, nx))
    for k in range(4):
        W[k] = states[q, k]
    return W


def random_prim(nx, ny, seed, rho=(0.3, 2.0), p=(0.2, 3.0), vel=(-1.5, 1.5), ndim=2):
    """Rough, cell-by-cell independent states: exercises every reconstruction
    and Riemann-solver branch (subsonic/supersonic, both contact signs)."""
    g = np.random.default_rng(seed)
    if ndim == 1:
        W = np.empty((3, 1, nx))
        W[0] = g.uniform(*rho, size=(1, nx))
        W[1] = g.uniform(*vel, size=(1, nx))
        W[2] = g.uniform(*p, size=(1, nx))
        return W
    W = np.empty((4, ny, nx))
    W[0] = g.uniform(*rho, size=(ny, nx))
    W[1] = g.uniform(*vel, size=(ny, nx))
    W[2] = g.uniform(*vel, size=(ny, nx))
    W[3] = g.uniform(*p, size=(ny, nx))
    return W


def smooth_prim(nx, ny, seed, amp=0.2, domain=(0.0, 1.0, 0.0, 1.0)):
    """Smooth periodic states: a few random Fourier modes on a uniform base."""
    g = np.random.default_rng(seed)
    x = centres(nx, domain[0], domain[1])[None, :]
    y = centres(ny, domain[2], domain[3])[:, None]
    Lx, Ly = domain[1] - domain[0], domain[3] - domain[2]
    base = (1.0, 0.3, -0.2, 1.0)
    W = np.empty((4, ny, nx))
    for k in range(4):
        f = np.full((ny, nx), base[k])
        for _ in range(3):
            kx, ky = g.integers(0, 3, size=2)
            ph = g.uniform(0, 2 * np.pi)
            f = f + amp * g.uniform(-1, 1) * np.sin(2 * np.pi * (kx * x / Lx + ky * y / Ly) + ph)
        W[k] = f
    return W


def circle_phi(nx, ny, domain, centre, radius):
    """Signed distance to a circle at the cell centres (negative inside)."""
    x = centres(nx, domain[0], domain[1])[None, :]
    y = centres(ny, domain[2], domain[3])[:, None]
    return np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2) - radius


def plane_phi(nx, ny, domain, y_wall):
    """Signed distance to the horizontal wall y = y_wall, solid below it."""
    y = centres(ny, domain[2], domain[3])[:, None]
    return np.broadcast_to(y - y_wall, (ny, nx)).copy()


def shock_prim(nx, ny, domain, xs, post, pre):
    """Planar shock: primitive state `post` (rho, u, v, p) for cell centres
    with x < xs, `pre` elsewhere."""
    x = centres(nx, domain[0], domain[1])[None, :]
    W = np.empty((4, ny, nx))
    for k in range(4):
        W[k] = np.where(np.broadcast_to(x < xs, (ny, nx)), post[k], pre[k])
    return W


def riemann_batch_states(seeds, rho=(0.1, 1.5), p=(0.1, 1.5), vel=(-1.0, 1.0)):
    """Quadrant states for a batch of random 2D Riemann problems, one seed each."""
    out = []
    for s in seeds:
        g = np.random.default_rng(int(s))
        S = np.empty((4, 4))
        S[:, 0] = g.uniform(*rho, size=4)
        S[:, 1] = g.uniform(*vel, size=4)
        S[:, 2] = g.uniform(*vel, size=4)
        S[:, 3] = g.uniform(*p, size=4)
        out.append(S)
    return out


def shock_cylinder(nx, ny, post, domain=(0.0, 2.0, 0.0, 1.0), centre=(0.3, 0.5), radius=0.1, xs=0.1,
                   pre=(1.4, 0.0, 0.0, 1.0)):
    """Planar normal shock at x = xs moving into gas at rest `pre` towards a
    circular cylinder.  `post` is the post-shock primitive state (rho, u, v, p)
    supplied by the caller.  Returns the primitive field, the level set and
    the boundary rules: inflow (post-shock) on the left, transmissive on the
    right, reflective walls at the bottom and top (section 3 setup)."""
    W = shock_prim(nx, ny, domain, xs, post, pre)
    phi = circle_phi(nx, ny, domain, centre, radius)
    return dict(W=W, phi=phi, domain=domain, bc=(2, 0, 1, 1), inflow=tuple(post))


def paper_shock_cylinder(nx, ny):
    """The section 3 shock-cylinder set-up: [-0.5, 4] x [0, 2], cylinder of
    radius 0.25 at (0.6, 1), initial state (7, 4, 0, 29) for x < 0.3 and
    (1.4, 0, 0, 1) elsewhere (a Mach-5 shock, eq. Sod_ST), inflow of the left
    state on the left, outflow on the right, reflective walls at the bottom
    and top, slip wall on the cylinder."""
    dom = (-0.5, 4.0, 0.0, 2.0)
    post, pre = (7.0, 4.0, 0.0, 29.0), (1.4, 0.0, 0.0, 1.0)
    W = shock_prim(nx, ny, dom, 0.3, post, pre)
    phi = circle_phi(nx, ny, dom, (0.6, 1.0), 0.25)
    return dict(W=W, phi=phi, domain=dom, bc=(2, 0, 1, 1), inflow=post)


def cylinder_viscosity(mach, reynolds=1000.0, diameter=0.2, rho1=1.4, a1=1.0):
    """Dynamic viscosity giving Reynolds number `reynolds` on the cylinder
    diameter with the pre-shock density and the shock speed M a1."""
    return rho1 * mach * a1 * diameter / reynolds
