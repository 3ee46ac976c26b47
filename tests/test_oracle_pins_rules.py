"""Pins of the oracle parts that drive the automatic time step, the
Navier-Stokes terms, the wall and boundary rules, the per-face network and the
training pieces (restriction, unrolled loss, Adam).

As in test_oracle_pins.py each test checks the oracle against something other
than itself: closed forms, an independent evaluation, or an equivalent
problem (a grid extended by the ghost cells it should see).
"""
import math

import numpy as np
import pytest

from paper_2601_04400_amd import inputs

G = 1.4


def prim_field(nx, ny, W):
    out = np.empty((4, ny, nx))
    for k in range(4):
        out[k] = W[k]
    return out


# ------------------------------------------------------------- time step
def test_cfl_dt_sod_closed_form(orc):
    """Sod at t = 0 (section 3): u = 0 everywhere, the fastest cell is the
    left state with a = sqrt(1.4), so dt = CFL dx / sqrt(1.4)."""
    n = 200
    c = orc.config(ndim=1, nx=n, cfl=0.5)
    U = orc.prim_to_cons(c, inputs.sod_prim(n))
    dt = orc.cfl_dt(c, U)
    assert abs(dt - 0.5 * (1.0 / n) / math.sqrt(1.4)) <= 1e-15


def test_cfl_dt_two_dimensional_sum_form(orc):
    """A uniform 2D state on an anisotropic grid: dt = CFL / ((|u|+a)/dx +
    (|v|+a)/dy) -- the sum of the two directions, not their maximum, and each
    velocity component divided by its own spacing."""
    nx, ny = 20, 12
    c = orc.config(nx=nx, ny=ny, x1=2.0, y1=0.3, cfl=0.7)
    rho, u, v, p = 0.8, -1.3, 0.45, 2.1
    U = orc.prim_to_cons(c, prim_field(nx, ny, (rho, u, v, p)))
    a = math.sqrt(G * p / rho)
    dx, dy = 2.0 / nx, 0.3 / ny
    ref = 0.7 / ((abs(u) + a) / dx + (abs(v) + a) / dy)
    assert abs(orc.cfl_dt(c, U) - ref) <= 1e-14 * ref
    # the maximum over cells: one fast cell sets the step
    W = prim_field(nx, ny, (rho, u, v, p))
    W[1, 5, 7] = 4.0
    ref2 = 0.7 / ((4.0 + a) / dx + (abs(v) + a) / dy)
    assert abs(orc.cfl_dt(c, orc.prim_to_cons(c, W)) - ref2) <= 1e-14 * ref2


@pytest.mark.parametrize("prandtl", [0.72, 2.0])
def test_cfl_dt_viscous_limit(orc, prandtl):
    """Navier-Stokes: dt <= 0.25 h^2 rho_min / (mu max(4/3, gamma/Pr)) with
    h = min(dx, dy); Pr = 0.72 takes gamma/Pr, Pr = 2 takes 4/3.  The
    viscosity is large enough for this limit to bind."""
    nx, ny, mu = 16, 10, 0.5
    c = orc.config(nx=nx, ny=ny, x1=1.0, y1=0.5, viscous=1, mu=mu, prandtl=prandtl)
    W = prim_field(nx, ny, (1.0, 0.2, -0.1, 1.0))
    W[0, 3, 4] = 0.37  # the minimum density sets the limit
    U = orc.prim_to_cons(c, W)
    h = min(1.0 / nx, 0.5 / ny)
    ref = 0.25 * h * h * 0.37 / (mu * max(4.0 / 3.0, G / prandtl))
    dt = orc.cfl_dt(c, U)
    assert abs(dt - ref) <= 1e-14 * ref
    # with a tiny viscosity the convective limit binds again
    c2 = orc.config(nx=nx, ny=ny, x1=1.0, y1=0.5, viscous=1, mu=1e-9, prandtl=prandtl)
    a = np.sqrt(G * 1.0 / W[0])
    s = (np.abs(W[1]) + a) / (1.0 / nx) + (np.abs(W[2]) + a) / (0.5 / ny)
    ref2 = 0.5 / np.max(s)
    assert abs(orc.cfl_dt(c2, U) - ref2) <= 1e-14 * ref2


def test_cfl_dt_ignores_solid_and_ghost_cells(orc):
    """Only fluid cells enter the step: a wild state inside the body leaves
    it equal to the uniform fluid's closed form."""
    nx, ny = 40, 30
    dom = (0.0, 1.0, 0.0, 0.75)
    phi = inputs.circle_phi(nx, ny, dom, (0.5, 0.4), 0.17)
    c = orc.config(nx=nx, ny=ny, y1=0.75)
    W = prim_field(nx, ny, (1.1, 0.3, 0.2, 0.9))
    solid = phi < 0
    W[1][solid] = 40.0
    W[0][solid] = 0.01
    U = orc.prim_to_cons(c, W)
    a = math.sqrt(G * 0.9 / 1.1)
    ref = 0.5 / ((0.3 + a) * nx + (0.2 + a) * (ny / 0.75))
    assert abs(orc.cfl_dt(c, U, phi=phi) - ref) <= 1e-14 * ref
    assert orc.cfl_dt(c, U) < 0.1 * ref  # without the body the wild cells count


# -------------------------------------------------------- viscous terms
def viscous_part(orc, nx, ny, W, **kw):
    """Viscous contribution to the right-hand side: the viscous minus the
    inviscid oracle right-hand side on the same state."""
    cv = orc.config(nx=nx, ny=ny, viscous=1, **kw)
    kw.pop("mu", None)
    kw.pop("prandtl", None)
    ci = orc.config(nx=nx, ny=ny, viscous=0, **kw)
    U = orc.prim_to_cons(cv, W)
    return orc.rhs(cv, U)[0] - orc.rhs(ci, U)[0]


def test_viscous_normal_stress_heating(orc):
    """u = a x, v = b y at uniform rho, p (Stokes hypothesis): the stresses
    are uniform, tau_xx = mu (4/3 a - 2/3 b), tau_yy = mu (4/3 b - 2/3 a),
    tau_xy = 0, so the momentum equations get nothing and the energy equation
    gets a tau_xx + b tau_yy = (4/3) mu (a^2 - a b + b^2)."""
    nx, ny, a, b, mu = 14, 12, 0.6, -0.35, 0.03
    x = inputs.centres(nx, 0, 1)[None, :]
    y = inputs.centres(ny, 0, 1)[:, None]
    W = np.empty((4, ny, nx))
    W[0] = 1.0
    W[1] = a * x + 0 * y
    W[2] = b * y + 0 * x
    W[3] = 1.0
    D = viscous_part(orc, nx, ny, W, mu=mu, bc=(0, 0, 0, 0))
    inner = (slice(2, ny - 2), slice(2, nx - 2))
    assert np.max(np.abs(D[0][inner])) < 1e-13
    assert np.max(np.abs(D[1][inner])) < 1e-12 and np.max(np.abs(D[2][inner])) < 1e-12
    ref = 4.0 / 3.0 * mu * (a * a - a * b + b * b)
    np.testing.assert_allclose(D[3][inner], ref, rtol=1e-9)


@pytest.mark.parametrize("prandtl", [0.72, 1.5])
def test_heat_conduction_quadratic_temperature(orc, prandtl):
    """Gas at rest at uniform pressure with T = T0 + c x^2 (rho = p / T, gas
    constant 1): a stationary contact, so the inviscid right-hand side
    vanishes, and Fourier conduction gives the energy equation kappa T'' =
    2 kappa c with kappa = mu gamma / ((gamma - 1) Pr)."""
    nx, ny, mu, T0, cc, p = 16, 6, 0.02, 1.0, 0.8, 1.3
    x = inputs.centres(nx, 0, 1)[None, :]
    T = T0 + cc * x * x + 0.0 * np.zeros((ny, 1))
    W = np.empty((4, ny, nx))
    W[0] = p / T
    W[1] = 0.0
    W[2] = 0.0
    W[3] = p
    c = orc.config(nx=nx, ny=ny, viscous=1, mu=mu, prandtl=prandtl, bc=(0, 0, 3, 3))
    L = orc.rhs(c, orc.prim_to_cons(c, W))[0]
    inner = (slice(None), slice(2, nx - 2))
    kappa = mu * G / ((G - 1.0) * prandtl)
    assert np.max(np.abs(L[0][inner])) < 1e-13
    assert np.max(np.abs(L[1][inner])) < 1e-12 and np.max(np.abs(L[2][inner])) < 1e-13
    np.testing.assert_allclose(L[3][inner], 2.0 * kappa * cc, rtol=1e-9)


# ------------------------------------------------------------ wall rules
@pytest.mark.parametrize("wall", [0, 1])
def test_ibm_wall_rules_on_planar_wall(orc, wall):
    """A flat wall on a cell face: each ghost's image point is the centre of
    its mirror cell, so the filled ghost holds that cell's density and
    pressure with the normal velocity reversed (slip) or the whole velocity
    reversed (no-slip adiabatic); solid cells beyond the band keep their
    values."""
    nx, ny, jw = 10, 24, 9
    dom = (0.0, 1.0, 0.0, 1.0)
    c = orc.config(nx=nx, ny=ny, bc=(3, 3, 0, 0))
    phi = inputs.plane_phi(nx, ny, dom, jw / ny)
    W = inputs.random_prim(nx, ny, seed=11)
    U = orc.prim_to_cons(c, W)
    Uf = orc.ibm_fill(c, U, phi, wall=wall)
    Wf = orc.cons_to_prim(c, Uf)
    for k in range(3):
        g, m = jw - 1 - k, jw + k  # ghost row and its mirror row
        np.testing.assert_allclose(Wf[0, g], W[0, m], rtol=1e-13)
        np.testing.assert_allclose(Wf[3, g], W[3, m], rtol=1e-12)
        np.testing.assert_allclose(Wf[2, g], -W[2, m], rtol=1e-12, atol=1e-13)
        sgn = 1.0 if wall == 0 else -1.0
        np.testing.assert_allclose(Wf[1, g], sgn * W[1, m], rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(Uf[:, : jw - 3], U[:, : jw - 3])
    np.testing.assert_array_equal(Uf[:, jw:], U[:, jw:])


# -------------------------------------------------------- boundary rules
def ghost_cells(rule, W_edge_to_far, inflow):
    """The three ghost cells (nearest first) a boundary rule should produce,
    from the interior cells listed nearest first; normal velocity index 1."""
    out = []
    for g in range(3):
        if rule == "transmissive":
            w = W_edge_to_far[0].copy()
        elif rule == "reflective":
            w = W_edge_to_far[g].copy()
            w[1] = -w[1]
        else:  # inflow
            w = np.array(inflow, dtype=float)
        out.append(w)
    return out


RULES = {"transmissive": 0, "reflective": 1, "inflow": 2}


@pytest.mark.parametrize("rule", ["transmissive", "reflective", "inflow"])
@pytest.mark.parametrize("side", [0, 1, 2, 3])
def test_boundary_rule_equals_extended_grid(orc, rule, side):
    """A boundary rule is the same as three more cells holding the ghost
    values it should produce: the right-hand side of the original grid equals
    that of the extended grid on the original cells.  The opposite axis is
    periodic, the far side transmissive, the flow inviscid."""
    n_along, n_across = 11, 9
    inflow = (1.3, 0.4, -0.2, 1.7)
    Wd = inputs.random_prim(n_along, n_across, seed=20 + side)  # along = normal axis here
    # build everything in the (normal, tangential) frame, then lay it out
    axis_x = side < 2
    lo = side % 2 == 0
    nx, ny = (n_along, n_across) if axis_x else (n_across, n_along)
    W = Wd if axis_x else np.ascontiguousarray(np.stack([Wd[0].T, Wd[2].T, Wd[1].T, Wd[3].T]))
    # W in physical layout [4][ny][nx]; the normal velocity of this side:
    vn = 1 if axis_x else 2
    inflow_phys = inflow
    bc = [3, 3, 3, 3]
    if axis_x:
        bc[0], bc[1] = 0, 0
    else:
        bc[2], bc[3] = 0, 0
    bc[side] = RULES[rule]
    c = orc.config(nx=nx, ny=ny, bc=tuple(bc), inflow=inflow_phys)
    L = orc.rhs(c, orc.prim_to_cons(c, W))[0]
    # extended grid: three ghost cells added on `side`, transmissive there
    h = 1.0 / (nx if axis_x else ny)
    if axis_x:
        edge = [W[:, :, i] for i in (range(3) if lo else range(nx - 1, nx - 4, -1))]
    else:
        edge = [W[:, j, :] for j in (range(3) if lo else range(ny - 1, ny - 4, -1))]
    ghosts = []
    for g in range(3):
        if rule == "transmissive":
            w = edge[0].copy()
        elif rule == "reflective":
            w = edge[g].copy()
            w[vn] = -w[vn]
        else:
            w = np.empty_like(edge[0])
            for k in range(4):
                w[k] = inflow_phys[k]
        ghosts.append(w)
    if axis_x:
        cols = [gh[:, :, None] for gh in ghosts]
        We = np.concatenate(cols[::-1] + [W], axis=2) if lo else np.concatenate([W] + cols, axis=2)
        dom = (-3 * h, 1.0, 0.0, 1.0) if lo else (0.0, 1.0 + 3 * h, 0.0, 1.0)
        ce = orc.config(nx=nx + 3, ny=ny, x0=dom[0], x1=dom[1], bc=tuple(bc[:side] + [0] + bc[side + 1:]))
        Le = orc.rhs(ce, orc.prim_to_cons(ce, We))[0]
        Le = Le[:, :, 3:] if lo else Le[:, :, :nx]
    else:
        rows = [gh[:, None, :] for gh in ghosts]
        We = np.concatenate(rows[::-1] + [W], axis=1) if lo else np.concatenate([W] + rows, axis=1)
        dom = (0.0, 1.0, -3 * h, 1.0) if lo else (0.0, 1.0, 0.0, 1.0 + 3 * h)
        ce = orc.config(nx=nx, ny=ny + 3, y0=dom[2], y1=dom[3], bc=tuple(bc[:side] + [0] + bc[side + 1:]))
        Le = orc.rhs(ce, orc.prim_to_cons(ce, We))[0]
        Le = Le[:, 3:, :] if lo else Le[:, :ny, :]
    for k in range(4):
        scale = np.max(np.abs(L[k])) + 1e-300
        assert np.max(np.abs(Le[k] - L[k])) <= 1e-13 * scale, (rule, side, k)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_periodic_rule_equals_extended_grid(orc, axis):
    """Periodic boundaries: three wrapped cells on each side of an extended
    grid with transmissive ends give the same right-hand side."""
    nx, ny = 10, 8
    W = inputs.random_prim(nx, ny, seed=31)
    c = orc.config(nx=nx, ny=ny, bc=(3, 3, 3, 3))
    L = orc.rhs(c, orc.prim_to_cons(c, W))[0]
    if axis == "x":
        We = np.concatenate([W[:, :, -3:], W, W[:, :, :3]], axis=2)
        ce = orc.config(nx=nx + 6, ny=ny, x0=-0.3, x1=1.3, bc=(0, 0, 3, 3))
        Le = orc.rhs(ce, orc.prim_to_cons(ce, We))[0][:, :, 3:-3]
    else:
        We = np.concatenate([W[:, -3:, :], W, W[:, :3, :]], axis=1)
        ce = orc.config(nx=nx, ny=ny + 6, y0=-3 / 8, y1=1 + 3 / 8, bc=(3, 3, 0, 0))
        Le = orc.rhs(ce, orc.prim_to_cons(ce, We))[0][:, 3:-3, :]
    for k in range(4):
        scale = np.max(np.abs(L[k]))
        assert np.max(np.abs(Le[k] - L[k])) <= 1e-13 * scale


# ---------------------------------------------------------- network forward
def bf16_round(a):
    """bfloat16 rounding (nearest even) through float32 by integer masking."""
    f = np.asarray(a, dtype=np.float32).copy()
    u = f.view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))
    u &= np.uint32(0xFFFF0000)
    return f.astype(np.float64)


@pytest.mark.parametrize("emulate", [False, True])
def test_net_forward_matches_numpy_evaluation(orc, emulate):
    """The per-face network (24 -> 64 -> 64 -> 64 -> 4, ReLU, out_scale *
    tanh) evaluated with numpy matrix products from the parameter vector
    layout W0, b0, W1, b1, W2, b2, W3, b3; with emulation every product
    operand is rounded to bfloat16."""
    rng = np.random.default_rng(41)
    p = (rng.normal(size=orc.NET_PARAMS) * 0.3).astype(np.float32)
    mean = np.array([1.0, 0.1, -0.2, 1.1])
    inv = np.array([2.0, 1.5, 1.25, 0.9])
    net = orc.Net(p, mean, inv, 0.07, emulate_bf16=emulate)
    st = rng.uniform(0.2, 1.8, size=(9, 6, 4))
    got = net.forward(st)
    q = p.astype(np.float64)
    sizes = [(64, 24), (64, 64), (64, 64), (4, 64)]
    k = 0
    layers = []
    for o, i in sizes:
        Wl = q[k:k + o * i].reshape(o, i)
        k += o * i
        bl = q[k:k + o]
        k += o
        layers.append((Wl, bl))
    assert k == orc.NET_PARAMS
    r = bf16_round if emulate else (lambda a: a)
    h = ((st - mean) * inv).reshape(9, 24)
    for li, (Wl, bl) in enumerate(layers):
        h = r(h) @ r(Wl).T + bl
        if li < 3:
            h = np.maximum(h, 0.0)
    ref = 0.07 * np.tanh(h)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-15)


# --------------------------------------------------------- training pieces
def cell_avg_poly(x0, x1, y0, y1):
    """Exact cell average of f(x, y) = 1 + 2x - y + 3 x^2 y + y^3 over
    [x0,x1] x [y0,y1] (antiderivatives evaluated at the corners)."""
    def F(x, y):
        return x * y + x * x * y - 0.5 * x * y * y + 0.5 * x ** 3 * y * y + 0.25 * x * y ** 4
    area = (x1 - x0) * (y1 - y0)
    return (F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)) / area


def averages(nx, ny):
    xe = np.linspace(0, 1, nx + 1)
    ye = np.linspace(0, 0.5, ny + 1)
    A = np.empty((ny, nx))
    for j in range(ny):
        for i in range(nx):
            A[j, i] = cell_avg_poly(xe[i], xe[i + 1], ye[j], ye[j + 1])
    return A


@pytest.mark.parametrize("factor", [2, 4])
def test_restrict_maps_cell_averages_to_cell_averages(orc, factor):
    """The restriction d(U) of section 2 on nested uniform grids: the mean of
    exact fine cell averages is the exact coarse cell average, for any
    integrand; per plane, with batch and variable planes kept apart."""
    nxc, nyc = 5, 3
    fine = averages(nxc * factor, nyc * factor)
    coarse = averages(nxc, nyc)
    stack = np.stack([fine, 2.0 * fine - 1.0, np.full_like(fine, 0.7)])[None]  # [1][3][ny][nx]
    got = orc.restrict(stack, factor)
    assert got.shape == (1, 3, nyc, nxc)
    np.testing.assert_allclose(got[0, 0], coarse, rtol=1e-13)
    np.testing.assert_allclose(got[0, 1], 2.0 * coarse - 1.0, rtol=1e-13)
    np.testing.assert_allclose(got[0, 2], 0.7, rtol=1e-15)
    # block sums are conserved
    assert abs(got[0, 0].sum() * factor * factor - fine.sum()) <= 1e-12 * abs(fine.sum())


def test_mse_closed_form_and_gradient(orc):
    """Unrolled-loss term ||U - T||^2 / N per batch member: U = T + c gives
    c^2; the gradient matches central differences of the loss and scales
    linearly; batch members are independent."""
    rng = np.random.default_rng(5)
    T = rng.normal(size=(3, 4, 6, 5))
    U = T + np.array([0.1, -0.3, 0.0])[:, None, None, None]
    loss, Gr = orc.mse(U, T, nbatch=3)
    np.testing.assert_allclose(loss, [0.01, 0.09, 0.0], rtol=1e-13, atol=1e-17)
    U = T + rng.normal(size=T.shape) * 0.2
    loss, Gr = orc.mse(U, T, scale=0.5, nbatch=3)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 3, 4), (2, 3, 5, 1)]:
        Up, Um = U.copy(), U.copy()
        Up[idx] += h
        Um[idx] -= h
        b = idx[0]
        fd = (orc.mse(Up, T, nbatch=3, grad=False)[0][b] - orc.mse(Um, T, nbatch=3, grad=False)[0][b]) / (2 * h)
        assert abs(0.5 * fd - Gr[idx]) <= 1e-8 * max(1e-3, abs(Gr[idx]))
    # member 1's loss does not see member 0's entries
    U2 = U.copy()
    U2[0] += 1.0
    assert orc.mse(U2, T, nbatch=3, grad=False)[0][1] == loss[1]


def test_adam_constant_gradient_closed_form(orc):
    """Adam with bias correction under a constant gradient g: mhat = g and
    vhat = g^2 exactly at every step, so each step moves theta by
    lr g / (|g| + eps), and a zero gradient with zero moments moves
    nothing."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 0.5, -0.25, 2.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    for step in range(1, 8):
        th, m, v = orc.adam(th, g, m, v, lr, step, eps=eps)
    ref = np.array([1.0, 0.5, -0.25, 2.0]) - 7 * lr * g / (np.abs(g) + eps)
    np.testing.assert_allclose(th, ref, rtol=1e-13, atol=1e-15)
    assert th[3] == 2.0
    # first moment is (1 - b1^t) g, second (1 - b2^t) g^2
    np.testing.assert_allclose(m, (1 - 0.9 ** 7) * g, rtol=1e-13)
    np.testing.assert_allclose(v, (1 - 0.999 ** 7) * g * g, rtol=1e-12)


def test_degenerate_ghosts_counted(orc):
    """A solid plate one cell thick (signed distance |y - yc| - t/2, t < dy):
    at its cells the central difference of phi straddles the plate's middle
    and vanishes (up to rounding), so the ghosts have no normal and no image
    point -- every one is counted as degenerate; a cylinder many cells across
    has none."""
    from paper_2601_04400_amd import inputs
    n = 40
    dom = (0.0, 1.0, 0.0, 1.0)
    y = inputs.centres(n, 0.0, 1.0)[:, None]
    yc = y[n // 2, 0]
    phi = np.broadcast_to(np.abs(y - yc) - 0.4 / n, (n, n)).copy()
    c = orc.config(nx=n, ny=n)
    cls, ng = orc.ibm_classify(c, phi)
    assert ng == n and orc.ibm_degenerate(c, phi) == n
    phi_c = inputs.circle_phi(n, n, dom, (0.5, 0.5), 0.25)
    assert orc.ibm_degenerate(c, phi_c) == 0
