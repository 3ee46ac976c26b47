"""GPU parity of the immersed boundary and the viscous terms against the
oracle: cell classes and ghost lists bit-exact, right-hand sides to 1e-13,
trajectories to 1e-11 (per conserved field)."""
import numpy as np
import pytest

from paper_2601_04400_amd import inputs
from gpu_util import assert_fields, make_pair

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def to_np(U):
    torch.cuda.synchronize()
    return U.detach().to("cpu", torch.float64).numpy()


def setup(orc, nx, ny, mach=3.0, viscous=False, prec="f64", domain=(0.0, 2.0, 0.0, 1.0)):
    post_o = orc.rh_post_shock(mach)
    post = (post_o[0], post_o[1], 0.0, post_o[2])
    sc = inputs.shock_cylinder(nx, ny, post, domain=domain)
    mu = inputs.cylinder_viscosity(mach) if viscous else 0.0
    c, g = make_pair(orc, nx, ny, domain=domain, bc=sc["bc"], inflow=sc["inflow"], viscous=viscous,
                     mu=mu, prec=prec, ibm=True)
    return c, g, sc


def test_classes_and_ghost_count_bitwise(orc):
    for nx, ny in ((96, 48), (1024, 512), (77, 53)):
        c, g, sc = setup(orc, nx, ny)
        ng = g.set_levelset(torch.from_numpy(sc["phi"]), wall=0)
        cls_o, ng_o = orc.ibm_classify(c, sc["phi"])
        np.testing.assert_array_equal(g.classes().cpu().numpy(), cls_o)
        assert ng == ng_o > 0


@pytest.mark.parametrize("viscous,wall", [(False, 0), (True, 1), (False, 1), (True, 0)])
def test_rhs_with_ibm(orc, viscous, wall):
    nx, ny = 160, 80
    c, g, sc = setup(orc, nx, ny, viscous=viscous)
    # a rough state so every ghost interpolation and wall rule matters
    W = inputs.random_prim(nx, ny, seed=5)
    Uo = orc.prim_to_cons(c, W)
    Lo, Ufo, _ = orc.rhs(c, Uo, phi=sc["phi"], wall=wall)
    g.set_levelset(torch.from_numpy(sc["phi"]), wall=wall)
    Ug = torch.from_numpy(Uo).to(g.device).reshape(g.shape).contiguous()
    Lg = to_np(g.rhs(Ug))[0]
    # the right-hand side forms the ghost values as it loads them and leaves U as it is
    assert np.array_equal(to_np(Ug)[0], Uo)
    assert_fields(Lg, Lo, 1e-13, f"ibm rhs viscous={viscous} wall={wall}")
    # the separate refill stores the same ghost values the right-hand side used
    assert_fields(to_np(g.ib_fill(Ug))[0], Ufo, 1e-14, "ghost-filled state")
    assert np.array_equal(to_np(g.rhs(Ug))[0], Lg)


@pytest.mark.parametrize("viscous,wall", [(False, 0), (True, 1)])
def test_ibm_bodies_across_periodic_edges(orc, viscous, wall):
    """Two bodies cut by the periodic domain edges (one across x = 0, one
    across y = 0) on a 160 x 80 grid of 32 x 8 stage tiles: the tiles along
    the opposite edges reach those bodies' solid and ghost cells only through
    the periodic wrap of their halo, so they must keep the immersed-boundary
    handling that tiles of all-fluid cells skip.  Right-hand side on a rough
    state and one fixed-step RK3 step on a smooth one, against the oracle."""
    nx, ny = 160, 80
    dom = (0.0, 2.0, 0.0, 1.0)
    phi = np.minimum(inputs.circle_phi(nx, ny, dom, (0.0, 0.5), 0.12),
                     inputs.circle_phi(nx, ny, dom, (1.0, 0.0), 0.12))
    mu = 2e-3 if viscous else 0.0
    c, g = make_pair(orc, nx, ny, domain=dom, bc=(3, 3, 3, 3), viscous=viscous, mu=mu, ibm=True)
    assert g.set_levelset(torch.from_numpy(phi), wall=wall) == orc.ibm_classify(c, phi)[1] > 0
    W = inputs.random_prim(nx, ny, seed=17)
    Uo = orc.prim_to_cons(c, W)
    Lo, _, _ = orc.rhs(c, Uo, phi=phi, wall=wall)
    Ug = torch.from_numpy(Uo).to(g.device).reshape(g.shape).contiguous()
    assert_fields(to_np(g.rhs(Ug))[0], Lo, 1e-13, f"periodic-edge bodies rhs viscous={viscous}")
    Uo = orc.prim_to_cons(c, inputs.smooth_prim(nx, ny, seed=18, amp=0.3, domain=dom))
    dt = 0.4 * orc.cfl_dt(c, Uo, phi=phi)
    U1o, _ = orc.rk3_step(c, Uo, dt, phi=phi, wall=wall)
    Ug = torch.from_numpy(Uo).to(g.device).reshape(g.shape).contiguous()
    g.step(Ug, dt)
    assert_fields(to_np(Ug)[0], U1o, 1e-13, f"periodic-edge bodies step viscous={viscous}")


@pytest.mark.parametrize("viscous,wall", [(True, 1), (False, 0)])
def test_ibm_batch_members_step_independently(orc, viscous, wall):
    """Two batch members share one body: the Mach-3 shock already at the
    cylinder, and a smooth periodic-mode state.  Ten automatic steps of the
    batched grid (each member its own step size, every member covering all of
    the body-first tile order) against the oracle per member, and member 1
    bit for bit against the same state stepped on a one-member grid."""
    nx, ny = 160, 80
    post_o = orc.rh_post_shock(3.0)
    sc = inputs.shock_cylinder(nx, ny, (post_o[0], post_o[1], 0.0, post_o[2]), xs=0.25)
    mu = inputs.cylinder_viscosity(3.0) if viscous else 0.0
    kw = dict(domain=sc["domain"], bc=sc["bc"], inflow=sc["inflow"], viscous=viscous, mu=mu, ibm=True)
    c, g = make_pair(orc, nx, ny, nbatch=2, **kw)
    _, g1 = make_pair(orc, nx, ny, **kw)
    for gg in (g, g1):
        gg.set_levelset(torch.from_numpy(sc["phi"]), wall=wall)
    W1 = inputs.smooth_prim(nx, ny, seed=21, amp=0.3, domain=sc["domain"])
    Ug = g.prim_to_cons(torch.from_numpy(np.stack([sc["W"], W1])))
    U1 = g1.prim_to_cons(torch.from_numpy(W1))
    g.set_time(0.0, 1.0)
    g1.set_time(0.0, 1.0)
    for _ in range(10):
        g.step(Ug)
        g1.step(U1)
    assert torch.equal(Ug[1], U1[0]), "batch member 1 differs from the one-member grid"
    for b, W in enumerate((sc["W"], W1)):
        Ue, te, steps_o, fbo = orc.run(c, orc.prim_to_cons(c, W), 1.0, max_steps=10, phi=sc["phi"], wall=wall)
        t, _, steps = g.get_time(b)
        assert steps == steps_o == 10 and abs(t - te) <= 1e-14 * te and fbo == 0
        errs = assert_fields(to_np(Ug)[b], Ue, 1e-11, f"batch member {b}, 10 steps")
        print(f"ibm batch member {b} viscous={viscous}: per-field errors {errs}", flush=True)
    assert g.poll_faults() == (0, 0)


@pytest.mark.parametrize("viscous,wall", [(False, 0), (True, 1), (True, 0)])
def test_ibm_body_cut_by_reflective_wall(orc, viscous, wall):
    """The restricted shock-cylinder geometry (the cylinder centred on the
    reflecting top edge): halo slots above that edge reach ghost cells
    through the wall's mirror rule, so their refilled values take its sign
    flip.  Right-hand side on a rough state and one step with the shock
    inside the body, against the oracle."""
    from paper_2601_04400_amd import infer
    nx, ny = 120, 80
    sc = infer.restricted_cylinder(nx, ny)
    dom = sc["domain"]
    mu = 2e-3 if viscous else 0.0
    c, g = make_pair(orc, nx, ny, domain=dom, bc=sc["bc"], inflow=sc["inflow"], viscous=viscous, mu=mu, ibm=True)
    assert g.set_levelset(torch.from_numpy(sc["phi"]), wall=wall) == orc.ibm_classify(c, sc["phi"])[1] > 0
    Uo = orc.prim_to_cons(c, inputs.random_prim(nx, ny, seed=23))
    Lo, _, _ = orc.rhs(c, Uo, phi=sc["phi"], wall=wall)
    Ug = torch.from_numpy(Uo).to(g.device).reshape(g.shape).contiguous()
    assert_fields(to_np(g.rhs(Ug))[0], Lo, 1e-13, f"wall-cut body rhs viscous={viscous} wall={wall}")
    Uo = orc.prim_to_cons(c, inputs.shock_prim(nx, ny, dom, 0.5, sc["inflow"], infer.PRE))
    dt = 0.4 * orc.cfl_dt(c, Uo, phi=sc["phi"])
    U1o, _ = orc.rk3_step(c, Uo, dt, phi=sc["phi"], wall=wall)
    Ug = torch.from_numpy(Uo).to(g.device).reshape(g.shape).contiguous()
    g.step(Ug, dt)
    assert_fields(to_np(Ug)[0], U1o, 1e-13, f"wall-cut body step viscous={viscous} wall={wall}")


@pytest.mark.parametrize("prec,viscous", [("f32", False), ("mixed", False), ("mixed", True)])
def test_ibm_single_precision_storage(orc, prec, viscous):
    """The immersed boundary with FP32 storage (FP32 or FP64 arithmetic):
    right-hand side and one step with the Mach-3 shock inside the body's
    front, against the oracle run on the FP32-rounded state, to 1e-5 per
    field.  FP32 arithmetic is held on the smooth side of the bar: its
    right-hand side is taken before the shock reaches the body."""
    nx, ny = 160, 80
    post_o = orc.rh_post_shock(3.0)
    post = (post_o[0], post_o[1], 0.0, post_o[2])
    xs = 0.1 if prec == "f32" else 0.25
    sc = inputs.shock_cylinder(nx, ny, post, xs=xs)
    mu = inputs.cylinder_viscosity(3.0) if viscous else 0.0
    c, g = make_pair(orc, nx, ny, domain=sc["domain"], bc=sc["bc"], inflow=sc["inflow"], viscous=viscous, mu=mu,
                     prec=prec, ibm=True)
    assert g.set_levelset(torch.from_numpy(sc["phi"]), wall=1 if viscous else 0) > 0
    wall = 1 if viscous else 0
    Uo = orc.prim_to_cons(c, sc["W"]).astype(np.float32).astype(np.float64)  # what FP32 storage holds
    Lo, _, _ = orc.rhs(c, Uo, phi=sc["phi"], wall=wall)
    Ug = torch.from_numpy(Uo).to(device=g.device, dtype=g.dtype).reshape(g.shape).contiguous()
    assert_fields(to_np(g.rhs(Ug))[0], Lo, 1e-5, f"ibm rhs {prec} viscous={viscous}")
    dt = 0.4 * orc.cfl_dt(c, Uo, phi=sc["phi"])
    U1o, _ = orc.rk3_step(c, Uo, dt, phi=sc["phi"], wall=wall)
    g.step(Ug, dt)
    errs = assert_fields(to_np(Ug)[0], U1o, 1e-5, f"ibm step {prec} viscous={viscous}")
    print(f"ibm {prec} viscous={viscous}: step per-field errors {errs}", flush=True)


def test_shock_cylinder_ns_trajectory_small(orc):
    """Mach-3 shock on the cylinder, Navier-Stokes, no-slip adiabatic wall, at
    160x80, 40 automatic steps (the shock reaches the cylinder)."""
    nx, ny = 160, 80
    c, g, sc = setup(orc, nx, ny, viscous=True)
    Uo = orc.prim_to_cons(c, sc["W"])
    Ue, te, steps_o, fbo = orc.run(c, Uo, 1.0, max_steps=40, phi=sc["phi"], wall=1)
    g.set_levelset(torch.from_numpy(sc["phi"]), wall=1)
    Ug = g.prim_to_cons(torch.from_numpy(sc["W"]))
    g.set_time(0.0, 1.0)
    for _ in range(40):
        g.step(Ug)
    t, done, steps = g.get_time()
    assert steps == steps_o == 40 and abs(t - te) <= 1e-14 * te
    assert_fields(to_np(Ug)[0], Ue, 1e-11, "NS shock-cylinder trajectory")
    assert g.poll_faults() == (0, 0) and fbo == 0


def test_shock_cylinder_ns_full_size_step(orc):
    """1024x512 (the Navier-Stokes cylinder size): one right-hand side and one
    automatic step from the initial condition."""
    nx, ny = 1024, 512
    c, g, sc = setup(orc, nx, ny, viscous=True)
    Uo = orc.prim_to_cons(c, sc["W"])
    g.set_levelset(torch.from_numpy(sc["phi"]), wall=1)
    Ug = g.prim_to_cons(torch.from_numpy(sc["W"]))
    Lo, _, _ = orc.rhs(c, Uo, phi=sc["phi"], wall=1)
    U0 = Ug.clone()
    assert_fields(to_np(g.rhs(U0))[0], Lo, 1e-13, "1024x512 rhs")
    dto = orc.cfl_dt(c, Uo, phi=sc["phi"])
    U1o, _ = orc.rk3_step(c, Uo, dto, phi=sc["phi"], wall=1)
    dts = torch.zeros(1, dtype=torch.float64, device=g.device)
    g.set_time(0.0, 1.0)
    g.step(Ug, dt_out=dts)
    assert float(dts.cpu()[0]) == dto
    assert_fields(to_np(Ug)[0], U1o, 1e-13, "1024x512 step")


@pytest.mark.parametrize("viscous,wall", [(True, 1), (False, 0)])
def test_ibm_automatic_step_equals_fixed_step_bitwise(orc, viscous, wall):
    """With an immersed boundary the automatic step runs fused into the three
    stage kernels, each refilling its ghost cells while loading its tile; the
    same steps given as fixed steps run the plain three stages.  Both must
    produce the same states bit for bit (and the oracle's to 1e-11)."""
    nx, ny = 160, 80
    c, g, sc = setup(orc, nx, ny, viscous=viscous)
    _, g2, _ = setup(orc, nx, ny, viscous=viscous)
    for gg in (g, g2):
        gg.set_levelset(torch.from_numpy(sc["phi"]), wall=wall)
    Ua = g.prim_to_cons(torch.from_numpy(sc["W"]))
    Ub = Ua.clone()
    g.set_time(0.0, 1.0)
    dts = []
    for k in range(30):
        dt = torch.zeros(1, dtype=torch.float64, device=g.device)
        g.step(Ua, dt_out=dt)
        g2.step(Ub, dt=dt.clone())
        dts.append(float(dt.cpu()[0]))
        assert torch.equal(Ua, Ub), f"step {k}: fused and fixed-step states differ"
    Uo = orc.prim_to_cons(c, sc["W"])
    for dt in dts:
        Uo, _ = orc.rk3_step(c, Uo, dt, phi=sc["phi"], wall=wall)
    errs = assert_fields(to_np(Ua)[0], Uo, 1e-11, "30 steps with the immersed boundary")
    print(f"ibm fused steps viscous={viscous}: per-field errors {errs}", flush=True)


def test_shock_cylinder_ns_full_size_at_body(orc):
    """1024x512 Navier-Stokes cylinder with the Mach-3 shock already inside
    the body's leading part (shock at x = 0.25; the cylinder spans 0.2..0.4),
    so the no-slip wall, the ghost refill and the viscous terms act on a
    moving, shocked gas: five automatic steps against the oracle."""
    nx, ny = 1024, 512
    post_o = orc.rh_post_shock(3.0)
    post = (post_o[0], post_o[1], 0.0, post_o[2])
    sc = inputs.shock_cylinder(nx, ny, post, xs=0.25)
    mu = inputs.cylinder_viscosity(3.0)
    c, g = make_pair(orc, nx, ny, domain=sc["domain"], bc=sc["bc"], inflow=sc["inflow"], viscous=True, mu=mu,
                     ibm=True)
    g.set_levelset(torch.from_numpy(sc["phi"]), wall=1)
    Ug = g.prim_to_cons(torch.from_numpy(sc["W"]))
    Uo = orc.prim_to_cons(c, sc["W"])
    Ue, te, steps_o, fbo = orc.run(c, Uo, 1.0, max_steps=5, phi=sc["phi"], wall=1)
    g.set_time(0.0, 1.0)
    for _ in range(5):
        g.step(Ug)
    t, done, steps = g.get_time()
    assert steps == steps_o == 5 and abs(t - te) <= 1e-14 * te
    errs = assert_fields(to_np(Ug)[0], Ue, 1e-11, "1024x512 shock at the body, 5 steps")
    print(f"1024x512 shock at the body: per-field errors {errs}", flush=True)
    assert g.poll_faults() == (0, 0) and fbo == 0


def test_quiescent_cylinder_stays_at_rest_gpu(orc):
    nx, ny = 96, 96
    dom = (0.0, 1.0, 0.0, 1.0)
    phi = inputs.circle_phi(nx, ny, dom, (0.45, 0.52), 0.2)
    c, g = make_pair(orc, nx, ny, domain=dom, bc=(1, 1, 1, 1), viscous=True, mu=1e-3, ibm=True)
    W = np.zeros((4, ny, nx)); W[0] = 1.0; W[3] = 1.0
    g.set_levelset(torch.from_numpy(phi), wall=1)
    U = g.prim_to_cons(torch.from_numpy(W))
    g.set_time(0.0, 1.0)
    for _ in range(10):
        g.step(U)
    u = to_np(U)[0]
    fl = phi >= 0
    assert np.max(np.abs(u[1][fl])) < 1e-14 and np.max(np.abs(u[2][fl])) < 1e-14


def test_paper_shock_cylinder_line_profile_self_converges():
    """Section 3 Mach-5 shock-cylinder set-up at three resolutions: the density
    along the transverse line x = 0.2 at t = 0.3 converges under refinement
    (successive differences shrink), the run reaches t = 0.3 exactly with
    finite values, and the profile is mirror-
    symmetric about y = 1 (the set-up is) up to rounding."""
    import torch
    from paper_2601_04400_amd import Grid
    profiles = {}
    for nx in (256, 512, 1024):
        ny = nx // 2
        sc = inputs.paper_shock_cylinder(nx, ny)
        g = Grid(nx, ny, domain=sc["domain"], bc=sc["bc"], inflow=sc["inflow"], ibm=True)
        g.set_levelset(torch.from_numpy(sc["phi"]), wall=0)
        U = g.prim_to_cons(torch.from_numpy(sc["W"]))
        t, steps = g.advance(U, 0.3, chunk=128)
        assert t == 0.3
        flags, fb = g.poll_faults()
        assert flags & 1 == 0  # finite (the Mach-5 reflection may use the positivity fallback)
        rho = U[0, 0].cpu().numpy()
        x = inputs.centres(nx, -0.5, 4.0)
        i = int(np.searchsorted(x, 0.2)) - 1  # x[i] <= 0.2 < x[i + 1]
        w = (0.2 - x[i]) / (x[i + 1] - x[i])
        col = (1 - w) * rho[:, i] + w * rho[:, i + 1]
        profiles[nx] = col
        # mirror symmetry up to rounding (mirrored faces associate their sums
        # differently, so it is not bitwise)
        np.testing.assert_allclose(col, col[::-1], rtol=1e-8, atol=1e-8)
    # compare on the coarsest cells: average the finer profile pairwise
    def down(p):
        return 0.5 * (p[0::2] + p[1::2])
    d1 = np.mean(np.abs(down(profiles[512]) - profiles[256]))
    d2 = np.mean(np.abs(down(profiles[1024]) - profiles[512]))
    assert d2 < d1, (d1, d2)


def test_paper_shock_cylinder_full_size(orc):
    """The section 3 Mach-5 shock-cylinder at its full 4096 x 2048 size
    (slip wall, inflow / outflow / reflective walls): cell classes and ghost
    count bit-exact, one right-hand side and one automatic step from the
    initial condition against the oracle."""
    nx, ny = 4096, 2048
    sc = inputs.paper_shock_cylinder(nx, ny)
    c, g = make_pair(orc, nx, ny, domain=sc["domain"], bc=sc["bc"], inflow=sc["inflow"], ibm=True)
    ng = g.set_levelset(torch.from_numpy(sc["phi"]), wall=0)
    cls_o, ng_o = orc.ibm_classify(c, sc["phi"])
    np.testing.assert_array_equal(g.classes().cpu().numpy(), cls_o)
    assert ng == ng_o > 0
    Uo = orc.prim_to_cons(c, sc["W"])
    Ug = g.prim_to_cons(torch.from_numpy(sc["W"]))
    Lo, _, _ = orc.rhs(c, Uo, phi=sc["phi"], wall=0)
    assert_fields(to_np(g.rhs(Ug.clone()))[0], Lo, 1e-13, "4096x2048 rhs")
    dto = orc.cfl_dt(c, Uo, phi=sc["phi"])
    U1o, _ = orc.rk3_step(c, Uo, dto, phi=sc["phi"], wall=0)
    dts = torch.zeros(1, dtype=torch.float64, device=g.device)
    g.set_time(0.0, 1.2)
    g.step(Ug, dt_out=dts)
    assert float(dts.cpu()[0]) == dto
    assert_fields(to_np(Ug)[0], U1o, 1e-13, "4096x2048 step")
