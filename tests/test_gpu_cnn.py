"""GPU convolutional learned correction (section 2's 2D neural flux: 3x3
layers 4-16-32-4 over the images of x-faces and transposed y-faces, bfloat16
matrix cores, FP32 accumulation) against the oracle's double-precision
network with every product operand rounded to bfloat16.

Tolerances as for the per-face network: 4e-3 of the largest reference value
(one bfloat16 unit); the input images, which both sides round to bfloat16
from double values, agree to one bfloat16 unit.
"""
import numpy as np
import pytest

from paper_2601_04400_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def make_cnn(orc, seed, scale_out=1.0, zero_output=False):
    import paper_2601_04400_amd.learn as L
    theta = L.init_cnn_theta(seed, zero_output=zero_output)
    theta[L.CNN_NP - 4 - 1152:L.CNN_NP - 4] *= 10.0 * scale_out  # a lively output layer for the comparison
    inv = [1.0 / s for s in L.CNN_STD]
    gpu = L.FluxCnn(theta, L.CNN_MEAN, inv, 0.1)
    ref = orc.Cnn(theta, L.CNN_MEAN, inv, 0.1, emulate_bf16=True)
    return gpu, ref, theta


def bf16_round(a):
    f = np.asarray(a, dtype=np.float32).copy()
    u = f.view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))
    u &= np.uint32(0xFFFF0000)
    return f.astype(np.float64)


# ragged multi-tile grids, and periodic images smaller than the fused forward's
# 22 x 22 halo region (its windows then wrap around more than once)
CASES = [((37, 21), (3, 3, 3, 3)), ((37, 21), (0, 0, 0, 0)), ((34, 18), (2, 0, 1, 1)), ((40, 17), (3, 3, 1, 1)),
         ((5, 4), (3, 3, 3, 3)), ((7, 3), (3, 3, 0, 0))]


def setup(orc, shape, bc, seed=6):
    from paper_2601_04400_amd import Grid
    nx, ny = shape
    dom = (0.0, 1.0, 0.0, ny / nx)
    inflow = (1.3, 0.7, -0.2, 1.1)
    c = orc.config(nx=nx, ny=ny, y1=dom[3], bc=bc, inflow=inflow)
    g = Grid(nx, ny, domain=dom, bc=bc, inflow=inflow, flux_net=2, adjoint=True)
    U = orc.prim_to_cons(c, inputs.smooth_prim(nx, ny, seed=seed, amp=0.3, domain=dom))
    return c, g, U


@pytest.mark.parametrize("shape,bc", CASES)
def test_input_images_vs_oracle(orc, shape, bc):
    """The network's input images (normalised conservative means of the two
    WENO5 face states, face frame; y-faces transposed; one column less along
    a periodic axis) equal the oracle's to one bfloat16 unit, on grids of
    several ragged 16 x 16 tiles."""
    c, g, U = setup(orc, shape, bc)
    net, ref, _ = make_cnn(orc, 1)
    g.set_flux_cnn(net)
    Xx, Xy = g.flux_cnn_images(torch.from_numpy(U).cuda().reshape(g.shape))
    Ox, Oy = orc.cnn_images(c, U, ref)
    for got, want in ((to_np(Xx)[0], Ox), (to_np(Xy)[0], Oy)):
        assert got.shape == want.shape
        # equal, or one bfloat16 unit apart where the double values straddle a rounding boundary
        assert np.max(np.abs(got - bf16_round(want)) / np.maximum(np.abs(want), 1e-3)) <= 1.01 * 2.0 ** -7


@pytest.mark.parametrize("shape,bc", CASES)
def test_cnn_forward_vs_oracle(orc, shape, bc):
    """Per-face correction: the oracle network on the oracle's images (the
    last face of a periodic row repeats the first), every face."""
    c, g, U = setup(orc, shape, bc)
    nx, ny = shape
    net, ref, _ = make_cnn(orc, 2)
    g.set_flux_cnn(net)
    dF = to_np(g.flux_cnn_eval(torch.from_numpy(U).cuda().reshape(g.shape)))[0].astype(np.float64)
    Ox, Oy = orc.cnn_images(c, U, ref)
    perx, pery = bc[0] == 3, bc[2] == 3
    fx = ref.forward(Ox, wrap=(pery, perx))
    fy = ref.forward(Oy, wrap=(perx, pery))
    want = np.zeros_like(dF)
    for j in range(ny):
        for fi in range(nx + 1):
            want[j * (nx + 1) + fi] = fx[j, fi % fx.shape[1]]
    base = (nx + 1) * ny
    for fj in range(ny + 1):
        for i in range(nx):
            want[base + fj * nx + i] = fy[i, fj % fy.shape[1]]
    scale = np.max(np.abs(want))
    assert scale > 1e-3
    assert np.max(np.abs(dF - want)) <= 4e-3 * scale


def face_bar(lam, dx, dy, bc):
    """Face-flux adjoint (face frame) from a right-hand-side adjoint, zero
    beyond non-periodic boundaries."""
    _, ny, nx = lam.shape
    px, py = bc[0] == 3, bc[2] == 3

    def at(j, i):
        if (i < 0 or i >= nx) and not px or (j < 0 or j >= ny) and not py:
            return np.zeros(4)
        return lam[:, j % ny, i % nx]
    out = []
    for j in range(ny):
        for f in range(nx + 1):
            d = (at(j, f) - at(j, f - 1)) / dx
            out.append(d)
    for f in range(ny + 1):
        for i in range(nx):
            d = (at(f, i) - at(f - 1, i)) / dy
            out.append(d[[0, 2, 1, 3]])
    return np.array(out)


@pytest.mark.parametrize("shape,bc", [((37, 21), (3, 3, 3, 3)), ((34, 18), (0, 0, 0, 0)), ((5, 4), (3, 3, 3, 3))])
def test_cnn_parameter_gradient_vs_oracle(orc, shape, bc):
    """Parameter gradient of the network alone (per layer block) for face
    adjoints formed from a random right-hand-side adjoint, against the
    oracle's reverse pass on its images."""
    c, g, U = setup(orc, shape, bc)
    nx, ny = shape
    net, ref, _ = make_cnn(orc, 4)
    g.set_flux_cnn(net)
    lam = np.random.default_rng(2).normal(size=U.shape)
    grad = torch.zeros(6388, dtype=torch.float32, device="cuda")
    g.flux_cnn_vjp(torch.from_numpy(U).cuda().reshape(g.shape), torch.from_numpy(lam).cuda().reshape(g.shape), grad)
    Fb = face_bar(lam, 1.0 / nx, (ny / nx) / ny, bc)
    Ox, Oy = orc.cnn_images(c, U, ref)
    perx, pery = bc[0] == 3, bc[2] == 3
    # a pixel's output adjoint: its face's (lam_right - lam_left) / h; along
    # a periodic axis the first face's wrapped difference already holds both
    # uses of the pixel (as the first and as the last face of the row)
    Dx = np.zeros_like(Ox)
    Dy = np.zeros_like(Oy)
    for j in range(ny):
        for fi in range(Ox.shape[1]):
            Dx[j, fi] = Fb[j * (nx + 1) + fi]
    base = (nx + 1) * ny
    for fj in range(Oy.shape[1]):
        for i in range(nx):
            Dy[i, fj] = Fb[base + fj * nx + i]
    gx, _ = ref.backward(Ox, Dx, wrap=(pery, perx))
    gy, _ = ref.backward(Oy, Dy, wrap=(perx, pery))
    gref = gx + gy
    gg = to_np(grad).astype(np.float64)
    for lo, hi in ((0, 576), (576, 592), (592, 5200), (5200, 5232), (5232, 6384), (6384, 6388)):
        s = np.max(np.abs(gref[lo:hi]))
        assert np.max(np.abs(gg[lo:hi] - gref[lo:hi])) <= 4e-3 * s + 1e-12, (lo, hi)


def test_zero_output_layer_gives_plain_solver(orc):
    import paper_2601_04400_amd.learn as L
    from paper_2601_04400_amd import Grid
    n = 40
    W = inputs.riemann2d_prim(n, n)
    net = L.FluxCnn(L.init_cnn_theta(1, zero_output=True))
    ga = Grid(n, n, flux_net=2)
    ga.set_flux_cnn(net)
    gb = Grid(n, n)
    Ua = ga.prim_to_cons(torch.from_numpy(W))
    Ub = gb.prim_to_cons(torch.from_numpy(W))
    for _ in range(4):
        ga.step(Ua, 1e-3)
        gb.step(Ub, 1e-3)
    np.testing.assert_array_equal(to_np(Ua), to_np(Ub))


@pytest.mark.parametrize("shape,bc", [((37, 21), (3, 3, 3, 3)), ((34, 18), (2, 0, 1, 1))])
def test_rhs_with_cnn_vs_oracle(orc, shape, bc):
    """Right-hand side with the convolutional correction against the oracle's:
    within one bfloat16 unit of what the network changes, plus FP64
    rounding; on a periodic grid the corrected scheme stays conservative."""
    c, g, U = setup(orc, shape, bc)
    net, ref, _ = make_cnn(orc, 3)
    g.set_flux_cnn(net)
    got = to_np(g.rhs(torch.from_numpy(U).cuda().reshape(g.shape)))[0]
    want = orc.rhs(c, U, net=ref)[0]
    plain = orc.rhs(c, U)[0]
    effect = np.max(np.abs(want - plain))
    assert effect > 1e-3 * np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 4e-3 * effect + 1e-11 * np.max(np.abs(want))
    if bc == (3, 3, 3, 3):
        assert np.max(np.abs(got.sum(axis=(1, 2)))) <= 1e-11 * np.max(np.abs(got)) * got[0].size


@pytest.mark.parametrize("bc", [(3, 3, 3, 3), (0, 0, 0, 0)])
def test_step_adjoint_with_cnn_vs_oracle_jacobian(orc, bc):
    """Vector-Jacobian product of one RK3 step with the convolutional
    correction (its reverse pass chained through the input images and the
    WENO5 reverse into the stencils) against the oracle's dense Jacobian,
    entry by entry: within one bfloat16 unit of the network's share (the
    reverse pass rounds its signals to bfloat16 like every product operand;
    a dot product with a random vector would magnify that by its
    cancellation)."""
    nx, ny = 16, 10
    from paper_2601_04400_amd import Grid
    dom = (0.0, 1.0, 0.0, ny / nx)
    c = orc.config(nx=nx, ny=ny, y1=dom[3], bc=bc)
    g = Grid(nx, ny, domain=dom, bc=bc, flux_net=2, adjoint=True)
    net, ref, _ = make_cnn(orc, 5)
    g.set_flux_cnn(net)
    U = orc.prim_to_cons(c, inputs.smooth_prim(nx, ny, seed=8, amp=0.3, domain=dom))
    dt = 0.4 * orc.cfl_dt(c, U)
    J = orc.rk3_step_jacobian(c, U, dt, net=ref)
    J0 = orc.rk3_step_jacobian(c, U, dt)
    lam = np.random.default_rng(3).normal(size=U.shape)
    n = U.size
    want = (J.T @ lam.ravel())[:n]
    net_part = want - (J0.T @ lam.ravel())[:n]
    assert np.max(np.abs(net_part)) > 1e-3 * np.max(np.abs(want))  # the network matters here
    Ub = torch.from_numpy(lam).cuda().reshape(g.shape).clone()
    g.step_adjoint(torch.from_numpy(U).cuda().reshape(g.shape), dt, Ub, g.param_bar())
    got = to_np(Ub).ravel()
    assert np.max(np.abs(got - want)) <= 4e-3 * np.max(np.abs(net_part)) + 1e-10 * np.max(np.abs(want))


def cylinder_case(orc, nx, ny):
    """The restricted shock-cylinder set-up of section 3 (a Mach-5 shock,
    the cylinder centred on the top symmetry edge, slip wall) at nx x ny,
    the shock moved to x = 0.5, into the body's front, so every ghost cell
    sees a moving, shocked gas."""
    from paper_2601_04400_amd import Grid, infer
    sc = infer.restricted_cylinder(nx, ny)
    sc["W"] = inputs.shock_prim(nx, ny, sc["domain"], 0.5, sc["inflow"], infer.PRE)
    dom = sc["domain"]
    c = orc.config(nx=nx, ny=ny, x0=dom[0], x1=dom[1], y0=dom[2], y1=dom[3], bc=sc["bc"], inflow=sc["inflow"])
    g = Grid(nx, ny, domain=dom, bc=sc["bc"], inflow=sc["inflow"], flux_net=2, adjoint=True, ibm=True)
    assert g.set_levelset(torch.from_numpy(sc["phi"]), wall=0) == orc.ibm_classify(c, sc["phi"])[1] > 0
    return c, g, sc, orc.prim_to_cons(c, sc["W"])


def test_rhs_with_cnn_and_body_vs_oracle(orc):
    """The convolutional correction on a grid with a body (its input images
    read the refilled ghost cells; solid and ghost cells keep a zero
    right-hand side) against the oracle's, to one bfloat16 unit of what the
    network changes."""
    c, g, sc, U = cylinder_case(orc, 48, 32)
    net, ref, _ = make_cnn(orc, 3)
    g.set_flux_cnn(net)
    Ug = torch.from_numpy(U).cuda().reshape(g.shape).contiguous()
    got = to_np(g.rhs(Ug))[0]
    assert np.array_equal(to_np(Ug)[0], U)  # the state is left as it was
    want = orc.rhs(c, U, phi=sc["phi"], wall=0, net=ref)[0]
    plain = orc.rhs(c, U, phi=sc["phi"], wall=0)[0]
    effect = np.max(np.abs(want - plain))
    assert effect > 1e-4 * np.max(np.abs(want))  # the shock's own terms reach 2e4
    err = np.max(np.abs(got - want))
    print(f"cnn + body rhs: error {err:.3e}, network effect {effect:.3e}", flush=True)
    assert err <= 4e-3 * effect + 1e-11 * np.max(np.abs(want))


def test_step_adjoint_with_cnn_and_body_vs_oracle_tangent(orc):
    """Vector-Jacobian product of one RK3 step with the convolutional
    correction on a grid with a body (the refill transpose and the network's
    reverse pass together) against the oracle, entry by entry on a sample:
    entry i of J^T lam is <lam, J e_i>, one forward-mode oracle step.  The
    sample takes every variable of ghost cells, of fluid cells next to them
    (the refill's sources) and of cells away from the body; the bar is one
    bfloat16 unit of the network's share."""
    nx, ny = 24, 16
    c, g, sc, U = cylinder_case(orc, nx, ny)
    net, ref, _ = make_cnn(orc, 5)
    g.set_flux_cnn(net)
    dt = 0.4 * orc.cfl_dt(c, U, phi=sc["phi"])
    lam = np.random.default_rng(4).normal(size=U.shape)
    Ub = torch.from_numpy(lam).cuda().reshape(g.shape).clone()
    g.step_adjoint(torch.from_numpy(U).cuda().reshape(g.shape), dt, Ub, g.param_bar())
    got = to_np(Ub)[0]
    cls = orc.ibm_classify(c, sc["phi"])[0]
    rng = np.random.default_rng(9)
    ghosts = np.argwhere(cls == 2)
    near = np.zeros_like(cls, dtype=bool)
    for j, i in ghosts:
        near[max(j - 2, 0):j + 3, max(i - 2, 0):i + 3] = True
    near &= cls == 0
    pick = [tuple(x) for x in ghosts[rng.choice(len(ghosts), 12, replace=False)]]
    pick += [tuple(x) for x in rng.permutation(np.argwhere(near))[:12]]
    pick += [tuple(x) for x in rng.permutation(np.argwhere(~near & (cls == 0)))[:4]]
    want, share, gv = [], [], []
    for (j, i) in pick:
        for v in range(4):
            e = np.zeros_like(U)
            e[v, j, i] = 1.0
            w = float(np.sum(lam * orc.rk3_step_jvp(c, U, e, dt, phi=sc["phi"], wall=0, net=ref)[1]))
            w0 = float(np.sum(lam * orc.rk3_step_jvp(c, U, e, dt, phi=sc["phi"], wall=0)[1]))
            want.append(w)
            share.append(w - w0)
            gv.append(got[v, j, i])
    want, share, gv = np.array(want), np.array(share), np.array(gv)
    assert np.max(np.abs(share)) > 1e-3 * np.max(np.abs(want))
    err = np.max(np.abs(gv - want))
    print(f"cnn + body step adjoint: {len(want)} entries, error {err:.3e}, "
          f"network share {np.max(np.abs(share)):.3e}", flush=True)
    assert err <= 4e-3 * np.max(np.abs(share)) + 1e-10 * np.max(np.abs(want))


def test_cnn_training_reduces_loss_and_beats_plain_solver():
    """Reduced convolutional training run: 16 random Riemann problems on
    64 x 32 against 128 x 64 restricted 2 x 2, m = 8 unrolled steps, the
    output layer starting at zero.  The unrolled training loss falls and on
    8 held-out problems the corrected solver ends closer to the restricted
    fine solution than the uncorrected one."""
    import paper_2601_04400_amd.learn as L
    data = L.Dataset(list(range(16)), nc=64, ny=32, factor=2, nsnap=12)
    net = L.FluxCnn(L.init_cnn_theta(0, zero_output=True))
    before = L.dataset_loss(net, data, m=4)
    L.train(net, data, iters=300, m=8, lr=1e-3, log_every=50, log=lambda s: print(s, flush=True))
    after = L.dataset_loss(net, data, m=4)
    print("cnn training-set loss", before, after, flush=True)
    assert after < before
    ev = L.evaluate(net, list(range(1000, 1008)), nc=64, ny=32, factor=2, nsteps=12)
    print(ev, flush=True)
    assert ev["learned"]["mse"] < ev["plain"]["mse"]


def test_cylinder_learned_flux_case_runs_and_zero_output_is_plain():
    """The shock-cylinder learned-flux data set (coarse 32 x 16 against
    64 x 32 restricted 2 x 2, both with the body, fixed steps to t = 0.2):
    the step count lands on t = 0.2 within the CFL bound, the snapshots
    stay finite, and a network whose output layer is zero (a zero correction)
    reproduces the uncorrected coarse run exactly in the evaluation."""
    import paper_2601_04400_amd.learn as L
    data = L.Dataset(None, nc=32, factor=2, case="cylinder", t_end=0.2, cfl_frac=0.5)
    assert (data.nx, data.ny) == (32, 16)
    assert abs(float(data.dt_c[0]) * data.nsnap - 0.2) < 1e-12
    assert bool(torch.isfinite(data.snaps).all())
    mean, inv = L.cnn_norm_from(data)
    net = L.FluxCnn(L.init_cnn_theta(0, zero_output=True), mean, inv, out_scale=0.1)
    ev = L.evaluate_cylinder(net, data)
    print(ev, flush=True)
    for t in ev["plain"]["errors"]:
        assert ev["learned"]["errors"][t] == ev["plain"]["errors"][t]
        assert np.isfinite(ev["plain"]["errors"][t]["mse_fluid"])


def test_graph_replays_with_cnn_equal_eager_steps(orc):
    """Automatic-step RK3 steps with the convolutional correction captured in
    a HIP graph (network forward and corrected stage per stage, no memory
    fills): every replay, with eager work and synchronisations between the
    replays, gives the eager steps' state bit for bit."""
    from paper_2601_04400_amd import Grid
    n, k = 48, 4
    net, _, _ = make_cnn(orc, 5)
    g = Grid(n, n, flux_net=2)
    g.set_flux_cnn(net)
    U0 = g.prim_to_cons(torch.from_numpy(inputs.riemann2d_prim(n, n)))
    Ue = U0.clone()
    g.set_time(0.0, 1e30)
    for _ in range(k):
        g.step(Ue)
    want = to_np(Ue)
    U = U0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g.set_time(0.0, 1e30)
        g.step(U)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(k):
            g.step(U)
    for rep in range(3):
        U.copy_(U0)
        g.set_time(0.0, 1e30)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(U), want, err_msg=f"replay {rep}")
        Ue.mul_(1.0)  # eager work between replays


def test_cnn_forward_full_size_training_batch(orc):
    """The convolutional workload at full size: 64 random four-quadrant
    problems at 128 x 64 (the training batch) in one launch; the per-face
    corrections of members 0 and 63 against the oracle network on the
    oracle's images."""
    import paper_2601_04400_amd.learn as L
    from paper_2601_04400_amd import Grid
    nx, ny, nb = 128, 64, 64
    dom = (0.0, 1.0, 0.0, ny / nx)
    W = L.riemann_batch(list(range(nb)), nx, "cpu", ny=ny).numpy()
    c = orc.config(nx=nx, ny=ny, y1=dom[3])
    g = Grid(nx, ny, nbatch=nb, domain=dom, flux_net=2)
    net, ref, _ = make_cnn(orc, 3)
    g.set_flux_cnn(net)
    U = np.stack([orc.prim_to_cons(c, W[b]) for b in range(nb)])
    dF = to_np(g.flux_cnn_eval(torch.from_numpy(U).cuda().reshape(g.shape))).astype(np.float64)
    for b in (0, nb - 1):
        Ox, Oy = orc.cnn_images(c, U[b], ref)
        fx = ref.forward(Ox, wrap=(False, False))
        fy = ref.forward(Oy, wrap=(False, False))
        want = np.concatenate([fx.reshape(-1, 4), np.transpose(fy, (1, 0, 2)).reshape(-1, 4)])
        scale = np.max(np.abs(want))
        assert scale > 1e-3
        assert np.max(np.abs(dF[b] - want)) <= 4e-3 * scale, b
