"""GPU characteristic-wise WENO5 (the reconstruction variant the paper leaves
open: WENO on the characteristic fields of the face-normal flux Jacobian at
the Roe average of the two adjacent cells) against the oracle's, FP64.

Tolerances (per conserved field, max|x - o| / max|o|): one right-hand side
1e-12 (the projection and back-projection add rounding to the primitive-wise
path's 1e-13), trajectories 1e-11 (the target bound)."""
import numpy as np
import pytest

from paper_2601_04400_amd import inputs
from gpu_util import assert_fields, make_pair

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def to_gpu(g, U):
    return torch.from_numpy(np.ascontiguousarray(U)).to(device=g.device, dtype=g.dtype).reshape(g.shape)


def to_np(U):
    torch.cuda.synchronize()
    return U.detach().to("cpu", torch.float64).numpy()


@pytest.mark.parametrize("shape", [(37, 29), (70, 17)])
@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (3, 3, 3, 3), (2, 0, 1, 1), (2, 1, 3, 3)])
def test_rhs_char_f64(orc, shape, bc):
    nx, ny = shape
    inflow = (1.3, 0.7, -0.2, 1.1)
    c, g = make_pair(orc, nx, ny, bc=bc, inflow=inflow, domain=(0.0, 1.0, 0.0, ny / nx), weno_char=True)
    Uo = orc.prim_to_cons(c, inputs.random_prim(nx, ny, seed=nx * 7 + ny))
    Lo, _, fbo = orc.rhs(c, Uo)
    Lg = to_np(g.rhs(to_gpu(g, Uo)))[0]
    assert_fields(Lg, Lo, 1e-12, f"rhs char {shape} {bc}")
    assert g.poll_faults()[1] == fbo
    # the variant differs from the primitive-wise reconstruction
    cp, _ = make_pair(orc, nx, ny, bc=bc, inflow=inflow, domain=(0.0, 1.0, 0.0, ny / nx))
    assert np.max(np.abs(orc.rhs(cp, Uo)[0] - Lo)) > 1e-3 * np.max(np.abs(Lo))


def test_rhs_char_1d_and_viscous(orc):
    for nx, bc in ((200, (0, 0, 0, 0)), (301, (1, 2, 0, 0)), (64, (3, 3, 0, 0))):
        c, g = make_pair(orc, nx, ndim=1, bc=bc, inflow=(1.2, 0.3, 0.0, 1.5), weno_char=True)
        Uo = orc.prim_to_cons(c, inputs.random_prim(nx, 1, seed=nx, ndim=1))
        Lg = to_np(g.rhs(to_gpu(g, Uo)))[0]
        assert_fields(Lg, orc.rhs(c, Uo)[0], 1e-12, f"rhs char 1d {nx} {bc}")
    nx, ny = 45, 33
    c, g = make_pair(orc, nx, ny, bc=(2, 0, 1, 1), inflow=(1.3, 0.7, -0.2, 1.1), viscous=True, mu=0.01,
                     domain=(0.0, 1.0, 0.0, ny / nx), weno_char=True)
    Uo = orc.prim_to_cons(c, inputs.smooth_prim(nx, ny, seed=5, amp=0.3, domain=(0.0, 1.0, 0.0, ny / nx)))
    Lg = to_np(g.rhs(to_gpu(g, Uo)))[0]
    assert_fields(Lg, orc.rhs(c, Uo)[0], 1e-12, "rhs char viscous")


def test_sod_char_trajectory(orc):
    """Sod, 200 cells, CFL 0.5 to t = 0.2 with the characteristic variant:
    identical step count and end time, per-field error within 1e-11."""
    n = 200
    c, g = make_pair(orc, n, ndim=1, weno_char=True)
    W = inputs.sod_prim(n)
    Uo = orc.prim_to_cons(c, W)
    Ue, te, steps_o, fbo = orc.run(c, Uo, 0.2)
    Ug = g.prim_to_cons(torch.from_numpy(W))
    tg, steps_g = g.advance(Ug, 0.2)
    assert steps_g == steps_o and tg == te == 0.2
    assert_fields(to_np(Ug)[0], Ue, 1e-11, "sod char")


def test_riemann2d_char_trajectory(orc):
    """Four-quadrant problem, 64 x 48, 20 automatic steps (the fused
    step sequence) with the characteristic variant, per-field error within
    1e-11."""
    nx, ny = 64, 48
    dom = (0.0, 1.0, 0.0, ny / nx)
    c, g = make_pair(orc, nx, ny, domain=dom, weno_char=True)
    W = inputs.riemann2d_prim(nx, ny, split=(0.5, 0.5 * ny / nx), domain=dom)
    Uo = orc.prim_to_cons(c, W)
    Ue, te, steps_o, _ = orc.run(c, Uo, 10.0, max_steps=20)
    Ug = g.prim_to_cons(torch.from_numpy(W))
    g.set_time(0.0, 10.0)
    for _ in range(20):
        g.step(Ug)
    assert_fields(to_np(Ug)[0], Ue, 1e-11, "riemann2d char")


def test_char_rejects_what_it_does_not_support():
    from paper_2601_04400_amd import Grid
    for kw in (dict(prec="f32"), dict(adjoint=True), dict(flux_net=True)):
        with pytest.raises(Exception):
            Grid(32, 16, weno_char=True, **kw)


def test_char_full_size_step(orc):
    """512^2 four-quadrant problem (the size `bench.py --weno char` times):
    one right-hand side and one automatic step against the oracle."""
    n = 512
    c, g = make_pair(orc, n, n, weno_char=True)
    W = inputs.riemann2d_prim(n, n)
    Uo = orc.prim_to_cons(c, W)
    Ug = g.prim_to_cons(torch.from_numpy(W))
    Lo, _, _ = orc.rhs(c, Uo)
    assert_fields(to_np(g.rhs(Ug.clone()))[0], Lo, 1e-12, "512^2 char rhs")
    dto = orc.cfl_dt(c, Uo)
    U1o, _ = orc.rk3_step(c, Uo, dto)
    dts = torch.zeros(1, dtype=torch.float64, device=g.device)
    g.set_time(0.0, 1.0)
    g.step(Ug, dt_out=dts)
    assert float(dts.cpu()[0]) == dto
    assert_fields(to_np(Ug)[0], U1o, 1e-12, "512^2 char step")
