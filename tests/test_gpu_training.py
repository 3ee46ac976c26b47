"""GPU training pieces of the learned correction (section 2: the restriction
d(U) of fine data, the unrolled-loss term and its gradient; section 3: Adam)
against the oracle's double-precision versions, through the C ABI.

Tolerances:
  - restriction: bit-exact (both sides sum a block row by row, then divide by
    factor^2 in double);
  - loss: 1e-13 relative (the GPU sums in a different fixed order);
    gradient: 1e-15 relative (one rounding of the product order);
  - Adam: the GPU runs in FP32 on FP32 parameters, the oracle in double on
    the same FP32 values, so theta, m and v agree to a few FP32 units:
    2e-6 relative to |theta| + |update| (the update is evaluated in FP32),
    to |v| and, for m (whose two terms can cancel), to |b1 m| + |(1 - b1) g|.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("shape,factor", [((3, 4, 40, 56), 2), ((2, 4, 64, 48), 4), ((1, 3, 12, 9), 3),
                                          ((64, 4, 16, 16), 4)])
def test_restrict_vs_oracle(orc, shape, factor):
    from paper_2601_04400_amd._lib import lib
    rng = np.random.default_rng(7)
    fine = rng.uniform(-2.0, 3.0, size=shape)
    nb, nv, ny, nx = shape
    f = torch.from_numpy(fine).cuda()
    out = torch.full((nb, nv, ny // factor, nx // factor), np.nan, dtype=torch.float64, device="cuda")
    assert lib().shk_restrict(_p(f), _p(out), nx, ny, factor, nv, nb, _stream()) == 0
    torch.cuda.synchronize()
    ref = orc.restrict(fine, factor)
    got = out.cpu().numpy()
    print(f"restrict {shape} /{factor}: max diff {np.max(np.abs(got - ref)):.3e}", flush=True)
    assert np.array_equal(got, ref)


def test_restrict_rejects_bad_sizes():
    from paper_2601_04400_amd._lib import lib
    f = torch.zeros(1, 4, 10, 12, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, 4, 3, 3, dtype=torch.float64, device="cuda")
    assert lib().shk_restrict(_p(f), _p(out), 12, 10, 4, 4, 1, _stream()) == 1  # 10 not a multiple of 4
    assert lib().shk_restrict(_p(f), _p(out), 12, 10, 0, 4, 1, _stream()) == 1


@pytest.mark.parametrize("nbatch,per", [(1, 1000), (3, 4 * 37 * 21), (64, 4 * 128 * 2), (65, 333), (128, 4 * 64),
                                        (5, 4 * 512 * 300)])
def test_mse_vs_oracle(orc, nbatch, per):
    from paper_2601_04400_amd._lib import lib
    rng = np.random.default_rng(nbatch * 1000 + per % 997)
    U = rng.normal(size=(nbatch, per))
    T = U + rng.normal(scale=0.3, size=(nbatch, per))
    G0 = rng.normal(size=(nbatch, per))
    loss0 = rng.uniform(size=nbatch)
    scale = 0.37
    Ud, Td = torch.from_numpy(U).cuda(), torch.from_numpy(T).cuda()
    Gd, lossd = torch.from_numpy(G0.copy()).cuda(), torch.from_numpy(loss0.copy()).cuda()
    part = torch.empty(nbatch * 256, dtype=torch.float64, device="cuda")
    assert lib().shk_mse(_p(Ud), _p(Td), _p(Gd), scale, per, nbatch, _p(part), _p(lossd), _stream()) == 0
    # a second call without the gradient accumulates the loss again
    assert lib().shk_mse(_p(Ud), _p(Td), None, scale, per, nbatch, _p(part), _p(lossd), _stream()) == 0
    torch.cuda.synchronize()
    l_ref, g_ref = orc.mse(U, T, scale=scale, nbatch=nbatch)
    want_loss = loss0 + 2.0 * l_ref
    want_G = G0 + g_ref
    got_loss, got_G = lossd.cpu().numpy(), Gd.cpu().numpy()
    el = np.max(np.abs(got_loss - want_loss) / np.abs(want_loss))
    eg = np.max(np.abs(got_G - want_G)) / np.max(np.abs(want_G))
    print(f"mse nbatch={nbatch} per={per}: loss rel {el:.3e}, grad rel {eg:.3e}", flush=True)
    assert el <= 1e-13
    assert eg <= 1e-15


def test_mse_rejects_bad_sizes():
    from paper_2601_04400_amd._lib import lib
    U = torch.zeros(10, dtype=torch.float64, device="cuda")
    part = torch.zeros(256, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert lib().shk_mse(_p(U), _p(U), None, 1.0, 0, 1, _p(part), _p(loss), _stream()) == 1
    assert lib().shk_mse(_p(U), _p(U), None, 1.0, 10, 0, _p(part), _p(loss), _stream()) == 1
    assert lib().shk_mse(_p(U), _p(U), None, 1.0, 10, 1, None, _p(loss), _stream()) == 1


@pytest.mark.parametrize("n", [1, 255, 10180, 6388])
def test_adam_vs_oracle(orc, n):
    from paper_2601_04400_amd._lib import lib
    rng = np.random.default_rng(n)
    theta = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    th_d, m_d, v_d = (torch.from_numpy(a.copy()).cuda() for a in (theta, m, v))
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    for step in range(1, 13):
        g = (rng.normal(size=n) * (10.0 ** rng.uniform(-6, 1, size=n))).astype(np.float32)
        if step == 5:
            g[: max(1, n // 7)] = 0.0  # zero gradients: only the moments' decay moves the parameter
        g_d = torch.from_numpy(g).cuda()
        assert lib().shk_adam(_p(th_d), _p(g_d), _p(m_d), _p(v_d), n, lr, b1, b2, eps, step, _stream()) == 0
        torch.cuda.synchronize()
        # the oracle runs one step in double from the GPU's FP32 state before the step,
        # with the hyperparameters the ABI passes as FP32 (1 - 0.999f differs from
        # 1 - 0.999 by 1.3e-5 relative)
        f32 = lambda x: float(np.float32(x))
        th_ref, m_ref, v_ref = orc.adam(theta, g, m, v, f32(lr), step, f32(b1), f32(b2), f32(eps))
        th_got, m_got, v_got = (t.cpu().numpy().astype(np.float64) for t in (th_d, m_d, v_d))
        # m = b1 m + (1 - b1) g can cancel, so its error is measured against the
        # size of the two terms; v adds two non-negative terms
        m_scale = np.abs(f32(b1) * m.astype(np.float64)) + np.abs((1.0 - f32(b1)) * g.astype(np.float64))
        # theta - lr mhat / (sqrt(vhat) + eps) in FP32: a few units of the
        # update's size plus one rounding of the result
        th_scale = np.abs(th_ref) + np.abs(theta.astype(np.float64) - th_ref)
        for name, got, ref, scale in (("theta", th_got, th_ref, np.maximum(th_scale, 1e-30)),
                                      ("m", m_got, m_ref, np.maximum(m_scale, 1e-30)),
                                      ("v", v_got, v_ref, np.maximum(np.abs(v_ref), 1e-30))):
            err = np.max(np.abs(got - ref) / scale)
            assert err <= 2e-6, f"adam step {step} n={n}: {name} rel error {err:.3e}"
        theta, m, v = (t.cpu().numpy() for t in (th_d, m_d, v_d))
    print(f"adam n={n}: 12 steps within 2e-6", flush=True)
