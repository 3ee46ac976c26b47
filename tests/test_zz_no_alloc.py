"""The allocation-free unrolled-loss entry point (shk_mse_noalloc, for
callers that cannot allocate memory) against shk_mse with a caller buffer:
the same kernels, so the loss and the gradient must agree bit for bit, on two
calls in a row (the second smaller, so the static partials hold the first
call's values where the second does not write), and sizes past the static
array's limit are rejected."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _call_both(lib, nbatch, per, seed):
    rng = np.random.default_rng(seed)
    U = torch.from_numpy(rng.normal(size=(nbatch, per))).cuda()
    T = torch.from_numpy(rng.normal(size=(nbatch, per))).cuda()
    G0 = rng.normal(size=(nbatch, per))
    l0 = rng.uniform(size=nbatch)
    G_a, G_b = torch.from_numpy(G0.copy()).cuda(), torch.from_numpy(G0.copy()).cuda()
    l_a, l_b = torch.from_numpy(l0.copy()).cuda(), torch.from_numpy(l0.copy()).cuda()
    part = torch.empty(nbatch * 256, dtype=torch.float64, device="cuda")
    assert lib.shk_mse(_p(U), _p(T), _p(G_a), 0.5, per, nbatch, _p(part), _p(l_a), _stream()) == 0
    assert lib.shk_mse_noalloc(_p(U), _p(T), _p(G_b), 0.5, per, nbatch, _p(l_b), _stream()) == 0
    torch.cuda.synchronize()
    return (l_a.cpu().numpy(), G_a.cpu().numpy()), (l_b.cpu().numpy(), G_b.cpu().numpy())


def test_mse_noalloc_matches_mse_twice():
    from paper_2601_04400_amd._lib import lib
    L = lib()
    # first call: 200 members of 65536 entries (256 partials each); second:
    # 3 members of 1000 entries (4 partials each)
    for nbatch, per, seed in ((200, 65536, 1), (3, 1000, 2)):
        print(f"mse_noalloc nbatch={nbatch} per={per}", flush=True)
        (la, Ga), (lb, Gb) = _call_both(L, nbatch, per, seed)
        assert np.array_equal(la, lb), (la - lb)
        assert np.array_equal(Ga, Gb)


def test_mse_noalloc_rejects_sizes_beyond_limit():
    from paper_2601_04400_amd._lib import lib
    L = lib()
    U = torch.zeros(257 * 4, dtype=torch.float64, device="cuda")
    loss = torch.zeros(257, dtype=torch.float64, device="cuda")
    assert L.shk_mse_noalloc(_p(U), _p(U), None, 1.0, 4, 257, _p(loss), _stream()) == 1
    assert L.shk_mse_noalloc(_p(U), _p(U), None, 1.0, 4, 0, _p(loss), _stream()) == 1
    assert L.shk_mse_noalloc(_p(U), None, None, 1.0, 4, 1, _p(loss), _stream()) == 1
    torch.cuda.synchronize()
    assert float(loss.abs().sum()) == 0.0
