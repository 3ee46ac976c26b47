"""Host-side checks of the C ABI: the library loads, exports every symbol
declared in include/shk.h, and validates arguments before touching the GPU
(no compute call is made here)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "shk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(shk_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_2601_04400_amd import _lib
    return _lib.lib()


def test_library_exports_every_declared_symbol(L):
    from paper_2601_04400_amd import _lib
    decl = declared_symbols()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTS) == decl


def desc(**kw):
    from paper_2601_04400_amd._lib import GridDesc
    d = GridDesc()
    d.ndim, d.nx, d.ny, d.nbatch = 2, 64, 32, 1
    d.x0, d.x1, d.y0, d.y1 = 0.0, 1.0, 0.0, 0.5
    d.prec, d.gamma, d.cfl, d.weno_eps = 0, 1.4, 0.5, 1e-6
    d.prandtl = 0.72
    for k, v in kw.items():
        if k == "bc":
            for i in range(4):
                d.bc[i] = v[i]
        else:
            setattr(d, k, v)
    return d


def test_workspace_bytes_validates_descriptor(L):
    good = L.shk_workspace_bytes(ctypes.byref(desc()))
    # two state copies of 4 x 64 x 32 doubles at least
    assert good >= 2 * 4 * 64 * 32 * 8
    assert L.shk_workspace_bytes(ctypes.byref(desc(prec=1))) < good
    assert L.shk_workspace_bytes(ctypes.byref(desc(ibm=1))) > good
    for bad in (dict(ndim=3), dict(nx=0), dict(nx=2), dict(ny=2), dict(ndim=1, ny=1, nx=2), dict(gamma=1.0),
                dict(ndim=1, ny=4), dict(prec=7),
                dict(bc=(3, 0, 0, 0)), dict(viscous=1, ndim=1, ny=1), dict(x1=-1.0), dict(cfl=0.0)):
        assert L.shk_workspace_bytes(ctypes.byref(desc(**bad))) == 0, bad
    assert L.shk_workspace_bytes(None) == 0


def test_init_rejects_bad_arguments_without_gpu(L):
    h = ctypes.c_void_p()
    d = desc()
    n = L.shk_workspace_bytes(ctypes.byref(d))
    assert L.shk_init_grid(ctypes.byref(d), None, n, None, ctypes.byref(h)) == 1      # null workspace
    assert L.shk_init_grid(ctypes.byref(desc(nx=0)), ctypes.c_void_p(256), n, None, ctypes.byref(h)) == 1
    assert L.shk_init_grid(ctypes.byref(d), ctypes.c_void_p(256), n - 1, None, ctypes.byref(h)) == 6  # ESPACE
    assert L.shk_init_grid(ctypes.byref(d), ctypes.c_void_p(257), n, None, ctypes.byref(h)) == 1      # misaligned
    assert L.shk_init_grid(ctypes.byref(d), ctypes.c_void_p(256), n, None, None) == 1
    for fn, args in (("shk_rhs", (None, None, None)), ("shk_rk3_step", (None, None, None, None)),
                     ("shk_set_ib_levelset", (None, None, 0)), ("shk_poll_faults", (None, None, None))):
        assert getattr(L, fn)(*args) == 1
    assert L.shk_status_string(6) == b"SHK_ESPACE"


def test_normal_shock_state_host_function(orc):
    from paper_2601_04400_amd import normal_shock_state
    for M, g in ((5.0, 1.4), (3.0, 1.4), (2.8, 1.3), (3.0, 5.0 / 3.0)):
        out, dM, dg = normal_shock_state(M, g)
        ref = orc.rh_post_shock(M, g)
        for k in range(3):
            assert abs(out[k] - ref[k]) <= 4e-16 * abs(ref[k]) + 1e-300
        h = 1e-6
        fm = [normal_shock_state(M + s * h, g)[0] for s in (1, -1)]
        fg = [normal_shock_state(M, g + s * h)[0] for s in (1, -1)]
        for k in range(3):
            assert math.isclose((fm[0][k] - fm[1][k]) / (2 * h), dM[k], rel_tol=1e-8, abs_tol=1e-9)
            assert math.isclose((fg[0][k] - fg[1][k]) / (2 * h), dg[k], rel_tol=1e-8, abs_tol=1e-9)
