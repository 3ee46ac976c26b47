"""Oracle: a plain serial FP64 CPU implementation of the WENO5 / HLLC /
immersed-boundary / SSP-RK3 path, used ONLY as test infrastructure.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may load it.  It shares no code with the GPU library; the C++ sources
next to this file cite the part of the paper each function follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_p = ctypes.c_void_p


class Config(ctypes.Structure):
    _fields_ = [
        ("ndim", _i), ("nx", _i), ("ny", _i),
        ("x0", _d), ("x1", _d), ("y0", _d), ("y1", _d),
        ("gamma", _d), ("cfl", _d), ("weno_eps", _d),
        ("viscous", _i), ("mu", _d), ("prandtl", _d), ("nu_art", _d),
        ("bc", _i * 4), ("inflow", _d * 4), ("weno_char", _i),
    ]


TRANSMISSIVE, REFLECTIVE, INFLOW, PERIODIC = 0, 1, 2, 3


def lib():
    global _lib
    if _lib is None:
        if _build.needs_build():
            _build.build()
        _lib = ctypes.CDLL(_build.LIB)
        _lib.orc_cfl_dt.restype = _d
        _lib.orc_weno5_left.restype = _d
        _lib.orc_net_create.restype = _p
        _lib.orc_net_create.argtypes = [_p, _p, _p, _d, _i]
        _lib.orc_net_destroy.argtypes = [_p]
        _lib.orc_net_forward.argtypes = [_p, _i, _p, _p]
        _lib.orc_net_backward.argtypes = [_p, _i, _p, _p, _p, _p]
        _lib.orc_cnn_create.restype = _p
        _lib.orc_cnn_create.argtypes = [_p, _p, _p, _d, _i]
        _lib.orc_cnn_destroy.argtypes = [_p]
        _lib.orc_cnn_forward.argtypes = [_p, _i, _i, _i, _i, _p, _p]
        _lib.orc_cnn_backward.argtypes = [_p, _i, _i, _i, _i, _p, _p, _p, _p]
        _lib.orc_cnn_images.argtypes = [_p, _p, _p, _i, _p, _p, _p]
        _lib.orc_char_basis.argtypes = [_d, _p, _p, _p, _p]
        _lib.orc_threads.argtypes = [_i]
        _lib.orc_threads.restype = _i
    return _lib


def threads(n=0):
    """Set (n >= 1) and return the oracle's OpenMP thread count."""
    return lib().orc_threads(int(n))


def config(ndim=2, nx=64, ny=64, x0=0.0, x1=1.0, y0=0.0, y1=1.0, gamma=1.4, cfl=0.5,
           weno_eps=1e-6, viscous=0, mu=0.0, prandtl=0.72, nu_art=0.0,
           bc=(0, 0, 0, 0), inflow=(1.0, 0.0, 0.0, 1.0), weno_char=0):
    c = Config()
    c.ndim, c.nx, c.ny = ndim, nx, (1 if ndim == 1 else ny)
    c.x0, c.x1, c.y0, c.y1 = x0, x1, y0, y1
    c.gamma, c.cfl, c.weno_eps = gamma, cfl, weno_eps
    c.viscous, c.mu, c.prandtl, c.nu_art = viscous, mu, prandtl, nu_art
    for k in range(4):
        c.bc[k] = bc[k]
        c.inflow[k] = inflow[k]
    c.weno_char = int(weno_char)
    return c


def _nvar(c):
    return 3 if c.ndim == 1 else 4


def _arr(x, shape=None):
    a = np.ascontiguousarray(x, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_p)


def _shape(c):
    return (_nvar(c), c.ny, c.nx)


def prim_to_cons(c, W):
    W = _arr(W, _shape(c))
    U = np.empty_like(W)
    assert lib().orc_prim_to_cons(ctypes.byref(c), _ptr(W), _ptr(U)) == 0
    return U


def cons_to_prim(c, U):
    U = _arr(U, _shape(c))
    W = np.empty_like(U)
    assert lib().orc_cons_to_prim(ctypes.byref(c), _ptr(U), _ptr(W)) == 0
    return W


def _phi(c, phi):
    return None if phi is None else _arr(phi, (c.ny, c.nx))


def rhs(c, U, phi=None, wall=0, net=None):
    """Return (dU/dt, U with IBM ghosts filled, positivity-fallback count)."""
    U = _arr(U, _shape(c))
    L = np.empty_like(U)
    Uf = np.empty_like(U)
    fb = ctypes.c_long(0)
    phi = _phi(c, phi)
    rc = lib().orc_rhs(ctypes.byref(c), _ptr(U), _ptr(L), _ptr(phi), _i(wall),
                       _p(net.handle) if net else None, _ptr(Uf), ctypes.byref(fb))
    assert rc == 0
    return L, Uf, fb.value


def rk3_step(c, U, dt, phi=None, wall=0, net=None):
    U = _arr(U, _shape(c)).copy()
    fb = ctypes.c_long(0)
    phi = _phi(c, phi)
    rc = lib().orc_rk3_step(ctypes.byref(c), _ptr(U), _d(dt), _ptr(phi), _i(wall),
                            _p(net.handle) if net else None, ctypes.byref(fb))
    assert rc == 0
    return U, fb.value


def cfl_dt(c, U, phi=None, wall=0):
    U = _arr(U, _shape(c))
    phi = _phi(c, phi)
    return lib().orc_cfl_dt(ctypes.byref(c), _ptr(U), _ptr(phi), _i(wall))


def run(c, U, t_end, t0=0.0, max_steps=10 ** 9, phi=None, wall=0, net=None):
    """Advance to t_end with CFL steps. Returns (U, t, steps, fallback count)."""
    U = _arr(U, _shape(c)).copy()
    t = _d(0.0)
    steps = _i(0)
    fb = ctypes.c_long(0)
    phi = _phi(c, phi)
    rc = lib().orc_run(ctypes.byref(c), _ptr(U), _d(t0), _d(t_end), _i(int(min(max_steps, 2 ** 31 - 1))),
                       _ptr(phi), _i(wall), _p(net.handle) if net else None,
                       ctypes.byref(t), ctypes.byref(steps), ctypes.byref(fb))
    assert rc == 0
    return U, t.value, steps.value, fb.value


def weno5_left(f5, eps=1e-6):
    f5 = _arr(f5, (5,))
    return lib().orc_weno5_left(_ptr(f5), _d(eps))


def hllc_x(WL, WR, gamma=1.4):
    WL, WR = _arr(WL, (4,)), _arr(WR, (4,))
    F = np.empty(4)
    lib().orc_hllc_x(_ptr(WL), _ptr(WR), _d(gamma), _ptr(F))
    return F


def riemann_star(left, right, gamma=1.4):
    out = np.empty(4)
    it = _i(0)
    lib().orc_riemann_star(*[_d(v) for v in (*left, *right, gamma)], _ptr(out), ctypes.byref(it))
    return dict(p=out[0], u=out[1], rhoL=out[2], rhoR=out[3], iterations=it.value)


def riemann_sample(left, right, x, t, xd=0.5, gamma=1.4):
    x = _arr(x)
    r, u, p = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    lib().orc_riemann_sample(*[_d(v) for v in (*left, *right, gamma, xd, t)], _i(x.size),
                             _ptr(x), _ptr(r), _ptr(u), _ptr(p))
    return r, u, p


def rh_post_shock(mach, gamma=1.4, rho1=1.4, p1=1.0):
    out = np.empty(3)
    lib().orc_rh_post_shock(_d(mach), _d(gamma), _d(rho1), _d(p1), _ptr(out))
    return out


def ibm_classify(c, phi):
    phi = _phi(c, phi)
    cls = np.empty((c.ny, c.nx), dtype=np.uint8)
    n = lib().orc_ibm_classify(ctypes.byref(c), _ptr(phi), cls.ctypes.data_as(_p))
    assert n >= 0
    return cls, n


def ibm_ghosts(c, phi):
    phi = _phi(c, phi)
    cap = c.nx * c.ny
    ij = np.empty((cap, 2), dtype=np.int32)
    nrm = np.empty((cap, 2))
    src = np.empty((cap, 4), dtype=np.int32)
    w = np.empty((cap, 4))
    n = lib().orc_ibm_ghosts(ctypes.byref(c), _ptr(phi), _i(cap), ij.ctypes.data_as(_p), _ptr(nrm),
                             src.ctypes.data_as(_p), _ptr(w))
    return dict(ij=ij[:n], normal=nrm[:n], src=src[:n], w=w[:n])


def ibm_degenerate(c, phi):
    """Number of ghosts whose image point is undefined (vanishing grad phi or
    no fluid cell to interpolate from)."""
    return lib().orc_ibm_degenerate(ctypes.byref(c), _ptr(_phi(c, phi)))


def ibm_fill(c, U, phi, wall=0):
    U = _arr(U, _shape(c)).copy()
    assert lib().orc_ibm_fill(ctypes.byref(c), _ptr(U), _ptr(_phi(c, phi)), _i(wall)) == 0
    return U


def rhs_jvp(c, U, Udot, gdot=0.0, indot=(0, 0, 0, 0), phi=None, wall=0, net=None):
    U, Udot = _arr(U, _shape(c)), _arr(Udot, _shape(c))
    L, Ld = np.empty_like(U), np.empty_like(U)
    ind = _arr(indot, (4,))
    rc = lib().orc_rhs_jvp(ctypes.byref(c), _ptr(U), _ptr(Udot), _d(gdot), _ptr(ind), _ptr(_phi(c, phi)),
                           _i(wall), _ptr(L), _ptr(Ld), _net(net))
    assert rc == 0
    return L, Ld


def _net(net):
    return _p(net.handle) if net is not None else None


def rhs_jacobian(c, U, phi=None, wall=0, net=None):
    """Dense Jacobian of the RHS (small grids): columns = state entries, then
    gamma and the inflow primitives (rho, u, v, p)."""
    U = _arr(U, _shape(c))
    n = U.size
    J = np.empty((n, n + 5))
    assert lib().orc_rhs_jacobian(ctypes.byref(c), _ptr(U), _ptr(_phi(c, phi)), _i(wall), _ptr(J), _net(net)) == 0
    return J


def rk3_step_jacobian(c, U, dt, phi=None, wall=0, net=None):
    """Dense Jacobian of one fixed-dt RK3 step (small grids), columns as in
    rhs_jacobian."""
    U = _arr(U, _shape(c))
    n = U.size
    J = np.empty((n, n + 5))
    assert lib().orc_rk3_step_jacobian(ctypes.byref(c), _ptr(U), _d(dt), _ptr(_phi(c, phi)), _i(wall),
                                       _ptr(J), _net(net)) == 0
    return J


def rk3_step_jvp(c, U, Udot, dt, gdot=0.0, indot=(0, 0, 0, 0), phi=None, wall=0, net=None):
    U, Udot = _arr(U, _shape(c)).copy(), _arr(Udot, _shape(c)).copy()
    ind = _arr(indot, (4,))
    rc = lib().orc_rk3_step_jvp(ctypes.byref(c), _ptr(U), _ptr(Udot), _d(dt), _d(gdot), _ptr(ind),
                                _ptr(_phi(c, phi)), _i(wall), _net(net))
    assert rc == 0
    return U, Udot


def shock_tangent(c, phi, mach, xs, nsteps, dt, target_rho, wall=0, rho1=1.4, p1=1.0):
    """J = mean_fluid (rho - target)^2 after nsteps; returns (J, dJ/dM, dJ/dgamma, U)."""
    J = _d(0.0)
    dJ = np.empty(2)
    U = np.empty((4, c.ny, c.nx))
    tgt = _arr(target_rho, (c.ny, c.nx))
    rc = lib().orc_shock_tangent(ctypes.byref(c), _ptr(_phi(c, phi)), _i(wall), _d(mach), _d(xs),
                                 _d(rho1), _d(p1), _i(nsteps), _d(dt), _ptr(tgt), ctypes.byref(J),
                                 _ptr(dJ), _ptr(U))
    assert rc == 0
    return J.value, dJ[0], dJ[1], U


NET_PARAMS = 10180


class Net:
    """The learned face-flux correction, evaluated in double precision with
    optional bfloat16 rounding of every matrix-product operand."""

    def __init__(self, params, mean, inv_std, out_scale, emulate_bf16=True):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == NET_PARAMS
        self._keep = (p, _arr(mean, (4,)), _arr(inv_std, (4,)))
        self.handle = lib().orc_net_create(_ptr(p), _ptr(self._keep[1]), _ptr(self._keep[2]),
                                           _d(out_scale), _i(1 if emulate_bf16 else 0))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.orc_net_destroy(_p(self.handle))
            self.handle = None

    def forward(self, st):
        st = _arr(st).reshape(-1, 6, 4)
        dF = np.empty((st.shape[0], 4))
        lib().orc_net_forward(_p(self.handle), _i(st.shape[0]), _ptr(st), _ptr(dF))
        return dF

    def backward(self, st, dFbar):
        st = _arr(st).reshape(-1, 6, 4)
        dFbar = _arr(dFbar).reshape(-1, 4)
        g = np.zeros(NET_PARAMS)
        dst = np.empty_like(st)
        lib().orc_net_backward(_p(self.handle), _i(st.shape[0]), _ptr(st), _ptr(dFbar), _ptr(g), _ptr(dst))
        return g, dst


CNN_PARAMS = 6388


class Cnn:
    """The convolutional learned correction (section 2's 2D form), evaluated
    in double precision with optional bfloat16 rounding of every product
    operand.  Pass it as `net` to rhs / rk3_step / the Jacobians."""

    def __init__(self, params, mean, inv_std, out_scale, emulate_bf16=True):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == CNN_PARAMS
        self._keep = (p, _arr(mean, (4,)), _arr(inv_std, (4,)))
        self.handle = lib().orc_cnn_create(_ptr(p), _ptr(self._keep[1]), _ptr(self._keep[2]),
                                           _d(out_scale), _i(1 if emulate_bf16 else 0))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.orc_cnn_destroy(_p(self.handle))
            self.handle = None

    def forward(self, x, wrap=(False, False)):
        """x: normalised inputs [H][W][4] -> corrections [H][W][4]; wrap:
        (rows, columns) periodic."""
        x = _arr(x)
        H, W = x.shape[:2]
        out = np.empty((H, W, 4))
        lib().orc_cnn_forward(_p(self.handle), _i(H), _i(W), _i(int(wrap[0])), _i(int(wrap[1])), _ptr(x), _ptr(out))
        return out

    def backward(self, x, dout, wrap=(False, False)):
        """(parameter gradient, input gradient) for upstream gradient dout."""
        x, dout = _arr(x), _arr(dout)
        H, W = x.shape[:2]
        g = np.zeros(CNN_PARAMS)
        dx = np.empty((H, W, 4))
        lib().orc_cnn_backward(_p(self.handle), _i(H), _i(W), _i(int(wrap[0])), _i(int(wrap[1])), _ptr(x),
                               _ptr(dout), _ptr(g), _ptr(dx))
        return g, dx


def cnn_images(c, U, net, phi=None, wall=0):
    """The convolutional network's input images of state U: x-faces
    [ny][wx][4] and transposed y-faces [nx][wy][4] (wx = nx + 1, or nx when x
    is periodic; likewise wy)."""
    U = _arr(U)
    wx = c.nx if c.bc[0] == 3 else c.nx + 1
    wy = c.ny if c.bc[2] == 3 else c.ny + 1
    Xx = np.empty((c.ny, wx, 4))
    Xy = np.empty((c.nx, wy, 4))
    assert lib().orc_cnn_images(ctypes.byref(c), _ptr(U), _ptr(_phi(c, phi)), _i(wall), _p(net.handle),
                                _ptr(Xx), _ptr(Xy)) == 0
    return Xx, Xy


def char_basis(Wa, Wb, gamma=1.4):
    """Left and right eigenvector matrices (face frame) of the characteristic
    reconstruction at the Roe average of primitive states Wa, Wb."""
    Wa, Wb = _arr(Wa, (4,)), _arr(Wb, (4,))
    L, R = np.empty((4, 4)), np.empty((4, 4))
    lib().orc_char_basis(_d(gamma), _ptr(Wa), _ptr(Wb), _ptr(L), _ptr(R))
    return L, R


# ------------------------------------------------------------- training
def restrict(fine, factor):
    """Restriction d(U) of section 2: block mean of factor x factor fine
    cells.  fine [..., ny_f, nx_f] -> [..., ny_f/factor, nx_f/factor]."""
    fine = np.ascontiguousarray(fine, dtype=np.float64)
    *lead, nyf, nxf = fine.shape
    lead = tuple(lead)
    npl = int(np.prod(lead)) if lead else 1
    out = np.empty(lead + (nyf // factor, nxf // factor))
    assert lib().orc_restrict(_ptr(fine), _i(nxf), _i(nyf), _i(factor), _i(npl), _i(1), _ptr(out)) == 0
    return out


def mse(U, T, scale=1.0, nbatch=1, grad=True):
    """Unrolled-loss term of section 2 per batch member: (loss [nbatch],
    gradient scale * 2 (U - T) / N or None), N = entries per member."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    assert U.shape == T.shape and U.size % nbatch == 0
    loss = np.zeros(nbatch)
    G = np.zeros_like(U) if grad else None
    lib().orc_mse.argtypes = [_p, _p, ctypes.c_longlong, _i, _d, _p, _p]
    assert lib().orc_mse(_ptr(U), _ptr(T), U.size // nbatch, nbatch, float(scale), _ptr(loss), _ptr(G)) == 0
    return loss, G


def adam(theta, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on copies: returns (theta, m, v) after the update."""
    th = np.array(theta, dtype=np.float64)
    mm = np.array(m, dtype=np.float64)
    vv = np.array(v, dtype=np.float64)
    gg = np.ascontiguousarray(g, dtype=np.float64)
    assert lib().orc_adam(_ptr(th), _ptr(gg), _ptr(mm), _ptr(vv), _i(th.size), _d(lr), _d(b1), _d(b2),
                          _d(eps), _i(step)) == 0
    return th, mm, vv
