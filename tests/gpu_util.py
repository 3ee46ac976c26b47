"""Shared helpers of the GPU tests: build matching oracle / GPU configurations
from one description and compare fields."""
import numpy as np


def field_errors(gpu, ref):
    """Per-field error max|x - o| / max|o|.  A field whose oracle values are
    all below 1e-8 of the largest field (zero in exact arithmetic, e.g. the
    transverse momentum of a planar problem, so both sides hold only
    round-off) is measured against the largest field instead."""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, (g.shape, r.shape)
    top = max(float(np.max(np.abs(r[k]))) for k in range(r.shape[0]))
    errs = []
    for k in range(r.shape[0]):
        scale = float(np.max(np.abs(r[k])))
        if scale < 1e-8 * top:
            scale = top
        diff = float(np.max(np.abs(g[k] - r[k])))
        errs.append(diff / scale if scale > 0 else diff)
    return errs


def assert_fields(gpu, ref, tol, what=""):
    errs = field_errors(gpu, ref)
    assert all(e <= tol for e in errs), f"{what}: per-field errors {errs} exceed {tol}"
    return errs


def make_pair(orc, nx, ny=1, ndim=2, domain=(0.0, 1.0, 0.0, 1.0), prec="f64", bc=(0, 0, 0, 0),
              inflow=(1.0, 0.0, 0.0, 1.0), gamma=1.4, cfl=0.5, viscous=False, mu=0.0, prandtl=0.72,
              ibm=False, nbatch=1, nu_art=0.0, weno_char=False):
    """Oracle config and GPU Grid for the same problem."""
    from paper_2601_04400_amd import Grid
    c = orc.config(ndim=ndim, nx=nx, ny=ny, x0=domain[0], x1=domain[1], y0=domain[2], y1=domain[3],
                   gamma=gamma, cfl=cfl, viscous=int(viscous), mu=mu, prandtl=prandtl, bc=bc,
                   inflow=inflow, nu_art=nu_art, weno_char=int(weno_char))
    g = Grid(nx, ny, ndim=ndim, nbatch=nbatch, domain=domain, prec=prec, gamma=gamma, cfl=cfl,
             viscous=viscous, mu=mu, prandtl=prandtl, bc=bc, inflow=inflow, ibm=ibm, nu_art=nu_art,
             weno_char=weno_char)
    return c, g
