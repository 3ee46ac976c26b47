// Per-face device helpers shared by the network kernels and the adjoint:
// the face-frame primitive stencil of a face read from a global state, and
// the reverse of one WENO5-JS reconstruction.
#pragma once
#include <hip/hip_runtime.h>

#include "flux.hpp"
#include "grid.hpp"

namespace shk {

// Primitive state (rho, u_n, u_t, p) of grid cell (gi, gj) of batch member
// Ub in the frame of an x-face (isx) or a y-face.  Indices outside the
// domain are ghost cells by the boundary rules of the stage kernel
// (reflection with the normal velocity negated, inflow state, periodic
// wrap, zero-gradient outflow), clamped into the domain beyond the ghost
// layers.
__device__ __forceinline__ void cell_prim_frame(const GridArgs& a, const double* __restrict__ Ub, int gi, int gj,
                                                bool isx, double w[4]) {
  double q[4];
  int fx = 0, fy = 0;
  auto src = [](int g, int n, int lo, int hi, int& flag) {
    if (g >= 0 && g < n) return g;
    const bool l = g < 0;
    const int bc = l ? lo : hi;
    const int depth = l ? -g : g - (n - 1);
    int r;
    switch (bc) {
      case BC_REFL: r = l ? depth - 1 : n - depth; flag |= 1; break;
      case BC_INFLOW: r = l ? 0 : n - 1; flag = 2; break;
      case BC_PERIODIC: r = ((g % n) + n) % n; break;
      default: r = l ? 0 : n - 1; break;
    }
    return r < 0 ? 0 : (r >= n ? n - 1 : r);
  };
  const int si = src(gi, a.nx, a.bc[0], a.bc[1], fx);
  const int sj = src(gj, a.ny, a.bc[2], a.bc[3], fy);
  if (fx == 2 || fy == 2) {
    for (int v = 0; v < 4; ++v) q[v] = a.inflow_cons[v];
  } else {
    const long long c = (long long)sj * a.nx + si;
    q[0] = Ub[c]; q[1] = Ub[a.ncell + c]; q[2] = Ub[2 * a.ncell + c]; q[3] = Ub[3 * a.ncell + c];
    if (fx & 1) q[1] = -q[1];
  }
  if (fy & 1) q[2] = -q[2];
  // the same conversion as the stage kernel's tile load, so the network sees
  // bit-identical inputs on both paths
  const Prim<double> p = to_prim(q[0], q[1], q[2], q[3], a.gamma - 1.0);
  w[0] = p.r;
  w[1] = isx ? p.un : p.ut;
  w[2] = isx ? p.ut : p.un;
  w[3] = p.p;
}

// Primitive state (rho, u_n, u_t, p) of stencil cell s (0..5) of face f of
// batch member Ub; x-faces first ((nx+1) per row), then y-faces (nx per row).
// The faces of one batch member are indexed in 32 bits.
__device__ __forceinline__ void face_cell_prim(const GridArgs& a, const double* __restrict__ Ub, long long f, int s,
                                               double w[4]) {
  const int fi = (int)f, nxf = (a.nx + 1) * a.ny;
  if (fi < nxf) {
    const int gj = fi / (a.nx + 1);
    cell_prim_frame(a, Ub, fi - gj * (a.nx + 1) - 3 + s, gj, true, w);
  } else {
    const int g = fi - nxf;
    const int r = g / a.nx;
    cell_prim_frame(a, Ub, g - r * a.nx, r - 3 + s, false, w);
  }
}

// Reverse of one WENO5-JS reconstruction f(a,b,c,d,e) (the forward value is
// recomputed): d f / d beta_k = -2 omega_k (q_k - f) / (eps + beta_k).
__device__ __forceinline__ void weno5_vjp(double a, double b, double c, double d, double e, double eps,
                                          double fb, double& ga, double& gb, double& gc, double& gd,
                                          double& ge) {
  const double k13 = 13.0 / 12.0;
  const double s0 = a - 2.0 * b + c, t0 = a - 4.0 * b + 3.0 * c;
  const double s1 = b - 2.0 * c + d, t1 = b - d;
  const double s2 = c - 2.0 * d + e, t2 = 3.0 * c - 4.0 * d + e;
  const double g0 = eps + (k13 * s0 * s0 + 0.25 * t0 * t0);
  const double g1 = eps + (k13 * s1 * s1 + 0.25 * t1 * t1);
  const double g2 = eps + (k13 * s2 * s2 + 0.25 * t2 * t2);
  const double h0 = g0 * g0, h1 = g1 * g1, h2 = g2 * g2;
  const double w0 = 0.1 * (h1 * h2), w1 = 0.6 * (h0 * h2), w2 = 0.3 * (h0 * h1);
  // one reciprocal serves the normalisation and the three 1/g_k:
  // r = 1/(S P) with S = w0 + w1 + w2 and P = g0 g1 g2 (both positive and
  // far from the double range limits since g_k >= eps)
  const double S = w0 + w1 + w2, P = g0 * g1 * g2;
  const double r = qrcp(S * P);
  const double is = P * r, iP = S * r;
  const double o0 = w0 * is, o1 = w1 * is, o2 = w2 * is;
  const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
  const double q1 = (5.0 * c - b + 2.0 * d) * (1.0 / 6.0);
  const double q2 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
  const double f = o0 * q0 + o1 * q1 + o2 * q2;
  const double qb0 = fb * o0, qb1 = fb * o1, qb2 = fb * o2;
  const double m2 = -2.0 * fb * iP;
  const double bb0 = m2 * o0 * (q0 - f) * (g1 * g2);
  const double bb1 = m2 * o1 * (q1 - f) * (g0 * g2);
  const double bb2 = m2 * o2 * (q2 - f) * (g0 * g1);
  const double sb0 = bb0 * (2.0 * k13) * s0, tb0 = bb0 * 0.5 * t0;
  const double sb1 = bb1 * (2.0 * k13) * s1, tb1 = bb1 * 0.5 * t1;
  const double sb2 = bb2 * (2.0 * k13) * s2, tb2 = bb2 * 0.5 * t2;
  ga += qb0 * (2.0 / 6.0) + sb0 + tb0;
  gb += qb0 * (-7.0 / 6.0) + qb1 * (-1.0 / 6.0) - 2.0 * sb0 - 4.0 * tb0 + sb1 + tb1;
  gc += qb0 * (11.0 / 6.0) + qb1 * (5.0 / 6.0) + qb2 * (2.0 / 6.0) + sb0 + 3.0 * tb0 - 2.0 * sb1 + sb2 +
        3.0 * tb2;
  gd += qb1 * (2.0 / 6.0) + qb2 * (5.0 / 6.0) + sb1 - tb1 - 2.0 * sb2 - 4.0 * tb2;
  ge += qb2 * (-1.0 / 6.0) + sb2 + tb2;
}

}  // namespace shk
