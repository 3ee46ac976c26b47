// Oracle: plain serial CPU solver for the compressible Euler / Navier-Stokes
// right-hand side, the SSP-RK3 step and the ghost-cell immersed boundary.
//
// TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library: it is
// loaded by the test suite, by the package's smoke check and by the CPU
// baseline leg of the benchmark, and by nothing else.  It shares no code,
// header, table or constant with the GPU path.
//
// Everything is written for readability, in the order the method states it:
//   * state, flux tensor and ideal-gas equation of state: paper section 2,
//     eq. (euler) and the equation of state that follows it;
//   * reconstruction of primitive variables with fifth-order WENO
//     (Jiang-Shu weights, eps = 1e-6 by default: the paper cites Johnsen &
//     Colonius for the WENO + HLLC combination but prints no weights);
//   * HLLC flux in the compact sign(s*) form of section 2, with Davis wave
//     speeds and the standard contact speed; the star-state energy row is the
//     Rankine-Hugoniot-consistent one E + (s*-u)(rho s* + p/(s-u)) (the energy
//     row as printed does not satisfy the jump condition across the s wave);
//   * conservative update of section 2, advanced with Shu-Osher SSP-RK3;
//   * ghost-cell immersed boundary (section 2, Mittal & Iaccarino) with a
//     mirrored image point and fluid-only bilinear interpolation.
// It is templated on the scalar type so that the same code instantiated with
// forward-mode dual numbers gives exact tangents of the discrete map.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "correction.hpp"
#include "dual.hpp"

namespace orc {

using std::fabs;
using std::tanh;
using std::sqrt;

constexpr int NG = 3;  // ghost layers: a 6-cell WENO5 stencil reaches 3 cells out

enum Bc { BC_TRANSMISSIVE = 0, BC_REFLECTIVE = 1, BC_INFLOW = 2, BC_PERIODIC = 3 };
enum CellClass { FLUID = 0, SOLID = 1, GHOST = 2 };

// Plain description of a grid and its physics (all doubles; C layout).
struct Config {
  int ndim, nx, ny;          // ndim 1 => ny == 1, external state has 3 fields
  double x0, x1, y0, y1;     // cell-centred uniform grid on [x0,x1]x[y0,y1]
  double gamma, cfl, weno_eps;
  int viscous;               // 1 => Navier-Stokes viscous and heat fluxes
  double mu, prandtl, nu_art;  // dynamic viscosity, Prandtl number, Laplacian nu
  int bc[4];                 // x-lo, x-hi, y-lo, y-hi (enum Bc)
  double inflow[4];          // (rho, u, v, p) of an inflow boundary
  int weno_char;             // 1 => WENO5 on characteristic variables (else on primitives)
};

// The differentiable physical parameters (gamma and the inflow state).
template <class T>
struct Params {
  T gamma;
  T inflow[4];
};

template <class T>
Params<T> params_from(const Config& c) {
  Params<T> p;
  p.gamma = T(c.gamma);
  for (int k = 0; k < 4; ++k) p.inflow[k] = T(c.inflow[k]);
  return p;
}

// Conservative state with NG ghost layers on every side, 4 planes
// (rho, rho u, rho v, E).  In 1D the rho v plane is identically zero.
template <class T>
struct Field {
  int nx = 0, ny = 0, px = 0, py = 0;
  std::vector<T> q;
  Field() {}
  Field(int nx_, int ny_) : nx(nx_), ny(ny_), px(nx_ + 2 * NG), py(ny_ + 2 * NG),
                            q(size_t(4) * (nx_ + 2 * NG) * (ny_ + 2 * NG), T(0.0)) {}
  T& at(int v, int i, int j) { return q[(size_t(v) * py + (j + NG)) * px + (i + NG)]; }
  const T& at(int v, int i, int j) const { return q[(size_t(v) * py + (j + NG)) * px + (i + NG)]; }
};

inline double dx_of(const Config& c) { return (c.x1 - c.x0) / c.nx; }
inline double dy_of(const Config& c) { return c.ndim == 1 ? 1.0 : (c.y1 - c.y0) / c.ny; }

// ---------------------------------------------------------------- layout I/O
// External layout: planes [nvar][ny][nx], x fastest; nvar = 3 in 1D
// (rho, rho u, E) and 4 in 2D (rho, rho u, rho v, E).
inline int nvar_ext(const Config& c) { return c.ndim == 1 ? 3 : 4; }
inline int ext_plane(const Config& c, int v) {  // internal plane -> external, -1 if absent
  if (c.ndim == 2) return v;
  return v == 0 ? 0 : v == 1 ? 1 : v == 3 ? 2 : -1;
}

template <class T>
void load_state(const Config& c, const T* U, Field<T>& f) {
  const size_t n = size_t(c.nx) * c.ny;
  for (int v = 0; v < 4; ++v) {
    int e = ext_plane(c, v);
    for (int j = 0; j < c.ny; ++j)
      for (int i = 0; i < c.nx; ++i)
        f.at(v, i, j) = e < 0 ? T(0.0) : U[e * n + size_t(j) * c.nx + i];
  }
}

template <class T>
void store_state(const Config& c, const Field<T>& f, T* U) {
  const size_t n = size_t(c.nx) * c.ny;
  for (int v = 0; v < 4; ++v) {
    int e = ext_plane(c, v);
    if (e < 0) continue;
    for (int j = 0; j < c.ny; ++j)
      for (int i = 0; i < c.nx; ++i) U[e * n + size_t(j) * c.nx + i] = f.at(v, i, j);
  }
}

// ------------------------------------------------------ equation of state
// Primitive (rho, u, v, p) from conservative, ideal gas (section 2, the
// equation of state under eq. (euler)).
template <class T>
void cons_to_prim(const T U[4], const T& gamma, T W[4]) {
  W[0] = U[0];
  W[1] = U[1] / U[0];
  W[2] = U[2] / U[0];
  W[3] = (gamma - 1.0) * (U[3] - 0.5 * U[0] * (W[1] * W[1] + W[2] * W[2]));
}

// Conservative from primitive: E = p/(gamma-1) + rho (u^2+v^2)/2.
template <class T>
void prim_to_cons(const T W[4], const T& gamma, T U[4]) {
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = W[3] / (gamma - 1.0) + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2]);
}

// Physical x-flux of eq. (euler): first column of the flux tensor.
template <class T>
void euler_flux_x(const T W[4], const T U[4], T F[4]) {
  F[0] = U[1];
  F[1] = U[1] * W[1] + W[3];
  F[2] = U[1] * W[2];
  F[3] = W[1] * (U[3] + W[3]);
}

// ---------------------------------------------------------------- WENO5-JS
// Left-biased reconstruction at face i+1/2 from the five cell values
// f[0..4] = f_{i-2}, ..., f_{i+2}: three third-order candidates, Jiang-Shu
// smoothness indicators, ideal weights (1/10, 6/10, 3/10), alpha = d/(eps+beta)^2.
template <class T>
T weno5_left(const T f[5], double eps) {
  const T& a = f[0]; const T& b = f[1]; const T& c = f[2]; const T& d = f[3]; const T& e = f[4];
  T q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  T q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  T q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  T s0 = a - 2.0 * b + c, t0 = a - 4.0 * b + 3.0 * c;
  T s1 = b - 2.0 * c + d, t1 = b - d;
  T s2 = c - 2.0 * d + e, t2 = 3.0 * c - 4.0 * d + e;
  T beta0 = (13.0 / 12.0) * (s0 * s0) + 0.25 * (t0 * t0);
  T beta1 = (13.0 / 12.0) * (s1 * s1) + 0.25 * (t1 * t1);
  T beta2 = (13.0 / 12.0) * (s2 * s2) + 0.25 * (t2 * t2);
  T g0 = eps + beta0, g1 = eps + beta1, g2 = eps + beta2;
  T alpha0 = 0.1 / (g0 * g0);
  T alpha1 = 0.6 / (g1 * g1);
  T alpha2 = 0.3 / (g2 * g2);
  T sum = alpha0 + alpha1 + alpha2;
  T w0 = alpha0 / sum, w1 = alpha1 / sum, w2 = alpha2 / sum;
  return w0 * q0 + w1 * q1 + w2 * q2;
}

// Right state at face i+1/2: the mirror image, from f_{i+3}, ..., f_{i-1}.
template <class T>
T weno5_right(const T f6[6], double eps) {  // f6 = f_{i-2..i+3}
  T m[5] = {f6[5], f6[4], f6[3], f6[2], f6[1]};
  return weno5_left(m, eps);
}

// ------------------------------------------- characteristic-wise WENO5
// The variant the paper leaves open: reconstruction in characteristic
// variables.  At a face the conservative stencil (face frame, u normal) is
// projected on the left eigenvectors of the face-normal flux Jacobian at the
// Roe average of the two adjacent cells, each characteristic field is
// reconstructed by WENO5-JS, and the two face states are projected back.
// Right eigenvectors (columns, for u - c, u, u, u + c), q = (u^2 + v^2)/2:
//   (1, u - c, v, H - u c), (1, u, v, q), (0, 0, 1, v), (1, u + c, v, H + u c)
// and the left ones (rows of the inverse), b1 = (gamma - 1)/c^2, b2 = b1 q:
//   ((b2 + u/c)/2, -(b1 u + 1/c)/2, -b1 v/2, b1/2), (1 - b2, b1 u, b1 v, -b1),
//   (-v, 0, 1, 0), ((b2 - u/c)/2, -(b1 u - 1/c)/2, -b1 v/2, b1/2).
template <class T>
void char_basis(const T Wa[4], const T Wb[4], const T& gamma, T Lm[4][4], T Rm[4][4]) {
  const T ra = sqrt(Wa[0]), rb_ = sqrt(Wb[0]);
  const T Ha = gamma / (gamma - 1.0) * Wa[3] / Wa[0] + 0.5 * (Wa[1] * Wa[1] + Wa[2] * Wa[2]);
  const T Hb = gamma / (gamma - 1.0) * Wb[3] / Wb[0] + 0.5 * (Wb[1] * Wb[1] + Wb[2] * Wb[2]);
  const T u = (ra * Wa[1] + rb_ * Wb[1]) / (ra + rb_);
  const T v = (ra * Wa[2] + rb_ * Wb[2]) / (ra + rb_);
  const T H = (ra * Ha + rb_ * Hb) / (ra + rb_);
  const T q = 0.5 * (u * u + v * v);
  const T c = sqrt((gamma - 1.0) * (H - q));
  const T b1 = (gamma - 1.0) / (c * c), b2 = b1 * q;
  const T R[4][4] = {{T(1.0), T(1.0), T(0.0), T(1.0)},
                     {u - c, u, T(0.0), u + c},
                     {v, v, T(1.0), v},
                     {H - u * c, q, v, H + u * c}};
  const T L[4][4] = {{0.5 * (b2 + u / c), -0.5 * (b1 * u + 1.0 / c), -0.5 * b1 * v, 0.5 * b1},
                     {1.0 - b2, b1 * u, b1 * v, -b1},
                     {-v, T(0.0), T(1.0), T(0.0)},
                     {0.5 * (b2 - u / c), -0.5 * (b1 * u - 1.0 / c), -0.5 * b1 * v, 0.5 * b1}};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) { Lm[i][j] = L[i][j]; Rm[i][j] = R[i][j]; }
}

// Face states (primitive, face frame) from the six-cell stencil by the
// characteristic-wise reconstruction.
template <class T>
void char_weno(const T Wst[6][4], const T& gamma, double eps, T WL[4], T WR[4]) {
  T U[6][4], w[6][4], L[4][4], R[4][4];
  for (int s = 0; s < 6; ++s) prim_to_cons(Wst[s], gamma, U[s]);
  char_basis(Wst[2], Wst[3], gamma, L, R);
  for (int s = 0; s < 6; ++s)
    for (int m = 0; m < 4; ++m) {
      T acc = T(0.0);
      for (int k = 0; k < 4; ++k) acc = acc + L[m][k] * U[s][k];
      w[s][m] = acc;
    }
  T wl[4], wr[4];
  for (int m = 0; m < 4; ++m) {
    T f5[5] = {w[0][m], w[1][m], w[2][m], w[3][m], w[4][m]};
    T f6[6] = {w[0][m], w[1][m], w[2][m], w[3][m], w[4][m], w[5][m]};
    wl[m] = weno5_left(f5, eps);
    wr[m] = weno5_right(f6, eps);
  }
  T UL[4], UR[4];
  for (int k = 0; k < 4; ++k) {
    T al = T(0.0), ar = T(0.0);
    for (int m = 0; m < 4; ++m) {
      al = al + R[k][m] * wl[m];
      ar = ar + R[k][m] * wr[m];
    }
    UL[k] = al;
    UR[k] = ar;
  }
  cons_to_prim(UL, gamma, WL);
  cons_to_prim(UR, gamma, WR);
}

// ------------------------------------------------------------------- HLLC
// x-direction HLLC flux between primitive states WL, WR (section 2).
// Davis estimates sL = min(uL-aL, uR-aR), sR = max(uL+aL, uR+aR); contact
// speed s* as printed; star states U*k = (sk-uk)/(sk-s*) [rho, rho s*, rho v,
// E + (s*-u)(rho s* + p/(sk-uk))].  The compact form
//   F = (1+sign s*)/2 [FL + s-(U*L-UL)] + (1-sign s*)/2 [FR + s+(U*R-UR)]
// is evaluated by its branches (s- = min(0,sL), s+ = max(0,sR)); at s* = 0
// the sign is zero and the flux is the mean of both brackets.
template <class T>
void hllc_x(const T WL[4], const T WR[4], const T& gamma, T F[4]) {
  T UL[4], UR[4], FL[4], FR[4];
  prim_to_cons(WL, gamma, UL);
  prim_to_cons(WR, gamma, UR);
  euler_flux_x(WL, UL, FL);
  euler_flux_x(WR, UR, FR);
  T aL = sqrt(gamma * WL[3] / WL[0]);
  T aR = sqrt(gamma * WR[3] / WR[0]);
  T sL = std::min(WL[1] - aL, WR[1] - aR);
  T sR = std::max(WL[1] + aL, WR[1] + aR);
  T num = WR[3] - WL[3] + WL[0] * WL[1] * (sL - WL[1]) - WR[0] * WR[1] * (sR - WR[1]);
  T den = WL[0] * (sL - WL[1]) - WR[0] * (sR - WR[1]);
  T ss = num / den;

  auto left_bracket = [&](T out[4]) {
    if (sL >= 0.0) { for (int k = 0; k < 4; ++k) out[k] = FL[k]; return; }
    T chi = (sL - WL[1]) / (sL - ss);
    T Us[4] = {chi * WL[0], chi * (WL[0] * ss), chi * (WL[0] * WL[2]),
               chi * (UL[3] + (ss - WL[1]) * (WL[0] * ss + WL[3] / (sL - WL[1])))};
    for (int k = 0; k < 4; ++k) out[k] = FL[k] + sL * (Us[k] - UL[k]);
  };
  auto right_bracket = [&](T out[4]) {
    if (sR <= 0.0) { for (int k = 0; k < 4; ++k) out[k] = FR[k]; return; }
    T chi = (sR - WR[1]) / (sR - ss);
    T Us[4] = {chi * WR[0], chi * (WR[0] * ss), chi * (WR[0] * WR[2]),
               chi * (UR[3] + (ss - WR[1]) * (WR[0] * ss + WR[3] / (sR - WR[1])))};
    for (int k = 0; k < 4; ++k) out[k] = FR[k] + sR * (Us[k] - UR[k]);
  };
  if (ss > 0.0) {
    left_bracket(F);
  } else if (ss < 0.0) {
    right_bracket(F);
  } else {
    T A[4], B[4];
    left_bracket(A);
    right_bracket(B);
    for (int k = 0; k < 4; ++k) F[k] = 0.5 * (A[k] + B[k]);
  }
}

// ------------------------------------------------------- domain boundaries
// Fill the NG ghost layers of the conservative state.  x-ghosts over the
// interior rows first, then y-ghosts over every column (x-ghosts included).
template <class T>
void apply_bc(const Config& c, const Params<T>& P, Field<T>& f) {
  T Uin[4];
  prim_to_cons(P.inflow, P.gamma, Uin);
  auto side_x = [&](int side) {
    int bc = c.bc[side];
    for (int j = 0; j < c.ny; ++j)
      for (int g = 1; g <= NG; ++g) {
        int ig = side == 0 ? -g : c.nx - 1 + g;  // ghost index
        for (int v = 0; v < 4; ++v) {
          T val;
          if (bc == BC_TRANSMISSIVE) {
            val = f.at(v, side == 0 ? 0 : c.nx - 1, j);
          } else if (bc == BC_REFLECTIVE) {
            int im = side == 0 ? g - 1 : c.nx - g;
            val = f.at(v, im, j);
            if (v == 1) val = -val;
          } else if (bc == BC_INFLOW) {
            val = Uin[v];
          } else {
            int ip = side == 0 ? c.nx - g : g - 1;
            val = f.at(v, ip, j);
          }
          f.at(v, ig, j) = val;
        }
      }
  };
  auto side_y = [&](int side) {
    int bc = c.bc[2 + side];
    for (int i = -NG; i < c.nx + NG; ++i)
      for (int g = 1; g <= NG; ++g) {
        int jg = side == 0 ? -g : c.ny - 1 + g;
        for (int v = 0; v < 4; ++v) {
          T val;
          if (bc == BC_TRANSMISSIVE) {
            val = f.at(v, i, side == 0 ? 0 : c.ny - 1);
          } else if (bc == BC_REFLECTIVE) {
            int jm = side == 0 ? g - 1 : c.ny - g;
            val = f.at(v, i, jm);
            if (v == 2) val = -val;
          } else if (bc == BC_INFLOW) {
            val = Uin[v];
          } else {
            int jp = side == 0 ? c.ny - g : g - 1;
            val = f.at(v, i, jp);
          }
          f.at(v, i, jg) = val;
        }
      }
  };
  side_x(0);
  side_x(1);
  if (c.ndim == 2) {
    side_y(0);
    side_y(1);
  }
}

// ----------------------------------------------------- immersed boundary
// Ghost-cell IBM on a signed-distance level set phi sampled at cell centres
// (phi < 0 inside the solid).  Classes: fluid (phi >= 0), solid (phi < 0),
// ghost (solid with a fluid cell within NG cells along +-x or +-y).
struct Ibm {
  bool active = false;
  int wall = 0;                 // 0 slip, 1 no-slip adiabatic
  std::vector<uint8_t> cls;     // [ny][nx]
  struct GhostPt {
    int i, j;
    double nx_, ny_;            // unit normal from grad phi
    int src[4];                 // flat indices of the interpolation cells (-1 unused)
    double w[4];                // renormalised fluid-only weights
  };
  std::vector<GhostPt> ghosts;
  // ghosts whose image point is undefined: the central-difference gradient
  // of the signed distance is far from unit length (|grad phi| < 1/2: the
  // difference straddles the solid's medial axis -- a solid thinner than
  // about two cells, a body a few cells across), or no fluid cell is found
  // around the image point or along the normal
  int degenerate = 0;
};

inline Ibm build_ibm(const Config& c, const double* phi, int wall) {
  Ibm ib;
  if (!phi) return ib;
  ib.active = true;
  ib.wall = wall;
  const int nx = c.nx, ny = c.ny;
  const double dx = dx_of(c), dy = dy_of(c);
  auto P = [&](int i, int j) { return phi[size_t(j) * nx + i]; };
  auto is_fluid = [&](int i, int j) { return P(i, j) >= 0.0; };
  ib.cls.assign(size_t(nx) * ny, FLUID);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      if (is_fluid(i, j)) continue;
      bool near = false;
      for (int k = 1; k <= NG && !near; ++k) {
        if (i - k >= 0 && is_fluid(i - k, j)) near = true;
        if (i + k < nx && is_fluid(i + k, j)) near = true;
        if (j - k >= 0 && is_fluid(i, j - k)) near = true;
        if (j + k < ny && is_fluid(i, j + k)) near = true;
      }
      ib.cls[size_t(j) * nx + i] = near ? GHOST : SOLID;
    }
  // Per ghost: normal, image point at twice the wall distance, stencil.
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      if (ib.cls[size_t(j) * nx + i] != GHOST) continue;
      Ibm::GhostPt g;
      g.i = i; g.j = j;
      int il = std::max(i - 1, 0), ir = std::min(i + 1, nx - 1);
      int jl = std::max(j - 1, 0), jr = std::min(j + 1, ny - 1);
      double gx = (P(ir, j) - P(il, j)) / ((ir - il) * dx);
      double gy = (P(i, jr) - P(i, jl)) / ((jr - jl) * dy);
      double gn = std::sqrt(gx * gx + gy * gy);
      g.nx_ = gx / gn; g.ny_ = gy / gn;
      double xg = c.x0 + (i + 0.5) * dx, yg = c.y0 + (j + 0.5) * dy;
      double dist = 2.0 * std::fabs(P(i, j));
      double xi = xg + dist * g.nx_, yi = yg + dist * g.ny_;
      // enclosing cell centres: (i0,j0) .. (i0+1,j0+1)
      double fx = (xi - c.x0) / dx - 0.5, fy = (yi - c.y0) / dy - 0.5;
      int i0 = int(std::floor(fx)), j0 = int(std::floor(fy));
      double tx = fx - i0, ty = fy - j0;
      double wb[4] = {(1.0 - tx) * (1.0 - ty), tx * (1.0 - ty), (1.0 - tx) * ty, tx * ty};
      int ci[4] = {i0, i0 + 1, i0, i0 + 1}, cj[4] = {j0, j0, j0 + 1, j0 + 1};
      double wsum = 0.0;
      for (int k = 0; k < 4; ++k) {
        g.src[k] = -1; g.w[k] = 0.0;
        if (ci[k] < 0 || ci[k] >= nx || cj[k] < 0 || cj[k] >= ny) continue;
        if (!is_fluid(ci[k], cj[k])) continue;
        g.src[k] = cj[k] * nx + ci[k];
        g.w[k] = wb[k];
        wsum += wb[k];
      }
      if (wsum > 0.0) {
        for (int k = 0; k < 4; ++k) g.w[k] = g.w[k] / wsum;
      } else {
        // No fluid weight: nearest fluid cell met walking out along the normal.
        for (int k = 0; k < 4; ++k) { g.src[k] = -1; g.w[k] = 0.0; }
        double h = 0.5 * std::min(dx, dy);
        for (int m = 0; m < 64; ++m) {
          double s = std::fabs(P(i, j)) + m * h;
          double xs = xg + s * g.nx_, ys = yg + s * g.ny_;
          int is = int(std::floor((xs - c.x0) / dx)), js = int(std::floor((ys - c.y0) / dy));
          if (is < 0 || is >= nx || js < 0 || js >= ny) break;
          if (is_fluid(is, js)) { g.src[0] = js * nx + is; g.w[0] = 1.0; break; }
        }
      }
      bool resolved = false;
      for (int k = 0; k < 4; ++k) resolved = resolved || g.src[k] >= 0;
      if (!(gn >= 0.5) || !resolved) ++ib.degenerate;
      ib.ghosts.push_back(g);
    }
  return ib;
}

// Refill every ghost cell of f from the fluid state at its image point.
template <class T>
void ibm_fill(const Config& c, const Params<T>& P, const Ibm& ib, Field<T>& f) {
  if (!ib.active) return;
  // each ghost reads fluid cells only, so the ghosts are independent
#pragma omp parallel for schedule(static)
  for (size_t gk = 0; gk < ib.ghosts.size(); ++gk) {
    const auto& g = ib.ghosts[gk];
    T Wi[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
    for (int k = 0; k < 4; ++k) {
      if (g.src[k] < 0) continue;
      int si = g.src[k] % c.nx, sj = g.src[k] / c.nx;
      T U[4] = {f.at(0, si, sj), f.at(1, si, sj), f.at(2, si, sj), f.at(3, si, sj)};
      T W[4];
      cons_to_prim(U, P.gamma, W);
      for (int v = 0; v < 4; ++v) Wi[v] = Wi[v] + g.w[k] * W[v];
    }
    T Wg[4] = {Wi[0], Wi[1], Wi[2], Wi[3]};
    if (ib.wall == 0) {  // slip: reflect the normal velocity, keep the tangential one
      T un = Wi[1] * g.nx_ + Wi[2] * g.ny_;
      Wg[1] = Wi[1] - 2.0 * un * g.nx_;
      Wg[2] = Wi[2] - 2.0 * un * g.ny_;
    } else {             // no-slip adiabatic: velocity reversed, rho and p kept
      Wg[1] = -Wi[1];
      Wg[2] = -Wi[2];
    }
    T Ug[4];
    prim_to_cons(Wg, P.gamma, Ug);
    for (int v = 0; v < 4; ++v) f.at(v, g.i, g.j) = Ug[v];
  }
}

// ------------------------------------------------------------- face fluxes
// Optional learned correction hooks (correction.hpp tags which one): the
// per-face network dF = net(stencil), stencil = 6 cells x (rho, u_n, u_t, p)
// in the face-normal frame, or the convolutional network over the images of
// x-faces and (transposed) y-faces; either correction is in the face frame
// and is added to the HLLC flux.
struct FluxNet;  // defined in mlp.hpp
template <class T>
void flux_net_apply(const FluxNet* net, const T stencil[6][4], T dF[4]);
struct FluxCnn;  // defined in cnn.hpp
template <class T>
void cnn_apply(const FluxCnn& n, const std::vector<T>& x, int H, int Wd, const bool wrap[2], std::vector<T>& out);
template <class T>
T cnn_norm(const FluxCnn* n, int v, const T& x);  // (x - mean[v]) * inv_std[v]

// Numerical flux across one face.  Wst holds the 6 primitive cell states
// i-2..i+3 along the face normal, already rotated so that component 1 is the
// normal velocity and component 2 the tangential one.
template <class T>
void face_flux(const Config& c, const Params<T>& P, const T Wst[6][4], const FluxNet* net,
               T F[4], long* fallback_count, T* WLout = nullptr, T* WRout = nullptr) {
  T WL[4], WR[4];
  if (c.weno_char) {
    char_weno(Wst, P.gamma, c.weno_eps, WL, WR);
  } else {
    for (int v = 0; v < 4; ++v) {
      T f5[5] = {Wst[0][v], Wst[1][v], Wst[2][v], Wst[3][v], Wst[4][v]};
      T f6[6] = {Wst[0][v], Wst[1][v], Wst[2][v], Wst[3][v], Wst[4][v], Wst[5][v]};
      WL[v] = weno5_left(f5, c.weno_eps);
      WR[v] = weno5_right(f6, c.weno_eps);
    }
  }
  // Positivity fallback: a non-positive reconstructed density or pressure
  // reverts both states of this face to the adjacent cell values.
  if (WL[0] <= 0.0 || WL[3] <= 0.0 || WR[0] <= 0.0 || WR[3] <= 0.0) {
    for (int v = 0; v < 4; ++v) { WL[v] = Wst[2][v]; WR[v] = Wst[3][v]; }
    if (fallback_count) ++*fallback_count;
  }
  if (WLout)
    for (int v = 0; v < 4; ++v) { WLout[v] = WL[v]; WRout[v] = WR[v]; }
  hllc_x(WL, WR, P.gamma, F);
  if (net) {
    T dF[4];
    flux_net_apply(net, Wst, dF);
    for (int v = 0; v < 4; ++v) F[v] = F[v] + dF[v];
  }
}

// Viscous face flux (Newtonian, Stokes hypothesis, Fourier conduction with
// gas constant 1 so T = p/rho).  Normal derivatives by the two-point
// difference across the face, tangential ones by averaging the central
// differences of the two adjacent cells.  Returned in the face-normal frame:
// [0, tau_nn, tau_nt, u_n tau_nn + u_t tau_nt - q_n].
template <class T>
void viscous_face(const Config& c, const T& gamma,
                  const T Wa[4], const T Wb[4],          // the two cells across the face
                  const T Wa_p[4], const T Wa_m[4],      // tangential neighbours of a (+, -)
                  const T Wb_p[4], const T Wb_m[4],      // tangential neighbours of b
                  double dn, double dt_, T Fv[4]) {
  const double mu = c.mu;
  const T kappa = mu * gamma / ((gamma - 1.0) * c.prandtl);
  T un_n = (Wb[1] - Wa[1]) / dn;
  T ut_n = (Wb[2] - Wa[2]) / dn;
  T T_n = (Wb[3] / Wb[0] - Wa[3] / Wa[0]) / dn;
  T un_t = (Wa_p[1] - Wa_m[1] + Wb_p[1] - Wb_m[1]) / (4.0 * dt_);
  T ut_t = (Wa_p[2] - Wa_m[2] + Wb_p[2] - Wb_m[2]) / (4.0 * dt_);
  T tau_nn = mu * ((4.0 / 3.0) * un_n - (2.0 / 3.0) * ut_t);
  T tau_nt = mu * (un_t + ut_n);
  T q_n = -kappa * T_n;
  T un = 0.5 * (Wa[1] + Wb[1]);
  T ut = 0.5 * (Wa[2] + Wb[2]);
  Fv[0] = T(0.0);
  Fv[1] = tau_nn;
  Fv[2] = tau_nt;
  Fv[3] = un * tau_nn + ut * tau_nt - q_n;
}

// ---------------------------------------------------------------- the RHS
// L(U) = -(F_{i+1/2}-F_{i-1/2})/dx - (G_{j+1/2}-G_{j-1/2})/dy + nu lap(U).
// f must hold the stage state with ghost cells of the IBM already filled;
// the domain ghost layers are (re)filled here.  L is zero at solid and ghost
// cells.  Each face flux is computed once, so the update telescopes exactly.
template <class T>
void rhs(const Config& c, const Params<T>& P, const Ibm& ib, Field<T>& f, Field<T>& L,
         const Correction* corr, long* fallback_count, std::vector<T>* images = nullptr) {
  const FluxNet* net = corr && corr->kind == CORR_MLP ? reinterpret_cast<const FluxNet*>(corr) : nullptr;
  const FluxCnn* cnn = corr && corr->kind == CORR_CNN ? reinterpret_cast<const FluxCnn*>(corr) : nullptr;
  apply_bc(c, P, f);
  const int nx = c.nx, ny = c.ny;
  const double dx = dx_of(c), dy = dy_of(c);
  // primitives everywhere (interior and ghost layers)
  Field<T> w(nx, ny);
  const int jlo = c.ndim == 2 ? -NG : 0, jhi = c.ndim == 2 ? ny + NG : ny;
  // Rows are independent: with OpenMP the loops below are shared out over
  // threads (each value is computed exactly as in a serial run; the learned
  // corrections stay serial).
  const bool par = !net && !cnn;
  long fbl = 0;  // positivity fallbacks of this call
#pragma omp parallel for schedule(static)
  for (int j = jlo; j < jhi; ++j)
    for (int i = -NG; i < nx + NG; ++i) {
      T U[4] = {f.at(0, i, j), f.at(1, i, j), f.at(2, i, j), f.at(3, i, j)};
      T W[4];
      cons_to_prim(U, P.gamma, W);
      for (int v = 0; v < 4; ++v) w.at(v, i, j) = W[v];
    }
  auto Wat = [&](int i, int j, T out[4]) { for (int v = 0; v < 4; ++v) out[v] = w.at(v, i, j); };

  // x-faces: face index fi = 0..nx is the left face of cell fi.
  std::vector<T> Fx(size_t(4) * (nx + 1) * ny), Fy;
  // inputs of the convolutional correction: per face, the normalised
  // conservative mean of the two reconstructed states (face frame)
  // (a periodic axis holds each face once: the last face is the first)
  const bool perx = c.bc[0] == BC_PERIODIC, pery = c.ndim == 2 && c.bc[2] == BC_PERIODIC;
  const int wx = perx ? nx : nx + 1, wy = pery ? ny : ny + 1;
  std::vector<T> Xx, Xy;
  if (cnn) Xx.resize(size_t(4) * wx * ny);
  auto cnn_input = [&](const T WL[4], const T WR[4], T* x) {
    T UL[4], UR[4];
    prim_to_cons(WL, P.gamma, UL);
    prim_to_cons(WR, P.gamma, UR);
    for (int v = 0; v < 4; ++v) x[v] = cnn_norm(cnn, v, T(0.5) * (UL[v] + UR[v]));
  };
#pragma omp parallel for schedule(static) if (par) reduction(+ : fbl)
  for (int j = 0; j < ny; ++j)
    for (int fi = 0; fi <= nx; ++fi) {
      T st[6][4];
      for (int s = 0; s < 6; ++s) Wat(fi - 3 + s, j, st[s]);
      T F[4], WL[4], WR[4];
      face_flux(c, P, st, net, F, &fbl, WL, WR);
      if (cnn && fi < wx) cnn_input(WL, WR, &Xx[(size_t(j) * wx + fi) * 4]);
      if (c.viscous) {
        T a[4], b[4], ap[4], am[4], bp[4], bm[4], Fv[4];
        Wat(fi - 1, j, a); Wat(fi, j, b);
        Wat(fi - 1, j + 1, ap); Wat(fi - 1, j - 1, am);
        Wat(fi, j + 1, bp); Wat(fi, j - 1, bm);
        viscous_face(c, P.gamma, a, b, ap, am, bp, bm, dx, dy, Fv);
        for (int v = 0; v < 4; ++v) F[v] = F[v] - Fv[v];
      }
      for (int v = 0; v < 4; ++v) Fx[(size_t(v) * ny + j) * (nx + 1) + fi] = F[v];
    }
  // y-faces: rotate (u, v) -> (v, u), compute, rotate the momentum back.
  if (c.ndim == 2) {
    Fy.resize(size_t(4) * nx * (ny + 1));
    if (cnn) Xy.resize(size_t(4) * nx * wy);
#pragma omp parallel for schedule(static) if (par) reduction(+ : fbl)
    for (int fj = 0; fj <= ny; ++fj)
      for (int i = 0; i < nx; ++i) {
        T st[6][4];
        for (int s = 0; s < 6; ++s) {
          T W[4];
          Wat(i, fj - 3 + s, W);
          st[s][0] = W[0]; st[s][1] = W[2]; st[s][2] = W[1]; st[s][3] = W[3];
        }
        T G[4], WL[4], WR[4];
        face_flux(c, P, st, net, G, &fbl, WL, WR);
        if (cnn && fj < wy) cnn_input(WL, WR, &Xy[(size_t(i) * wy + fj) * 4]);  // transposed image
        if (c.viscous) {
          T a[4], b[4], ap[4], am[4], bp[4], bm[4], Fv[4], t[4];
          auto rot = [&](int ii, int jj, T o[4]) { Wat(ii, jj, t); o[0] = t[0]; o[1] = t[2]; o[2] = t[1]; o[3] = t[3]; };
          rot(i, fj - 1, a); rot(i, fj, b);
          rot(i + 1, fj - 1, ap); rot(i - 1, fj - 1, am);
          rot(i + 1, fj, bp); rot(i - 1, fj, bm);
          viscous_face(c, P.gamma, a, b, ap, am, bp, bm, dy, dx, Fv);
          for (int v = 0; v < 4; ++v) G[v] = G[v] - Fv[v];
        }
        T Gs[4] = {G[0], G[2], G[1], G[3]};
        for (int v = 0; v < 4; ++v) Fy[(size_t(v) * (ny + 1) + fj) * nx + i] = Gs[v];
      }
  }
  if (fallback_count) *fallback_count += fbl;
  if (cnn && images) {  // the network's input images (x-faces, transposed y-faces)
    images[0] = Xx;
    images[1] = Xy;
  }
  if (cnn) {
    std::vector<T> ox, oy;
    const bool wrapx[2] = {pery, perx}, wrapy[2] = {perx, pery};
    cnn_apply(*cnn, Xx, ny, wx, wrapx, ox);
    for (int j = 0; j < ny; ++j)
      for (int fi = 0; fi <= nx; ++fi)
        for (int v = 0; v < 4; ++v) {
          T& F = Fx[(size_t(v) * ny + j) * (nx + 1) + fi];
          F = F + ox[(size_t(j) * wx + fi % wx) * 4 + v];
        }
    if (c.ndim == 2) {
      cnn_apply(*cnn, Xy, nx, wy, wrapy, oy);
      const int glob[4] = {0, 2, 1, 3};  // face frame (rho, n, t, E) -> (rho, x, y, E)
      for (int i = 0; i < nx; ++i)
        for (int fj = 0; fj <= ny; ++fj)
          for (int v = 0; v < 4; ++v) {
            T& G = Fy[(size_t(glob[v]) * (ny + 1) + fj) * nx + i];
            G = G + oy[(size_t(i) * wy + fj % wy) * 4 + v];
          }
    }
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        T r = -(Fx[(size_t(v) * ny + j) * (nx + 1) + i + 1] - Fx[(size_t(v) * ny + j) * (nx + 1) + i]) / dx;
        if (c.ndim == 2)
          r = r - (Fy[(size_t(v) * (ny + 1) + j + 1) * nx + i] - Fy[(size_t(v) * (ny + 1) + j) * nx + i]) / dy;
        if (c.nu_art != 0.0) {
          T lap = (f.at(v, i + 1, j) - 2.0 * f.at(v, i, j) + f.at(v, i - 1, j)) / (dx * dx);
          if (c.ndim == 2) lap = lap + (f.at(v, i, j + 1) - 2.0 * f.at(v, i, j) + f.at(v, i, j - 1)) / (dy * dy);
          r = r + c.nu_art * lap;
        }
        if (ib.active && ib.cls[size_t(j) * nx + i] != FLUID) r = T(0.0);
        L.at(v, i, j) = r;
      }
}

// ------------------------------------------------------------------ SSP-RK3
// Shu-Osher three-stage scheme with a fixed association (left to right):
//   U1 = Un + dt L(Un)
//   U2 = 0.75 Un + 0.25 U1 + (0.25 dt) L(U1)
//   U  = (1/3) Un + (2/3) U2 + ((2/3) dt) L(U2)
// IBM ghost cells are refilled in place before every stage's RHS.
template <class T>
void rk3_step(const Config& c, const Params<T>& P, const Ibm& ib, Field<T>& un, const T& dt,
              const Correction* net, long* fb) {
  Field<T> L(c.nx, c.ny), u1(c.nx, c.ny), u2(c.nx, c.ny);
  ibm_fill(c, P, ib, un);
  rhs(c, P, ib, un, L, net, fb);
#pragma omp parallel for collapse(2) schedule(static)
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < c.ny; ++j)
      for (int i = 0; i < c.nx; ++i) u1.at(v, i, j) = un.at(v, i, j) + dt * L.at(v, i, j);
  ibm_fill(c, P, ib, u1);
  rhs(c, P, ib, u1, L, net, fb);
  const T dt2 = 0.25 * dt;
#pragma omp parallel for collapse(2) schedule(static)
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < c.ny; ++j)
      for (int i = 0; i < c.nx; ++i)
        u2.at(v, i, j) = 0.75 * un.at(v, i, j) + 0.25 * u1.at(v, i, j) + dt2 * L.at(v, i, j);
  ibm_fill(c, P, ib, u2);
  rhs(c, P, ib, u2, L, net, fb);
  const T dt3 = (2.0 / 3.0) * dt;
#pragma omp parallel for collapse(2) schedule(static)
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < c.ny; ++j)
      for (int i = 0; i < c.nx; ++i)
        un.at(v, i, j) = (1.0 / 3.0) * un.at(v, i, j) + (2.0 / 3.0) * u2.at(v, i, j) + dt3 * L.at(v, i, j);
}

// ------------------------------------------------------------- time step
// dt = CFL / max over fluid cells of (|u|+a)/dx + (|v|+a)/dy (1D: x term
// only); Navier-Stokes adds the explicit viscous limit
// dt <= 0.25 min(dx,dy)^2 min(rho) / (mu max(4/3, gamma/Pr)).
inline double cfl_dt(const Config& c, const Ibm& ib, const Field<double>& f) {
  const double dx = dx_of(c), dy = dy_of(c);
  double smax = 0.0, rmin = 1e300;
  // max and min are exact, so the reduction order does not matter
#pragma omp parallel for schedule(static) reduction(max : smax) reduction(min : rmin)
  for (int j = 0; j < c.ny; ++j)
    for (int i = 0; i < c.nx; ++i) {
      if (ib.active && ib.cls[size_t(j) * c.nx + i] != FLUID) continue;
      double U[4] = {f.at(0, i, j), f.at(1, i, j), f.at(2, i, j), f.at(3, i, j)}, W[4];
      cons_to_prim(U, c.gamma, W);
      double a = std::sqrt(c.gamma * W[3] / W[0]);
      double s = (std::fabs(W[1]) + a) / dx;
      if (c.ndim == 2) s = s + (std::fabs(W[2]) + a) / dy;
      smax = std::max(smax, s);
      rmin = std::min(rmin, W[0]);
    }
  double dt = c.cfl / smax;
  if (c.viscous && c.mu > 0.0) {
    double h = c.ndim == 2 ? std::min(dx, dy) : dx;
    double dv = 0.25 * h * h * rmin / (c.mu * std::max(4.0 / 3.0, c.gamma / c.prandtl));
    dt = std::min(dt, dv);
  }
  return dt;
}

}  // namespace orc
