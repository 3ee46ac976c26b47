// Device building blocks of the face flux: primitive conversion, WENO5-JS
// reconstruction and the HLLC Riemann flux, written for gfx950.
//
// All functions are templated on the arithmetic type C (double or float) and
// work in the face-normal frame: component 1 is the normal velocity and
// component 2 the tangential one, so the same code serves x- and y-faces.
#pragma once
#include <hip/hip_runtime.h>

namespace shk {

// Quotient a / b without the IEEE division sequence.  double: the hardware
// reciprocal estimate (relative error below 2^-23) refined by one Newton
// step (below 2^-46), then one correction step on the quotient, which leaves
// an error of about one unit in the last place for normal operands; float:
// hardware reciprocal times a (about one unit in the last place).  Operands
// here are finite and b != 0.
__device__ __forceinline__ double qdiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  double x = a * r;
  return fma(fma(-b, x, a), r, x);
}
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qrcp(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  return fma(fma(-b, r, 1.0), r, r);
}
__device__ __forceinline__ float qrcp(float b) { return __builtin_amdgcn_rcpf(b); }
// Square root: IEEE sequence in double, the hardware estimate in float.
__device__ __forceinline__ double qsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float qsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// 1/sqrt(x) for finite x > 0.  double: the hardware estimate refined by two
// Newton steps y <- y + y (1 - x y^2) / 2 (each squares the relative error),
// which leaves a few units in the last place; float: the hardware estimate.
__device__ __forceinline__ double qrsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-(x * y), y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-(x * y), y, 1.0);
  return fma(0.5 * y, e, y);
}
__device__ __forceinline__ float qrsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
// Speed of sound sqrt(gamma p / rho), formed as gamma p / sqrt(gamma p rho):
// one reciprocal square root instead of a quotient and a square root.
template <class C>
__device__ __forceinline__ C sound_speed(C gamma, C p, C rho) {
  const C gp = gamma * p;
  return gp * qrsqrt(gp * rho);
}

template <class C>
struct Prim {
  C r, un, ut, p;
};

// Ideal-gas primitives from conservative variables (section 2 equation of
// state).  mn/mt are the normal/tangential momenta.
template <class C>
__device__ __forceinline__ Prim<C> to_prim(C rho, C mn, C mt, C E, C gm1) {
  Prim<C> w;
  C ir = qrcp(rho);
  w.r = rho;
  w.un = mn * ir;
  w.ut = mt * ir;
  w.p = gm1 * (E - C(0.5) * rho * (w.un * w.un + w.ut * w.ut));
  return w;
}

// Unnormalised nonlinear weights of a stencil set from G_m = (eps + beta_m)^2:
// the product form (G1 G2, G0 G2, G0 G1) in double, which needs no division
// (every weight is d_m/G_m times the same factor G0 G1 G2); the reciprocals
// (1/G0, 1/G1, 1/G2) in float, where the products, of the order of the
// eighth power of the jump across the stencil, would overflow for jumps
// above about 1e4 (a float reciprocal is one instruction).
__device__ __forceinline__ void weno_products(double g0, double g1, double g2, double P[3]) {
  P[0] = g1 * g2;
  P[1] = g0 * g2;
  P[2] = g0 * g1;
}
__device__ __forceinline__ void weno_products(float g0, float g1, float g2, float P[3]) {
  P[0] = qrcp(g0);
  P[1] = qrcp(g1);
  P[2] = qrcp(g2);
}

// Indicator terms.  In double the Jiang-Shu indicators are formed four
// times over, beta' = 4 beta = (13/3) s^2 + t^2 (s the curvature of the
// triple, t its one-sided slope term), with eps' = 4 eps: every nonlinear
// weight d_m / (eps + beta_m)^2 then carries the same factor 16, which the
// normalisation removes, and the 1/4 of the slope term and the separate eps
// addition disappear (eps' is added once to each triple's curvature term,
// which the two biased values of a face share).  Float keeps the unscaled
// form eps + ((13/12) s^2 + t^2 / 4), whose rounding near strong shocks is
// the one the single-precision path was validated with.
// weno_kterm: the curvature term of the triple (x, y, z); weno_gterm: eps +
// beta from it and the slope term t.
__device__ __forceinline__ double weno_kterm(double x, double y, double z, double eps) {
  const double s = x - 2.0 * y + z;
  return fma((13.0 / 3.0) * s, s, 4.0 * eps);
}
__device__ __forceinline__ double weno_gterm(double t, double k, double) { return fma(t, t, k); }
__device__ __forceinline__ float weno_kterm(float x, float y, float z, float) {
  const float s = x - 2.f * y + z;
  return (13.f / 12.f) * s * s;
}
__device__ __forceinline__ float weno_gterm(float t, float k, float eps) { return eps + (k + 0.25f * t * t); }

// Both WENO5-JS values at the face between c and d of the six cells
// a b c d e f (Jiang-Shu indicators, ideal weights 1/10, 6/10, 3/10, eps):
// the left-biased one from a..e and the right-biased one from the mirrored
// stencil f..b.  The two share the curvature terms of the triples (b,c,d)
// and (c,d,e) and two of the six candidate polynomials, which are formed
// once.  The nonlinear weights d_k/(eps+beta_k)^2 are normalised as
// weno_products describes, which leaves a single division per value.
template <class C>
__device__ __forceinline__ void weno5_pair(C a, C b, C c, C d, C e, C f, C eps, C& left, C& right) {
  // curvature terms of the four triples, symmetric under mirroring
  const C kA = weno_kterm(a, b, c, eps), kB = weno_kterm(b, c, d, eps);
  const C kC = weno_kterm(c, d, e, eps), kD = weno_kterm(d, e, f, eps);
  // left: triples A, B, C
  C g0 = weno_gterm(a - C(4) * b + C(3) * c, kA, eps);
  C g1 = weno_gterm(b - d, kB, eps);
  C g2 = weno_gterm(C(3) * c - C(4) * d + e, kC, eps);
  // right (mirrored): triples D, C, B
  C h0 = weno_gterm(f - C(4) * e + C(3) * d, kD, eps);
  C h1 = weno_gterm(e - c, kC, eps);
  C h2 = weno_gterm(C(3) * d - C(4) * c + b, kB, eps);
  // candidate polynomials (x6); the centred ones coincide across the pair
  const C qm = C(5) * c - b + C(2) * d;  // left q1 = right q2
  const C qp = C(2) * c + C(5) * d - e;  // left q2 = right q1
  const C q0 = C(2) * a - C(7) * b + C(11) * c;
  const C r0 = C(2) * f - C(7) * e + C(11) * d;
  g0 = g0 * g0; g1 = g1 * g1; g2 = g2 * g2;
  h0 = h0 * h0; h1 = h1 * h1; h2 = h2 * h2;
  C Pg[3], Ph[3];
  weno_products(g0, g1, g2, Pg);
  weno_products(h0, h1, h2, Ph);
  const C w0 = C(0.1) * Pg[0], w1 = C(0.6) * Pg[1], w2 = C(0.3) * Pg[2];
  const C v0 = C(0.1) * Ph[0], v1 = C(0.6) * Ph[1], v2 = C(0.3) * Ph[2];
  left = qdiv(w0 * q0 + w1 * qm + w2 * qp, C(6) * (w0 + w1 + w2));
  right = qdiv(v0 * r0 + v1 * qp + v2 * qm, C(6) * (v0 + v1 + v2));
}

// WENO5-JS states of NF consecutive faces from the NF + 5 cells c0.. (the
// stride st apart from f): face k lies between cells k+2 and k+3, its left
// state comes from cells k..k+4 and its right state from the mirrored
// k+5..k+1 -- as weno5_pair on cells k..k+5.  The indicators of a face's
// right state are those of the next face's left state (the same three
// triples of cells, with the ideal weights in reverse order), so NF faces
// need NF + 1 indicator sets instead of 2 NF, and the NF + 3 triples'
// curvature terms are formed once.  Set j (cells j..j+4) holds the weight
// factors P0, P1, P2 (proportional to 1/G0, 1/G1, 1/G2; weno_products) of
// G_m = (eps + beta_m)^2 of the triples starting at j, j+1, j+2 (indicators
// in the left-state orientation, formed by weno_kterm and weno_gterm); the
// left state of face j has the weights (0.1 P0, 0.6 P1, 0.3 P2) on the
// candidates (q0, q1, q2) of cells j..j+4, and the right state of face j-1
// the weights (0.1 P2, 0.6 P1, 0.3 P0) on its candidates (r0, q2, q1).
template <int NF, class C>
__device__ __forceinline__ void weno5_run(const C* f, int st, C eps, C L[NF], C R[NF]) {
  C c[NF + 5];
#pragma unroll
  for (int m = 0; m < NF + 5; ++m) c[m] = f[m * st];
  C kc[NF + 3];  // curvature term of the triple starting at cell t
#pragma unroll
  for (int t = 0; t < NF + 3; ++t) kc[t] = weno_kterm(c[t], c[t + 1], c[t + 2], eps);
  C P[NF + 1][3];
#pragma unroll
  for (int j = 0; j < NF + 1; ++j) {
    C g0 = weno_gterm(c[j] - C(4) * c[j + 1] + C(3) * c[j + 2], kc[j], eps);
    C g1 = weno_gterm(c[j + 1] - c[j + 3], kc[j + 1], eps);
    C g2 = weno_gterm(C(3) * c[j + 2] - C(4) * c[j + 3] + c[j + 4], kc[j + 2], eps);
    g0 = g0 * g0; g1 = g1 * g1; g2 = g2 * g2;
    weno_products(g0, g1, g2, P[j]);
  }
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const C q0 = C(2) * c[k] - C(7) * c[k + 1] + C(11) * c[k + 2];
    const C q1 = C(5) * c[k + 2] - c[k + 1] + C(2) * c[k + 3];
    const C q2 = C(2) * c[k + 2] + C(5) * c[k + 3] - c[k + 4];
    const C r0 = C(2) * c[k + 5] - C(7) * c[k + 4] + C(11) * c[k + 3];
    const C w0 = C(0.1) * P[k][0], w1 = C(0.6) * P[k][1], w2 = C(0.3) * P[k][2];
    const C v0 = C(0.1) * P[k + 1][2], v1 = C(0.6) * P[k + 1][1], v2 = C(0.3) * P[k + 1][0];
    L[k] = qdiv(w0 * q0 + w1 * q1 + w2 * q2, C(6) * (w0 + w1 + w2));
    R[k] = qdiv(v0 * r0 + v1 * q2 + v2 * q1, C(6) * (v0 + v1 + v2));
  }
}

// HLLC flux (section 2) in the face-normal frame, components
// (mass, normal momentum, tangential momentum, energy).
//   wave speeds (Davis): sL = min(uL-aL, uR-aR), sR = max(uL+aL, uR+aR)
//   contact: s* = (pR - pL + rL uL (sL-uL) - rR uR (sR-uR)) / (rL (sL-uL) - rR (sR-uR))
//   star state on side k: (sk-uk)/(sk-s*) [r, r s*, r ut, E + (s*-uk)(r s* + p/(sk-uk))]
// The sign(s*) blend picks the left bracket FL + min(0,sL)(U*L-UL) for
// s* > 0, the right bracket FR + max(0,sR)(U*R-UR) for s* < 0 and their mean
// at s* = 0.
template <class C>
struct Flux4 {
  C f0, f1, f2, f3;
};

// One bracket, evaluated without branches.  With su = s - u and chi = su /
// (s - s*), the star energy chi (E + (s* - u)(rho s* + p / su)) is (su (E +
// (s* - u) rho s*) + (s* - u) p) / (s - s*): su cancels, so one reciprocal
// serves the whole bracket.  On a supersonic side the bracket is the
// physical flux alone: the wave speed and the reciprocal are set to zero
// there, which keeps the star differences finite (whatever s - s* is) and
// adds exactly zero, so lanes of a wavefront never diverge here.
template <class C>
__device__ __forceinline__ Flux4<C> hllc_side(const Prim<C>& w, C E, C s, C ss, bool supersonic) {
  // physical flux of this side
  C mn = w.r * w.un;
  Flux4<C> F;
  F.f0 = mn;
  F.f1 = mn * w.un + w.p;
  F.f2 = mn * w.ut;
  F.f3 = w.un * (E + w.p);
  C su = s - w.un;
  const C id = supersonic ? C(0) : qrcp(s - ss);
  const C se = supersonic ? C(0) : s;
  C chi = su * id;
  C rs = chi * w.r;
  C d0 = rs - w.r;
  C d1 = rs * ss - mn;
  C d2 = d0 * w.ut;
  C du = ss - w.un;
  C d3 = (su * (E + du * (w.r * ss)) + du * w.p) * id - E;
  return Flux4<C>{F.f0 + se * d0, F.f1 + se * d1, F.f2 + se * d2, F.f3 + se * d3};
}

template <class C>
__device__ __forceinline__ C total_energy(const Prim<C>& w, C igm1) {
  return w.p * igm1 + C(0.5) * w.r * (w.un * w.un + w.ut * w.ut);
}

template <class C>
__device__ __forceinline__ Flux4<C> hllc(const Prim<C>& L, const Prim<C>& R, C gamma, C igm1) {
  C aL = sound_speed(gamma, L.p, L.r);
  C aR = sound_speed(gamma, R.p, R.r);
  C sL = fmin(L.un - aL, R.un - aR);
  C sR = fmax(L.un + aL, R.un + aR);
  C dL = sL - L.un, dR = sR - R.un;
  C ss = qdiv(R.p - L.p + L.r * L.un * dL - R.r * R.un * dR, L.r * dL - R.r * dR);
  if (ss == C(0)) {
    // contact exactly at rest: the mean of the two brackets (rare)
    Flux4<C> A = hllc_side(L, total_energy(L, igm1), sL, ss, sL >= C(0));
    Flux4<C> B = hllc_side(R, total_energy(R, igm1), sR, ss, sR <= C(0));
    return Flux4<C>{C(0.5) * (A.f0 + B.f0), C(0.5) * (A.f1 + B.f1), C(0.5) * (A.f2 + B.f2),
                    C(0.5) * (A.f3 + B.f3)};
  }
  // s* > 0: left bracket; s* < 0 (or not a number): right bracket.  The side
  // is chosen first so only one bracket (and one energy) is evaluated per face.
  const bool left = ss > C(0);
  const Prim<C> W{left ? L.r : R.r, left ? L.un : R.un, left ? L.ut : R.ut, left ? L.p : R.p};
  const C s = left ? sL : sR;
  return hllc_side(W, total_energy(W, igm1), s, ss, left ? sL >= C(0) : sR <= C(0));
}

}  // namespace shk
