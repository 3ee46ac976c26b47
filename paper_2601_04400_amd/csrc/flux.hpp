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

// Both WENO5-JS values at the face between c and d of the six cells
// a b c d e f (Jiang-Shu indicators, ideal weights 1/10, 6/10, 3/10, eps):
// the left-biased one from a..e and the right-biased one from the mirrored
// stencil f..b.  The two share the curvature terms of the triples (b,c,d)
// and (c,d,e) and two of the six candidate polynomials, which are formed
// once.  The nonlinear weights d_k/(eps+beta_k)^2 are normalised as
// weno_products describes, which leaves a single division per value.
template <class C>
__device__ __forceinline__ void weno5_pair(C a, C b, C c, C d, C e, C f, C eps, C& left, C& right) {
  const C k13 = C(13) / C(12);
  // curvature (second difference) of each triple, symmetric under mirroring
  const C sA = a - C(2) * b + c, sB = b - C(2) * c + d, sC = c - C(2) * d + e, sD = d - C(2) * e + f;
  const C kB = k13 * sB * sB, kC = k13 * sC * sC;
  // left: triples A, B, C
  C g0 = eps + (k13 * sA * sA + C(0.25) * (a - C(4) * b + C(3) * c) * (a - C(4) * b + C(3) * c));
  C g1 = eps + (kB + C(0.25) * (b - d) * (b - d));
  C g2 = eps + (kC + C(0.25) * (C(3) * c - C(4) * d + e) * (C(3) * c - C(4) * d + e));
  // right (mirrored): triples D, C, B
  C h0 = eps + (k13 * sD * sD + C(0.25) * (f - C(4) * e + C(3) * d) * (f - C(4) * e + C(3) * d));
  C h1 = eps + (kC + C(0.25) * (e - c) * (e - c));
  C h2 = eps + (kB + C(0.25) * (C(3) * d - C(4) * c + b) * (C(3) * d - C(4) * c + b));
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

// WENO5-JS states of three consecutive faces from the eight cells c0..c7 (the
// stride st apart from f): face k (k = 0, 1, 2) lies between cells k+2 and
// k+3, its left state comes from cells k..k+4 and its right state from the
// mirrored k+5..k+1 -- as weno5_pair on cells k..k+5.  The indicators of a
// face's right state are those of the next face's left state (the same three
// triples of cells, with the ideal weights in reverse order), so three faces
// need four indicator sets instead of six, and the six triples' curvature
// terms are formed once.  Set j (cells j..j+4) holds the weight factors
// P0, P1, P2 (proportional to 1/G0, 1/G1, 1/G2; weno_products) of G_m =
// (eps + beta_m)^2 of the triples starting at j, j+1, j+2 (Jiang-Shu
// indicators in the left-state orientation); the left state of face j has
// the weights (0.1 P0, 0.6 P1, 0.3 P2) on the
// candidates (q0, q1, q2) of cells j..j+4, and the right state of face j-1
// the weights (0.1 P2, 0.6 P1, 0.3 P0) on its candidates (r0, q2, q1).
template <class C>
__device__ __forceinline__ void weno5_triple(const C* f, int st, C eps, C L[3], C R[3]) {
  const C k13 = C(13) / C(12);
  C c[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) c[m] = f[m * st];
  C kc[6];  // 13/12 (curvature)^2 of the triple starting at cell t
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const C sc = c[t] - C(2) * c[t + 1] + c[t + 2];
    kc[t] = k13 * sc * sc;
  }
  C P[4][3];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const C t0 = c[j] - C(4) * c[j + 1] + C(3) * c[j + 2];
    const C t1 = c[j + 1] - c[j + 3];
    const C t2 = C(3) * c[j + 2] - C(4) * c[j + 3] + c[j + 4];
    C g0 = eps + (kc[j] + C(0.25) * t0 * t0);
    C g1 = eps + (kc[j + 1] + C(0.25) * t1 * t1);
    C g2 = eps + (kc[j + 2] + C(0.25) * t2 * t2);
    g0 = g0 * g0; g1 = g1 * g1; g2 = g2 * g2;
    weno_products(g0, g1, g2, P[j]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
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

// One bracket, evaluated without branches: the star correction is always
// formed and selected away on a supersonic side (its value there is never
// used, whatever it is), so lanes of a wavefront never diverge here.  With
// su = s - u and chi = su / (s - s*), the star energy chi (E + (s* - u)(rho s*
// + p / su)) is (su (E + (s* - u) rho s*) + (s* - u) p) / (s - s*): su
// cancels, so one reciprocal serves the whole bracket.
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
  C id = qrcp(s - ss);
  C chi = su * id;
  C rs = chi * w.r;
  C d0 = rs - w.r;
  C d1 = rs * ss - mn;
  C d2 = d0 * w.ut;
  C du = ss - w.un;
  C d3 = (su * (E + du * (w.r * ss)) + du * w.p) * id - E;
  Flux4<C> G;
  G.f0 = supersonic ? F.f0 : F.f0 + s * d0;
  G.f1 = supersonic ? F.f1 : F.f1 + s * d1;
  G.f2 = supersonic ? F.f2 : F.f2 + s * d2;
  G.f3 = supersonic ? F.f3 : F.f3 + s * d3;
  return G;
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
