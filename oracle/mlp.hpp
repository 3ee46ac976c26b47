// Oracle: the learned face-flux correction (TEST INFRASTRUCTURE ONLY).
//
// Section 2 adds a neural flux F^Neural(U_norm | theta) to the HLLC flux
// inside the divergence, with one parameter set theta shared by the x and y
// directions.  This oracle follows the per-face multilayer-perceptron form:
// input = the 6-cell stencil of primitive states (rho, u_n, u_t, p) in the
// face-normal frame, normalised per variable by a fixed affine map; three
// hidden layers of width 64 with ReLU; a 4-wide output squashed by tanh (the
// paper's final activation) and scaled by a fixed factor.  Weights are
// bfloat16 values; with emulation on, every matrix-product input (weights and
// activations) is rounded to bfloat16 (round to nearest even, via float),
// while sums are carried in double.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "correction.hpp"
#include "dual.hpp"

namespace orc {

using std::tanh;

constexpr int NET_IN = 24, NET_HID = 64, NET_OUT = 4;

struct FluxNet : Correction {
  FluxNet() { kind = CORR_MLP; }
  // Row-major weights: W0 [64][24], W1 [64][64], W2 [64][64], W3 [4][64].
  std::vector<double> W0, W1, W2, W3, b0, b1, b2, b3;
  double mean[4] = {0, 0, 0, 0}, inv_std[4] = {1, 1, 1, 1};
  double out_scale = 1.0;
  bool emulate_bf16 = true;
};

// Round to bfloat16: first to float (nearest even), then to the 8-bit
// significand (nearest even on the dropped 16 bits).
inline double round_bf16(double x) {
  float f = static_cast<float>(x);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return f;  // inf / nan unchanged
  uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7fffu + lsb) & 0xffff0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}
inline double rb(const FluxNet& n, double x) { return n.emulate_bf16 ? round_bf16(x) : x; }
template <int N> inline Dual<N> rb(const FluxNet& n, const Dual<N>& x) {
  Dual<N> r = x;  // rounding changes the value only (straight-through tangent)
  r.v = rb(n, x.v);
  return r;
}

template <class T>
void dense(const FluxNet& n, const std::vector<double>& W, const std::vector<double>& b,
           const T* x, int nin, int nout, bool relu, T* y) {
  for (int o = 0; o < nout; ++o) {
    T acc = T(0.0);
    for (int k = 0; k < nin; ++k) acc = acc + rb(n, W[size_t(o) * nin + k]) * rb(n, x[k]);
    acc = acc + b[o];
    y[o] = (relu && acc < 0.0) ? T(0.0) : acc;
  }
}

template <class T>
void flux_net_apply(const FluxNet* net, const T st[6][4], T dF[4]) {
  const FluxNet& n = *net;
  T x[NET_IN], h1[NET_HID], h2[NET_HID], h3[NET_HID], z[NET_OUT];
  for (int s = 0; s < 6; ++s)
    for (int v = 0; v < 4; ++v) x[s * 4 + v] = (st[s][v] - n.mean[v]) * n.inv_std[v];
  dense(n, n.W0, n.b0, x, NET_IN, NET_HID, true, h1);
  dense(n, n.W1, n.b1, h1, NET_HID, NET_HID, true, h2);
  dense(n, n.W2, n.b2, h2, NET_HID, NET_HID, true, h3);
  dense(n, n.W3, n.b3, h3, NET_HID, NET_OUT, false, z);
  for (int k = 0; k < NET_OUT; ++k) dF[k] = n.out_scale * tanh(z[k]);
}

}  // namespace orc

namespace orc {

// Reverse-mode gradient of the correction for one face, written out by hand:
// given the upstream gradient dFbar of the 4 outputs, accumulate the
// parameter gradient into g (layout W0,b0,W1,b1,W2,b2,W3,b3) and return the
// gradient with respect to the 6x4 stencil.  With emulation on, every
// matrix-product operand (weights, activations and the backward signals) is
// rounded to bfloat16, the rounding being passed through unchanged.
inline void flux_net_backward(const FluxNet& n, const double st[6][4], const double dFbar[4],
                              double* g, double dst[6][4]) {
  double x[NET_IN], a1[NET_HID], h1[NET_HID], a2[NET_HID], h2[NET_HID], a3[NET_HID], h3[NET_HID], z[NET_OUT];
  for (int s = 0; s < 6; ++s)
    for (int v = 0; v < 4; ++v) x[s * 4 + v] = (st[s][v] - n.mean[v]) * n.inv_std[v];
  auto fwd = [&](const std::vector<double>& W, const std::vector<double>& b, const double* in, int nin,
                 int nout, double* pre, double* post, bool relu) {
    for (int o = 0; o < nout; ++o) {
      double acc = 0.0;
      for (int k = 0; k < nin; ++k) acc += rb(n, W[size_t(o) * nin + k]) * rb(n, in[k]);
      acc += b[o];
      pre[o] = acc;
      if (post) post[o] = (relu && acc < 0.0) ? 0.0 : acc;
    }
  };
  fwd(n.W0, n.b0, x, NET_IN, NET_HID, a1, h1, true);
  fwd(n.W1, n.b1, h1, NET_HID, NET_HID, a2, h2, true);
  fwd(n.W2, n.b2, h2, NET_HID, NET_HID, a3, h3, true);
  fwd(n.W3, n.b3, h3, NET_HID, NET_OUT, z, nullptr, false);
  const size_t oW0 = 0, ob0 = oW0 + NET_HID * NET_IN, oW1 = ob0 + NET_HID, ob1 = oW1 + NET_HID * NET_HID,
               oW2 = ob1 + NET_HID, ob2 = oW2 + NET_HID * NET_HID, oW3 = ob2 + NET_HID,
               ob3 = oW3 + NET_OUT * NET_HID;
  double dz[NET_OUT];
  for (int k = 0; k < NET_OUT; ++k) {
    double t = std::tanh(z[k]);
    dz[k] = dFbar[k] * n.out_scale * (1.0 - t * t);
  }
  // layer 3
  double dh3[NET_HID];
  for (int k = 0; k < NET_HID; ++k) dh3[k] = 0.0;
  for (int o = 0; o < NET_OUT; ++o) {
    g[ob3 + o] += dz[o];
    for (int k = 0; k < NET_HID; ++k) {
      g[oW3 + size_t(o) * NET_HID + k] += rb(n, dz[o]) * rb(n, h3[k]);
      dh3[k] += rb(n, n.W3[size_t(o) * NET_HID + k]) * rb(n, dz[o]);
    }
  }
  auto back = [&](const std::vector<double>& W, size_t oW, size_t ob, const double* pre,
                  const double* dpost, const double* in, int nin, int nout, double* din) {
    double da[NET_HID];
    for (int o = 0; o < nout; ++o) da[o] = pre[o] > 0.0 ? dpost[o] : 0.0;
    for (int k = 0; k < nin; ++k) din[k] = 0.0;
    for (int o = 0; o < nout; ++o) {
      g[ob + o] += da[o];
      for (int k = 0; k < nin; ++k) {
        g[oW + size_t(o) * nin + k] += rb(n, da[o]) * rb(n, in[k]);
        din[k] += rb(n, W[size_t(o) * nin + k]) * rb(n, da[o]);
      }
    }
  };
  double dh2[NET_HID], dh1[NET_HID], dx[NET_IN];
  back(n.W2, oW2, ob2, a3, dh3, h2, NET_HID, NET_HID, dh2);
  back(n.W1, oW1, ob1, a2, dh2, h1, NET_HID, NET_HID, dh1);
  back(n.W0, oW0, ob0, a1, dh1, x, NET_IN, NET_HID, dx);
  for (int s = 0; s < 6; ++s)
    for (int v = 0; v < 4; ++v) dst[s][v] = dx[s * 4 + v] * n.inv_std[v];
}

}  // namespace orc
