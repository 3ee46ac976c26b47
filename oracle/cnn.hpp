// Oracle: the convolutional form of the learned flux correction (TEST
// INFRASTRUCTURE ONLY).
//
// Section 2: for 2D runs the neural flux is a fully convolutional network of
// three 3x3 layers -- ReLU, ReLU, tanh -- with 6,388 parameters and SAME
// (zero) padding, applied pixel by pixel to the normalised WENO-reconstructed
// states of each direction, one parameter set serving both directions.  Here
// (channels 4 -> 16 -> 32 -> 4):
//  * the pixels of direction x are the x-faces, an image of ny rows and
//    nx + 1 columns; those of direction y are the y-faces transposed, nx rows
//    and ny + 1 columns, so that the face normal runs along the image's
//    second axis in both;
//  * the 3x3 windows are padded with zeros (SAME) at domain boundaries and
//    wrap around across periodic ones; along a periodic axis the image
//    holds each face once (nx columns: the last face is the first), so the
//    corrected scheme stays conservative on periodic grids;
//  * a face's input is the conservative form of the mean of its two
//    reconstructed states, in the face frame (rho, rho u_n, rho u_t, E),
//    normalised per channel by a fixed affine map;
//  * its output is the face-frame flux correction out_scale * tanh(z).
// Weights are bfloat16 values; with emulation on, every product operand
// (weights and activations, forward and backward) is rounded to bfloat16 and
// sums are carried in double, as in the per-face network.
#pragma once
#include <cmath>
#include <vector>

#include "mlp.hpp"

namespace orc {

constexpr int CNN_C0 = 4, CNN_C1 = 16, CNN_C2 = 32, CNN_C3 = 4;
// Parameter vector: W1 [16][3][3][4], b1 [16], W2 [32][3][3][16], b2 [32],
// W3 [4][3][3][32], b3 [4].
constexpr int CNN_PARAMS = 16 * 9 * 4 + 16 + 32 * 9 * 16 + 32 + 4 * 9 * 32 + 4;

struct FluxCnn : Correction {
  std::vector<double> W1, b1, W2, b2, W3, b3;
  double mean[4] = {0, 0, 0, 0}, inv_std[4] = {1, 1, 1, 1};
  double out_scale = 1.0;
  bool emulate_bf16 = true;
  FluxCnn() { kind = CORR_CNN; }
};

inline double rb(const FluxCnn& n, double x) { return n.emulate_bf16 ? round_bf16(x) : x; }
template <int N> inline Dual<N> rb(const FluxCnn& n, const Dual<N>& x) {
  Dual<N> r = x;  // rounding changes the value only (straight-through tangent)
  r.v = rb(n, x.v);
  return r;
}

// An image axis of n pixels: index k of a 3x3 window, wrapped when the axis
// is periodic, -1 (zero padding) when it falls outside otherwise.
inline int cnn_pixel(int k, int n, bool wrap) {
  if (k >= 0 && k < n) return k;
  return wrap ? (k + n) % n : -1;
}

// Pre-activations of one 3x3 layer on an H x Wd image, channels last:
// pre[r][c][co] = b[co] + sum over the 3x3 window and the input channels of
// W[co][dr][dc][ci] * in[r + dr - 1][c + dc - 1][ci], the window padded with
// zeros (SAME) or wrapped around along a periodic axis (wrap[0]: rows,
// wrap[1]: columns).
template <class T>
void conv3x3(const FluxCnn& n, const std::vector<double>& W, const std::vector<double>& b, const std::vector<T>& in,
             int H, int Wd, const bool wrap[2], int cin, int cout, std::vector<T>& pre) {
  pre.assign(size_t(H) * Wd * cout, T(0.0));
  for (int r = 0; r < H; ++r)
    for (int c = 0; c < Wd; ++c)
      for (int co = 0; co < cout; ++co) {
        T acc = T(0.0);
        for (int dr = 0; dr < 3; ++dr)
          for (int dc = 0; dc < 3; ++dc) {
            const int rr = cnn_pixel(r + dr - 1, H, wrap[0]), cc = cnn_pixel(c + dc - 1, Wd, wrap[1]);
            if (rr < 0 || cc < 0) continue;
            for (int ci = 0; ci < cin; ++ci)
              acc = acc + rb(n, W[((size_t(co) * 3 + dr) * 3 + dc) * cin + ci]) *
                              rb(n, in[(size_t(rr) * Wd + cc) * cin + ci]);
          }
        pre[(size_t(r) * Wd + c) * cout + co] = acc + b[co];
      }
}

template <class T>
T cnn_norm(const FluxCnn* n, int v, const T& x) {
  return (x - n->mean[v]) * n->inv_std[v];
}

template <class T>
void relu_inplace(std::vector<T>& a) {
  for (auto& x : a)
    if (x < 0.0) x = T(0.0);
}

// The correction of every pixel of one image: x = normalised inputs
// [H][Wd][4], out = out_scale * tanh(z) [H][Wd][4].
template <class T>
void cnn_apply(const FluxCnn& n, const std::vector<T>& x, int H, int Wd, const bool wrap[2], std::vector<T>& out) {
  std::vector<T> h1, h2, z;
  conv3x3(n, n.W1, n.b1, x, H, Wd, wrap, CNN_C0, CNN_C1, h1);
  relu_inplace(h1);
  conv3x3(n, n.W2, n.b2, h1, H, Wd, wrap, CNN_C1, CNN_C2, h2);
  relu_inplace(h2);
  conv3x3(n, n.W3, n.b3, h2, H, Wd, wrap, CNN_C2, CNN_C3, z);
  out.resize(z.size());
  for (size_t k = 0; k < z.size(); ++k) out[k] = n.out_scale * tanh(z[k]);
}

// Reverse mode for one image, written out by hand: given the upstream
// gradient dOut of the outputs, add the parameter gradient to g (layout
// W1, b1, W2, b2, W3, b3) and return the gradient with respect to the
// normalised inputs.  Every product operand is rounded as in the forward
// pass (the backward signals included); bias gradients are the unrounded
// sums of the pre-activation gradients.
inline void cnn_backward(const FluxCnn& n, const std::vector<double>& x, int H, int Wd, const bool wrap[2],
                         const std::vector<double>& dOut, double* g, std::vector<double>& dx) {
  std::vector<double> a1, h1, a2, h2, z;
  conv3x3(n, n.W1, n.b1, x, H, Wd, wrap, CNN_C0, CNN_C1, a1);
  h1 = a1;
  relu_inplace(h1);
  conv3x3(n, n.W2, n.b2, h1, H, Wd, wrap, CNN_C1, CNN_C2, a2);
  h2 = a2;
  relu_inplace(h2);
  conv3x3(n, n.W3, n.b3, h2, H, Wd, wrap, CNN_C2, CNN_C3, z);
  const size_t oW1 = 0, ob1 = oW1 + 16 * 9 * 4, oW2 = ob1 + 16, ob2 = oW2 + 32 * 9 * 16, oW3 = ob2 + 32,
               ob3 = oW3 + 4 * 9 * 32;
  std::vector<double> dz(z.size());
  for (size_t k = 0; k < z.size(); ++k) {
    const double t = std::tanh(z[k]);
    dz[k] = dOut[k] * n.out_scale * (1.0 - t * t);
  }
  // one layer: da = gradient of its pre-activations, in = its input image;
  // adds dW, db and returns din (before the mask of the layer below)
  auto back = [&](const std::vector<double>& W, size_t oW, size_t ob, const std::vector<double>& da,
                  const std::vector<double>& in, int cin, int cout, std::vector<double>& din) {
    din.assign(size_t(H) * Wd * cin, 0.0);
    for (int r = 0; r < H; ++r)
      for (int c = 0; c < Wd; ++c)
        for (int co = 0; co < cout; ++co) {
          const double d = da[(size_t(r) * Wd + c) * cout + co];
          g[ob + co] += d;
          const double dr_ = rb(n, d);
          for (int dr = 0; dr < 3; ++dr)
            for (int dc = 0; dc < 3; ++dc) {
              const int rr = cnn_pixel(r + dr - 1, H, wrap[0]), cc = cnn_pixel(c + dc - 1, Wd, wrap[1]);
              if (rr < 0 || cc < 0) continue;
              for (int ci = 0; ci < cin; ++ci) {
                const size_t wi = ((size_t(co) * 3 + dr) * 3 + dc) * cin + ci;
                const size_t ii = (size_t(rr) * Wd + cc) * cin + ci;
                g[oW + wi] += dr_ * rb(n, in[ii]);
                din[ii] += rb(n, W[wi]) * dr_;
              }
            }
        }
  };
  std::vector<double> dh2, dh1;
  back(n.W3, oW3, ob3, dz, h2, CNN_C2, CNN_C3, dh2);
  for (size_t k = 0; k < dh2.size(); ++k)
    if (!(a2[k] > 0.0)) dh2[k] = 0.0;
  back(n.W2, oW2, ob2, dh2, h1, CNN_C1, CNN_C2, dh1);
  for (size_t k = 0; k < dh1.size(); ++k)
    if (!(a1[k] > 0.0)) dh1[k] = 0.0;
  back(n.W1, oW1, ob1, dh1, x, CNN_C0, CNN_C1, dx);
}

}  // namespace orc
