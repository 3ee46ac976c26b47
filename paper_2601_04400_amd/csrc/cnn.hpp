// Convolutional learned flux correction: parameter layouts and launchers
// shared by the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "grid.hpp"

namespace shk {

// Packed parameter vector theta (FP32, the order of gradients and Adam):
// W1 [16][3][3][4], b1 [16], W2 [32][3][3][16], b2 [32], W3 [4][3][3][32], b3 [4].
constexpr int CNN_G_W1 = 0, CNN_G_B1 = 576, CNN_G_W2 = 592, CNN_G_B2 = 5200, CNN_G_W3 = 5232, CNN_G_B3 = 6384,
              CNN_NP = 6388;
// Device weights (bf16), each a row-major matrix used as the MFMA A operand
// [rows][K] with K = 3x3 taps x channels (k = tap * C + c, tap = 3 dr + dc):
//   F1 [16][48]  layer 1 forward (k >= 36 zero)
//   F2 [32][144] layer 2 forward
//   F3 [16][288] layer 3 forward (rows >= 4 zero)
//   B3 [32][48]  input gradient of layer 3: row = its input channel, taps
//                mirrored, k = tap * 4 + output channel (k >= 36 zero)
//   B2 [16][288] input gradient of layer 2
//   B1 [16][144] input gradient of layer 1 (rows >= 4 zero)
constexpr int CNN_F1 = 0, CNN_F2 = 768, CNN_F3 = 5376, CNN_B3 = 9984, CNN_B2 = 11520, CNN_B1 = 16128, CNN_NW = 18432;
// FP32 biases: b1 [16], b2 [32], b3 [16] (4 used)
constexpr int CNN_BB1 = 0, CNN_BB2 = 16, CNN_BB3 = 48, CNN_NB = 64;
constexpr int CNN_BLOCKS = 512;  // workgroups (and parameter partials) of the weight-gradient kernels
// hidden-layer bias sums of the input-gradient layers: one row of CNN_BROW
// per workgroup (b1 at 0..15, b2 at 16..47), at most CNN_BMAX workgroups
constexpr int CNN_BROW = 48, CNN_BMAX = 8192;

struct CnnArgs {
  const unsigned short* w;  // [CNN_NW] bf16
  const float* bias;        // [CNN_NB]
  double mean[4], inv_std[4];
  float out_scale;
};

// The two images of a batch member: x-faces (ny rows, wx columns) and the
// y-faces transposed (nx rows, wy columns); a periodic axis holds each face
// once (wx = nx, else nx + 1; likewise wy).  Pixel p of member b, channel c
// of a C-channel buffer: [(b * npix + p) * C + c], image 1 after image 0.
struct CnnGeom {
  int H[2], W[2];
  int wrapR[2], wrapC[2];
  int tilesR[2], tilesC[2];  // 16 x 16 tiles per image
  int npix, tiles;           // pixels and tiles per batch member
  int nbatch;
};

CnnGeom cnn_geom(const GridArgs& a);
// workspace of one grid: images and per-block partials, in bytes
size_t cnn_workspace_bytes(const GridArgs& a);

struct CnnBufs {
  unsigned short *x, *h1, *h2, *dz, *da2, *da1;  // bf16 images: 4, 16, 32, 4, 32, 16 channels
  float *t;                                       // tanh of the output layer [npix][4]
  float *dx;                                      // input gradient [npix][4]
  float *part;                                    // [CNN_BLOCKS][CNN_NP]
  float *bpart;                                   // [CNN_BMAX][CNN_BROW]
};
CnnBufs cnn_bufs(const GridArgs& a, char* base);

hipError_t launch_cnn_pack(const float* theta, unsigned short* w, float* bias, hipStream_t st);
// forward: correction of every face dF [nbatch][nface][4] (face frame) from
// the state U; with keep, also the activations in bufs for the reverse pass
hipError_t launch_cnn_forward(const GridArgs& a, const CnnArgs& n, const double* U, float* dF, const CnnBufs& b,
                              bool keep, hipStream_t st);
// reverse: from the right-hand-side adjoint lam (scaled by clam_f * dt[b]),
// recomputes the forward, writes the stencil gradient of every face
// dX [nbatch][nface][24] (face frame, w.r.t. the primitive states) and adds
// the parameter gradient to grad (fixed-order sums), if grad is set
hipError_t launch_cnn_backward(const GridArgs& a, const CnnArgs& n, const double* U, const double* lam,
                               double clam_f, const double* dtp, float* dX, float* dF, const CnnBufs& b, float* grad,
                               hipStream_t st);
// the input images as float [nbatch][npix][4] (the bf16 values), for tests
hipError_t launch_cnn_images(const GridArgs& a, const CnnArgs& n, const double* U, const CnnBufs& b, float* out,
                             hipStream_t st);

}  // namespace shk
