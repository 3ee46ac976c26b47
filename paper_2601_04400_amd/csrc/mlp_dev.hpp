// Device building blocks of the per-face MLP on gfx950 matrix cores
// (bfloat16 MFMA, FP32 accumulation), shared by the face-batched network
// kernels and the stage kernel that evaluates the network inside its tile.
#pragma once
#include <hip/hip_runtime.h>

#include "grid.hpp"
#include "mlp.hpp"

namespace shk {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned int u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// A operand: rows r0..r0+15 (lane & 15), columns k0 + 4 (lane >> 4) + 0..3 of a
// row-major bf16 matrix with leading dimension ld.
__device__ __forceinline__ bf16x4 ldA(const unsigned short* m, int ld, int r0, int k0, int lane) {
  const unsigned short* p = m + (r0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4);
  return bf16x4{(short)p[0], (short)p[1], (short)p[2], (short)p[3]};
}

// A operand of the transpose: (M^T)[r][k] = M[k][r].
__device__ __forceinline__ bf16x4 ldAT(const unsigned short* m, int ld, int r0, int k0, int lane) {
  const int r = r0 + (lane & 15), k = k0 + 4 * (lane >> 4);
  return bf16x4{(short)m[k * ld + r], (short)m[(k + 1) * ld + r], (short)m[(k + 2) * ld + r],
                (short)m[(k + 3) * ld + r]};
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  return bf16x4{(short)f2bf(a), (short)f2bf(b), (short)f2bf(c), (short)f2bf(d)};
}

// Network input of one 16-face tile from the face's six stencil cells:
// prim(s, w) gives the primitive state (rho, u_n, u_t, p) of stencil cell s
// in the face frame.  Lane (q = lane >> 4, face = lane & 15) holds the
// normalised inputs 4q..4q+3 (cell q) in k-tile 0 and those of cell 4 + q
// (q < 2; zero padding above input 24) in k-tile 1.
template <class Prim6>
__device__ __forceinline__ void net_inputs(const NetArgs& n, int lane, Prim6 prim, bf16x4& x0, bf16x4& x1) {
  const int q = lane >> 4;
  double w[4];
  float xv[4];
  prim(q, w);
#pragma unroll
  for (int v = 0; v < 4; ++v) xv[v] = float((w[v] - n.mean[v]) * n.inv_std[v]);
  x0 = pack4(xv[0], xv[1], xv[2], xv[3]);
  if (q < 2) {
    prim(4 + q, w);
#pragma unroll
    for (int v = 0; v < 4; ++v) xv[v] = float((w[v] - n.mean[v]) * n.inv_std[v]);
    x1 = pack4(xv[0], xv[1], xv[2], xv[3]);
  } else {
    x1 = bf16x4{0, 0, 0, 0};
  }
}

__device__ __forceinline__ void load_net_lds(const NetArgs& n, unsigned short* sw, float* sb) {
  for (int k = threadIdx.x; k < NET_NW; k += blockDim.x) sw[k] = n.w[k];
  for (int k = threadIdx.x; k < NET_NB; k += blockDim.x) sb[k] = n.bias[k];
}

// Forward of one 64-face batch held by a wave.  Returns, for lanes with
// lane>>4 == 0, the pre-tanh outputs z[ft][0..3] of face ft*16 + (lane&15);
// optionally keeps the activations and ReLU masks for the reverse pass.
struct Acts {
  bf16x4 x[2][4];
  bf16x4 h[3][4][4];        // layer, neuron tile, face tile
  unsigned int mask[3][4];  // bit (nt*4 + i) of face tile ft: pre-activation > 0
};

__device__ __forceinline__ void net_forward_batch(const unsigned short* sw, const float* sb, int lane, Acts& A,
                                                  f32x4 z[4]) {
  const int q = lane >> 4;
  // layer 1: 64 x 32
#pragma unroll
  for (int ft = 0; ft < 4; ++ft) A.mask[0][ft] = 0u;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(ldA(sw + NET_OFF_W0, 32, nt * 16, 0, lane), A.x[0][ft], acc);
      acc = mfma(ldA(sw + NET_OFF_W0, 32, nt * 16, 16, lane), A.x[1][ft], acc);
      float hv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float pre = acc[i] + sb[NET_OFF_B0 + nt * 16 + 4 * q + i];
        hv[i] = pre > 0.f ? pre : 0.f;
        if (pre > 0.f) A.mask[0][ft] |= 1u << (nt * 4 + i);
      }
      A.h[0][nt][ft] = pack4(hv[0], hv[1], hv[2], hv[3]);
    }
  // layers 2 and 3: 64 x 64
#pragma unroll
  for (int l = 1; l < 3; ++l) {
    const unsigned short* W = sw + (l == 1 ? NET_OFF_W1 : NET_OFF_W2);
    const float* B = sb + (l == 1 ? NET_OFF_B1 : NET_OFF_B2);
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) A.mask[l][ft] = 0u;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int ft = 0; ft < 4; ++ft) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) acc = mfma(ldA(W, 64, nt * 16, kt * 16, lane), A.h[l - 1][kt][ft], acc);
        float hv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float pre = acc[i] + B[nt * 16 + 4 * q + i];
          hv[i] = pre > 0.f ? pre : 0.f;
          if (pre > 0.f) A.mask[l][ft] |= 1u << (nt * 4 + i);
        }
        A.h[l][nt][ft] = pack4(hv[0], hv[1], hv[2], hv[3]);
      }
  }
  // output layer: 16 (4 used) x 64
#pragma unroll
  for (int ft = 0; ft < 4; ++ft) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) acc = mfma(ldA(sw + NET_OFF_W3, 64, 0, kt * 16, lane), A.h[2][kt][ft], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = acc[i] + sb[NET_OFF_B3 + 4 * q + i];
    z[ft] = acc;
  }
}


}  // namespace shk
