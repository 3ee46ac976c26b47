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

// float -> bfloat16 bits, round to nearest even (the hardware conversion,
// v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ unsigned short f2bf(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// K = 32 products (v_mfma_f32_16x16x32_bf16, twice the rate of the K = 16
// form on gfx950).  The 32 k-slots of lane (q = lane >> 4) are ordered
// 4q..4q+3, 16+4q..16+4q+3 within the block: the concatenation of two
// K = 16 B tiles, i.e. of two D tiles of the layer below, so activations
// still chain from layer to layer without leaving the registers; the A
// operand reads the weight columns in the same order.
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ s16x8 cat8(bf16x4 lo, bf16x4 hi) { return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7); }

__device__ __forceinline__ f32x4 mfma32(s16x8 a, s16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// A operand of K block kb: rows r0 + (lane & 15), columns 32 kb + 4q + 0..3
// and 32 kb + 16 + 4q + 0..3 of a row-major bf16 matrix (ld multiple of 4,
// 8-byte aligned).
__device__ __forceinline__ s16x8 ldA32(const unsigned short* m, int ld, int r0, int kb, int lane) {
  const unsigned short* p = m + (r0 + (lane & 15)) * ld + 32 * kb + 4 * (lane >> 4);
  return cat8(*reinterpret_cast<const bf16x4*>(p), *reinterpret_cast<const bf16x4*>(p + 16));
}

// A operand: rows r0..r0+15 (lane & 15), columns k0 + 4 (lane >> 4) + 0..3 of a
// row-major bf16 matrix with leading dimension ld.
// (ld and k0 are multiples of 4 and m is 8-byte aligned: one 64-bit load.)
__device__ __forceinline__ bf16x4 ldA(const unsigned short* m, int ld, int r0, int k0, int lane) {
  const unsigned short* p = m + (r0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4);
  return *reinterpret_cast<const bf16x4*>(p);
}

// A operand of the transpose: (M^T)[r][k] = M[k][r].
__device__ __forceinline__ bf16x4 ldAT(const unsigned short* m, int ld, int r0, int k0, int lane) {
  const int r = r0 + (lane & 15), k = k0 + 4 * (lane >> 4);
  return bf16x4{(short)m[k * ld + r], (short)m[(k + 1) * ld + r], (short)m[(k + 2) * ld + r],
                (short)m[(k + 3) * ld + r]};
}

// Four floats to bfloat16 (round to nearest even) as two packed conversions
// (v_cvt_pk_bf16_f32 takes a pair).
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  typedef float f32x4v __attribute__((ext_vector_type(4)));
  typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));
  return __builtin_bit_cast(bf16x4, __builtin_convertvector(f32x4v{a, b, c, d}, bf16x4v));
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

// Weights into LDS with the padded row strides (NET_LNW elements; the
// padding columns are never read), biases as they are.
__device__ __forceinline__ void load_net_lds(const NetArgs& n, unsigned short* sw, float* sb) {
  for (int k = threadIdx.x; k < NET_NW; k += blockDim.x) {
    int d;
    if (k < NET_OFF_W1) d = NET_L_W0 + (k >> 5) * NET_LD_W0 + (k & 31);
    else if (k < NET_OFF_W2) d = NET_L_W1 + ((k - NET_OFF_W1) >> 6) * NET_LD_H + (k & 63);
    else if (k < NET_OFF_W3) d = NET_L_W2 + ((k - NET_OFF_W2) >> 6) * NET_LD_H + (k & 63);
    else d = NET_L_W3 + ((k - NET_OFF_W3) >> 6) * NET_LD_H + (k & 63);
    sw[d] = n.w[k];
  }
  for (int k = threadIdx.x; k < NET_NB; k += blockDim.x) sb[k] = n.bias[k];
}

// Forward of one 64-face batch held by a wave.  Returns, for lanes with
// lane>>4 == 0, the pre-tanh outputs z[ft][0..3] of face ft*16 + (lane&15);
// optionally keeps the activations and ReLU masks for the reverse pass.
template <int FT = 4>
struct ActsT {
  bf16x4 x[2][FT];
  bf16x4 h[3][4][FT];        // layer, neuron tile, face tile
  unsigned int mask[3][FT];  // bit 15 - (nt*4 + i) of face tile ft: pre-activation > 0
};
typedef ActsT<4> Acts;

// max(x, 0) as one integer maximum of the bit pattern: every non-negative
// float orders like its bits taken as a signed integer and every negative
// one (-0 included) is below zero, so the result is max(x, 0) with -0 giving
// +0 for every number (a floating-point maximum first quiets a NaN operand,
// a second instruction); a NaN of positive sign passes through, which
// carries it to the network output and its non-finite check.
__device__ __forceinline__ float relu0(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// ReLU of one accumulator tile.  MASK (the reverse pass): the activations
// and the mask bits shifted into m (the tile's four rows in order, each
// appended at bit 0; set where the pre-activation is positive), a select on
// the comparison.  Otherwise the activations alone (relu0).
template <bool MASK>
__device__ __forceinline__ void relu_tile(f32x4 acc, float hv[4], unsigned int& m) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (MASK) {
      const bool pos = acc[i] > 0.f;
      hv[i] = pos ? acc[i] : 0.f;
      m = m * 2u + (pos ? 1u : 0u);
    } else {
      hv[i] = relu0(acc[i]);
    }
  }
}

// FT face tiles of 16 faces per call (FT = 4: 64 faces per wave); MASK:
// keep the ReLU masks (the reverse pass).
template <int FT = 4, bool MASK = false>
__device__ __forceinline__ void net_forward_batch(const unsigned short* sw, const float* sb, int lane, ActsT<FT>& A,
                                                  f32x4 z[FT]) {
  const int q = lane >> 4;
  // layer 1: 64 x 32
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) A.mask[0][ft] = 0u;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      // the accumulator starts at the bias of its four rows
      const float* b0 = sb + NET_OFF_B0 + nt * 16 + 4 * q;
      f32x4 acc = {b0[0], b0[1], b0[2], b0[3]};
      acc = mfma32(ldA32(sw + NET_L_W0, NET_LD_W0, nt * 16, 0, lane), cat8(A.x[0][ft], A.x[1][ft]), acc);
      float hv[4];
      relu_tile<MASK>(acc, hv, A.mask[0][ft]);
      A.h[0][nt][ft] = pack4(hv[0], hv[1], hv[2], hv[3]);
    }
  // layers 2 and 3: 64 x 64
#pragma unroll
  for (int l = 1; l < 3; ++l) {
    const unsigned short* W = sw + (l == 1 ? NET_L_W1 : NET_L_W2);
    const float* B = sb + (l == 1 ? NET_OFF_B1 : NET_OFF_B2);
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) A.mask[l][ft] = 0u;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) {
        const float* bl = B + nt * 16 + 4 * q;
        f32x4 acc = {bl[0], bl[1], bl[2], bl[3]};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
          acc = mfma32(ldA32(W, NET_LD_H, nt * 16, kb, lane), cat8(A.h[l - 1][2 * kb][ft], A.h[l - 1][2 * kb + 1][ft]), acc);
        float hv[4];
        relu_tile<MASK>(acc, hv, A.mask[l][ft]);
        A.h[l][nt][ft] = pack4(hv[0], hv[1], hv[2], hv[3]);
      }
  }
  // output layer: 16 (4 used) x 64
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) {
    const float* b3 = sb + NET_OFF_B3 + 4 * q;
    f32x4 acc = {b3[0], b3[1], b3[2], b3[3]};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
      acc = mfma32(ldA32(sw + NET_L_W3, NET_LD_H, 0, kb, lane), cat8(A.h[2][2 * kb][ft], A.h[2][2 * kb + 1][ft]), acc);
    z[ft] = acc;
  }
}


}  // namespace shk
