// Learned face-flux correction on gfx950 matrix cores (bfloat16 MFMA, FP32
// accumulation): forward per face, reverse (input and parameter gradients),
// plus the small training kernels (restriction, loss, Adam, BF16 packing).
//
// Section 2 adds a neural flux F^Neural(U_norm | theta) to the HLLC flux in
// the divergence, with one parameter set shared by the x and y directions.
// Here the network is a per-face multilayer perceptron: input = 6-cell
// stencil x (rho, u_n, u_t, p) in the face-normal frame, normalised per
// variable (24 inputs, padded to 32); three hidden layers of 64 with ReLU;
// 4 outputs (padded to 16) through tanh (the paper's last activation) times a
// fixed scale; the correction is in the face frame and rotated back like the
// HLLC flux.
//
// Each wave evaluates 64 faces as four 16-face tiles.  A layer is computed as
// D = W . H^T on the matrix cores: the rows of D are the layer's neurons and
// its columns the faces, which is exactly the B-operand layout of the next
// layer, so activations stay in registers from layer to layer.  The reverse
// pass chains D = W^T . dA the same way; weight gradients are contractions
// over faces (K = faces) whose operands the four waves of a workgroup
// exchange through LDS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "face_dev.hpp"
#include "flux.hpp"
#include "grid.hpp"
#include "mlp.hpp"
#include "mlp_dev.hpp"

namespace shk {

namespace {

__device__ __forceinline__ void build_inputs(const GridArgs& a, const NetArgs& n, const double* __restrict__ Ub,
                                             long long f, int lane, bf16x4& x0, bf16x4& x1) {
  net_inputs(n, lane, [&](int s, double w[4]) { face_cell_prim(a, Ub, f, s, w); }, x0, x1);
}

}  // namespace

// dF[b][face][4] = correction of every face (face frame).  A non-finite
// output is replaced by zero (the uncorrected flux) and flagged.
__global__ void __launch_bounds__(256) net_forward_kernel(GridArgs a, NetArgs n, const double* __restrict__ U,
                                                          float* __restrict__ dF, long long nface) {
  __shared__ __attribute__((aligned(16))) unsigned short sw[NET_LNW];
  __shared__ float sb[NET_NB];
  load_net_lds(n, sw, sb);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b = blockIdx.y;
  const double* __restrict__ Ub = U + (long long)b * 4 * a.ncell;
  float* __restrict__ dFb = dF + (long long)b * nface * 4;
  bool bad = false;
  for (long long base = ((long long)blockIdx.x * 4 + wv) * 64; base < nface; base += (long long)gridDim.x * 256) {
    Acts A;
    for (int ft = 0; ft < 4; ++ft) {
      long long f = base + ft * 16 + (lane & 15);
      if (f >= nface) f = nface - 1;
      build_inputs(a, n, Ub, f, lane, A.x[0][ft], A.x[1][ft]);
    }
    f32x4 z[4];
    net_forward_batch(sw, sb, lane, A, z);
    if ((lane >> 4) == 0) {
      for (int ft = 0; ft < 4; ++ft) {
        const long long f = base + ft * 16 + (lane & 15);
        if (f >= nface) continue;
        float o[4];
        bool ok = true;
        for (int i = 0; i < 4; ++i) {
          o[i] = n.out_scale * tanhf(z[ft][i]);
          ok = ok && isfinite(o[i]);
        }
        if (!ok) { o[0] = o[1] = o[2] = o[3] = 0.f; bad = true; }
        for (int i = 0; i < 4; ++i) dFb[f * 4 + i] = o[i];
      }
    }
  }
  if (bad) atomicOr(&a.glob->fault, 8u);
}

namespace {

// Row stride (bf16 elements) of the reverse pass's exchange tiles: a
// multiple of 4 (8-byte operand reads) that puts the 16 rows of a read on
// distinct LDS bank pairs.
constexpr int TR_LD = 20;

// ReLU mask of the layer below: bit 15 - (tile * 4 + i) of m (relu_tile's
// order), sign-extended to a whole word (all ones or zero) and applied to
// the value's bits.
__device__ __forceinline__ f32x4 relu_mask(f32x4 v, unsigned int m, int tile) {
  f32x4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned int keep = (unsigned int)((int)(m << (16 + tile * 4 + i)) >> 31);
    r[i] = __uint_as_float(__float_as_uint(v[i]) & keep);
  }
  return r;
}

// Sum over the 16 faces of a row group (lanes q*16 .. q*16+15), in a fixed
// order, of a per-lane value.
__device__ __forceinline__ float face_sum16(float v) {
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
  return v;
}

// dH = W^T . dA for a 64 x 64 layer (W^T rows in LDS; dA as bf16 tiles),
// masked by the ReLU of the layer below.
__device__ __forceinline__ void hidden_input_grad(const unsigned short* wT, const bf16x4 (&dA)[4], unsigned int mask,
                                                  f32x4 (&dB)[4], int lane) {
  const s16x8 b0 = cat8(dA[0], dA[1]), b1 = cat8(dA[2], dA[3]);
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma32(ldA32(wT, NET_LD_H, it * 16, 0, lane), b0, acc);
    acc = mfma32(ldA32(wT, NET_LD_H, it * 16, 1, lane), b1, acc);
    dB[it] = relu_mask(acc, mask, it);
  }
}

}  // namespace

// Reverse of the correction.  The upstream gradient of every face flux is
// formed from the right-hand-side adjoint lam (scaled by clam_f * dt[b]), as
// in the flux-difference transpose.  Writes the stencil gradient of every
// face (dX[b][face][6][4], face frame, w.r.t. the primitive states) and this
// block's parameter gradient to part[block][NET_NP].
//
// The four waves of a workgroup take one 16-face tile each per round (tiles
// of all batch members in a fixed order) and run the network forward and
// backward on it.  At each layer they exchange their tiles' pre-activation
// gradients dZ and layer inputs H through LDS (neuron-major, so an operand
// slice of four faces is one 8-byte read), and each wave accumulates one
// quarter of the layer's weight gradient dW += dZ . H^T over the four
// tiles: output rows 16 wv .. 16 wv + 15 of the hidden and first layers,
// input columns 16 wv .. 16 wv + 15 of the output layer (44 accumulator
// values per lane instead of the whole 176).  The bias gradients are FP32
// running sums of each lane's own pre-activation gradients, summed over the
// lanes of a row group and then over the waves in wave order.  Every
// parameter's sum runs in a fixed order: the result is reproducible bit for
// bit.  The reverse products dH = W^T dA read a transposed copy of the
// weights.
__global__ void __launch_bounds__(256, 2) net_backward_kernel(GridArgs a, NetArgs n, const double* __restrict__ U,
                                                           const double* __restrict__ lam, double clam_f,
                                                           const double* __restrict__ dtp, float* __restrict__ dX,
                                                           float* __restrict__ part, long long nface) {
  __shared__ __attribute__((aligned(16))) unsigned short sw[NET_LNW];
  __shared__ __attribute__((aligned(16))) unsigned short swT[NET_TNW];  // W0^T [32][64], W1^T, W2^T, W3^T [64][16]
  __shared__ float sb[NET_NB];
  // per wave: rows 0..63 dZ of the current layer, rows 64..127 its input
  constexpr int XR = 128;
  __shared__ __attribute__((aligned(16))) unsigned short xch[4][XR * TR_LD];
  __shared__ float bred[4][NET_NB];
  load_net_lds(n, sw, sb);
  // transposed copy: element (o, i) of W_l goes to row i, column o
  for (int k = threadIdx.x; k < NET_NW; k += blockDim.x) {
    int d;
    if (k < NET_OFF_W1) {
      d = NET_T_W0 + (k & 31) * NET_LD_H + (k >> 5);
    } else if (k < NET_OFF_W3) {
      const int base = k < NET_OFF_W2 ? NET_OFF_W1 : NET_OFF_W2, kk = k - base;
      d = (k < NET_OFF_W2 ? NET_T_W1 : NET_T_W2) + (kk & 63) * NET_LD_H + (kk >> 6);
    } else {
      const int kk = k - NET_OFF_W3;
      d = NET_T_W3 + (kk & 63) * NET_LD_O + (kk >> 6);
    }
    swT[d] = n.w[k];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, fl = lane & 15;
  unsigned short* xw = xch[wv];
  const int nxf = (a.nx + 1) * a.ny;
  const bool perx = a.bc[0] == BC_PERIODIC, pery = a.bc[2] == BC_PERIODIC;
  // this wave's quarter of the weight gradients
  f32x4 g0[2], g1[4], g2[4], g3;
  f32x4 bs0[4], bs1[4], bs2[4], bs3;  // bias sums of the lane's own faces: [neuron tile] rows 4q..4q+3
  bs3 = g3 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) bs0[ot] = bs1[ot] = bs2[ot] = g1[ot] = g2[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
  g0[0] = g0[1] = f32x4{0.f, 0.f, 0.f, 0.f};
  // D-layout tile (lane (face c, q) holds rows r0 + 4q .. + 3) into this
  // wave's exchange rows, bf16
  auto put = [&](int r0, bf16x4 v) {
#pragma unroll
    for (int i = 0; i < 4; ++i) xw[(r0 + 4 * q + i) * TR_LD + fl] = (unsigned short)v[i];
  };
  // operand slice of wave j's exchange rows: row r0 + (lane & 15), faces 4q .. 4q + 3
  auto get = [&](int j, int r0) { return *reinterpret_cast<const bf16x4*>(&xch[j][(r0 + fl) * TR_LD + 4 * q]); };
  const long long per_b = (nface + 15) / 16;
  const long long total = per_b * a.nbatch;
  // every wave of the workgroup runs the same rounds (a wave past the last
  // tile computes zeros), so the barriers are uniform
  // XCD-aware order: workgroups are dealt to the eight XCDs round-robin, so
  // the k-th workgroup an XCD receives takes block slot start + k of a
  // contiguous run; in each round an XCD then covers one contiguous run of
  // face tiles, whose stencil cells mostly stay in its own L2
  int blk;
  {
    const int n = gridDim.x, x = blockIdx.x & 7, k = blockIdx.x >> 3, qn = n >> 3, rn = n & 7;
    blk = x * qn + (x < rn ? x : rn) + k;
  }
  for (long long t0 = (long long)blk * 4; t0 < total; t0 += (long long)gridDim.x * 4) {
    const long long t = t0 + wv;
    const bool tok = t < total;
    const long long tc = tok ? t : total - 1;
    const int b = (int)(tc / per_b);
    const long long f = (tc % per_b) * 16 + fl;
    const bool fok = tok && f < nface;
    const long long fc = f < nface ? f : nface - 1;
    const double* __restrict__ Ub = U + (long long)b * 4 * a.ncell;
    const double* __restrict__ Lb = lam + (long long)b * 4 * a.ncell;
    // component v of the adjoint of a cell beside the face (zero outside the
    // domain unless periodic, and in solid cells)
    auto lam_cell = [&](int gi, int gj, int v) {
      bool ok = true;
      if (gi < 0 || gi >= a.nx) {
        ok = perx;
        gi += gi < 0 ? a.nx : -a.nx;
      }
      if (gj < 0 || gj >= a.ny) {
        ok = ok && pery;
        gj += gj < 0 ? a.ny : -a.ny;
      }
      const int c = gj * a.nx + gi;
      if (ok && a.cls != nullptr) ok = a.cls[c] == CELL_FLUID;
      return ok ? Lb[(long long)v * a.ncell + c] : 0.0;
    };
    // upstream gradient of the face flux (face frame): lane (face fl, q)
    // forms component q; loaded before the forward so the loads overlap it
    double fbq = 0.0;
    if (fok) {
      const double clam = clam_f * (dtp ? dtp[b] : 1.0);
      const int fi = (int)f;
      if (fi < nxf) {
        const int gj = fi / (a.nx + 1), gf = fi - gj * (a.nx + 1);
        const double sc = clam * a.inv_dx;
        fbq = sc * (lam_cell(gf, gj, q) - lam_cell(gf - 1, gj, q));
      } else {
        const int g = fi - nxf, gf = g / a.nx, gi = g - gf * a.nx;
        const int vy = q == 1 ? 2 : (q == 2 ? 1 : q);
        const double sc = clam * a.inv_dy;
        fbq = sc * (lam_cell(gi, gf, vy) - lam_cell(gi, gf - 1, vy));
      }
    }
    ActsT<1> A;
    f32x4 z[1];
    build_inputs(a, n, Ub, fc, lane, A.x[0][0], A.x[1][0]);
    net_forward_batch<1, true>(sw, sb, lane, A, z);
    // d3 = gradient of the pre-tanh outputs.  Lanes q == 0 hold the outputs
    // z[0][0..3] of face fl; lane (fl, q) takes output q through this wave's
    // exchange rows (nothing reads them before this wave's first barrier of
    // the round), forms its component there, and lanes q == 0 gather the
    // four back.  One wave's LDS operations complete in order.
    f32x4 d3 = {0.f, 0.f, 0.f, 0.f};
    {
      float* zx = reinterpret_cast<float*>(xw);  // [face][4]
      if (q == 0) *reinterpret_cast<f32x4*>(zx + 4 * fl) = z[0];
      const float th = tanhf(zx[4 * fl + q]);
      zx[4 * fl + q] = float(fbq) * n.out_scale * (1.f - th * th);
      if (q == 0) d3 = *reinterpret_cast<const f32x4*>(zx + 4 * fl);
    }
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    f32x4 dA[4], dB[4];
    // every gradient tile is rounded to bf16 once, for the exchange and for
    // the next product
    bf16x4 pk[4];
    // output layer (16 rows, 4 used): dZ3 and H2 out, dH2 = W3^T dZ3
    {
      const bf16x4 b3 = pack4(d3[0], d3[1], d3[2], d3[3]);
      put(0, b3);
#pragma unroll
      for (int it = 0; it < 4; ++it) put(64 + it * 16, A.h[2][it][0]);
      bs3 += d3;
#pragma unroll
      for (int it = 0; it < 4; ++it)
        dA[it] = relu_mask(mfma(ldA(swT + NET_T_W3, NET_LD_O, it * 16, 0, lane), b3, zero), A.mask[2][0], it);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) g3 = mfma(get(j, 0), get(j, 64 + 16 * wv), g3);
    __syncthreads();
    // layer 2: dZ2 = dA, input H1
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
      pk[ot] = pack4(dA[ot][0], dA[ot][1], dA[ot][2], dA[ot][3]);
      put(ot * 16, pk[ot]);
      put(64 + ot * 16, A.h[1][ot][0]);
      bs2[ot] += dA[ot];
    }
    hidden_input_grad(swT + NET_T_W2, pk, A.mask[1][0], dB, lane);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf16x4 ga = get(j, 16 * wv);
#pragma unroll
      for (int it = 0; it < 4; ++it) g2[it] = mfma(ga, get(j, 64 + it * 16), g2[it]);
    }
    __syncthreads();
    // layer 1: dZ1 = dB, input H0
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
      pk[ot] = pack4(dB[ot][0], dB[ot][1], dB[ot][2], dB[ot][3]);
      put(ot * 16, pk[ot]);
      put(64 + ot * 16, A.h[0][ot][0]);
      bs1[ot] += dB[ot];
    }
    hidden_input_grad(swT + NET_T_W1, pk, A.mask[0][0], dA, lane);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf16x4 ga = get(j, 16 * wv);
#pragma unroll
      for (int it = 0; it < 4; ++it) g1[it] = mfma(ga, get(j, 64 + it * 16), g1[it]);
    }
    __syncthreads();
    // first layer (inputs 0..23; 24..31 are zero padding): dZ0 = dA, input X
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
      pk[ot] = pack4(dA[ot][0], dA[ot][1], dA[ot][2], dA[ot][3]);
      put(ot * 16, pk[ot]);
      bs0[ot] += dA[ot];
    }
    put(64, A.x[0][0]);
    put(80, A.x[1][0]);
    {
      // stencil gradient dX = W0^T dA (every lane takes part in the products;
      // the stores are masked)
      const s16x8 b0 = cat8(pk[0], pk[1]), b1 = cat8(pk[2], pk[3]);
      f32x4 dx[2];
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        dx[it] = mfma32(ldA32(swT + NET_T_W0, NET_LD_H, it * 16, 0, lane), b0, zero);
        dx[it] = mfma32(ldA32(swT + NET_T_W0, NET_LD_H, it * 16, 1, lane), b1, dx[it]);
      }
      if (fok) {
        float* out = dX + ((long long)b * nface + f) * 24;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          // input 4*(it*4+q)+i = stencil cell it*4+q, variable i
          const int cell = it * 4 + q;
          if (cell < 6)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[cell * 4 + i] = dx[it][i] * float(n.inv_std[i]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf16x4 ga = get(j, 16 * wv);
      g0[0] = mfma(ga, get(j, 64), g0[0]);
      g0[1] = mfma(ga, get(j, 80), g0[1]);
    }
    __syncthreads();
  }
  // this wave's weight-gradient quarter (lane (in = it * 16 + fl, q) holds
  // output rows 16 wv + 4q .. + 3)
  float* pb = part + (long long)blk * NET_NP;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = 16 * wv + 4 * q + i;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int in = it * 16 + fl;
      pb[NET_G_W1 + o * 64 + in] = g1[it][i];
      pb[NET_G_W2 + o * 64 + in] = g2[it][i];
    }
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int in = it * 16 + fl;
      if (in < 24) pb[NET_G_W0 + o * 24 + in] = g0[it][i];
    }
  }
  if (q == 0)
#pragma unroll
    for (int i = 0; i < 4; ++i) pb[NET_G_W3 + i * 64 + 16 * wv + fl] = g3[i];
  // bias sums: the 16 faces of a row group, then the waves in wave order
#pragma unroll
  for (int ot = 0; ot < 4; ++ot)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = ot * 16 + 4 * q + i;
      const float s0 = face_sum16(bs0[ot][i]), s1 = face_sum16(bs1[ot][i]), s2 = face_sum16(bs2[ot][i]);
      if (fl == 0) {
        bred[wv][o] = s0;
        bred[wv][64 + o] = s1;
        bred[wv][128 + o] = s2;
      }
    }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float s3 = face_sum16(bs3[i]);
    if (q == 0 && fl == 0) bred[wv][192 + i] = s3;
  }
  __syncthreads();
  if (threadIdx.x < 196) {
    const int k = threadIdx.x;
    const float s = ((bred[0][k] + bred[1][k]) + bred[2][k]) + bred[3][k];
    const int dst = k < 64 ? NET_G_B0 + k : (k < 128 ? NET_G_B1 + k - 64 : (k < 192 ? NET_G_B2 + k - 128 : NET_G_B3 + k - 192));
    pb[dst] = s;
  }
}

// grad[k] += sum over the nblk block partials of part, in a fixed order:
// each of the 16 waves of a workgroup sums every 16th partial of 64
// parameters, then the 16 wave sums are added in wave order.
__global__ void __launch_bounds__(1024) net_grad_reduce_kernel(const float* __restrict__ part, int nblk,
                                                               float* __restrict__ grad) {
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (k < NET_NP)
    for (int j = wv; j < nblk; j += 16) s += part[(long long)j * NET_NP + k];
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && k < NET_NP) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w][lane];
    grad[k] += float(t);
  }
}

// bf16 weights (padded MFMA layout) and biases from FP32 master parameters in
// the packed order W0[64][24], b0, W1[64][64], b1, W2[64][64], b2, W3[4][64], b3.
__global__ void __launch_bounds__(256) net_pack_kernel(const float* __restrict__ theta, unsigned short* __restrict__ w,
                                                       float* __restrict__ bias) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < NET_NW) {
    float v = 0.f;
    if (k < NET_OFF_W1) {
      const int o = k / 32, i = k % 32;
      v = i < 24 ? theta[NET_G_W0 + o * 24 + i] : 0.f;
    } else if (k < NET_OFF_W2) {
      v = theta[NET_G_W1 + (k - NET_OFF_W1)];
    } else if (k < NET_OFF_W3) {
      v = theta[NET_G_W2 + (k - NET_OFF_W2)];
    } else {
      const int o = (k - NET_OFF_W3) / 64, i = (k - NET_OFF_W3) % 64;
      v = o < 4 ? theta[NET_G_W3 + o * 64 + i] : 0.f;
    }
    w[k] = f2bf(v);
  }
  if (k < NET_NB) {
    float v = 0.f;
    if (k < 64) v = theta[NET_G_B0 + k];
    else if (k < 128) v = theta[NET_G_B1 + k - 64];
    else if (k < 192) v = theta[NET_G_B2 + k - 128];
    else if (k < 196) v = theta[NET_G_B3 + k - 192];
    bias[k] = v;
  }
}

// Adam (bias-corrected) on the FP32 master parameters.  ic1 = 1/(1 - b1^step)
// and ic2 = 1/(1 - b2^step) come from the host in double: 1 - b2^step
// evaluated in FP32 loses most of its digits to cancellation at small steps.
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ theta, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                   float b1, float b2, float eps, float ic1, float ic2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = grad[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  const float mh = mk * ic1;
  const float vh = vk * ic2;
  theta[k] = theta[k] - lr * mh / (sqrtf(vh) + eps);
}

// Block average of a fine state onto a grid coarser by `factor` in x and y
// (the restriction d(U) of section 2, applied to conservative variables).
__global__ void __launch_bounds__(256) restrict_kernel(const double* __restrict__ fine, double* __restrict__ coarse,
                                                       int nxf, int nyf, int factor, int nvar, int nbatch) {
  const int nxc = nxf / factor, nyc = nyf / factor;
  const long long total = (long long)nbatch * nvar * nxc * nyc;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(k % nxc);
    const int j = (int)((k / nxc) % nyc);
    const long long pv = k / ((long long)nxc * nyc);  // batch * nvar + var
    const double* src = fine + pv * (long long)nxf * nyf;
    double s = 0.0;
    for (int jj = 0; jj < factor; ++jj)
      for (int ii = 0; ii < factor; ++ii) s += src[(long long)(j * factor + jj) * nxf + i * factor + ii];
    coarse[k] = s / double(factor * factor);
  }
}

// Unrolled loss term ||U - T||^2 / N (N = entries per batch member) per batch
// member (block-partial sums, fixed order) and its gradient added to G.
__global__ void __launch_bounds__(256) mse_kernel(const double* __restrict__ U, const double* __restrict__ T,
                                                  double* __restrict__ G, double scale, long long per_b,
                                                  double* __restrict__ part) {
  __shared__ double red[4];
  const int b = blockIdx.y;
  const double* Ub = U + (long long)b * per_b;
  const double* Tb = T + (long long)b * per_b;
  double* Gb = G ? G + (long long)b * per_b : nullptr;
  double s = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < per_b;
       k += (long long)gridDim.x * blockDim.x) {
    const double d = Ub[k] - Tb[k];
    s += d * d;
    if (Gb) Gb[k] += scale * 2.0 * d / double(per_b);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) / double(per_b);
}

// One thread per batch member, 64 members per workgroup.
__global__ void __launch_bounds__(64) mse_finalize_kernel(const double* __restrict__ part, int nblk, int nbatch,
                                                          double* __restrict__ loss) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= nbatch) return;
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += part[(long long)b * nblk + k];
  loss[b] += s;
}

// Block partials of launch_mse_noalloc: one copy per GPU, kept until the
// process ends.  Host code never passes this name to a kernel (on the host it
// is a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns on each device.
static __device__ __align__(256) double scratch[MSE_NOALLOC_MAX_BATCH * 256];

// ------------------------------------------------------------------ launchers
long long net_face_count(const GridArgs& a) {
  return (long long)(a.nx + 1) * a.ny + (long long)a.nx * (a.ny + 1);
}

static unsigned int net_blocks(long long nface) {
  long long nb = (nface + 255) / 256;
  if (nb > 1024) nb = 1024;
  return (unsigned int)(nb < 1 ? 1 : nb);
}

// Reverse pass: 64-face batches of all members over at most NET_BWD_BLOCKS
// workgroups (one parameter partial each).
unsigned int net_backward_blocks(const GridArgs& a) {
  const long long tiles = (net_face_count(a) + 15) / 16 * a.nbatch;
  long long nb = (tiles + 3) / 4;
  if (nb > NET_BWD_BLOCKS) nb = NET_BWD_BLOCKS;
  return (unsigned int)(nb < 1 ? 1 : nb);
}

hipError_t launch_net_forward(const GridArgs& a, const NetArgs& n, const double* U, float* dF, hipStream_t st) {
  const long long nf = net_face_count(a);
  if (nf > 0x7fffffffLL) return hipErrorInvalidValue;  // faces of a batch member are indexed in 32 bits
  hipLaunchKernelGGL(net_forward_kernel, dim3(net_blocks(nf), a.nbatch), dim3(256), 0, st, a, n, U, dF, nf);
  return hipGetLastError();
}

hipError_t launch_net_backward(const GridArgs& a, const NetArgs& n, const double* U, const double* lam, double clam_f,
                               const double* dtp, float* dX, float* part, float* grad, hipStream_t st) {
  const long long nf = net_face_count(a);
  if (nf > 0x7fffffffLL) return hipErrorInvalidValue;  // faces of a batch member are indexed in 32 bits
  const unsigned int nb = net_backward_blocks(a);
  hipLaunchKernelGGL(net_backward_kernel, dim3(nb), dim3(256), 0, st, a, n, U, lam, clam_f, dtp, dX, part, nf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !grad) return e;
  hipLaunchKernelGGL(net_grad_reduce_kernel, dim3((NET_NP + 63) / 64), dim3(1024), 0, st, part, (int)nb, grad);
  return hipGetLastError();
}

hipError_t launch_net_pack(const float* theta, unsigned short* w, float* bias, hipStream_t st) {
  hipLaunchKernelGGL(net_pack_kernel, dim3((NET_NW + 255) / 256), dim3(256), 0, st, theta, w, bias);
  return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st) {
  const float ic1 = float(1.0 / (1.0 - std::pow(double(b1), step)));
  const float ic2 = float(1.0 / (1.0 - std::pow(double(b2), step)));
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, theta, grad, m, v, n, lr, b1, b2, eps,
                     ic1, ic2);
  return hipGetLastError();
}

hipError_t launch_restrict(const double* fine, double* coarse, int nxf, int nyf, int factor, int nvar, int nbatch,
                           hipStream_t st) {
  const long long total = (long long)nbatch * nvar * (nxf / factor) * (nyf / factor);
  long long nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(restrict_kernel, dim3((unsigned int)(nb < 1 ? 1 : nb)), dim3(256), 0, st, fine, coarse, nxf, nyf,
                     factor, nvar, nbatch);
  return hipGetLastError();
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
double* scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call on that device.
hipError_t scratch_address(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

hipError_t launch_mse_noalloc(const double* U, const double* T, double* G, double scale, long long per_b, int nbatch,
                              double* loss, hipStream_t st) {
  if (nbatch < 1 || nbatch > MSE_NOALLOC_MAX_BATCH) return hipErrorInvalidValue;
  double* part = nullptr;
  hipError_t e = scratch_address(&part);
  if (e != hipSuccess) return e;
  // mse_kernel writes every partial launch_mse's finaliser reads, so the
  // array needs no clearing between calls.
  return launch_mse(U, T, G, scale, per_b, nbatch, part, loss, st);
}

hipError_t launch_mse(const double* U, const double* T, double* G, double scale, long long per_b, int nbatch,
                      double* part, double* loss, hipStream_t st) {
  unsigned int nb = (unsigned int)((per_b + 255) / 256);
  if (nb > 256) nb = 256;
  hipLaunchKernelGGL(mse_kernel, dim3(nb, nbatch), dim3(256), 0, st, U, T, G, scale, per_b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mse_finalize_kernel, dim3((nbatch + 63) / 64), dim3(64), 0, st, part, (int)nb, nbatch, loss);
  return hipGetLastError();
}

}  // namespace shk
