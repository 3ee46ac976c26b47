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
// D = W . H^T with v_mfma_f32_16x16x16_bf16: the rows of D are the layer's
// neurons and its columns the faces, which is exactly the B-operand layout
// of the next layer, so activations stay in registers from layer to layer.
// The reverse pass chains D = W^T . dA the same way; weight gradients are
// contractions over faces (K = faces) whose operands are transposed through a
// small per-wave LDS tile.
#include <hip/hip_runtime.h>

#include <cmath>

#include "flux.hpp"
#include "grid.hpp"
#include "mlp.hpp"
#include "mlp_dev.hpp"

namespace shk {

namespace {

// Primitive state (rho, u_n, u_t, p) of stencil cell s (0..5) of face f of
// batch member Ub; x-faces first ((nx+1) per row), then y-faces (nx per row).
__device__ __forceinline__ void face_cell_prim(const GridArgs& a, const double* __restrict__ Ub, long long f, int s,
                                               double w[4]) {
  const long long nxf = (long long)(a.nx + 1) * a.ny;
  int gi, gj;
  bool isx = f < nxf;
  if (isx) {
    gj = (int)(f / (a.nx + 1));
    gi = (int)(f % (a.nx + 1)) - 3 + s;
  } else {
    const long long g = f - nxf;
    gj = (int)(g / a.nx) - 3 + s;
    gi = (int)(g % a.nx);
  }
  double q[4];
  // boundary rules as in the stage kernel
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

__device__ __forceinline__ void build_inputs(const GridArgs& a, const NetArgs& n, const double* __restrict__ Ub,
                                             long long f, int lane, bf16x4& x0, bf16x4& x1) {
  net_inputs(n, lane, [&](int s, double w[4]) { face_cell_prim(a, Ub, f, s, w); }, x0, x1);
}

}  // namespace

// dF[b][face][4] = correction of every face (face frame).  A non-finite
// output is replaced by zero (the uncorrected flux) and flagged.
__global__ void __launch_bounds__(256) net_forward_kernel(GridArgs a, NetArgs n, const double* __restrict__ U,
                                                          float* __restrict__ dF, long long nface) {
  __shared__ __attribute__((aligned(16))) unsigned short sw[NET_NW];
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

struct BwdCtx {
  const unsigned short* sw;
  float* gsum;
  unsigned short* trA;
  unsigned short* trH;
  int lane, wv;
  bool live;
};

// Reverse of layer L (0 = first hidden, 3 = output): adds the parameter
// gradient of the wave's 64 faces to the block's LDS sums (waves in a fixed
// order), then maps dA to the gradient of the layer input, applying the ReLU
// mask of the layer below (or returning it in dX for the network input).
template <int L>
__device__ __forceinline__ void bwd_layer(const BwdCtx& c, const Acts& A, f32x4 (&dA)[4][4],
                                          f32x4 (*dX)[4] = nullptr) {
  constexpr int NOUT = L == 3 ? 1 : 4;
  constexpr int NIN = L == 0 ? 2 : 4;
  constexpr int LD = L == 0 ? 32 : 64;
  constexpr int IN_REAL = L == 0 ? 24 : 64;
  constexpr int OUT_REAL = L == 3 ? 4 : 64;
  constexpr int OFFW = L == 0 ? NET_OFF_W0 : L == 1 ? NET_OFF_W1 : L == 2 ? NET_OFF_W2 : NET_OFF_W3;
  constexpr int GW = L == 0 ? NET_G_W0 : L == 1 ? NET_G_W1 : L == 2 ? NET_G_W2 : NET_G_W3;
  constexpr int GB = L == 0 ? NET_G_B0 : L == 1 ? NET_G_B1 : L == 2 ? NET_G_B2 : NET_G_B3;
  const int lane = c.lane, q = lane >> 4, fl = lane & 15;
  const unsigned short* W = c.sw + OFFW;
  f32x4 gw[NOUT][NIN];
  float gb[NOUT][4];
#pragma unroll
  for (int ot = 0; ot < NOUT; ++ot) {
#pragma unroll
    for (int it = 0; it < NIN; ++it) gw[ot][it] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float s = 0.f;
#pragma unroll
      for (int ft = 0; ft < 4; ++ft) s += dA[ot][ft][i];
      for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);  // the 16 faces of a lane group
      gb[ot][i] = s;
    }
  }
  if (c.live) {
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) {
#pragma unroll
      for (int ot = 0; ot < NOUT; ++ot) {
        // dA tile (rows = outputs, columns = faces) -> A operand [output][face]
#pragma unroll
        for (int i = 0; i < 4; ++i) c.trA[(4 * q + i) * 16 + fl] = f2bf(dA[ot][ft][i]);
        __builtin_amdgcn_wave_barrier();
        const bf16x4 aop = ldA(c.trA, 16, 0, 0, lane);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int it = 0; it < NIN; ++it) {
          const bf16x4 hin = L == 0 ? A.x[it][ft] : A.h[L == 0 ? 0 : L - 1][it][ft];
#pragma unroll
          for (int i = 0; i < 4; ++i) c.trH[(4 * q + i) * 16 + fl] = (unsigned short)hin[i];
          __builtin_amdgcn_wave_barrier();
          const bf16x4 bop = ldA(c.trH, 16, 0, 0, lane);  // B[face][input]
          __builtin_amdgcn_wave_barrier();
          gw[ot][it] = mfma(aop, bop, gw[ot][it]);
        }
      }
    }
  }
  for (int w2 = 0; w2 < 4; ++w2) {
    if (c.wv == w2 && c.live) {
#pragma unroll
      for (int ot = 0; ot < NOUT; ++ot) {
#pragma unroll
        for (int it = 0; it < NIN; ++it)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int o = ot * 16 + 4 * q + i, in = it * 16 + fl;
            if (o < OUT_REAL && in < IN_REAL) c.gsum[GW + o * IN_REAL + in] += gw[ot][it][i];
          }
        if (fl == 0)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int o = ot * 16 + 4 * q + i;
            if (o < OUT_REAL) c.gsum[GB + o] += gb[ot][i];
          }
      }
    }
    __syncthreads();
  }
  // input gradient: dH = W^T dA, then the ReLU mask of the layer below
  f32x4 dH[NIN][4];
#pragma unroll
  for (int it = 0; it < NIN; ++it)
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ot = 0; ot < NOUT; ++ot) {
        const bf16x4 bop = pack4(dA[ot][ft][0], dA[ot][ft][1], dA[ot][ft][2], dA[ot][ft][3]);
        acc = mfma(ldAT(W, LD, it * 16, ot * 16, lane), bop, acc);
      }
      dH[it][ft] = acc;
    }
  if (L > 0) {
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dA[it][ft][i] = ((A.mask[L == 0 ? 0 : L - 1][ft] >> (it * 4 + i)) & 1u) ? dH[it < NIN ? it : 0][ft][i] : 0.f;
  } else {
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
      for (int ft = 0; ft < 4; ++ft) dX[it][ft] = dH[it][ft];
  }
}

}  // namespace

// Reverse of the correction.  The upstream gradient of every face flux is
// formed from the right-hand-side adjoint lam (scaled by clam_f * dt[b]), as
// in the flux-difference transpose.  Writes the stencil gradient of every
// face (dX[b][face][6][4], face frame, w.r.t. the primitive states) and adds
// this block's parameter gradient to part[block][NET_NP] (fixed order).
__global__ void __launch_bounds__(256) net_backward_kernel(GridArgs a, NetArgs n, const double* __restrict__ U,
                                                           const double* __restrict__ lam, double clam_f,
                                                           const double* __restrict__ dtp, float* __restrict__ dX,
                                                           float* __restrict__ part, long long nface) {
  __shared__ __attribute__((aligned(16))) unsigned short sw[NET_NW];
  __shared__ float sb[NET_NB];
  __shared__ float gsum[NET_NP];
  __shared__ __attribute__((aligned(16))) unsigned short tr[4][2][16 * 16];  // per wave: dA tile, H tile, [row][face]
  load_net_lds(n, sw, sb);
  for (int k = threadIdx.x; k < NET_NP; k += blockDim.x) gsum[k] = 0.f;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, fl = lane & 15;
  const long long nxf = (long long)(a.nx + 1) * a.ny;
  const bool perx = a.bc[0] == BC_PERIODIC, pery = a.bc[2] == BC_PERIODIC;
  const double* __restrict__ Lb = lam;
  auto lam_at = [&](int v, int gi, int gj) -> double {
    if (gi < 0 || gi >= a.nx) {
      if (!perx) return 0.0;
      gi = ((gi % a.nx) + a.nx) % a.nx;
    }
    if (gj < 0 || gj >= a.ny) {
      if (!pery) return 0.0;
      gj = ((gj % a.ny) + a.ny) % a.ny;
    }
    const long long c = (long long)gj * a.nx + gi;
    if (a.cls != nullptr && a.cls[c] != CELL_FLUID) return 0.0;
    return Lb[v * a.ncell + c];
  };
  unsigned short* trA = tr[wv][0];
  unsigned short* trH = tr[wv][1];
  // 64-face batches of all batch members, dealt to the blocks in a fixed
  // order (every block runs the same number of rounds)
  const long long per_b = (nface + 63) / 64;
  const long long total = per_b * a.nbatch;
  for (long long g0 = (long long)blockIdx.x * 4; g0 < total; g0 += (long long)gridDim.x * 4) {
    const long long gb = g0 + wv;
    const bool live = gb < total;
    const int b = live ? (int)(gb / per_b) : 0;
    const long long base = live ? (gb % per_b) * 64 : 0;
    const double* __restrict__ Ub = U + (long long)b * 4 * a.ncell;
    Lb = lam + (long long)b * 4 * a.ncell;
    const double clam = clam_f * (dtp ? dtp[b] : 1.0);
    Acts A;
    f32x4 z[4];
    float Fb[4][4];
    for (int ft = 0; ft < 4; ++ft)
      for (int i = 0; i < 4; ++i) Fb[ft][i] = 0.f;
    if (live) {
      for (int ft = 0; ft < 4; ++ft) {
        long long f = base + ft * 16 + fl;
        if (f >= nface) f = nface - 1;
        build_inputs(a, n, Ub, f, lane, A.x[0][ft], A.x[1][ft]);
      }
      net_forward_batch(sw, sb, lane, A, z);
      // upstream gradient of the face fluxes (face frame), lanes q == 0
      for (int ft = 0; ft < 4; ++ft) {
        const long long f = base + ft * 16 + fl;
        for (int i = 0; i < 4; ++i) Fb[ft][i] = 0.f;
        if (q != 0 || f >= nface) continue;
        double fb[4];
        if (f < nxf) {
          const int gj = (int)(f / (a.nx + 1)), gf = (int)(f % (a.nx + 1));
          const double sc = clam * a.inv_dx;
          fb[0] = sc * (lam_at(0, gf, gj) - lam_at(0, gf - 1, gj));
          fb[1] = sc * (lam_at(1, gf, gj) - lam_at(1, gf - 1, gj));
          fb[2] = sc * (lam_at(2, gf, gj) - lam_at(2, gf - 1, gj));
          fb[3] = sc * (lam_at(3, gf, gj) - lam_at(3, gf - 1, gj));
        } else {
          const long long g = f - nxf;
          const int gf = (int)(g / a.nx), gi = (int)(g % a.nx);
          const double sc = clam * a.inv_dy;
          fb[0] = sc * (lam_at(0, gi, gf) - lam_at(0, gi, gf - 1));
          fb[1] = sc * (lam_at(2, gi, gf) - lam_at(2, gi, gf - 1));
          fb[2] = sc * (lam_at(1, gi, gf) - lam_at(1, gi, gf - 1));
          fb[3] = sc * (lam_at(3, gi, gf) - lam_at(3, gi, gf - 1));
        }
        for (int i = 0; i < 4; ++i) {
          const float t = tanhf(z[ft][i]);
          Fb[ft][i] = float(fb[i]) * n.out_scale * (1.f - t * t);
        }
      }
    }
    // reverse layer by layer; dA holds the gradient w.r.t. the current layer's
    // pre-activations (D layout)
    f32x4 dA[4][4];  // [neuron tile][face tile]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int ft = 0; ft < 4; ++ft) dA[nt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
      if (q == 0) dA[0][ft] = f32x4{Fb[ft][0], Fb[ft][1], Fb[ft][2], Fb[ft][3]};
    BwdCtx c{sw, gsum, trA, trH, lane, wv, live};
    bwd_layer<3>(c, A, dA);
    bwd_layer<2>(c, A, dA);
    bwd_layer<1>(c, A, dA);
    f32x4 dXt[2][4];
    bwd_layer<0>(c, A, dA, dXt);
    if (live) {
      // stencil gradient: input 4*(it*4+q)+i = cell it*4+q, variable i
#pragma unroll
      for (int ft = 0; ft < 4; ++ft) {
        const long long f = base + ft * 16 + fl;
        if (f >= nface) continue;
        float* out = dX + ((long long)b * nface + f) * 24;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          const int cell = it * 4 + q;
          if (cell >= 6) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) out[cell * 4 + i] = dXt[it][ft][i] * float(n.inv_std[i]);
        }
      }
    }
  }
  __syncthreads();
  float* pb = part + (long long)blockIdx.x * NET_NP;
  for (int k = threadIdx.x; k < NET_NP; k += blockDim.x) pb[k] = gsum[k];
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

// Adam (bias-corrected) on the FP32 master parameters.
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ theta, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                   float b1, float b2, float eps, int step) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = grad[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  const float mh = mk / (1.f - powf(b1, (float)step));
  const float vh = vk / (1.f - powf(b2, (float)step));
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

__global__ void __launch_bounds__(64) mse_finalize_kernel(const double* __restrict__ part, int nblk, int nbatch,
                                                          double* __restrict__ loss) {
  const int b = threadIdx.x;
  if (b >= nbatch) return;
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += part[(long long)b * nblk + k];
  loss[b] += s;
}

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
  const long long batches = (net_face_count(a) + 63) / 64 * a.nbatch;
  long long nb = (batches + 3) / 4;
  if (nb > NET_BWD_BLOCKS) nb = NET_BWD_BLOCKS;
  return (unsigned int)(nb < 1 ? 1 : nb);
}

hipError_t launch_net_forward(const GridArgs& a, const NetArgs& n, const double* U, float* dF, hipStream_t st) {
  const long long nf = net_face_count(a);
  hipLaunchKernelGGL(net_forward_kernel, dim3(net_blocks(nf), a.nbatch), dim3(256), 0, st, a, n, U, dF, nf);
  return hipGetLastError();
}

hipError_t launch_net_backward(const GridArgs& a, const NetArgs& n, const double* U, const double* lam, double clam_f,
                               const double* dtp, float* dX, float* part, float* grad, hipStream_t st) {
  const long long nf = net_face_count(a);
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
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, theta, grad, m, v, n, lr, b1, b2, eps,
                     step);
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

hipError_t launch_mse(const double* U, const double* T, double* G, double scale, long long per_b, int nbatch,
                      double* part, double* loss, hipStream_t st) {
  unsigned int nb = (unsigned int)((per_b + 255) / 256);
  if (nb > 256) nb = 256;
  hipLaunchKernelGGL(mse_kernel, dim3(nb, nbatch), dim3(256), 0, st, U, T, G, scale, per_b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mse_finalize_kernel, dim3(1), dim3(64 * ((nbatch + 63) / 64)), 0, st, part, (int)nb, nbatch, loss);
  return hipGetLastError();
}

}  // namespace shk
