// Convolutional learned flux correction on gfx950 matrix cores (bfloat16
// MFMA, FP32 accumulation): section 2's 2D neural flux, three 3x3 layers
// (4 -> 16 -> 32 -> 4 channels; ReLU, ReLU, tanh; 6,388 parameters) applied
// pixel by pixel to the normalised WENO-reconstructed states, one parameter
// set for both directions.
//
// The pixels are faces.  Image 0 holds the x-faces (ny rows, nx + 1
// columns), image 1 the y-faces transposed (nx rows, ny + 1 columns), so the
// face normal runs along the columns of both; a face's input is the
// normalised conservative mean of its two reconstructed states in the face
// frame, its output the face-frame flux correction out_scale * tanh(z).  The
// 3x3 windows are padded with zeros at domain boundaries and wrap around
// across periodic ones, where the image holds each face once (the last face
// of a periodic row is its first).
//
// The forward pass is two kernels: the face images (the stencil primitives
// of a 16 x 16 pixel tile staged once in LDS, FP64 reconstruction, bf16
// inputs), then the three layers fused over a tile with a three-pixel halo,
// each an implicit GEMM D[out channel][pixel] = W[out channel][tap, in
// channel] . X[tap, in channel][pixel] on the matrix cores (16 pixels per
// product, N = 16), activations channels-last in LDS so that an operand
// slice is one 8-byte LDS read.  The reverse pass runs a layer kernel with
// the mirrored, channel-swapped weights for the input gradients (masked by
// the forward ReLU) and a second kernel for the weight gradients, a
// contraction over pixels whose operands are read channel-major from LDS.
// Parameter gradients go to one FP32 partial per workgroup (fixed tile order
// per workgroup, fixed wave order inside it) and are summed in a fixed
// order: the gradients are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cnn.hpp"
#include "face_dev.hpp"
#include "flux.hpp"
#include "grid.hpp"
#include "mlp_dev.hpp"

namespace shk {

namespace {

enum { EPI_BWD_HIDDEN = 0, EPI_BWD_IN = 1 };

struct ConvOut {
  unsigned short* out_bf;            // bf16 image of COUT channels (EPI_BWD_HIDDEN)
  float* out_f;                      // FP32 image of 4 channels (EPI_BWD_IN)
  const unsigned short* mask_src;    // forward activation of the same pixels (EPI_BWD_HIDDEN)
  float* part;                       // [workgroup][CNN_BROW] (EPI_BWD_HIDDEN: bias sums)
  int part_off;
  int cout;                          // real output channels
};

// Pixel index along an image axis of n pixels for a 3x3 window position k
// (k in -1 .. n): wrapped along a periodic axis, -1 (zero padding) outside
// otherwise.  Positions further out are never read by a valid output.
__device__ __forceinline__ int pix_src(int k, int n, int wrap) {
  if (k >= 0 && k < n) return k;
  if (!wrap || k < -1 || k > n) return -1;
  return k < 0 ? n - 1 : 0;
}

struct TileLoc {
  int b, img, r0, c0, H, W, wr, wc;
  long long pbase;  // pixel index of the image's first pixel in the member-major buffer
};

__device__ __forceinline__ TileLoc tile_loc(const CnnGeom& g, long long t) {
  TileLoc L;
  L.b = (int)(t / g.tiles);
  int tt = (int)(t % g.tiles);
  const int t0 = g.tilesR[0] * g.tilesC[0];
  L.img = tt < t0 ? 0 : 1;
  if (L.img) tt -= t0;
  L.H = g.H[L.img];
  L.W = g.W[L.img];
  L.wr = g.wrapR[L.img];
  L.wc = g.wrapC[L.img];
  L.r0 = (tt / g.tilesC[L.img]) * 16;
  L.c0 = (tt % g.tilesC[L.img]) * 16;
  L.pbase = (long long)L.b * g.npix + (L.img ? g.H[0] * g.W[0] : 0);
  return L;
}

// The face of pixel (R, C) of an image, in the solver's face numbering
// (x-faces (nx + 1) per row, then y-faces nx per row).
__device__ __forceinline__ long long pixel_face(int img, int R, int C, int nx, int ny) {
  return img == 0 ? (long long)R * (nx + 1) + C : (long long)(nx + 1) * ny + (long long)C * nx + R;
}

// Input gradient of one 3x3 layer (the forward kernel with mirrored,
// channel-swapped weights; used for the 4-channel output layer, the wider
// layers take cnn_conv32_kernel below) as an implicit GEMM over 16 x 16
// pixel tiles;
// MT output-channel tiles of 16, KB K-blocks of 16 (k = tap * CIN +
// channel, taps >= 9 are zero padding).  Each lane keeps its weight
// fragments in registers for the whole launch; a wave computes its four
// pixel rows as four independent accumulation chains.  The tile is staged in
// planes of 16 channels ([plane][pixel][16]), so the 16 pixels x 4 channel
// groups of one operand read cover the LDS banks evenly.  Workgroups take
// tiles of every batch member and both images in a fixed order.
template <int CIN, int MT, int KB, int EPI>
__global__ void __launch_bounds__(256) cnn_conv_kernel(CnnGeom g, const unsigned short* __restrict__ in,
                                                       const unsigned short* __restrict__ wm, ConvOut o) {
  static_assert(CIN % 4 == 0, "channels come in groups of four");
  constexpr int CP = CIN >= 16 ? 16 : CIN;  // channels per plane
  constexpr int NPL = CIN / CP;             // planes
  __shared__ __attribute__((aligned(16))) unsigned short tile[NPL * 324 * CP];
  __shared__ float red[4][MT * 16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, fl = lane & 15;
  bf16x4 Aw[MT][KB];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) Aw[mt][kb] = ldA(wm, KB * 16, mt * 16, kb * 16, lane);
  f32x4 bs[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) bs[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const long long ntile = (long long)g.tiles * g.nbatch;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const TileLoc L = tile_loc(g, t);
    __syncthreads();  // the previous tile's readers are done
    for (int k = threadIdx.x; k < 324 * (CIN / 4); k += blockDim.x) {
      const int pq = k / (CIN / 4), cq = k - pq * (CIN / 4);
      const int tr = pq / 18, tc = pq - tr * 18;
      const int R = pix_src(L.r0 + tr - 1, L.H, L.wr), C = pix_src(L.c0 + tc - 1, L.W, L.wc);
      bf16x4 v = {0, 0, 0, 0};
      if (R >= 0 && C >= 0) v = *reinterpret_cast<const bf16x4*>(in + (L.pbase + (long long)R * L.W + C) * CIN + 4 * cq);
      const int pl = (4 * cq) / CP, c = 4 * cq - pl * CP;
      *reinterpret_cast<bf16x4*>(tile + (pl * 324 + pq) * CP + c) = v;
    }
    __syncthreads();
    // rows beyond the image hold zeros or wrapped pixels: computed, not stored
    f32x4 acc[4][MT];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[rr][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k0 = kb * 16 + 4 * q, tap = k0 / CIN, ci0 = k0 - tap * CIN;
      const int dr = tap / 3, dc = tap - 3 * dr, pl = ci0 / CP, c = ci0 - pl * CP;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        bf16x4 B = {0, 0, 0, 0};
        if (tap < 9) B = *reinterpret_cast<const bf16x4*>(tile + (pl * 324 + (wv * 4 + rr + dr) * 18 + fl + dc) * CP + c);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[rr][mt] = mfma(Aw[mt][kb], B, acc[rr][mt]);
      }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      // lane (pixel fl of the row, q) holds output channels 16 mt + 4q .. + 3
      const int R = L.r0 + wv * 4 + rr, C = L.c0 + fl;
      const bool valid = R < L.H && C < L.W;
      const long long pix = L.pbase + (long long)R * L.W + C;
      if (EPI == EPI_BWD_HIDDEN) {
        if (valid)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int c0 = mt * 16 + 4 * q;
            f32x4 d = acc[rr][mt];
            const bf16x4 h = *reinterpret_cast<const bf16x4*>(o.mask_src + pix * (MT * 16) + c0);
#pragma unroll
            for (int i = 0; i < 4; ++i) d[i] = h[i] > 0 ? d[i] : 0.f;  // bf16 bits: positive iff > 0 as int16
            *reinterpret_cast<bf16x4*>(o.out_bf + pix * (MT * 16) + c0) = pack4(d[0], d[1], d[2], d[3]);
            bs[mt] = bs[mt] + d;
          }
      } else {  // EPI_BWD_IN
        if (valid && q == 0) *reinterpret_cast<f32x4*>(o.out_f + pix * 4) = acc[rr][0];
      }
    }
  }
  if (EPI == EPI_BWD_HIDDEN) {
    // this workgroup's bias sums: the 16 pixels of a row group, then the
    // four waves in order
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float s = bs[mt][i];
        for (int m = 8; m >= 1; m >>= 1) s += __shfl_xor(s, m, 16);
        if (fl == 0) red[wv][mt * 16 + 4 * q + i] = s;
      }
    __syncthreads();
    if ((int)threadIdx.x < o.cout)
      o.part[(long long)blockIdx.x * CNN_BROW + o.part_off + threadIdx.x] =
          ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
  }
}

// The same input-gradient layer for CIN = 16 or 32 input channels on
// v_mfma_f32_16x16x32_bf16: a lane's eight k-slots are eight consecutive
// channels of one tap (one tap of 32 channels per block, or two taps of 16
// with the ninth tap as one K = 16 block), so that every operand is one
// 16-byte read of the weights or of the channels-last tile, whose pixel
// stride (CIN + 8 elements) puts the 16 pixels of a read on distinct LDS
// banks.
template <int CIN, int MT, int EPI>
__global__ void __launch_bounds__(256) cnn_conv32_kernel(CnnGeom g, const unsigned short* __restrict__ in,
                                                         const unsigned short* __restrict__ wm, ConvOut o) {
  static_assert(CIN == 16 || CIN == 32, "16 or 32 input channels");
  constexpr int PS = CIN + 8;                // pixel stride of the tile (elements)
  constexpr int K = 9 * CIN;                 // weight row length
  constexpr int KB = CIN == 32 ? 9 : 4;      // K = 32 blocks
  __shared__ __attribute__((aligned(16))) unsigned short tile[324 * PS];
  __shared__ float red[4][MT * 16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, fl = lane & 15;
  auto ld16 = [](const unsigned short* p) { return *reinterpret_cast<const s16x8*>(p); };
  s16x8 Aw[MT][KB];
  bf16x4 At[MT];  // tap 8 of the 16-channel layer
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) Aw[mt][kb] = ld16(wm + (mt * 16 + fl) * K + 32 * kb + 8 * q);
    At[mt] = CIN == 16 ? ldA(wm, K, mt * 16, 128, lane) : bf16x4{0, 0, 0, 0};
  }
  // this lane's tap offset (pixels) and channel offset in each K = 32 block
  int toff[KB], coff[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const int tap = CIN == 32 ? kb : 2 * kb + (q >> 1), dr = tap / 3, dc = tap - 3 * dr;
    toff[kb] = dr * 18 + dc;
    coff[kb] = CIN == 32 ? 8 * q : 8 * (q & 1);
  }
  f32x4 bs[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) bs[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const long long ntile = (long long)g.tiles * g.nbatch;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const TileLoc L = tile_loc(g, t);
    __syncthreads();  // the previous tile's readers are done
    for (int k = threadIdx.x; k < 324 * (CIN / 4); k += blockDim.x) {
      const int pq = k / (CIN / 4), cq = k - pq * (CIN / 4);
      const int tr = pq / 18, tc = pq - tr * 18;
      const int R = pix_src(L.r0 + tr - 1, L.H, L.wr), C = pix_src(L.c0 + tc - 1, L.W, L.wc);
      bf16x4 v = {0, 0, 0, 0};
      if (R >= 0 && C >= 0) v = *reinterpret_cast<const bf16x4*>(in + (L.pbase + (long long)R * L.W + C) * CIN + 4 * cq);
      *reinterpret_cast<bf16x4*>(tile + pq * PS + 4 * cq) = v;
    }
    __syncthreads();
    // rows beyond the image hold zeros or wrapped pixels: computed, not stored
    f32x4 acc[4][MT];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[rr][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const s16x8 B = ld16(tile + ((wv * 4 + rr) * 18 + fl + toff[kb]) * PS + coff[kb]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[rr][mt] = mfma32(Aw[mt][kb], B, acc[rr][mt]);
      }
    if (CIN == 16)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const bf16x4 B = *reinterpret_cast<const bf16x4*>(tile + ((wv * 4 + rr + 2) * 18 + fl + 2) * PS + 4 * q);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[rr][mt] = mfma(At[mt], B, acc[rr][mt]);
      }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      // lane (pixel fl of the row, q) holds output channels 16 mt + 4q .. + 3
      const int R = L.r0 + wv * 4 + rr, C = L.c0 + fl;
      const bool valid = R < L.H && C < L.W;
      const long long pix = L.pbase + (long long)R * L.W + C;
      if (EPI == EPI_BWD_HIDDEN) {
        if (valid)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int c0 = mt * 16 + 4 * q;
            f32x4 d = acc[rr][mt];
            const bf16x4 h = *reinterpret_cast<const bf16x4*>(o.mask_src + pix * (MT * 16) + c0);
#pragma unroll
            for (int i = 0; i < 4; ++i) d[i] = h[i] > 0 ? d[i] : 0.f;  // bf16 bits: positive iff > 0 as int16
            *reinterpret_cast<bf16x4*>(o.out_bf + pix * (MT * 16) + c0) = pack4(d[0], d[1], d[2], d[3]);
            bs[mt] = bs[mt] + d;
          }
      } else {  // EPI_BWD_IN
        if (valid && q == 0) *reinterpret_cast<f32x4*>(o.out_f + pix * 4) = acc[rr][0];
      }
    }
  }
  if (EPI == EPI_BWD_HIDDEN) {
    // this workgroup's bias sums: the 16 pixels of a row group, then the
    // four waves in order
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float s = bs[mt][i];
        for (int m = 8; m >= 1; m >>= 1) s += __shfl_xor(s, m, 16);
        if (fl == 0) red[wv][mt * 16 + 4 * q + i] = s;
      }
    __syncthreads();
    if ((int)threadIdx.x < o.cout)
      o.part[(long long)blockIdx.x * CNN_BROW + o.part_off + threadIdx.x] =
          ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
  }
}

// Pixel index along an image axis of n pixels for an unwrapped position k
// of a layer region: k itself inside, the wrapped pixel across a periodic
// edge, -1 (zero padding) outside otherwise.
__device__ __forceinline__ int wrap_pix(int k, int n, int wrap) {
  if (k >= 0 && k < n) return k;
  if (!wrap) return -1;
  return ((k % n) + n) % n;
}

// The forward network on one 16 x 16 output tile in a single pass: the
// input image with a three-pixel halo is staged in LDS, layer 1 is evaluated
// on the 20 x 20 pixels around the tile, layer 2 on 18 x 18 and layer 3 on
// the tile, each layer's activations kept in LDS.  Halo pixels outside the
// image are zero (the per-layer zero padding) unless they lie across a
// periodic edge, where they take the wrapped pixel's values.  The pixels of
// a region are taken 16 at a time in row-major order (one MFMA column
// each), so a region need not be a multiple of 16 wide.  Layers 2 and 3 use
// the K = 32 product with the eight k-slots of a lane on eight consecutive
// channels of one tap (two taps of 16 channels, or one tap of 32 per block):
// an operand is one 16-byte read of the weights or of the channels-last
// activations, whose pixel strides (48 and 80 bytes) put the 16 pixels of a
// read on distinct LDS banks.  The output layer's four channels are
// redistributed through LDS so that every lane evaluates tanh for one pixel.
// With KEEP the hidden activations and tanh values of the tile's own pixels
// are written out for the reverse pass.
template <bool KEEP>
__global__ void __launch_bounds__(256) cnn_forward_kernel(CnnGeom g, CnnArgs n, const unsigned short* __restrict__ xin,
                                                          float* __restrict__ dF, long long nface, int nx, int ny,
                                                          unsigned short* __restrict__ h1g,
                                                          unsigned short* __restrict__ h2g, float* __restrict__ tg,
                                                          unsigned int* fault) {
  constexpr int S1 = 24, S2 = 40;  // pixel strides (elements) of the layer-1 and layer-2 activations
  __shared__ __attribute__((aligned(16))) unsigned short sX[22 * 22 * 4];
  __shared__ __attribute__((aligned(16))) unsigned short sH1[20 * 20 * S1];
  __shared__ __attribute__((aligned(16))) unsigned short sH2[18 * 18 * S2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, fl = lane & 15;
  const unsigned short* __restrict__ w = n.w;
  auto bias4 = [&](int off) {
    const float* bp = n.bias + off + 4 * q;
    return f32x4{bp[0], bp[1], bp[2], bp[3]};
  };
  auto ld16 = [](const unsigned short* p) { return *reinterpret_cast<const s16x8*>(p); };
  bool bad = false;
  const long long ntile = (long long)g.tiles * g.nbatch;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const TileLoc L = tile_loc(g, t);
    __syncthreads();  // the previous tile's readers are done
    for (int k = threadIdx.x; k < 22 * 22; k += blockDim.x) {
      const int tr = k / 22, tc = k - tr * 22;
      const int R = wrap_pix(L.r0 - 3 + tr, L.H, L.wr), C = wrap_pix(L.c0 - 3 + tc, L.W, L.wc);
      bf16x4 v = {0, 0, 0, 0};
      if (R >= 0 && C >= 0) v = *reinterpret_cast<const bf16x4*>(xin + (L.pbase + (long long)R * L.W + C) * 4);
      *reinterpret_cast<bf16x4*>(sX + k * 4) = v;
    }
    __syncthreads();
    {  // layer 1 on 20 x 20: 25 groups, K = 3 blocks of four taps x 4 channels
      bf16x4 A1[3];
#pragma unroll
      for (int kb = 0; kb < 3; ++kb) A1[kb] = ldA(w + CNN_F1, 48, 0, kb * 16, lane);
      const f32x4 b1 = bias4(CNN_BB1);
      for (int gi = wv; gi < 25; gi += 4) {
        const int p = gi * 16 + fl, hr = p / 20, hc = p - hr * 20;
        f32x4 acc = b1;
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) {
          const int tap = 4 * kb + q, dr = tap / 3, dc = tap - 3 * dr;
          bf16x4 B = {0, 0, 0, 0};
          if (tap < 9) B = *reinterpret_cast<const bf16x4*>(sX + ((hr + dr) * 22 + hc + dc) * 4);
          acc = mfma(A1[kb], B, acc);
        }
        const int R = L.r0 - 2 + hr, C = L.c0 - 2 + hc;
        const bool live = wrap_pix(R, L.H, L.wr) >= 0 && wrap_pix(C, L.W, L.wc) >= 0;
        bf16x4 hv = {0, 0, 0, 0};
        if (live) hv = pack4(relu0(acc[0]), relu0(acc[1]), relu0(acc[2]), relu0(acc[3]));
        *reinterpret_cast<bf16x4*>(sH1 + p * S1 + 4 * q) = hv;
        if (KEEP && R >= L.r0 && R < L.r0 + 16 && C >= L.c0 && C < L.c0 + 16 && R < L.H && C < L.W)
          *reinterpret_cast<bf16x4*>(h1g + (L.pbase + (long long)R * L.W + C) * 16 + 4 * q) = hv;
      }
    }
    __syncthreads();
    {  // layer 2 on 18 x 18: 21 groups (the last holds 4 pixels), two at a time;
       // K = 32 block kb holds taps 2 kb (lanes q < 2) and 2 kb + 1 (q >= 2),
       // channels 8 (q & 1) .. + 7; tap 8 is one K = 16 block
      s16x8 A2[2][4];
      bf16x4 A2t[2];
      f32x4 b2[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) A2[mt][kb] = ld16(w + CNN_F2 + (mt * 16 + fl) * 144 + 32 * kb + 8 * q);
        A2t[mt] = ldA(w + CNN_F2, 144, mt * 16, 128, lane);
        b2[mt] = bias4(CNN_BB2 + mt * 16);
      }
      int toff[4];  // this lane's tap offset (elements) in K = 32 block kb
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int tap = 2 * kb + (q >> 1), dr = tap / 3, dc = tap - 3 * dr;
        toff[kb] = (dr * 20 + dc) * S1 + 8 * (q & 1);
      }
      for (int g0 = wv; g0 < 21; g0 += 8) {
        int p[2], base[2];
        f32x4 acc[2][2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          p[j] = (g0 + 4 * j) * 16 + fl;
          const int pc = p[j] < 324 ? p[j] : 323;
          const int hr = pc / 18, hc = pc - hr * 18;
          base[j] = (hr * 20 + hc) * S1;
          acc[j][0] = b2[0];
          acc[j][1] = b2[1];
        }
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const s16x8 B = ld16(sH1 + base[j] + toff[kb]);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) acc[j][mt] = mfma32(A2[mt][kb], B, acc[j][mt]);
          }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const bf16x4 B = *reinterpret_cast<const bf16x4*>(sH1 + base[j] + (2 * 20 + 2) * S1 + 4 * q);
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) acc[j][mt] = mfma(A2t[mt], B, acc[j][mt]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (p[j] >= 324) continue;
          const int hr = p[j] / 18, hc = p[j] - hr * 18;
          const int R = L.r0 - 1 + hr, C = L.c0 - 1 + hc;
          const bool live = wrap_pix(R, L.H, L.wr) >= 0 && wrap_pix(C, L.W, L.wc) >= 0;
          const bool own = KEEP && R >= L.r0 && R < L.r0 + 16 && C >= L.c0 && C < L.c0 + 16 && R < L.H && C < L.W;
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            const f32x4 a2 = acc[j][mt];
            bf16x4 hv = {0, 0, 0, 0};
            if (live) hv = pack4(relu0(a2[0]), relu0(a2[1]), relu0(a2[2]), relu0(a2[3]));
            *reinterpret_cast<bf16x4*>(sH2 + p[j] * S2 + mt * 16 + 4 * q) = hv;
            if (own) *reinterpret_cast<bf16x4*>(h2g + (L.pbase + (long long)R * L.W + C) * 32 + mt * 16 + 4 * q) = hv;
          }
        }
      }
    }
    __syncthreads();
    {  // layer 3 on the tile: rows 4 wv .. 4 wv + 3, one tap of 32 channels per K = 32 block
      s16x8 A3[9];
#pragma unroll
      for (int kb = 0; kb < 9; ++kb) A3[kb] = ld16(w + CNN_F3 + fl * 288 + 32 * kb + 8 * q);
      const f32x4 b3 = bias4(CNN_BB3);
      f32x4 acc[4];
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) acc[rr] = b3;
#pragma unroll
      for (int kb = 0; kb < 9; ++kb) {
        const int dr = kb / 3, dc = kb - 3 * dr;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          acc[rr] = mfma32(A3[kb], ld16(sH2 + ((wv * 4 + rr + dr) * 18 + fl + dc) * S2 + 8 * q), acc[rr]);
      }
      // lanes q = 0 hold the four output channels of rows 4 wv + rr; through
      // LDS (the layer-1 buffer, free now) lane (fl, q) takes row 4 wv + q
      float* red = reinterpret_cast<float*>(sH1) + wv * 256;
      if (q == 0)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) *reinterpret_cast<f32x4*>(red + (rr * 16 + fl) * 4) = acc[rr];
      __syncthreads();
      const f32x4 z = *reinterpret_cast<const f32x4*>(red + (q * 16 + fl) * 4);
      const int R = L.r0 + wv * 4 + q, C = L.c0 + fl;
      if (R < L.H && C < L.W) {
        float th[4], out[4];
        bool ok = true;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          th[i] = tanhf(z[i]);
          out[i] = n.out_scale * th[i];
          ok = ok && isfinite(out[i]);
        }
        if (!ok) {  // the uncorrected flux, with zero derivative
#pragma unroll
          for (int i = 0; i < 4; ++i) { out[i] = 0.f; th[i] = 1.f; }
          bad = true;
        }
        const long long pix = L.pbase + (long long)R * L.W + C;
        if (KEEP) *reinterpret_cast<f32x4*>(tg + pix * 4) = f32x4{th[0], th[1], th[2], th[3]};
        float* d = dF + ((long long)L.b * nface + pixel_face(L.img, R, C, nx, ny)) * 4;
        *reinterpret_cast<f32x4*>(d) = f32x4{out[0], out[1], out[2], out[3]};
        if (L.wc && C == 0) {  // the last face of a periodic row is this one
          float* d2 = dF + ((long long)L.b * nface + pixel_face(L.img, R, L.W, nx, ny)) * 4;
          *reinterpret_cast<f32x4*>(d2) = f32x4{out[0], out[1], out[2], out[3]};
        }
      }
    }
  }
  if (bad) atomicOr(fault, 8u);
}

// Weight gradient of one layer: D[out channel][tap, in channel] = sum over
// pixels of dA[pixel][out] X[pixel + tap][in], a contraction over the 16
// pixels of a tile row per product.  The operands are staged channel-major
// (pixels contiguous): dA without halo; X with a one-pixel halo of rows and
// in three copies shifted by the column offset of the tap, so that every
// operand slice (four pixels of one channel) is one aligned 8-byte LDS read.
// Channel row strides are 26 (mod 32) dwords (10 for dA): the 16 channels x
// 4 pixel groups of a read spread evenly over the banks, and the staging
// writes of channels four apart conflict at most two-way.
template <int CIN, int COUT, int MT, int NT>
__global__ void __launch_bounds__(256) cnn_wgrad_kernel(CnnGeom g, const unsigned short* __restrict__ dA,
                                                        const unsigned short* __restrict__ X,
                                                        float* __restrict__ part, int woff) {
  constexpr int K9 = 9 * CIN;
  constexpr int SA = 276;       // dA channel stride (elements): 256 pixels, padded to 138 dwords
  constexpr int SX = 308;       // X channel stride: 18 rows x 16 pixels, padded to 154 dwords
  constexpr int LDS_A = COUT * SA, LDS_X = 3 * CIN * SX;
  constexpr int LDS_U = (LDS_A + LDS_X) * 2 > COUT * K9 * 4 ? (LDS_A + LDS_X) : COUT * K9 * 2;
  __shared__ __attribute__((aligned(16))) unsigned short lds[LDS_U];
  unsigned short* tA = lds;           // [COUT][SA]
  unsigned short* tX = lds + LDS_A;   // [3][CIN][SX]: copy dc, channel, row * 16 + column
  float* red = reinterpret_cast<float*>(lds);  // [COUT][K9], after the last tile
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, fl = lane & 15;
  f32x4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const long long ntile = (long long)g.tiles * g.nbatch;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const TileLoc L = tile_loc(g, t);
    __syncthreads();
    for (int k = threadIdx.x; k < 256 * (COUT / 4); k += blockDim.x) {
      const int p = k / (COUT / 4), cq = k - p * (COUT / 4);
      const int R = L.r0 + (p >> 4), C = L.c0 + (p & 15);
      bf16x4 v = {0, 0, 0, 0};
      if (R < L.H && C < L.W) v = *reinterpret_cast<const bf16x4*>(dA + (L.pbase + (long long)R * L.W + C) * COUT + 4 * cq);
#pragma unroll
      for (int i = 0; i < 4; ++i) tA[(4 * cq + i) * SA + p] = (unsigned short)v[i];
    }
    for (int k = threadIdx.x; k < 324 * (CIN / 4); k += blockDim.x) {
      const int pq = k / (CIN / 4), cq = k - pq * (CIN / 4);
      const int tr = pq / 18, tc = pq - tr * 18;
      const int R = pix_src(L.r0 + tr - 1, L.H, L.wr), C = pix_src(L.c0 + tc - 1, L.W, L.wc);
      bf16x4 v = {0, 0, 0, 0};
      if (R >= 0 && C >= 0) v = *reinterpret_cast<const bf16x4*>(X + (L.pbase + (long long)R * L.W + C) * CIN + 4 * cq);
      // halo column tc lands at column tc - dc of copy dc
#pragma unroll
      for (int dc = 0; dc < 3; ++dc) {
        const int c = tc - dc;
        if (c >= 0 && c < 16)
#pragma unroll
          for (int i = 0; i < 4; ++i) tX[(dc * CIN + 4 * cq + i) * SX + tr * 16 + c] = (unsigned short)v[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int r = wv * 4 + rr;  // rows beyond the image are zeros in tA
      bf16x4 A[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        A[mt] = bf16x4{0, 0, 0, 0};
        if (mt * 16 + fl < COUT) A[mt] = *reinterpret_cast<const bf16x4*>(tA + (mt * 16 + fl) * SA + r * 16 + 4 * q);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int k = nt * 16 + fl, tap = k / CIN, ci = k - tap * CIN;
        bf16x4 B = {0, 0, 0, 0};
        if (tap < 9) {
          const int dr = tap / 3, dc = tap - 3 * dr;
          B = *reinterpret_cast<const bf16x4*>(tX + (dc * CIN + ci) * SX + (r + dr) * 16 + 4 * q);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma(A[mt], B, acc[mt][nt]);
      }
    }
  }
  // the four waves' sums in order, then this workgroup's partial
  for (int w2 = 0; w2 < 4; ++w2) {
    __syncthreads();
    if (wv == w2) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int co = mt * 16 + 4 * q + i, k = nt * 16 + fl;
            if (co < COUT && k < K9) {
              float& s = red[co * K9 + k];
              s = w2 == 0 ? acc[mt][nt][i] : s + acc[mt][nt][i];
            }
          }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < COUT * K9; k += blockDim.x)
    part[(long long)blockIdx.x * CNN_NP + woff + k] = red[k];
}

// The adjoint of the two cells beside a face: zero outside the domain unless
// periodic, and in solid cells.
__device__ __forceinline__ void lam_cell(const GridArgs& a, const double* __restrict__ Lb, int gi, int gj,
                                         double l[4]) {
  bool ok = true;
  if (gi < 0 || gi >= a.nx) {
    ok = a.bc[0] == BC_PERIODIC;
    gi += gi < 0 ? a.nx : -a.nx;
  }
  if (gj < 0 || gj >= a.ny) {
    ok = ok && a.bc[2] == BC_PERIODIC;
    gj += gj < 0 ? a.ny : -a.ny;
  }
  const long long c = (long long)gj * a.nx + gi;
  if (ok && a.cls != nullptr) ok = a.cls[c] == CELL_FLUID;
#pragma unroll
  for (int v = 0; v < 4; ++v) l[v] = ok ? Lb[v * a.ncell + c] : 0.0;
}

// Upstream gradient of one face's flux (face frame) from the RHS adjoint.
__device__ __forceinline__ void face_bar(const GridArgs& a, const double* __restrict__ Lb, double clam, int img,
                                         int R, int C, double fb[4]) {
  double lo[4], hi[4];
  if (img == 0) {  // x-face C of row R: cells C - 1 and C
    lam_cell(a, Lb, C - 1, R, lo);
    lam_cell(a, Lb, C, R, hi);
    const double sc = clam * a.inv_dx;
#pragma unroll
    for (int v = 0; v < 4; ++v) fb[v] = sc * (hi[v] - lo[v]);
  } else {  // y-face C of column R: cells C - 1 and C
    lam_cell(a, Lb, R, C - 1, lo);
    lam_cell(a, Lb, R, C, hi);
    const double sc = clam * a.inv_dy;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int vy = v == 1 ? 2 : (v == 2 ? 1 : v);
      fb[v] = sc * (hi[vy] - lo[vy]);
    }
  }
}

struct PixelLoc {
  int b, img, R, C, W, wc;
};

__device__ __forceinline__ PixelLoc pixel_loc(const CnnGeom& g, long long p) {
  PixelLoc P;
  P.b = (int)(p / g.npix);
  int q = (int)(p - (long long)P.b * g.npix);
  const int n0 = g.H[0] * g.W[0];
  P.img = q < n0 ? 0 : 1;
  if (P.img) q -= n0;
  P.W = g.W[P.img];
  P.wc = g.wrapC[P.img];
  P.R = q / P.W;
  P.C = q - P.R * P.W;
  return P;
}

// Primitive states (face frame) of the stencil cells of one 16 x 16 pixel
// tile: row tr of the tile, index c0 - 3 + tc (tc = 0..20) along the face
// normal.  Rows beyond the image are left unset (their pixels are skipped).
__device__ __forceinline__ void stage_tile_prims(const GridArgs& a, const TileLoc& L, const double* __restrict__ U,
                                                 double (*sp)[16][21]) {
  const double* __restrict__ Ub = U + (long long)L.b * 4 * a.ncell;
  for (int k = threadIdx.x; k < 16 * 21; k += blockDim.x) {
    const int tr = k / 21, tc = k - tr * 21;
    const int R = L.r0 + tr, nrm = L.c0 - 3 + tc;
    if (R >= L.H) continue;
    double w[4];
    if (L.img == 0) cell_prim_frame(a, Ub, nrm, R, true, w);
    else cell_prim_frame(a, Ub, R, nrm, false, w);
#pragma unroll
    for (int v = 0; v < 4; ++v) sp[v][tr][tc] = w[v];
  }
}

// The two reconstructed states of the face of pixel (tr, fl) of a staged
// tile, after the positivity fallback of the stage kernel.
__device__ __forceinline__ bool tile_face_states(const GridArgs& a, const double (*sp)[16][21], int tr, int fl,
                                                 double L[4], double R[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double* c = &sp[v][tr][fl];
    weno5_pair(c[0], c[1], c[2], c[3], c[4], c[5], a.eps, L[v], R[v]);
  }
  const bool fallback = !(L[0] > 0.0) || !(L[3] > 0.0) || !(R[0] > 0.0) || !(R[3] > 0.0);
  if (fallback)
#pragma unroll
    for (int v = 0; v < 4; ++v) { L[v] = sp[v][tr][fl + 2]; R[v] = sp[v][tr][fl + 3]; }
  return fallback;
}

// Normalised network input of every pixel: the conservative mean of the two
// reconstructed face states (positivity fallback as in the stage kernel),
// face frame, bfloat16.  One 16 x 16 pixel tile per workgroup pass: the
// primitive states of its 16 x 21 stencil cells are converted once into
// LDS, then each thread reconstructs one face.
__global__ void __launch_bounds__(256) cnn_inputs_kernel(GridArgs a, CnnGeom g, CnnArgs n,
                                                         const double* __restrict__ U,
                                                         unsigned short* __restrict__ x) {
  __shared__ double sp[4][16][21];
  const int tr = threadIdx.x >> 4, fl = threadIdx.x & 15;
  const long long ntile = (long long)g.tiles * g.nbatch;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const TileLoc L = tile_loc(g, t);
    __syncthreads();
    stage_tile_prims(a, L, U, sp);
    __syncthreads();
    const int R = L.r0 + tr, C = L.c0 + fl;
    if (R >= L.H || C >= L.W) continue;
    double Ls[4], Rs[4];
    tile_face_states(a, sp, tr, fl, Ls, Rs);
    const double gm1 = a.gamma - 1.0;
    const double uL[4] = {Ls[0], Ls[0] * Ls[1], Ls[0] * Ls[2],
                          Ls[3] / gm1 + 0.5 * Ls[0] * (Ls[1] * Ls[1] + Ls[2] * Ls[2])};
    const double uR[4] = {Rs[0], Rs[0] * Rs[1], Rs[0] * Rs[2],
                          Rs[3] / gm1 + 0.5 * Rs[0] * (Rs[1] * Rs[1] + Rs[2] * Rs[2])};
    float xv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) xv[v] = float((0.5 * (uL[v] + uR[v]) - n.mean[v]) * n.inv_std[v]);
    const long long pix = L.pbase + (long long)R * L.W + C;
    *reinterpret_cast<bf16x4*>(x + pix * 4) = pack4(xv[0], xv[1], xv[2], xv[3]);
  }
}

// Output-layer gradient dz = dF_bar out_scale (1 - tanh^2) per pixel,
// bfloat16, and this workgroup's sums of dz (bias b3).  dF_bar of a face is
// (lam_right - lam_left) / h with the periodic wrap, which for the first
// face of a periodic row already holds both of its uses (as the first and as
// the last face of the row).
__global__ void __launch_bounds__(256) cnn_head_kernel(GridArgs a, CnnGeom g, float out_scale,
                                                       const double* __restrict__ lam, double clam_f,
                                                       const double* __restrict__ dtp, const float* __restrict__ th,
                                                       unsigned short* __restrict__ dz, float* __restrict__ part) {
  __shared__ float red[4][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float bsum[4] = {0.f, 0.f, 0.f, 0.f};
  const long long total = (long long)g.npix * g.nbatch;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < total;
       p += (long long)gridDim.x * blockDim.x) {
    const PixelLoc P = pixel_loc(g, p);
    const double* __restrict__ Lb = lam + (long long)P.b * 4 * a.ncell;
    const double clam = clam_f * (dtp ? dtp[P.b] : 1.0);
    double fb[4];
    face_bar(a, Lb, clam, P.img, P.R, P.C, fb);
    const f32x4 t = *reinterpret_cast<const f32x4*>(th + p * 4);
    float d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      d[i] = float(fb[i]) * out_scale * (1.f - t[i] * t[i]);
      bsum[i] += d[i];
    }
    *reinterpret_cast<bf16x4*>(dz + p * 4) = pack4(d[0], d[1], d[2], d[3]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float s = bsum[i];
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) red[wv][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4)
    part[(long long)blockIdx.x * CNN_NP + CNN_G_B3 + threadIdx.x] =
        ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// Stencil gradient of every face (face frame, w.r.t. the six primitive
// states) from the gradient of its pixel's normalised input: the mean of
// the conservative forms of the two reconstructed states, through the
// WENO5 reverse (or the fallback's adjacent cells).  The last face of a
// periodic row is the first one seen from the other side and gets the same
// stencil gradient (the adjoint kernel takes each of the two copies for the
// cells on its own side).  Tiled as the input kernel; the reverse runs one
// primitive variable at a time from the staged states.
__global__ void __launch_bounds__(256) cnn_input_grad_kernel(GridArgs a, CnnGeom g, CnnArgs n,
                                                             const double* __restrict__ U,
                                                             const float* __restrict__ dx, float* __restrict__ dX,
                                                             long long nface) {
  __shared__ double sp[4][16][21];
  const int tr = threadIdx.x >> 4, fl = threadIdx.x & 15;
  const long long ntile = (long long)g.tiles * g.nbatch;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const TileLoc L = tile_loc(g, t);
    __syncthreads();
    stage_tile_prims(a, L, U, sp);
    __syncthreads();
    const int R = L.r0 + tr, C = L.c0 + fl;
    if (R >= L.H || C >= L.W) continue;
    double Ls[4], Rs[4];
    const bool fallback = tile_face_states(a, sp, tr, fl, Ls, Rs);
    const long long pix = L.pbase + (long long)R * L.W + C;
    const f32x4 d = *reinterpret_cast<const f32x4*>(dx + pix * 4);
    double du[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) du[v] = 0.5 * double(d[v]) * n.inv_std[v];
    // transpose of d(rho, rho u_n, rho u_t, E)/d(rho, u_n, u_t, p) at each side
    const double ig = 1.0 / (a.gamma - 1.0);
    auto side = [&](const double W[4], double o[4]) {
      o[0] = du[0] + du[1] * W[1] + du[2] * W[2] + du[3] * 0.5 * (W[1] * W[1] + W[2] * W[2]);
      o[1] = du[1] * W[0] + du[3] * W[0] * W[1];
      o[2] = du[2] * W[0] + du[3] * W[0] * W[2];
      o[3] = du[3] * ig;
    };
    double lb[4], rb[4];
    side(Ls, lb);
    side(Rs, rb);
    float sl[6][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double gs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (fallback) {
        gs[2] = lb[v];
        gs[3] = rb[v];
      } else {
        const double* c = &sp[v][tr][fl];
        weno5_vjp(c[0], c[1], c[2], c[3], c[4], a.eps, lb[v], gs[0], gs[1], gs[2], gs[3], gs[4]);
        weno5_vjp(c[5], c[4], c[3], c[2], c[1], a.eps, rb[v], gs[5], gs[4], gs[3], gs[2], gs[1]);
      }
#pragma unroll
      for (int s2 = 0; s2 < 6; ++s2) sl[s2][v] = float(gs[s2]);
    }
    const long long f = pixel_face(L.img, R, C, a.nx, a.ny);
    f32x4* o = reinterpret_cast<f32x4*>(dX + ((long long)L.b * nface + f) * 24);
#pragma unroll
    for (int s2 = 0; s2 < 6; ++s2) o[s2] = f32x4{sl[s2][0], sl[s2][1], sl[s2][2], sl[s2][3]};
    if (L.wc && C == 0) {
      f32x4* o2 = reinterpret_cast<f32x4*>(dX + ((long long)L.b * nface + pixel_face(L.img, R, L.W, a.nx, a.ny)) * 24);
#pragma unroll
      for (int s2 = 0; s2 < 6; ++s2) o2[s2] = f32x4{sl[s2][0], sl[s2][1], sl[s2][2], sl[s2][3]};
    }
  }
}

// The input images as floats (their bf16 values), for tests.
__global__ void __launch_bounds__(256) cnn_unpack_kernel(const unsigned short* __restrict__ x, float* __restrict__ out,
                                                         long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    out[k] = __uint_as_float((unsigned int)x[k] << 16);
}

// grad[k] += the CNN_BLOCKS partials of parameter k in block order (16 waves
// each take every 16th partial, then the wave sums in wave order); the
// hidden-layer biases b1, b2 come from the input-gradient layers' own
// partials (cnn_bias_reduce_kernel).
__global__ void __launch_bounds__(1024) cnn_grad_reduce_kernel(const float* __restrict__ part, float* __restrict__ grad) {
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const bool mine = k < CNN_NP && !(k >= CNN_G_B1 && k < CNN_G_B1 + 16) && !(k >= CNN_G_B2 && k < CNN_G_B2 + 32);
  double s = 0.0;
  if (mine)
    for (int j = wv; j < CNN_BLOCKS; j += 16) s += part[(long long)j * CNN_NP + k];
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && mine) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w][lane];
    grad[k] += float(t);
  }
}

// grad[b1, b2] += the nblk rows of bias sums: workgroup i takes bias i,
// thread t the rows t, t + 256, ..., then a fixed butterfly over each wave
// and the four waves in order.
__global__ void __launch_bounds__(256) cnn_bias_reduce_kernel(const float* __restrict__ bpart, int nblk,
                                                              float* __restrict__ grad) {
  __shared__ double red[4];
  const int i = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double s = 0.0;
#pragma unroll 4
  for (int j = threadIdx.x; j < nblk; j += 256) s += bpart[(long long)j * CNN_BROW + i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) red[wv] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = ((red[0] + red[1]) + red[2]) + red[3];
    grad[i < 16 ? CNN_G_B1 + i : CNN_G_B2 + i - 16] += float(t);
  }
}

// bf16 weight matrices and biases from the FP32 master parameters.
__global__ void __launch_bounds__(256) cnn_pack_kernel(const float* __restrict__ theta, unsigned short* __restrict__ w,
                                                       float* __restrict__ bias) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < CNN_NW) {
    float v = 0.f;
    auto W1 = [&](int co, int tap, int ci) { return theta[CNN_G_W1 + (co * 9 + tap) * 4 + ci]; };
    auto W2 = [&](int co, int tap, int ci) { return theta[CNN_G_W2 + (co * 9 + tap) * 16 + ci]; };
    auto W3 = [&](int co, int tap, int ci) { return theta[CNN_G_W3 + (co * 9 + tap) * 32 + ci]; };
    if (k < CNN_F2) {  // F1 [16][48]
      const int row = k / 48, kk = k % 48, tap = kk / 4, ci = kk % 4;
      if (tap < 9) v = W1(row, tap, ci);
    } else if (k < CNN_F3) {  // F2 [32][144]
      const int kk0 = k - CNN_F2, row = kk0 / 144, kk = kk0 % 144;
      v = W2(row, kk / 16, kk % 16);
    } else if (k < CNN_B3) {  // F3 [16][288]
      const int kk0 = k - CNN_F3, row = kk0 / 288, kk = kk0 % 288;
      if (row < 4) v = W3(row, kk / 32, kk % 32);
    } else if (k < CNN_B2) {  // B3 [32][48]: row = layer-3 input channel
      const int kk0 = k - CNN_B3, row = kk0 / 48, kk = kk0 % 48, tap = kk / 4, co = kk % 4;
      if (tap < 9) v = W3(co, 8 - tap, row);
    } else if (k < CNN_B1) {  // B2 [16][288]
      const int kk0 = k - CNN_B2, row = kk0 / 288, kk = kk0 % 288;
      v = W2(kk % 32, 8 - kk / 32, row);
    } else {  // B1 [16][144]
      const int kk0 = k - CNN_B1, row = kk0 / 144, kk = kk0 % 144;
      if (row < 4) v = W1(kk % 16, 8 - kk / 16, row);
    }
    w[k] = f2bf(v);
  }
  if (k < CNN_NB) {
    float v = 0.f;
    if (k < 16) v = theta[CNN_G_B1 + k];
    else if (k < 48) v = theta[CNN_G_B2 + k - 16];
    else if (k < 52) v = theta[CNN_G_B3 + k - 48];
    bias[k] = v;
  }
}

unsigned int tile_blocks(const CnnGeom& g) {
  const long long n = (long long)g.tiles * g.nbatch;
  return (unsigned int)(n < 1 ? 1 : (n > CNN_BMAX ? CNN_BMAX : n));
}

}  // namespace

CnnGeom cnn_geom(const GridArgs& a) {
  CnnGeom g{};
  const int perx = a.bc[0] == BC_PERIODIC, pery = a.bc[2] == BC_PERIODIC;
  g.H[0] = a.ny;
  g.W[0] = perx ? a.nx : a.nx + 1;
  g.wrapR[0] = pery;
  g.wrapC[0] = perx;
  g.H[1] = a.nx;
  g.W[1] = pery ? a.ny : a.ny + 1;
  g.wrapR[1] = perx;
  g.wrapC[1] = pery;
  for (int i = 0; i < 2; ++i) {
    g.tilesR[i] = (g.H[i] + 15) / 16;
    g.tilesC[i] = (g.W[i] + 15) / 16;
  }
  g.npix = g.H[0] * g.W[0] + g.H[1] * g.W[1];
  g.tiles = g.tilesR[0] * g.tilesC[0] + g.tilesR[1] * g.tilesC[1];
  g.nbatch = a.nbatch;
  return g;
}

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

size_t cnn_workspace_bytes(const GridArgs& a) {
  const CnnGeom g = cnn_geom(a);
  const size_t np = (size_t)g.npix * a.nbatch;
  // bf16 images: 4 + 16 + 32 + 4 + 32 + 16 channels; FP32: tanh and input gradient
  return al256(np * 4 * 2) + al256(np * 16 * 2) + al256(np * 32 * 2) + al256(np * 4 * 2) + al256(np * 32 * 2) +
         al256(np * 16 * 2) + al256(np * 4 * 4) + al256(np * 4 * 4) + al256((size_t)CNN_BLOCKS * CNN_NP * 4) +
         al256((size_t)CNN_BMAX * CNN_BROW * 4);
}

CnnBufs cnn_bufs(const GridArgs& a, char* base) {
  const CnnGeom g = cnn_geom(a);
  const size_t np = (size_t)g.npix * a.nbatch;
  CnnBufs b{};
  size_t o = 0;
  auto take = [&](size_t bytes) { char* p = base + o; o += al256(bytes); return p; };
  b.x = reinterpret_cast<unsigned short*>(take(np * 4 * 2));
  b.h1 = reinterpret_cast<unsigned short*>(take(np * 16 * 2));
  b.h2 = reinterpret_cast<unsigned short*>(take(np * 32 * 2));
  b.dz = reinterpret_cast<unsigned short*>(take(np * 4 * 2));
  b.da2 = reinterpret_cast<unsigned short*>(take(np * 32 * 2));
  b.da1 = reinterpret_cast<unsigned short*>(take(np * 16 * 2));
  b.t = reinterpret_cast<float*>(take(np * 4 * 4));
  b.dx = reinterpret_cast<float*>(take(np * 4 * 4));
  b.part = reinterpret_cast<float*>(take((size_t)CNN_BLOCKS * CNN_NP * 4));
  b.bpart = reinterpret_cast<float*>(take((size_t)CNN_BMAX * CNN_BROW * 4));
  return b;
}

hipError_t launch_cnn_pack(const float* theta, unsigned short* w, float* bias, hipStream_t st) {
  hipLaunchKernelGGL(cnn_pack_kernel, dim3((CNN_NW + 255) / 256), dim3(256), 0, st, theta, w, bias);
  return hipGetLastError();
}

hipError_t launch_cnn_forward(const GridArgs& a, const CnnArgs& n, const double* U, float* dF, const CnnBufs& b,
                              bool keep, hipStream_t st) {
  const CnnGeom g = cnn_geom(a);
  hipLaunchKernelGGL(cnn_inputs_kernel, dim3(tile_blocks(g)), dim3(256), 0, st, a, g, n, U, b.x);
  const long long nface = (long long)(a.nx + 1) * a.ny + (long long)a.nx * (a.ny + 1);
  if (keep)
    hipLaunchKernelGGL(cnn_forward_kernel<true>, dim3(tile_blocks(g)), dim3(256), 0, st, g, n, b.x, dF, nface, a.nx,
                       a.ny, b.h1, b.h2, b.t, &a.glob->fault);
  else
    hipLaunchKernelGGL(cnn_forward_kernel<false>, dim3(tile_blocks(g)), dim3(256), 0, st, g, n, b.x, dF, nface, a.nx,
                       a.ny, b.h1, b.h2, b.t, &a.glob->fault);
  return hipGetLastError();
}

hipError_t launch_cnn_backward(const GridArgs& a, const CnnArgs& n, const double* U, const double* lam,
                               double clam_f, const double* dtp, float* dX, float* dF, const CnnBufs& b, float* grad,
                               hipStream_t st) {
  hipError_t e = launch_cnn_forward(a, n, U, dF, b, true, st);
  if (e != hipSuccess) return e;
  const CnnGeom g = cnn_geom(a);
  const long long nface = (long long)(a.nx + 1) * a.ny + (long long)a.nx * (a.ny + 1);
  hipLaunchKernelGGL(cnn_head_kernel, dim3(CNN_BLOCKS), dim3(256), 0, st, a, g, n.out_scale, lam, clam_f, dtp, b.t,
                     b.dz, b.part);
  // the input-gradient layers take one tile per workgroup and leave their
  // bias sums (b2, then b1) in one bpart row per workgroup
  const unsigned int tb = tile_blocks(g);
  ConvOut o{};
  o.part = b.bpart;
  // layer 3: input gradient (32 channels, masked by the layer-2 ReLU) and weights
  o.out_bf = b.da2;
  o.mask_src = b.h2;
  o.part_off = 16;
  o.cout = 32;
  hipLaunchKernelGGL((cnn_conv_kernel<4, 2, 3, EPI_BWD_HIDDEN>), dim3(tb), dim3(256), 0, st, g, b.dz,
                     n.w + CNN_B3, o);
  hipLaunchKernelGGL((cnn_wgrad_kernel<32, 4, 1, 18>), dim3(CNN_BLOCKS), dim3(256), 0, st, g, b.dz, b.h2, b.part,
                     CNN_G_W3);
  // layer 2
  o.out_bf = b.da1;
  o.mask_src = b.h1;
  o.part_off = 0;
  o.cout = 16;
  hipLaunchKernelGGL((cnn_conv32_kernel<32, 1, EPI_BWD_HIDDEN>), dim3(tb), dim3(256), 0, st, g, b.da2,
                     n.w + CNN_B2, o);
  hipLaunchKernelGGL((cnn_wgrad_kernel<16, 32, 2, 9>), dim3(CNN_BLOCKS), dim3(256), 0, st, g, b.da2, b.h1, b.part,
                     CNN_G_W2);
  // layer 1: gradient of the normalised inputs, and weights
  ConvOut o1{};
  o1.out_f = b.dx;
  hipLaunchKernelGGL((cnn_conv32_kernel<16, 1, EPI_BWD_IN>), dim3(tile_blocks(g)), dim3(256), 0, st, g, b.da1,
                     n.w + CNN_B1, o1);
  hipLaunchKernelGGL((cnn_wgrad_kernel<4, 16, 1, 3>), dim3(CNN_BLOCKS), dim3(256), 0, st, g, b.da1, b.x, b.part,
                     CNN_G_W1);
  hipLaunchKernelGGL(cnn_input_grad_kernel, dim3(tile_blocks(g)), dim3(256), 0, st, a, g, n, U, b.dx, dX, nface);
  e = hipGetLastError();
  if (e != hipSuccess || grad == nullptr) return e;
  hipLaunchKernelGGL(cnn_grad_reduce_kernel, dim3((CNN_NP + 63) / 64), dim3(1024), 0, st, b.part, grad);
  hipLaunchKernelGGL(cnn_bias_reduce_kernel, dim3(CNN_BROW), dim3(256), 0, st, b.bpart, (int)tb, grad);
  return hipGetLastError();
}

hipError_t launch_cnn_images(const GridArgs& a, const CnnArgs& n, const double* U, const CnnBufs& b, float* out,
                             hipStream_t st) {
  const CnnGeom g = cnn_geom(a);
  hipLaunchKernelGGL(cnn_inputs_kernel, dim3(tile_blocks(g)), dim3(256), 0, st, a, g, n, U, b.x);
  const long long cnt = (long long)g.npix * g.nbatch * 4;
  hipLaunchKernelGGL(cnn_unpack_kernel, dim3((unsigned int)((cnt + 255) / 256 > 4096 ? 4096 : (cnt + 255) / 256)),
                     dim3(256), 0, st, b.x, out, cnt);
  return hipGetLastError();
}

}  // namespace shk
