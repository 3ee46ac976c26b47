// Learned face-flux correction: parameter layout shared by the host API and
// the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "grid.hpp"

namespace shk {

// Packed parameter vector theta (FP32, the order of gradients and Adam):
// W0[64][24], b0[64], W1[64][64], b1[64], W2[64][64], b2[64], W3[4][64], b3[4].
constexpr int NET_G_W0 = 0, NET_G_B0 = 1536, NET_G_W1 = 1600, NET_G_B1 = 5696, NET_G_W2 = 5760,
              NET_G_B2 = 9856, NET_G_W3 = 9920, NET_G_B3 = 10176, NET_NP = 10180;
// Device (MFMA) layout: bf16 W0[64][32] (inputs padded), W1[64][64], W2[64][64],
// W3[16][64] (outputs padded); FP32 biases b0[64], b1[64], b2[64], b3[16].
constexpr int NET_OFF_W0 = 0, NET_OFF_W1 = 2048, NET_OFF_W2 = 6144, NET_OFF_W3 = 10240, NET_NW = 11264;
constexpr int NET_OFF_B0 = 0, NET_OFF_B1 = 64, NET_OFF_B2 = 128, NET_OFF_B3 = 192, NET_NB = 208;
// The LDS copies pad each row (bf16 elements: 36 for W0's 32 inputs, 68 for
// 64, 20 for 16) so that the 16 rows of an operand read, each an 8-byte
// slice at the same column, fall on distinct LDS bank pairs (a row stride of
// 32 or 64 elements puts them all on one).
constexpr int NET_LD_W0 = 36, NET_LD_H = 68, NET_LD_O = 20;
constexpr int NET_L_W0 = 0, NET_L_W1 = 64 * NET_LD_W0, NET_L_W2 = NET_L_W1 + 64 * NET_LD_H,
              NET_L_W3 = NET_L_W2 + 64 * NET_LD_H, NET_LNW = NET_L_W3 + 16 * NET_LD_H;
// transposed copy for the reverse pass: W0^T [32][64], W1^T and W2^T [64][64], W3^T [64][16]
constexpr int NET_T_W0 = 0, NET_T_W1 = 32 * NET_LD_H, NET_T_W2 = NET_T_W1 + 64 * NET_LD_H,
              NET_T_W3 = NET_T_W2 + 64 * NET_LD_H, NET_TNW = NET_T_W3 + 64 * NET_LD_O;


// workgroups (and parameter partials) of the reverse pass: two per compute
// unit (its registers and LDS allow two workgroups per unit)
constexpr int NET_BWD_BLOCKS = 512;

long long net_face_count(const GridArgs& a);
unsigned int net_backward_blocks(const GridArgs& a);
hipError_t launch_net_forward(const GridArgs& a, const NetArgs& n, const double* U, float* dF, hipStream_t st);
hipError_t launch_net_backward(const GridArgs& a, const NetArgs& n, const double* U, const double* lam, double clam_f,
                               const double* dtp, float* dX, float* part, float* grad, hipStream_t st);
hipError_t launch_net_pack(const float* theta, unsigned short* w, float* bias, hipStream_t st);
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st);
hipError_t launch_restrict(const double* fine, double* coarse, int nxf, int nyf, int factor, int nvar, int nbatch,
                           hipStream_t st);
hipError_t launch_mse(const double* U, const double* T, double* G, double scale, long long per_b, int nbatch,
                      double* part, double* loss, hipStream_t st);
// Largest batch of launch_mse_noalloc: its block partials live in a static
// device array of MSE_NOALLOC_MAX_BATCH * 256 doubles (512 KiB per GPU).
constexpr int MSE_NOALLOC_MAX_BATCH = 256;
// launch_mse with the partials in that array (no caller buffer, no
// allocation).  The array's address on the current device is looked up once
// per device.  Calls that overlap on one GPU share the array and race.
hipError_t launch_mse_noalloc(const double* U, const double* T, double* G, double scale, long long per_b, int nbatch,
                              double* loss, hipStream_t st);

}  // namespace shk
