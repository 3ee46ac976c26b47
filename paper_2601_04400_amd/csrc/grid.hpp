// Internal (non-ABI) description of a grid shared by the host API and the
// kernels: sizes, physics constants, boundary rules and workspace pointers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shk {

enum : int { BC_TRANS = 0, BC_REFL = 1, BC_INFLOW = 2, BC_PERIODIC = 3 };
enum : uint8_t { CELL_FLUID = 0, CELL_SOLID = 1, CELL_GHOST = 2 };
constexpr int HALO = 3;
constexpr int STAGE_TX = 32, STAGE_TY = 8;  // cells of a 2D stage-kernel tile
constexpr int XSLOTS = 64;  // atomic targets the blocks of one reduction spread over

// Per-batch-member device scalars of the time loop.
struct alignas(64) StepScalars {
  double dt;                    // step used by the stages (0 => no-op)
  double t;                     // device time
  double t_end;                 // stop time
  unsigned long long smax_bits; // max wave-speed sum (bit pattern of a double >= 0)
  unsigned long long rmin_bits; // min density (bit pattern of a double > 0)
  int done;                     // t_end reached
  unsigned int blocks_done;     // last-block detection of the reduction
  int nsteps;                   // automatic steps taken with dt > 0
};

struct Globals {
  unsigned int fault;           // SHK_FAULT_* bits
  unsigned int pad;
  unsigned long long fallbacks; // positivity-fallback faces
};

// Ghost-cell table of the immersed boundary (structure of arrays).
struct GhostTable {
  int n;
  int* cell;        // flat index of the ghost
  int* src;         // [n][4] flat indices of the interpolation cells (-1 unused)
  double* w;        // [n][4] weights
  double* nrm;      // [n][2] unit normal
  int wall;         // 0 slip, 1 no-slip adiabatic
};

// Everything a kernel needs to know about the grid (passed by value).
struct GridArgs {
  int ndim, nx, ny, nbatch, nvar;
  long long ncell;      // nx * ny
  double x0, y0, dx, dy, inv_dx, inv_dy;
  double gamma, eps, cfl;
  int viscous;
  int weno_char;               // 1: characteristic-wise WENO5 (FP64 stage kernels)
  double mu, kappa, prandtl;   // kappa = mu gamma / ((gamma-1) Pr), gas constant 1
  double nu_art;
  int bc[4];
  double inflow_cons[4];       // conservative inflow state (rho, rho u, rho v, E)
  const uint8_t* cls;          // cell classes [ny][nx] or nullptr (no IBM)
  StepScalars* sc;             // [nbatch]
  double* dtbuf;               // [nbatch] step of the automatic time stepping
  double* dt_out;              // optional caller copy of the step (per call)
  void* stage_in_copy;         // MODE_STAGE1: optional copy of the stage input (storage type), or nullptr
  const int* ghost_of;         // immersed boundary: ghost index of each cell or -1 (else nullptr)
  const unsigned* tile_order;  // immersed boundary: the 2D stage tile (STAGE_TX x STAGE_TY cells; row-major
                               // index over the tile grid, bits 0..30) each workgroup of a stage launch
                               // takes, by workgroup index within a batch member, and in bit 31 the tile's
                               // body flag: set if a cell of the tile or a source cell its halo loads is not
                               // fluid (nullptr: the XCD-aware order of xcd_tile, and every tile checks its
                               // cells)
  GhostTable gt;               // immersed boundary: the ghost table (gt.n = 0 without)
  void* ghost_back;            // stage kernels: where the refilled ghost values of the stage
                               // state are written (storage type), or nullptr; when it is the
                               // stage state itself, the update reads them back from there
  unsigned long long* xslots;  // [nbatch][2][XSLOTS] spread extrema of the fused step
  const float* dXnet;          // its stencil gradient per face [nbatch][nface][24] or nullptr
  const float* dFext;          // precomputed face correction [nbatch][nface][4] (face frame) or nullptr
  long long nface;             // x-faces (nx+1)*ny then y-faces nx*(ny+1)
  Globals* glob;
};

// Learned face-flux correction: weights in the matrix-core layout (bf16),
// biases, input normalisation and output scale.
struct NetArgs {
  const unsigned short* w;  // bf16 bits, device layout of mlp.hpp
  const float* bias;
  double mean[4], inv_std[4];
  float out_scale;
};

// Host-side launchers (stage.hip, ibm.hip).
template <class S>
hipError_t launch_prim_to_cons(const GridArgs& a, const S* W, S* U, hipStream_t st);
template <class S>
hipError_t launch_cfl(const GridArgs& a, const S* U, double* dt_out, hipStream_t st);
// reverse mode of the primitive-to-conservative conversion (FP64); part:
// VJP_BLOCKS doubles per batch member
constexpr int VJP_BLOCKS = 256;
hipError_t launch_prim_to_cons_vjp(const GridArgs& a, const double* W, const double* Ubar, double* Wbar,
                                   double* param_bar, double* part, hipStream_t st);
template <class S>
hipError_t launch_stage(const GridArgs& a, int mode, const S* Us, const S* Un, S* Uout,
                        const double* dtp, const S* Lin, hipStream_t st);
hipError_t launch_init_scalars(const GridArgs& a, double t0, double t_end, hipStream_t st);
template <class S>
hipError_t launch_ibm_fill(const GridArgs& a, const GhostTable& gt, S* U, hipStream_t st);
hipError_t launch_ibm_classify(const GridArgs& a, const double* phi, uint8_t* cls, int* row_count,
                               hipStream_t st);
// per-tile flags of the stage kernel's immersed-boundary handling (a.cls set)
hipError_t launch_tile_body(const GridArgs& a, uint8_t* flags, hipStream_t st);
inline long long stage_tiles(int nx, int ny) {
  return (long long)((nx + STAGE_TX - 1) / STAGE_TX) * ((ny + STAGE_TY - 1) / STAGE_TY);
}
hipError_t launch_ibm_table(const GridArgs& a, const double* phi, const uint8_t* cls, const int* row_count,
                            int* row_off, GhostTable gt, int* nbad, hipStream_t st);
// Stage kernel with the learned correction evaluated inside the tile (2D,
// FP64, inviscid; modes MODE_RHS .. MODE_STAGE3).
hipError_t launch_stage_net(const GridArgs& a, const NetArgs& n, int mode, const double* Us, const double* Un,
                            double* Uout, const double* dtp, hipStream_t st);
hipError_t launch_stage_ext(const GridArgs& a, int mode, const double* Us, const double* Un, double* Uo,
                            const double* dtp, hipStream_t st);
hipError_t launch_stage_mixed(const GridArgs& a, int mode, const float* Us, const float* Un, float* Uout,
                              const double* dtp, const float* Lin, hipStream_t st);

// adjoint (adjoint.hip)
// Per-block partial derivatives of several launches, summed in one pass:
// slot s holds nblk[s] blocks per batch member at part + s * stride.
constexpr int MAX_PART_SLOTS = 6;
struct PartSlots {
  int n;
  int nblk[MAX_PART_SLOTS];
  long long stride;
};
// tile of the right-hand-side adjoint kernel (cells x, cells y, threads);
// the workspace sizes its per-block partials with the same tiles
constexpr int ADJ_TX = 32, ADJ_TY = 8, ADJ_NT = 768;
int adjoint_blocks(const GridArgs& a);
// With the immersed boundary (gW != nullptr, a.ghost_of set) the kernel also
// runs the first half of the refill transpose for the ghost cells it owns:
// their image-point adjoints go to gW and their own entries of out to zero.
hipError_t launch_rhs_adjoint(const GridArgs& a, const double* Us, const double* lam, double clam_f,
                              const double* dtp, const double* X1, double c1, const double* X2, double c2,
                              const double* X3, double c3, double* out, double* part, int* nblk,
                              const GhostTable& gt, double* gW, hipStream_t st);
hipError_t launch_ghost_index(const GridArgs& a, const GhostTable& gt, int* ghost_of, hipStream_t st);
hipError_t launch_partials_finalize(const double* part, const PartSlots& ps, int nbatch, double* param_bar,
                                    hipStream_t st);
hipError_t launch_ibm_entries(const GhostTable& gt, int* keys, int* vals, int* nvalid, hipStream_t st);
// Second half of the refill transpose (one workgroup per batch member): the
// source cells gather the image-point adjoints gW left by the adjoint
// kernel.  Its block partial goes to part (1 block per member).  With
// param_bar set it also finalises: param_bar += the slots of prior (which lie
// before part, at part - (prior.n - s) * prior.stride for slot s) plus its
// own partial.  The fill table: for source h < nsrc its cell fsrc[h], its
// entry count fcnt[h] <= m, and for entry slot t < fcnt[h] the ghost index
// fk[t * nsrc + h] and weight fw[t * nsrc + h], in entry order.
hipError_t launch_ibm_fill_adjoint(const GridArgs& a, const GhostTable& gt, const int* fsrc, const int* fcnt,
                                   const int* fk, const double* fw, int m, int nsrc, const double* Us, double* X,
                                   const double* gW, double* part, const PartSlots& prior, double* param_bar,
                                   hipStream_t st);
hipError_t launch_axpy(long long n, double alpha, const double* x, double* y, int accumulate, hipStream_t st);

// stage modes
enum : int { MODE_RHS = 0, MODE_STAGE1 = 1, MODE_STAGE2 = 2, MODE_STAGE3 = 3,
             MODE_S1L = 4, MODE_S2F = 5, MODE_S3F = 6 };
// learned correction inside the stage kernel: none, the per-face network
// evaluated in the tile, or a precomputed per-face correction (dFext)
enum : int { NET_NONE = 0, NET_MLP = 1, NET_EXT = 2 };

}  // namespace shk
