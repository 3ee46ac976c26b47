/*
 * shk.h -- C ABI of the MI355X (gfx950) WENO5 / HLLC / immersed-boundary /
 * SSP-RK3 library (libshk.so).
 *
 * The library evaluates the right-hand side of the compressible Euler (and,
 * optionally, Navier-Stokes) equations on a uniform Cartesian grid and
 * advances it with the three-stage strong-stability-preserving Runge-Kutta
 * scheme.  The method is the one of section 2 of arXiv 2601.04400:
 *   - state U = (rho, rho u, rho v, E), flux tensor and ideal-gas equation of
 *     state: eq. (euler) and the equation of state after it;
 *   - fifth-order WENO reconstruction of the primitive variables (rho,u,v,p),
 *     component by component, per dimension (Jiang-Shu weights);
 *   - HLLC flux of section 2 (Davis wave speeds, contact speed, star states;
 *     the star energy is the Rankine-Hugoniot-consistent
 *     E + (s*-u)(rho s* + p/(s-u)));
 *   - conservative flux-difference update of section 2 (with the optional
 *     Laplacian artificial viscosity nu lap U), advanced by Shu-Osher SSP-RK3;
 *   - ghost-cell immersed boundary (section 2, Mittal & Iaccarino) on a
 *     signed-distance level set.
 *
 * Conventions
 *   Ownership.  Every buffer (state, right-hand side, level set, workspace,
 *     time-step scalars) is allocated and owned by the caller.  The library
 *     never allocates device memory; it carves the caller's workspace.
 *   Pointers.  Unless stated otherwise every array argument is a DEVICE
 *     pointer; descriptors, handles and *_host outputs are host pointers.
 *   Layout.  A state is [nbatch][nvar][ny][nx], x fastest, with nvar = 3 in 1D
 *     (rho, rho u, E) and 4 in 2D (rho, rho u, rho v, E).  Element type is
 *     double for SHK_F64 and float for SHK_F32 and SHK_MIXED.  No ghost
 *     layers are stored: boundary values are produced on the fly.
 *   Asynchrony.  All work is enqueued on the grid's HIP stream; no call
 *     synchronises except shk_init_grid, shk_set_ib_levelset, shk_get_time
 *     and shk_poll_faults, which say so.
 *   Errors.  Every call returns a status; argument errors are detected before
 *     anything is enqueued.  shk_last_error gives a message.  Numerical
 *     faults during a run are latched in a device fault word
 *     (shk_poll_faults).
 *   Threads.  A handle must not be used by two host threads at once.
 */
#ifndef SHK_H
#define SHK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct shk_grid shk_grid;

typedef enum {
  SHK_OK = 0,
  SHK_EINVAL = 1,       /* bad argument (null pointer, size, enum value)       */
  SHK_ESTATE = 2,       /* call not valid in the handle's current state         */
  SHK_EHIP = 3,         /* a HIP runtime call failed                            */
  SHK_EFAULT = 4,       /* a numerical fault was latched (see shk_poll_faults)  */
  SHK_EUNSUPPORTED = 5, /* option combination not implemented                   */
  SHK_ESPACE = 6        /* workspace smaller than shk_workspace_bytes()         */
} shk_status;

typedef enum { SHK_F64 = 0, SHK_F32 = 1, SHK_MIXED = 2 } shk_precision;
/* SHK_MIXED: float storage, double arithmetic everywhere in the kernels.      */

typedef enum {
  SHK_BC_TRANSMISSIVE = 0, /* zero-order extrapolation of the nearest cell     */
  SHK_BC_REFLECTIVE = 1,   /* mirror, normal momentum negated                  */
  SHK_BC_INFLOW = 2,       /* fixed state inflow_prim                          */
  SHK_BC_PERIODIC = 3
} shk_bc;

/* Fault word bits (shk_poll_faults). */
#define SHK_FAULT_NONFINITE  0x1u  /* a non-finite value was written           */
#define SHK_FAULT_FALLBACK   0x2u  /* positivity fallback used at some face    */
#define SHK_FAULT_NONPHYS    0x4u  /* a cell with rho <= 0 or p <= 0 was read  */
#define SHK_FAULT_NET        0x8u  /* flux-net output rejected (fallback used) */

typedef struct {
  int ndim;            /* 1 or 2; ndim 1 requires ny == 1                     */
  int nx, ny;          /* interior cells; >= 3 along each axis of the grid    */
                       /* (boundary ghost layers are 3 interior cells deep)   */
  int nbatch;          /* independent grids sharing geometry and parameters   */
  double x0, x1, y0, y1; /* domain; cell centres at x0 + (i+1/2) dx           */
  int prec;            /* shk_precision                                       */
  double gamma;        /* ratio of specific heats (> 1)                       */
  double cfl;          /* Courant number of the automatic step                */
  double weno_eps;     /* WENO epsilon (1e-6 if <= 0)                         */
  int viscous;         /* 1: Navier-Stokes viscous and heat fluxes (2D only)  */
  double mu, prandtl;  /* constant dynamic viscosity; Prandtl number          */
  double nu_art;       /* Laplacian artificial viscosity nu (0 = off)         */
  int bc[4];           /* shk_bc for x-lo, x-hi, y-lo, y-hi                   */
  double inflow_prim[4]; /* (rho, u, v, p) used by SHK_BC_INFLOW              */
  int ibm;             /* 1: reserve immersed-boundary tables in the workspace */
  int adjoint;         /* 1: reserve adjoint buffers in the workspace          */
  int flux_net;        /* 1: per-face network, 2: convolutional network -- reserve
                          its buffers (ndim 2, SHK_F64, inviscid)            */
  int weno_char;       /* 1: WENO5 on characteristic variables (projection on
                          the eigenvectors of the face-normal flux Jacobian at
                          the Roe average of the two adjacent cells) instead
                          of on primitives; SHK_F64, no flux_net, no adjoint */
} shk_grid_desc;

/* Bytes of device workspace a grid with this descriptor needs (0 on a bad
 * descriptor).  The caller allocates it (256-byte aligned) and keeps it
 * alive until shk_destroy. */
size_t shk_workspace_bytes(const shk_grid_desc* desc);

/* Validate desc, carve workspace, initialise the device scalars (t = 0,
 * t_end = +inf) on hip_stream (a hipStream_t; NULL = default stream) and
 * return a handle in *out.  Synchronises the stream once.  Errors: SHK_EINVAL
 * (bad desc or null pointer), SHK_ESPACE (ws_bytes too small), SHK_EHIP. */
shk_status shk_init_grid(const shk_grid_desc* desc, void* workspace, size_t ws_bytes,
                         void* hip_stream, shk_grid** out);

/* Release the handle (not the caller's memory).  NULL is accepted. */
void shk_destroy(shk_grid* g);

/* Change the stream subsequent calls enqueue on. */
shk_status shk_set_stream(shk_grid* g, void* hip_stream);

/* Convert primitive planes W -> conservative planes U (same layout as a
 * state; in 1D W holds (rho, u, p)), E = p/(gamma-1) + rho (u^2+v^2)/2.
 * W and U are device arrays of the grid's element type; they may not alias. */
shk_status shk_prim_to_cons(shk_grid* g, const void* W, void* U);

/* Reverse mode of shk_prim_to_cons, to carry the gradient of a loss with
 * respect to a conservative state (the initial state of a differentiated
 * run, section 2 and the reverse learning of section 3) back to the
 * primitive variables it was built from and to gamma.  With U = (rho, rho u,
 * rho v, E), E = p/(gamma-1) + rho (u^2+v^2)/2 (1D: (rho, rho u, E), W =
 * (rho, u, p)):  W_bar += (dU/dW)^T U_bar cell by cell, and
 * param_bar[b][0] += sum over the cells of member b of (dU/dgamma) . U_bar,
 * summed in a fixed order.  W, U_bar, W_bar: device doubles in the state
 * layout (W_bar may alias neither); param_bar: device [nbatch][5] as for
 * shk_rhs_adjoint; W_bar or param_bar may be NULL.  SHK_F64 grids
 * (SHK_EUNSUPPORTED otherwise). */
shk_status shk_prim_to_cons_vjp(shk_grid* g, const void* W, const void* U_bar, void* W_bar, double* param_bar);

/* Immersed boundary on the signed-distance level set phi (device, double,
 * [ny][nx], phi < 0 inside the solid; shared by all batch members).
 * Classifies cells (fluid phi >= 0, solid, ghost = solid within 3 cells of a
 * fluid cell along x or y), and builds the per-ghost image-point table
 * (mirror point at twice the wall distance along grad phi, fluid-only
 * bilinear weights).  wall: 0 slip (normal velocity reflected), 1 no-slip
 * adiabatic (velocity reversed); rho and p are copied from the image point.
 * From then on ghost cells are refilled before every right-hand side and the
 * right-hand side is zero at solid and ghost cells.  Requires desc.ibm = 1
 * and ndim = 2.  Synchronises the stream once (to size the ghost list).
 * phi = NULL removes the immersed boundary.  SHK_EINVAL (and no immersed
 * boundary) when some ghost has no image point: the central-difference
 * gradient of phi there is far from unit length (|grad phi| < 1/2, where the
 * difference straddles the solid's medial axis: a solid thinner than about
 * two cells, a body a few cells across), or no fluid cell is found around
 * the image point or along the normal. */
shk_status shk_set_ib_levelset(shk_grid* g, const double* phi, int wall);

/* Change the ratio of specific heats gamma and, unless inflow_prim is NULL,
 * the inflow state (host, 4 doubles (rho, u, v, p)) of an existing grid, as
 * a parameter fit does between its iterations (section 3, reverse learning
 * of gamma).  Affects the calls enqueued after it; the level set, the
 * workspace and the network are kept.  SHK_EINVAL for gamma <= 1 or a
 * non-positive inflow density or pressure. */
shk_status shk_set_params(shk_grid* g, double gamma, const double* inflow_prim);

/* Number of ghost cells of the current immersed boundary (host output). */
shk_status shk_ib_ghost_count(const shk_grid* g, int* n_host);

/* Copy the cell classes (0 fluid, 1 solid, 2 ghost) into cls (device,
 * uint8 [ny][nx]). */
shk_status shk_ib_classes(shk_grid* g, uint8_t* cls);

/* Right-hand side dUdt = L(U) of the semi-discrete scheme (section 2
 * conservative update without the time step).  With an immersed boundary
 * the ghost cells take their refilled values (formed from the fluid cells
 * of U while the kernel loads them); U is not modified.  U and dUdt must not
 * alias. */
shk_status shk_rhs(shk_grid* g, const void* U, void* dUdt);

/* Refill the ghost cells of U in place from its fluid cells (the values
 * every right-hand side and stage uses for them).  SHK_ESTATE without an
 * immersed boundary. */
shk_status shk_ib_fill(shk_grid* g, void* U);

/* One SSP-RK3 step of U in place:
 *   U1 = U + dt L(U); U2 = 3/4 U + 1/4 U1 + dt/4 L(U1);
 *   U <- 1/3 U + 2/3 U2 + 2 dt/3 L(U2),
 * each stage state's ghost cells refilled before its right-hand side (the
 * refilled ghosts of U enter the last combination).
 * dt_in: device array of nbatch doubles with a fixed step, or NULL for the
 * automatic step dt = cfl / max_fluid[(|u|+a)/dx + (|v|+a)/dy] (plus the
 * explicit viscous limit), computed from U on the device and shortened so
 * that the device time lands exactly on t_end (after which steps are
 * no-ops).  dt_out: device array of nbatch doubles receiving the step used,
 * or NULL. */
shk_status shk_rk3_step(shk_grid* g, void* U, const double* dt_in, double* dt_out);

/* Discrete adjoint of shk_rhs (reverse mode).  The chain rule through the
 * unrolled solver (section 2, gradient of the unrolled loss through the
 * solver step S) is built from these vector-Jacobian products.  U: state at
 * which shk_rhs was evaluated (device, double; it is not modified, the
 * ghost refill is recomputed on a copy).  dUdt_bar: adjoint of the
 * right-hand side.  U_bar += (d rhs / d U)^T dUdt_bar, the map including the
 * immersed-boundary refill and the boundary rules.  param_bar (device,
 * [nbatch][5]) += derivatives with respect to (gamma, inflow rho, u, v, p).
 * Every branch is the one the forward evaluation takes; the WENO weights are
 * differentiated.  Reproducible bit for bit (no atomics in the sums).
 * Requires desc.adjoint = 1, prec SHK_F64, ndim 2, inviscid, nu_art = 0
 * (else SHK_ESTATE / SHK_EUNSUPPORTED). */
shk_status shk_rhs_adjoint(shk_grid* g, const void* U, const void* dUdt_bar, void* U_bar, double* param_bar);

/* Discrete adjoint of one fixed-step SSP-RK3 step.  U_n: the state the step
 * started from (device, double, not modified); dt: device array of nbatch
 * steps (treated as constants); U_bar: on entry the adjoint of the state
 * after the step, on return the adjoint of U_n; param_bar (device,
 * [nbatch][5]) += parameter derivatives as for shk_rhs_adjoint.  The stage
 * states are recomputed from U_n in the workspace.  Same requirements as
 * shk_rhs_adjoint. */
shk_status shk_rk3_step_adjoint(shk_grid* g, const void* U_n, const double* dt, void* U_bar, double* param_bar);

/* One SSP-RK3 step exactly as shk_rk3_step (fixed dt_in or automatic step,
 * dt_out as there) that also records the stage-start states for the reverse
 * pass: tape (device, double, caller-owned, 3 states = 3 * nbatch * 4 * ny *
 * nx entries) receives U^n, U1 and U2 (section 2 RK3 stages), each after the
 * immersed-boundary refill.  The automatic step is not fused into the stages
 * here (one extra reduction launch).  A step of zero length (dt_in 0, or the
 * end time already reached) leaves U and the tape untouched.  Same
 * requirements as shk_rhs_adjoint; SHK_EINVAL for a null U or tape. */
shk_status shk_rk3_step_record(shk_grid* g, void* U, const double* dt_in, double* dt_out, void* tape);

/* Discrete adjoint of one recorded step (as shk_rk3_step_adjoint, with the
 * stage states read from a tape written by shk_rk3_step_record instead of
 * recomputed).  dt: device array of the nbatch steps the recorded step used
 * (dt_in, or its dt_out).  The tape is not modified.  Same requirements as
 * shk_rhs_adjoint; SHK_EINVAL for a null tape, dt or U_bar. */
shk_status shk_rk3_step_adjoint_tape(shk_grid* g, const void* tape, const double* dt, void* U_bar,
                                     double* param_bar);

/* nsteps fixed-dt SSP-RK3 steps, each as shk_rk3_step_record: U advances in
 * place and tapes (device, double, caller-owned, nsteps * 3 states) receive
 * the stage-start states of step k at tapes + 3 k (one state = nbatch * 4 *
 * ny * nx entries).  dt: device array of nbatch steps used by every step.
 * The loop runs in the library (no per-step call overhead).  Same
 * requirements as shk_rhs_adjoint; SHK_EINVAL for null arrays or
 * nsteps < 0. */
shk_status shk_rk3_steps_record(shk_grid* g, void* U, int nsteps, const double* dt, void* tapes);

/* Reverse of nsteps recorded steps, last first: U_bar enters as the adjoint of
 * the state after the last step and leaves as the adjoint of the state before
 * the first; param_bar += the parameter derivatives of every step.  As
 * nsteps calls of shk_rk3_step_adjoint_tape on tapes + 3 k, k = nsteps-1..0. */
shk_status shk_rk3_steps_adjoint_tape(shk_grid* g, const void* tapes, int nsteps, const double* dt, void* U_bar,
                                      double* param_bar);

/* ---- Learned flux correction (section 2 neural flux, per-face MLP form) ----
 * F = F_HLLC + dF with dF = s_out tanh(MLP(x)), x = the 6-cell stencil of
 * (rho, u_n, u_t, p) in the face-normal frame normalised as (w - mean) *
 * inv_std; hidden layers 64-64-64 with ReLU; the same parameters for x- and
 * y-faces (u_n/u_t rotated).  Weights are bfloat16 and every matrix product
 * runs on the matrix cores with FP32 accumulation.
 * Parameter vector theta (FP32, 10180 entries, gradients and Adam use it):
 * W0[64][24], b0[64], W1[64][64], b1[64], W2[64][64], b2[64], W3[4][64], b3[4].
 * Device form used by the kernels (shk_flux_net_pack writes it): bf16
 * W0[64][32] (inputs zero-padded), W1[64][64], W2[64][64], W3[16][64]
 * (outputs zero-padded) = 11264 values, and FP32 biases b0[64], b1[64],
 * b2[64], b3[16] = 208 values. */

/* Enable (enable = 1) or disable the correction.  w_bf16 (device, 11264
 * bf16 bit patterns) and bias (device, 208 floats) stay owned by the caller
 * and must outlive their use; norm_host = host {mean[4], inv_std[4]};
 * out_scale = s_out.  While enabled, shk_rhs and shk_rk3_step evaluate the
 * network for every face of each stage state before the stage kernel (the
 * automatic step then uses the separate reduction), and the adjoint entry
 * points include its reverse pass.  A non-finite network output falls back to
 * the uncorrected flux at that face and sets SHK_FAULT_NET.  Requires
 * desc.flux_net = 1 (SHK_ESTATE otherwise). */
shk_status shk_set_flux_net(shk_grid* g, const uint16_t* w_bf16, const float* bias, const double* norm_host,
                            float out_scale, int enable);

/* Accumulate the parameter gradient (device, 10180 floats, theta order) of
 * every later adjoint call into grad (+=); NULL stops accumulating. */
shk_status shk_set_flux_net_grad(shk_grid* g, float* grad);

/* Network output for every face of state U (device double): dF (device,
 * [nbatch][nface][4] floats, face frame), faces ordered x-faces
 * (j*(nx+1)+i, i = 0..nx) then y-faces ((nx+1)*ny + j*nx + i, j = 0..ny). */
shk_status shk_flux_net_eval(shk_grid* g, const void* U, float* dF);

/* Reverse of the network alone: face-flux gradients formed from the
 * right-hand-side adjoint lam as in the flux difference (F_bar = (lam_right -
 * lam_left)/h, face frame); writes dX (device, [nbatch][nface][6][4] floats,
 * gradient w.r.t. the stencil primitives) and adds the parameter gradient to
 * grad (device, 10180 floats, may be NULL).  Requires desc.adjoint = 1. */
shk_status shk_flux_net_vjp(shk_grid* g, const void* U, const void* lam, float* dX, float* grad);

/* Device form (bf16 weights, FP32 biases) from theta; all device arrays. */
shk_status shk_flux_net_pack(const float* theta, uint16_t* w_bf16, float* bias, void* hip_stream);

/* ---- Learned flux correction, convolutional form (section 2: the paper's
 * 2D neural flux, a fully convolutional network of three 3x3 layers) ----
 * Channels 4 -> 16 -> 32 -> 4, ReLU, ReLU, tanh x s_out, 6388 parameters, one
 * parameter set for both directions.  Its pixels are faces: image 0 = the
 * x-faces (ny rows, nx + 1 columns), image 1 = the y-faces transposed (nx
 * rows, ny + 1 columns), so the face normal runs along the columns of both;
 * a periodic axis holds each face once (nx columns; the last face of a row
 * is its first) and wraps the 3x3 windows, other boundaries pad them with
 * zeros.  A pixel's input is the conservative form of the mean of the
 * face's two WENO5 states (after the positivity fallback), face frame
 * (rho, rho u_n, rho u_t, E), normalised as (x - mean) * inv_std; its
 * output is the face-frame correction added to the HLLC flux.  bf16
 * weights, FP32 accumulation on the matrix cores.
 * Parameter vector theta (FP32, 6388 entries): W1[16][3][3][4], b1[16],
 * W2[32][3][3][16], b2[32], W3[4][3][3][32], b3[4] (W[out][dy][dx][in]).
 * Device form (shk_flux_cnn_pack writes it): 18432 bf16 values (forward and
 * input-gradient weight matrices) and 64 FP32 biases. */

/* Enable (enable = 1) or disable the convolutional correction; arguments as
 * for shk_set_flux_net (device w_bf16 [18432], bias [64]; host norm_host =
 * {mean[4], inv_std[4]} of the conservative inputs; out_scale > 0).  While
 * enabled, every stage evaluates the network over the face images of its
 * state before the stage kernel, and the adjoint entry points include its
 * reverse pass; the parameter gradient goes to the buffer set by
 * shk_set_flux_net_grad (6388 floats).  A non-finite output falls back to the
 * uncorrected flux at that face and sets SHK_FAULT_NET.  Requires
 * desc.flux_net = 2 (SHK_ESTATE otherwise). */
shk_status shk_set_flux_cnn(shk_grid* g, const uint16_t* w_bf16, const float* bias, const double* norm_host,
                            float out_scale, int enable);

/* Network output for every face of state U: dF (device, [nbatch][nface][4]
 * floats, face frame, faces ordered as for shk_flux_net_eval). */
shk_status shk_flux_cnn_eval(shk_grid* g, const void* U, float* dF);

/* Reverse of the network alone, as shk_flux_net_vjp: dX (device,
 * [nbatch][nface][6][4]) = gradient w.r.t. each face's stencil primitives
 * through its input (the last face of a periodic row repeats the first);
 * adds the parameter gradient to grad (6388 floats, may be NULL).  The face
 * adjoints are (lam_right - lam_left) / h with the periodic wrap, so the
 * first face of a periodic row carries both of its uses. */
shk_status shk_flux_cnn_vjp(shk_grid* g, const void* U, const void* lam, float* dX, float* grad);

/* The network's input images of state U as floats (their bf16 values):
 * images (device, [nbatch][npix][4]), image 0's pixels row by row, then
 * image 1's.  *npix receives the pixels per batch member; with U and images
 * both NULL only *npix is set. */
shk_status shk_flux_cnn_images(shk_grid* g, const void* U, float* images, int* npix);

/* Device form (bf16 weight matrices, FP32 biases) from theta. */
shk_status shk_flux_cnn_pack(const float* theta, uint16_t* w_bf16, float* bias, void* hip_stream);

/* One Adam step on n parameters (Kingma & Ba, the optimiser of section 3;
 * device FP32 arrays; step counts from 1):
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   theta <- theta - lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps),
 * the two bias corrections formed in double on the host.  SHK_EINVAL for
 * null arrays, n < 1, step < 1, or beta1 / beta2 outside [0, 1). */
shk_status shk_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float beta1, float beta2,
                    float eps, int step, void* hip_stream);

/* Block average by factor x factor (the restriction d(U) of section 2):
 * fine [nbatch][nvar][ny_f][nx_f] -> coarse [nbatch][nvar][ny_f/factor][nx_f/factor],
 * device doubles; nx_f, ny_f must be multiples of factor. */
shk_status shk_restrict(const double* fine, double* coarse, int nx_f, int ny_f, int factor, int nvar, int nbatch,
                        void* hip_stream);

/* Unrolled-loss term of section 2 per batch member: loss[b] += ||U_b - T_b||^2
 * / per_batch, and G_b += scale * 2 (U_b - T_b) / per_batch if G is not NULL.
 * part: device scratch of nbatch * 256 doubles.  Fixed summation order. */
shk_status shk_mse(const double* U, const double* T, double* G, double scale, long long per_batch, int nbatch,
                   double* part, double* loss, void* hip_stream);

/* shk_mse for callers that cannot allocate memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid allocation): the same
 * kernels and the same result bit for bit, with the block partials in a
 * static device array of the library (SHK_MSE_NOALLOC_MAX_BATCH * 256
 * doubles, 512 KiB on each GPU it runs on, held until the process ends)
 * instead of a caller buffer.  Allocates nothing.  The stream must belong to
 * the current device.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (two streams, two threads) race and must be ordered by
 * the caller.  SHK_EINVAL for a null U, T or loss, per_batch < 1, or nbatch
 * outside 1..SHK_MSE_NOALLOC_MAX_BATCH. */
#define SHK_MSE_NOALLOC_MAX_BATCH 256
shk_status shk_mse_noalloc(const double* U, const double* T, double* G, double scale, long long per_batch,
                           int nbatch, double* loss, void* hip_stream);

/* Set the device time of every batch member to t0, the stop time to t_end
 * and the automatic-step counter to 0 (enqueued). */
shk_status shk_set_time(shk_grid* g, double t0, double t_end);

/* Read the device time, end flag and number of automatic steps taken since
 * shk_set_time of batch member b (host outputs, each may be NULL;
 * synchronises). */
shk_status shk_get_time(shk_grid* g, int b, double* t_host, int* done_host, int* steps_host);

/* Read and clear the fault word and the positivity-fallback face count
 * (synchronises). */
shk_status shk_poll_faults(shk_grid* g, uint32_t* flags_host, uint64_t* fallback_faces_host);

/* Kernel timing for performance reports.  With enable = 1 every later
 * shk_rk3_step brackets each of its kernels with HIP events on the grid's
 * stream (a small gap between launches results); enable = 0 stops and
 * discards the records.  shk_profile_read synchronises and returns, per kernel
 * class, the summed duration in milliseconds and the launch count:
 * index 0 time-step reduction, 1 stage 1, 2 stage 2, 3 stage 3, 4 ghost fill.
 * ms_host and count_host are host arrays of 5 entries. */
shk_status shk_profile(shk_grid* g, int enable);
shk_status shk_profile_read(shk_grid* g, double* ms_host, int* count_host);

/* Message of the last failed call on this handle ("" if none). */
const char* shk_last_error(const shk_grid* g);

/* Name of a status code. */
const char* shk_status_string(int status);

/* Post-shock state (rho2, u2, p2) behind a normal shock of Mach number
 * mach moving into gas at rest (rho1, p1) (normal-shock relations; the
 * paper's shock-cylinder inflow state is the Mach-5 case), and its
 * derivatives with respect to mach and gamma.  Host arrays; d_dmach and
 * d_dgamma may be NULL. */
shk_status shk_normal_shock_state(double mach, double gamma, double rho1, double p1, double* out3_host,
                                  double* d_dmach3_host, double* d_dgamma3_host);

#ifdef __cplusplus
}
#endif

#endif /* SHK_H */
