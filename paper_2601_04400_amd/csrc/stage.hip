// Fused right-hand-side / SSP-RK3 stage kernel, CFL reduction and
// primitive-to-conservative conversion for gfx950.
//
// One workgroup owns a TX x TY tile of cells.  It stages the tile plus a
// 3-cell halo of primitive variables in LDS (boundary rules applied while
// loading), computes every x- and y-face flux of the tile once (WENO5-JS on
// (rho, u, v, p), HLLC, optional viscous flux) into LDS, and finishes with the
// flux difference and the Runge-Kutta combination, writing each cell once.
// HBM traffic per stage is one read of the stage state (halo re-reads hit
// L2), one read of U^n for stages 2 and 3, and one write.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "flux.hpp"
#include "grid.hpp"
#include "ibm_dev.hpp"
#include "xcd.hpp"
#include "mlp.hpp"
#include "mlp_dev.hpp"

namespace shk {

// ----------------------------------------------------------- boundary rules
// Map a possibly out-of-range index along one axis to its source cell.
// flag: 0 copy, 1 copy and negate the momentum normal to this axis,
// 2 replace the whole state by the inflow state.
__device__ __forceinline__ int bc_source(int g, int n, int bc_lo, int bc_hi, int& flag) {
  if (g >= 0 && g < n) return g;
  const bool lo = g < 0;
  const int bc = lo ? bc_lo : bc_hi;
  const int depth = lo ? -g : g - (n - 1);  // 1 for the first ghost layer
  int s;
  switch (bc) {
    case BC_REFL: s = lo ? depth - 1 : n - depth; flag = flag | 1; break;
    case BC_INFLOW: s = lo ? 0 : n - 1; flag = 2; break;
    case BC_PERIODIC: s = ((g % n) + n) % n; break;
    default: s = lo ? 0 : n - 1; break;  // transmissive
  }
  return s < 0 ? 0 : (s >= n ? n - 1 : s);
}

// Refilled value of the immersed-boundary ghost cell of ghost index k of a stage state
// whose plane e of interior cell c is get(e, c), rounded to the storage type
// as the separate refill stores it.
template <class S, class C, class Get>
__device__ __forceinline__ void ghost_at(const GridArgs& a, int k, Get&& get, C q[4]) {
  double g[4];
  ghost_cons(a.gt, a.gamma, k, [&](int e, long long s) { return double(get(e, s)); }, g);
#pragma unroll
  for (int v = 0; v < 4; ++v) q[v] = C(S(g[v]));
}

// Conservative state (rho, m_x, m_y, E) of cell (gi, gj), which may lie in
// the ghost layers; x rules are applied first, then y rules (a y inflow
// overrides everything, as for a y-ghost layer filled after the x-ghosts).
// get(e, c) returns plane e of interior cell c.  An immersed-boundary ghost
// cell takes its refilled value, formed here from the fluid cells of the
// same state (they are complete when the stage starts).
// inside: (gi, gj) is known to be an interior cell (no boundary rule).
// DEFER: an immersed-boundary ghost cell is not refilled here; its ghost
// index goes to *ghost (else -1) and q holds its stored values.
template <class S, class C, int NDIM, bool GH, bool DEFER = false, class Get>
__device__ __forceinline__ void load_cons_f(const GridArgs& a, int gi, int gj, Get&& get, C q[4],
                                            bool inside = false, int* ghost = nullptr) {
  if (DEFER) *ghost = -1;
  int fx = 0, fy = 0;
  int si = gi, sj = NDIM == 2 ? gj : 0;
  if (!inside) {
    si = bc_source(gi, a.nx, a.bc[0], a.bc[1], fx);
    if (NDIM == 2) sj = bc_source(gj, a.ny, a.bc[2], a.bc[3], fy);
  }
  // scalars, not the array, along the branches (an array written on some
  // paths only is kept in scratch memory)
  C r, mx, my, E;
  if (fy == 2 || fx == 2) {
    r = C(a.inflow_cons[0]);
    mx = C(a.inflow_cons[1]);
    my = NDIM == 1 ? C(0) : C(a.inflow_cons[2]);
    E = C(a.inflow_cons[3]);
  } else {
    const long long c = (long long)sj * a.nx + si;
    // the state loads do not wait for the ghost test: they are issued beside
    // the ghost-index load (which itself marks a ghost cell), and a ghost
    // cell's values are then replaced by its refilled ones
    r = get(0, c);
    mx = get(1, c);
    if (NDIM == 2) {
      my = get(2, c);
      E = get(3, c);
    } else {
      my = C(0);
      E = get(2, c);
    }
    const int gk = GH && a.ghost_of != nullptr ? a.ghost_of[c] : -1;
    if (DEFER) {
      *ghost = gk;
    } else if (gk >= 0) {
      C g[4];
      ghost_at<S>(a, gk, get, g);
      r = g[0]; mx = g[1]; my = g[2]; E = g[3];
    }
    mx = (fx & 1) ? -mx : mx;
  }
  my = (fy & 1) ? -my : my;
  q[0] = r; q[1] = mx; q[2] = my; q[3] = E;
}

template <class S, class C, int NDIM, bool GH, bool DEFER = false>
__device__ __forceinline__ void load_cons(const GridArgs& a, const S* U, int gi, int gj, C q[4],
                                          bool inside = false, int* ghost = nullptr) {
  load_cons_f<S, C, NDIM, GH, DEFER>(a, gi, gj, [&](int e, long long c) { return C(U[e * a.ncell + c]); }, q,
                                     inside, ghost);
}

// Automatic step from the reduced maxima of a batch member (dt = cfl / max
// wave-speed sum, explicit viscous limit, shortened to land on t_end; 0 once
// t_end was reached).  *last tells whether this step reaches t_end.  Evaluated
// as written, without contraction, so every caller gets the same bits.
__device__ __forceinline__ double step_dt(const GridArgs& a, const StepScalars* sc, double sm,
                                                    double rm, bool* last) {
#pragma clang fp contract(off)
  *last = false;
  if (sc->done) return 0.0;
  double dt = a.cfl / sm;
  if (a.viscous && a.mu > 0.0) {
    const double h = a.ndim == 2 ? fmin(a.dx, a.dy) : a.dx;
    const double dv = 0.25 * h * h * rm / (a.mu * fmax(4.0 / 3.0, a.gamma / a.prandtl));
    dt = fmin(dt, dv);
  }
  if (sc->t + dt >= sc->t_end) {
    dt = sc->t_end - sc->t;
    *last = true;
  }
  return dt;
}

__device__ __forceinline__ double bits_to_double(unsigned long long u) { return __longlong_as_double((long long)u); }

// Wave-speed sum (|u|+a)/dx + (|v|+a)/dy of one cell (1D: x term), in double
// and in written order.
template <class S>
__device__ __forceinline__ double wave_speed_sum(const GridArgs& a, const S* __restrict__ U, long long c,
                                                            double* rho) {
#pragma clang fp contract(off)
  const double g = a.gamma;
  const double r = double(U[c]);
  const double u = double(U[a.ncell + c]) / r;
  const double v = a.ndim == 2 ? double(U[2 * a.ncell + c]) / r : 0.0;
  const double E = double(U[(a.nvar - 1) * a.ncell + c]);
  const double p = (g - 1.0) * (E - 0.5 * r * (u * u + v * v));
  const double cs = sqrt(g * p / r);
  double s = (fabs(u) + cs) / a.dx;
  if (a.ndim == 2) s = s + (fabs(v) + cs) / a.dy;
  *rho = r;
  return s;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// Extrema of the fused step, spread over XSLOTS atomic targets per batch
// member to avoid contention; every wave that calls this reduces all slots.
__device__ __forceinline__ void read_extrema(const GridArgs& a, int b, double* sm, double* rm) {
  const int lane = threadIdx.x & 63;
  const unsigned long long* xs = a.xslots + (long long)b * 2 * XSLOTS;
  *sm = wave_max(bits_to_double(xs[lane]));
  *rm = wave_min(bits_to_double(xs[XSLOTS + lane]));
}

template <class C>
__device__ __forceinline__ bool finite_val(C x) {
  return isfinite(x);
}

// Characteristic-wise WENO5 face states (the variant the paper leaves open):
// the six-cell stencil (face frame, primitive q0..q3 at stride st) in
// conservative form is projected on the left eigenvectors of the
// face-normal flux Jacobian at the Roe average of cells 2 and 3, each
// characteristic field is reconstructed like a primitive one, and the two
// states are projected back with the right eigenvectors:
//   R columns (u - c, u, u, u + c): (1, u - c, v, H - u c), (1, u, v, q),
//   (0, 0, 1, v), (1, u + c, v, H + u c);  L = R^-1 with b1 = (gamma-1)/c^2,
//   b2 = b1 q: ((b2 + u/c)/2, -(b1 u + 1/c)/2, -b1 v/2, b1/2),
//   (1 - b2, b1 u, b1 v, -b1), (-v, 0, 1, 0), ((b2 - u/c)/2, -(b1 u - 1/c)/2,
//   -b1 v/2, b1/2);  q = (u^2 + v^2)/2.
__device__ __forceinline__ void char_face_states(const double* q0, const double* q1, const double* q2,
                                                 const double* q3, int st, double eps, double gam,
                                                 Prim<double>& Lp, Prim<double>& Rp) {
  const double gm1 = gam - 1.0;
  const int ia = 2 * st, ib = 3 * st;
  const double ra = sqrt(q0[ia]), rb = sqrt(q0[ib]);
  const double Ha = gam / gm1 * q3[ia] / q0[ia] + 0.5 * (q1[ia] * q1[ia] + q2[ia] * q2[ia]);
  const double Hb = gam / gm1 * q3[ib] / q0[ib] + 0.5 * (q1[ib] * q1[ib] + q2[ib] * q2[ib]);
  const double iw = 1.0 / (ra + rb);
  const double u = (ra * q1[ia] + rb * q1[ib]) * iw, v = (ra * q2[ia] + rb * q2[ib]) * iw;
  const double H = (ra * Ha + rb * Hb) * iw;
  const double q = 0.5 * (u * u + v * v);
  const double c = sqrt(gm1 * (H - q));
  const double ic = 1.0 / c, b1 = gm1 * ic * ic, b2 = b1 * q;
  const double L[4][4] = {{0.5 * (b2 + u * ic), -0.5 * (b1 * u + ic), -0.5 * b1 * v, 0.5 * b1},
                          {1.0 - b2, b1 * u, b1 * v, -b1},
                          {-v, 0.0, 1.0, 0.0},
                          {0.5 * (b2 - u * ic), -0.5 * (b1 * u - ic), -0.5 * b1 * v, 0.5 * b1}};
  double wc[4][6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const double r = q0[s * st], un = q1[s * st], ut = q2[s * st], p = q3[s * st];
    const double U[4] = {r, r * un, r * ut, p / gm1 + 0.5 * r * (un * un + ut * ut)};
#pragma unroll
    for (int m = 0; m < 4; ++m) wc[m][s] = ((L[m][0] * U[0] + L[m][1] * U[1]) + L[m][2] * U[2]) + L[m][3] * U[3];
  }
  double wl[4], wr[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) weno5_pair(wc[m][0], wc[m][1], wc[m][2], wc[m][3], wc[m][4], wc[m][5], eps, wl[m], wr[m]);
  auto back = [&](const double w4[4], Prim<double>& P) {
    const double U0 = (w4[0] + w4[1]) + w4[3];
    const double U1 = ((u - c) * w4[0] + u * w4[1]) + (u + c) * w4[3];
    const double U2 = ((v * w4[0] + v * w4[1]) + w4[2]) + v * w4[3];
    const double U3 = (((H - u * c) * w4[0] + q * w4[1]) + v * w4[2]) + (H + u * c) * w4[3];
    P.r = U0;
    P.un = U1 / U0;
    P.ut = U2 / U0;
    P.p = gm1 * (U3 - 0.5 * U0 * (P.un * P.un + P.ut * P.ut));
  };
  back(wl, Lp);
  back(wr, Rp);
}

// Compile-time integer passed to a generic lambda.
template <int V>
struct IntC {
  static constexpr int value = V;
};

// ------------------------------------------------------------ stage kernel
// Modes: MODE_RHS writes L(U); MODE_STAGE1..3 are the three Shu-Osher stages
// with the step read from dtp[b].  The fused automatic-step sequence is
//   MODE_S1L: L0 = L(U^n) (written to Uout) and the block maxima of the
//             wave-speed sum and minima of the density of U^n;
//   MODE_S2F: dt from those extrema; U1 = U^n + dt L0 is formed while the
//             tile is loaded (never stored); writes U2;
//   MODE_S3F: stage 3 with the step of S2F; one block advances the device
//             time and clears the extrema for the next step.
//
// NET (learned face-flux correction, section 2 neural flux; added to each
// face flux in the face frame before the divergence):
//   NET_MLP: the per-face MLP, evaluated inside the tile on matrix cores from
//            the primitive halo the tile has already loaded;
//   NET_EXT: a correction computed beforehand for every face (the
//            convolutional network), read from a.dFext.
// CHAR: characteristic-wise WENO5 instead of the primitive-wise one (FP64).
// IBM: the grid has an immersed boundary (a.cls, a.ghost_of and a.gt set):
// ghost cells take their refilled values, formed from the stage state's
// fluid cells (in one pass over the tile's ghost slots after its plain
// loads), and their right-hand side is zero.  Tiles that a.tile_order marks
// all fluid skip this handling.
template <class S, class C, int NDIM, int TX, int TY, bool VISC, int MODE, int NET = NET_NONE, bool CHAR = false,
          bool IBM = false>
__global__ void __launch_bounds__(NDIM == 2 ? TX * TY : TX) stage_kernel(GridArgs a, const S* Us, const S* Un, S* Uout,
                                                    const double* __restrict__ dtp,
                                                    const S* __restrict__ Lin, NetArgs net) {
  // Us, Un and Uout may alias (stage 3 writes the step's result over U^n):
  // every cell is read before it is written, by the thread that writes it.
  // a.ghost_back may be Us: a ghost cell's refilled value is written there
  // by the workgroup whose tile holds the cell, in its ghost pass, and read
  // back only by that workgroup's update, after a barrier; any other read of
  // a ghost cell's stored value replaces it by the refilled one.
  constexpr int NT = NDIM == 2 ? TX * TY : TX;  // one thread per cell of the tile
  static_assert(NT % 64 == 0 && NT <= 1024, "whole waves");
  constexpr int H = HALO;
  constexpr int PX = TX + 2 * H;
  constexpr int PY = NDIM == 2 ? TY + 2 * H : 1;
  constexpr int NFX = (TX + 1) * TY;
  constexpr int NFY = NDIM == 2 ? TX * (TY + 1) : 0;
  constexpr int FYR = NDIM == 2 ? TY + 1 : 1;
  static_assert(NDIM == 2 || TY == 1, "1D tiles are one row");

  __shared__ C w[4][PY * PX];
  __shared__ C fxs[4][TY * (TX + 1)];
  __shared__ C fys[4][FYR * TX];
  __shared__ unsigned int blk_fallback, blk_fault;
  static_assert(NET == NET_NONE || (NDIM == 2 && !VISC), "learned correction: 2D inviscid tiles");
  constexpr bool MLP = NET == NET_MLP;
  constexpr bool GH = IBM && NDIM == 2;
  __shared__ __attribute__((aligned(16))) unsigned short net_w[MLP ? NET_LNW : 1];
  __shared__ float net_b[MLP ? NET_NB : 1];
  // normalised network inputs of every halo cell, bfloat16, in the x-face
  // frame (rho, u, v, p) and the y-face frame (rho, v, u, p): each cell feeds
  // twelve faces, so it is converted once here
  __shared__ bf16x4 net_in[MLP ? 2 : 1][MLP ? PY * PX : 1];
  __shared__ double red_s[NT / 64], red_r[NT / 64];
  // immersed boundary: the halo slots whose source is a ghost cell, with
  // its ghost index, refilled together after the plain loads
  __shared__ int gl_slot[GH ? PY * PX : 1], gl_idx[GH ? PY * PX : 1];
  __shared__ unsigned int gl_n;

  int bx, by, b;
  bool near_body = true;
  if (GH && TX == STAGE_TX && TY == STAGE_TY && a.tile_order != nullptr) {
    // grid with a body: the tiles near it first (host-built order); the
    // entry's top bit is the tile's body flag, so one load gives both
    const unsigned e = a.tile_order[blockIdx.x + gridDim.x * blockIdx.y];
    const int t = int(e & 0x7fffffffu);
    near_body = (e >> 31) != 0;
    bx = t % gridDim.x;
    by = t / gridDim.x;
    b = blockIdx.z;
  } else {
    xcd_tile(bx, by, b);
  }
  StepScalars* sc = a.sc + b;
  const bool lead = bx == 0 && by == 0 && threadIdx.x == 0;
  double dt = 0.0;
  if (MODE == MODE_STAGE1 || MODE == MODE_STAGE2 || MODE == MODE_STAGE3) {
    dt = dtp[b];
    if (dt == 0.0) return;  // end time reached: the step is a no-op
  } else if (MODE == MODE_S1L) {
    if (sc->done) return;
  } else if (MODE == MODE_S2F) {
    bool last;
    double sm, rm;
    read_extrema(a, b, &sm, &rm);
    dt = step_dt(a, sc, sm, rm, &last);
    if (lead) {
      a.dtbuf[b] = dt;
      if (a.dt_out) a.dt_out[b] = dt;
    }
    if (dt == 0.0) return;
  } else if (MODE == MODE_S3F) {
    dt = a.dtbuf[b];
    if (bx == 0 && by == 0) {
      // block 0 advances the device time and clears the extrema
      double sm, rm;
      read_extrema(a, b, &sm, &rm);
      __syncthreads();
      if (threadIdx.x == 0) {
        bool last;
        const double d2 = step_dt(a, sc, sm, rm, &last);
        if (d2 > 0.0) {
          sc->t = last ? sc->t_end : sc->t + d2;
          sc->nsteps = sc->nsteps + 1;
          if (last) sc->done = 1;
        }
        sc->dt = d2;
      }
      if (threadIdx.x < XSLOTS) {
        unsigned long long* xs = a.xslots + (long long)b * 2 * XSLOTS;
        xs[threadIdx.x] = 0ull;
        xs[XSLOTS + threadIdx.x] = (unsigned long long)__double_as_longlong(INFINITY);
      }
    }
    if (dt == 0.0) return;
  }
  if (threadIdx.x == 0) { blk_fallback = 0; blk_fault = 0; }
  const int i0 = bx * TX;
  const int j0 = by * TY;
  // immersed boundary: a tile whose cells and halo sources are all fluid
  // (the same for the whole workgroup) takes the plain path, reading no
  // cell classes
  const bool body = GH && a.cls != nullptr && near_body;
  const long long boff = (long long)b * a.nvar * a.ncell;
  const S* Ub = Us + boff;
  const S* __restrict__ Lb = MODE == MODE_S2F ? Lin + boff : nullptr;
  const C gm1 = C(a.gamma - 1.0);
  const C cdt = C(dt);
  // stage-1 state formed on the fly (fused sequence), rounded to storage and
  // evaluated like the stored stage-1 state of the three-stage path
  auto u1_at = [&](int e, long long c) {
#pragma clang fp contract(off)
    return C(S(C(Ub[e * a.ncell + c]) + cdt * C(Lb[e * a.ncell + c])));
  };

  if (MLP) load_net_lds(net, net_w, net_b);

  // 1. halo tile of primitives; a tile whose halo lies inside the domain
  // (the same for the whole workgroup) skips the boundary rules
  const bool inside = i0 >= H && i0 + TX + H <= a.nx && (NDIM == 1 || (j0 >= H && j0 + TY + H <= a.ny));
  bool nonphys = false;  // a loaded cell with rho <= 0 or p <= 0 (or not a number)
  // primitives of halo slot k into the tile (and the network's inputs)
  auto put = [&](int k, const C q[4]) {
    Prim<C> p = to_prim(q[0], q[1], q[2], q[3], gm1);
    nonphys = nonphys || !(p.r > C(0)) || !(p.p > C(0));
    w[0][k] = p.r;
    w[1][k] = p.un;
    w[2][k] = p.ut;
    w[3][k] = p.p;
    if (MLP) {
      const double pv[4] = {double(p.r), double(p.un), double(p.ut), double(p.p)};
      float xn[4], yn[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int vy = v == 1 ? 2 : (v == 2 ? 1 : v);  // y-face frame
        xn[v] = float((pv[v] - net.mean[v]) * net.inv_std[v]);
        yn[v] = float((pv[vy] - net.mean[v]) * net.inv_std[v]);
      }
      net_in[0][k] = pack4(xn[0], xn[1], xn[2], xn[3]);
      net_in[1][k] = pack4(yn[0], yn[1], yn[2], yn[3]);
    }
  };
  if (GH && body) {
    if (threadIdx.x == 0) gl_n = 0;
    __syncthreads();
  }
  for (int k = threadIdx.x; k < PY * PX; k += NT) {
    const int lx = k % PX, ly = k / PX;
    const bool inx = lx >= H && lx < TX + H;
    const bool iny = NDIM == 1 || (ly >= H && ly < TY + H);
    if (!VISC && !inx && !iny) continue;  // corner block: read only by viscous stencils
    const int gi = i0 + lx - H;
    const int gj = NDIM == 2 ? j0 + ly - H : 0;
    C q[4];
    int gk = -1;
    if (MODE == MODE_S2F) {
      if (body)
        load_cons_f<S, C, NDIM, GH, true>(a, gi, gj, u1_at, q, inside, &gk);
      else
        load_cons_f<S, C, NDIM, false>(a, gi, gj, u1_at, q, inside);
    } else {
      if (body)
        load_cons<S, C, NDIM, GH, true>(a, Ub, gi, gj, q, inside, &gk);
      else
        load_cons<S, C, NDIM, false>(a, Ub, gi, gj, q, inside);
    }
    if (GH && gk >= 0) {
      // a ghost cell's source: listed, and refilled in the pass below
      const unsigned int at = atomicAdd(&gl_n, 1u);
      gl_slot[at] = k;
      gl_idx[at] = gk;
      continue;
    }
    put(k, q);
  }
  if (GH && body) {
    // 1b. the listed ghost slots, all at once: each takes its ghost's
    // refilled value (from the stage state's fluid cells, complete when the
    // stage starts) and the boundary rule of its halo position
    __syncthreads();
    const int n = int(gl_n);
    for (int t = threadIdx.x; t < n; t += NT) {
      const int k = gl_slot[t];
      const int gi = i0 + k % PX - H, gj = j0 + k / PX - H;
      int fx = 0, fy = 0;
      if (!inside) {
        bc_source(gi, a.nx, a.bc[0], a.bc[1], fx);
        bc_source(gj, a.ny, a.bc[2], a.bc[3], fy);
      }
      C q[4];
      if (MODE == MODE_S2F)
        ghost_at<S>(a, gl_idx[t], u1_at, q);
      else
        ghost_at<S>(a, gl_idx[t], [&](int e, long long c) { return C(Ub[e * a.ncell + c]); }, q);
      const int lx = k % PX, ly = k / PX;
      if (MODE != MODE_S2F && a.ghost_back != nullptr && lx >= H && lx < TX + H && ly >= H && ly < TY + H &&
          gi < a.nx && gj < a.ny) {
        // a ghost cell of this tile (no boundary rule): its refilled value
        // is stored here; where that is the stage state, the update below
        // reads it back instead of forming it again
        const long long cell = (long long)gj * a.nx + gi;
#pragma unroll
        for (int v = 0; v < 4; ++v) static_cast<S*>(a.ghost_back)[boff + v * a.ncell + cell] = S(q[v]);
      }
      q[1] = (fx & 1) ? -q[1] : q[1];
      q[2] = (fy & 1) ? -q[2] : q[2];
      put(k, q);
    }
  }
  __syncthreads();

  // face k of the tile -> first stencil cell, stride, normal/tangential
  // velocity arrays and the index of its flux slot
  auto face_of = [&](int k, int& s0, int& st, int& cn, int& ct, int& oidx) {
    if (k < NFX) {
      const int fi = k % (TX + 1), y = k / (TX + 1);
      s0 = (NDIM == 2 ? (y + H) * PX : 0) + fi;
      st = 1; cn = 1; ct = 2;
      oidx = y * (TX + 1) + fi;
    } else {
      const int kk = k - NFX;
      const int x = kk % TX, fj = kk / TX;
      s0 = fj * PX + x + H;
      st = PX; cn = 2; ct = 1;
      oidx = fj * TX + x;
    }
  };

  if (MLP) {
    // 1b. learned correction of every face of the tile on the matrix cores,
    // 32 faces per wave and batch (the tile's 552 faces split evenly over
    // the four waves); the network output before its tanh is parked in the
    // flux arrays (face frame), and the face pass, one face per thread,
    // finishes it and adds it to the flux
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NF = NFX + NFY;
    constexpr int FT = 2;
    for (int bb = wv; bb * 16 * FT < NF; bb += NT / 64) {
      ActsT<FT> A;
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) {
        int k = bb * 16 * FT + ft * 16 + (lane & 15);
        if (k >= NF) k = NF - 1;
        int s0, st, cn, ct, oidx;
        face_of(k, s0, st, cn, ct, oidx);
        // B operand: lane (q, face) takes stencil cell q (k-tile 0) and 4 + q
        // (k-tile 1, q < 2), already normalised in this face's frame
        const int q = lane >> 4, fr = k < NFX ? 0 : 1;
        A.x[0][ft] = net_in[fr][s0 + q * st];
        A.x[1][ft] = q < 2 ? net_in[fr][s0 + (4 + q) * st] : bf16x4{0, 0, 0, 0};
      }
      f32x4 z[FT];
      net_forward_batch<FT>(net_w, net_b, lane, A, z);
      if ((lane >> 4) == 0) {
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) {
          const int k = bb * 16 * FT + ft * 16 + (lane & 15);
          if (k >= NF) continue;
          int s0, st, cn, ct, oidx;
          face_of(k, s0, st, cn, ct, oidx);
          if (k < NFX) {
#pragma unroll
            for (int i = 0; i < 4; ++i) fxs[i][oidx] = C(z[ft][i]);
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) fys[i][oidx] = C(z[ft][i]);
          }
        }
      }
    }
    __syncthreads();
  }

  // 2. face fluxes
  const C eps = C(a.eps);
  const C gam = C(a.gamma);
  const C igm1 = C(1.0 / (a.gamma - 1.0));
  unsigned int my_fallback = 0;
  bool net_bad = false;
  // Everything after the reconstruction for the face whose stencil starts at
  // LDS cell s0 (stride st; cn, ct: normal and tangential velocity arrays):
  // position fi along the normal and line (row of an x-face, column of a
  // y-face) in the tile; L, R its reconstructed states.
  auto face_flux = [&](bool isx, int s0, int st, int cn, int ct, int fi, int line, Prim<C> L, Prim<C> R) {
    int oidx;
    bool owned;  // this tile is the one that reports the face (fallback count)
    long long gface = -1;  // NET_EXT: the face's index, -1 outside the domain
    if (isx) {
      oidx = line * (TX + 1) + fi;
      const int gf = i0 + fi;
      owned = j0 + line < a.ny && gf <= a.nx && (fi < TX || gf == a.nx);
      if (NET == NET_EXT && j0 + line < a.ny && gf <= a.nx) gface = (long long)(j0 + line) * (a.nx + 1) + gf;
    } else {
      oidx = fi * TX + line;
      const int gf = j0 + fi;
      owned = i0 + line < a.nx && gf <= a.ny && (fi < TY || gf == a.ny);
      if (NET == NET_EXT && i0 + line < a.nx && gf <= a.ny)
        gface = (long long)(a.nx + 1) * a.ny + (long long)gf * a.nx + i0 + line;
    }
    if (!(L.r > C(0)) || !(L.p > C(0)) || !(R.r > C(0)) || !(R.p > C(0))) {
      // positivity fallback: first-order states from the two adjacent cells
      const int ia = s0 + 2 * st, ib = s0 + 3 * st;
      L = Prim<C>{w[0][ia], w[cn][ia], w[ct][ia], w[3][ia]};
      R = Prim<C>{w[0][ib], w[cn][ib], w[ct][ib], w[3][ib]};
      if (owned) ++my_fallback;
    }
    Flux4<C> F = hllc(L, R, gam, igm1);
    if (VISC) {
      // derivatives as products with the reciprocal spacings, the
      // temperature T = p / rho by the fast quotient (no IEEE division)
      const int ia = s0 + 2 * st, ib = s0 + 3 * st;
      const int tt = isx ? PX : 1;  // tangential LDS stride
      const C idn = C(isx ? a.inv_dx : a.inv_dy), idt4 = C(0.25 * (isx ? a.inv_dy : a.inv_dx));
      const C mu = C(a.mu), kap = C(a.kappa);
      const C un_n = (w[cn][ib] - w[cn][ia]) * idn;
      const C ut_n = (w[ct][ib] - w[ct][ia]) * idn;
      const C T_n = (qdiv(w[3][ib], w[0][ib]) - qdiv(w[3][ia], w[0][ia])) * idn;
      const C un_t = (w[cn][ia + tt] - w[cn][ia - tt] + w[cn][ib + tt] - w[cn][ib - tt]) * idt4;
      const C ut_t = (w[ct][ia + tt] - w[ct][ia - tt] + w[ct][ib + tt] - w[ct][ib - tt]) * idt4;
      const C tnn = mu * (C(4.0 / 3.0) * un_n - C(2.0 / 3.0) * ut_t);
      const C tnt = mu * (un_t + ut_n);
      const C qn = -kap * T_n;
      const C ubn = C(0.5) * (w[cn][ia] + w[cn][ib]);
      const C ubt = C(0.5) * (w[ct][ia] + w[ct][ib]);
      F.f1 = F.f1 - tnn;
      F.f2 = F.f2 - tnt;
      F.f3 = F.f3 - (ubn * tnn + ubt * tnt - qn);
    }
    if (NET == NET_EXT && gface >= 0) {
      const float* d = a.dFext + ((long long)b * a.nface + gface) * 4;
      F.f0 = F.f0 + C(d[0]);
      F.f1 = F.f1 + C(d[1]);
      F.f2 = F.f2 + C(d[2]);
      F.f3 = F.f3 + C(d[3]);
    }
    if (MLP) {
      // learned correction of this face (face frame): out_scale tanh of the
      // network output parked by pass 1b; a non-finite value leaves the
      // uncorrected flux and is flagged
      float o[4];
      bool ok = true;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = float(isx ? fxs[i][oidx] : fys[i][oidx]);
        o[i] = net.out_scale * tanhf(z);
        ok = ok && isfinite(o[i]);
      }
      if (!ok) {
        o[0] = o[1] = o[2] = o[3] = 0.f;
        if (owned) net_bad = true;
      }
      F.f0 = F.f0 + C(o[0]);
      F.f1 = F.f1 + C(o[1]);
      F.f2 = F.f2 + C(o[2]);
      F.f3 = F.f3 + C(o[3]);
    }
    if (isx) {
      fxs[0][oidx] = F.f0; fxs[1][oidx] = F.f1; fxs[2][oidx] = F.f2; fxs[3][oidx] = F.f3;
    } else {
      fys[0][oidx] = F.f0; fys[1][oidx] = F.f2; fys[2][oidx] = F.f1; fys[3][oidx] = F.f3;
    }
  };
  // One face per thread, k = x-faces first, then y-faces.  DIR 1 (x-faces)
  // and 2 (y-faces) fix the LDS stride and the velocity planes at compile
  // time, so the stencil reads take immediate offsets; DIR 0 decides per
  // lane.
  auto face_task = [&](int k, auto dirc) {
    constexpr int DIR = decltype(dirc)::value;
    const bool isx = DIR == 1 ? true : (DIR == 2 ? false : k < NFX);
    int s0, fi, line;
    if (isx) {
      fi = k % (TX + 1);
      line = k / (TX + 1);
      s0 = (NDIM == 2 ? (line + H) * PX : 0) + fi;
    } else {
      const int kk = k - NFX;
      line = kk % TX;
      fi = kk / TX;
      s0 = fi * PX + line + H;
    }
    const int st = isx ? 1 : PX;
    const int cn = isx ? 1 : 2, ct = isx ? 2 : 1;
    Prim<C> L, R;
    if constexpr (CHAR) {
      static_assert(sizeof(C) == 8, "characteristic reconstruction: FP64 tiles");
      char_face_states(w[0] + s0, w[cn] + s0, w[ct] + s0, w[3] + s0, st, a.eps, a.gamma, L, R);
    } else {
      {
        const C* f = w[0] + s0;
        weno5_pair(f[0], f[st], f[2 * st], f[3 * st], f[4 * st], f[5 * st], eps, L.r, R.r);
      }
      {
        const C* f = w[cn] + s0;
        weno5_pair(f[0], f[st], f[2 * st], f[3 * st], f[4 * st], f[5 * st], eps, L.un, R.un);
      }
      {
        const C* f = w[ct] + s0;
        weno5_pair(f[0], f[st], f[2 * st], f[3 * st], f[4 * st], f[5 * st], eps, L.ut, R.ut);
      }
      {
        const C* f = w[3] + s0;
        weno5_pair(f[0], f[st], f[2 * st], f[3 * st], f[4 * st], f[5 * st], eps, L.p, R.p);
      }
    }
    face_flux(isx, s0, st, cn, ct, fi, line, L, R);
  };
  if constexpr (NDIM == 2 && !CHAR && sizeof(C) == 4) {
    // FP32 arithmetic: three consecutive faces per thread along a row
    // (x-faces) or a column (y-faces), sharing indicator sets and curvature
    // terms (weno5_run); TX + 1 and TY + 1 are multiples of 3, so the tile's
    // faces split into NTX + NTY triples, one round of the workgroup.  Lanes
    // of a y-triple wave take neighbouring columns (consecutive LDS words).
    // DIR as for face_task, per wave.  FP64 tiles take one face per thread:
    // runs of three faces hold 24 face values through three flux evaluations
    // (about 165 registers), and even pairs (144 registers, three resident
    // waves per SIMD instead of four) were 4-6 % slower than single faces on
    // 512^2 and 4096 x 2048 grids; forced into 128 registers they spill.
    static_assert((TX + 1) % 3 == 0 && (TY + 1) % 3 == 0, "face triples need TX + 1 and TY + 1 divisible by 3");
    constexpr int TPR = (TX + 1) / 3;  // triples per row of x-faces
    constexpr int NTX = TPR * TY, NTY = (TY + 1) / 3 * TX;
    static_assert(NTX + NTY <= NT, "one round of face triples");
    auto triple_task = [&](int t, auto dirc) {
      constexpr int DIR = decltype(dirc)::value;
      const bool isx = DIR == 1 ? true : (DIR == 2 ? false : t < NTX);
      int s0, fa, line;
      if (isx) {
        line = t / TPR;
        fa = 3 * (t - line * TPR);
        s0 = (line + H) * PX + fa;
      } else {
        const int u = t - NTX;
        fa = 3 * (u / TX);
        line = u - (fa / 3) * TX;
        s0 = fa * PX + line + H;
      }
      const int st = isx ? 1 : PX;
      const int cn = isx ? 1 : 2, ct = isx ? 2 : 1;
      C lr[3], rr[3], lu[3], ru[3], lt[3], rt[3], lp[3], rp[3];
      weno5_run<3>(w[0] + s0, st, eps, lr, rr);
      weno5_run<3>(w[cn] + s0, st, eps, lu, ru);
      weno5_run<3>(w[ct] + s0, st, eps, lt, rt);
      weno5_run<3>(w[3] + s0, st, eps, lp, rp);
#pragma unroll
      for (int q = 0; q < 3; ++q)
        face_flux(isx, s0 + q * st, st, cn, ct, fa + q, line, Prim<C>{lr[q], lu[q], lt[q], lp[q]},
                  Prim<C>{rr[q], ru[q], rt[q], rp[q]});
    };
    const int t = threadIdx.x;
    if (t < NTX + NTY) {
      const int tw = t - (t & 63);  // first thread of this wave (wave-uniform)
      const int tl = min(tw + 63, NTX + NTY - 1);
      if (tl < NTX)
        triple_task(t, IntC<1>{});
      else if (tw >= NTX)
        triple_task(t, IntC<2>{});
      else
        triple_task(t, IntC<0>{});
    }
  } else {
    // A wave takes DIR 1 or 2 when all its faces lie in one direction, else
    // DIR 0 (at most one wave of a round straddles the x/y boundary).
    for (int k = threadIdx.x; k < NFX + NFY; k += NT) {
      const int kw = k - (threadIdx.x & 63);  // first face of this wave's block (wave-uniform)
      const int kl = min(kw + 63, NFX + NFY - 1);
      if (kl < NFX)
        face_task(k, IntC<1>{});
      else if (kw >= NFX)
        face_task(k, IntC<2>{});
      else
        face_task(k, IntC<0>{});
    }
  }
  if (my_fallback) atomicAdd(&blk_fallback, my_fallback);
  if (MLP && net_bad) atomicOr(&blk_fault, 8u);
  __syncthreads();

  // 3. flux difference and Runge-Kutta combination
  const C idx = C(a.inv_dx), idy = C(a.inv_dy);
  const S* Unb = Un + boff;
  S* Ob = Uout + boff;
  bool bad = false;
  double smax = 0.0, rmin = INFINITY;
  constexpr int NV = NDIM == 2 ? 4 : 3;  // stored planes
  for (int k = threadIdx.x; k < TX * TY; k += NT) {
    // Flux difference and stage combination are evaluated as written (no
    // fused multiply-add), so the fused and the three-stage sequences agree
    // bit for bit and the association is the oracle's.
#pragma clang fp contract(off)
    const int x = k % TX, y = k / TX;
    const int gi = i0 + x, gj = j0 + y;
    if (gi >= a.nx || gj >= a.ny) continue;
    const long long cell = (long long)gj * a.nx + gi;
    // the class (solid cells keep a zero right-hand side) and the ghost index
    // are independent loads, issued together
    const uint8_t cc = GH && body ? a.cls[cell] : CELL_FLUID;
    const int gk = GH && body ? a.ghost_of[cell] : -1;
    // the cell's stage-state and U^n values, all read before any write (the
    // output may overwrite U^n); a ghost cell takes its refilled stage value:
    // the one the ghost pass stored, where it stored it in the stage state,
    // else formed again (its stored one is loaded anyway, beside the ghost
    // index, and replaced)
    C us[4], un[4];
    if (MODE != MODE_RHS && MODE != MODE_S1L) {
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        const int v = (NDIM == 1 && e == 2) ? 3 : e;
        us[v] = MODE == MODE_S2F ? u1_at(e, cell) : C(Ub[e * a.ncell + cell]);
      }
      if (GH && gk >= 0) {
        if (MODE == MODE_S2F)
          ghost_at<S>(a, gk, u1_at, us);
        else if (a.ghost_back != static_cast<const void*>(Us))
          ghost_at<S>(a, gk, [&](int e, long long c) { return C(Ub[e * a.ncell + c]); }, us);
      }
    }
    if (MODE == MODE_STAGE2 || MODE == MODE_STAGE3 || MODE == MODE_S3F || MODE == MODE_S2F) {
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        const int v = (NDIM == 1 && e == 2) ? 3 : e;
        // S2F: U^n is the stage input itself (U1 is formed on the fly)
        un[v] = C(MODE == MODE_S2F ? Ub[e * a.ncell + cell] : Unb[e * a.ncell + cell]);
      }
    }
    C Lv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      C r = -(fxs[v][y * (TX + 1) + x + 1] - fxs[v][y * (TX + 1) + x]) * idx;
      if (NDIM == 2) r = r - (fys[v][(y + 1) * TX + x] - fys[v][y * TX + x]) * idy;
      Lv[v] = r;
    }
    if (a.nu_art != 0.0) {
      C c0[4], xm[4], xp[4];
      if (MODE == MODE_S2F) {
        load_cons_f<S, C, NDIM, GH>(a, gi, gj, u1_at, c0);
        load_cons_f<S, C, NDIM, GH>(a, gi - 1, gj, u1_at, xm);
        load_cons_f<S, C, NDIM, GH>(a, gi + 1, gj, u1_at, xp);
      } else {
        load_cons<S, C, NDIM, GH>(a, Ub, gi, gj, c0);
        load_cons<S, C, NDIM, GH>(a, Ub, gi - 1, gj, xm);
        load_cons<S, C, NDIM, GH>(a, Ub, gi + 1, gj, xp);
      }
      const C nu = C(a.nu_art);
      C ym[4], yp[4];
      if (NDIM == 2) {
        if (MODE == MODE_S2F) {
          load_cons_f<S, C, NDIM, GH>(a, gi, gj - 1, u1_at, ym);
          load_cons_f<S, C, NDIM, GH>(a, gi, gj + 1, u1_at, yp);
        } else {
          load_cons<S, C, NDIM, GH>(a, Ub, gi, gj - 1, ym);
          load_cons<S, C, NDIM, GH>(a, Ub, gi, gj + 1, yp);
        }
      }
      for (int v = 0; v < 4; ++v) {
        C lap = (xp[v] - C(2) * c0[v] + xm[v]) * (idx * idx);
        if (NDIM == 2) lap = lap + (yp[v] - C(2) * c0[v] + ym[v]) * (idy * idy);
        Lv[v] = Lv[v] + nu * lap;
      }
    }
    if (cc != CELL_FLUID) {
#pragma unroll
      for (int v = 0; v < 4; ++v) Lv[v] = C(0);
    }
    if (MODE == MODE_S1L && cc == CELL_FLUID) {
      double r;
      smax = fmax(smax, wave_speed_sum(a, Ub, cell, &r));
      rmin = fmin(rmin, r);
    }
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int v = (NDIM == 1 && e == 2) ? 3 : e;
      const long long o = (long long)e * a.ncell + cell;
      C out;
      if (MODE == MODE_RHS || MODE == MODE_S1L) {
        out = Lv[v];
      } else if (MODE == MODE_STAGE1) {
        // the reverse pass keeps the (refilled) stage input: copied here
        // from the value this thread holds anyway
        if (a.stage_in_copy != nullptr) static_cast<S*>(a.stage_in_copy)[boff + o] = S(us[v]);
        out = us[v] + cdt * Lv[v];
      } else if (MODE == MODE_STAGE2 || MODE == MODE_S2F) {
        out = C(0.75) * un[v] + C(0.25) * us[v] + C(0.25 * dt) * Lv[v];
      } else {
        out = C(1.0 / 3.0) * un[v] + C(2.0 / 3.0) * us[v] + C((2.0 / 3.0) * dt) * Lv[v];
      }
      bad = bad || !finite_val(out);
      Ob[o] = S(out);
    }
  }
  if (MODE == MODE_S1L) {
    smax = wave_max(smax);
    rmin = wave_min(rmin);
    if ((threadIdx.x & 63) == 0) { red_s[threadIdx.x >> 6] = smax; red_r[threadIdx.x >> 6] = rmin; }
  }
  if (bad) atomicOr(&blk_fault, 1u);
  if (nonphys) atomicOr(&blk_fault, 4u);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (MODE == MODE_S1L) {
      double s2 = red_s[0], r2 = red_r[0];
      for (int k = 1; k < NT / 64; ++k) { s2 = fmax(s2, red_s[k]); r2 = fmin(r2, red_r[k]); }
      unsigned long long* xs = a.xslots + (long long)b * 2 * XSLOTS;
      const int slot = (bx + by * gridDim.x) & (XSLOTS - 1);
      atomicMax(&xs[slot], (unsigned long long)__double_as_longlong(s2));
      atomicMin(&xs[XSLOTS + slot], (unsigned long long)__double_as_longlong(r2));
    }
    if (blk_fallback) {
      atomicAdd(&a.glob->fallbacks, (unsigned long long)blk_fallback);
      atomicOr(&a.glob->fault, 2u);
    }
    if (blk_fault) atomicOr(&a.glob->fault, blk_fault);
  }
}

// ------------------------------------------------- immersed-boundary tiles
// Flag of one 2D stage tile: 1 if any cell of the tile or any source cell
// its halo loads (the tile and three layers around it, corners included,
// mapped by the boundary rules) is not fluid.  One workgroup per tile.
__global__ void __launch_bounds__(256) tile_body_kernel(GridArgs a, uint8_t* __restrict__ flags) {
  constexpr int PX = STAGE_TX + 2 * HALO, PY = STAGE_TY + 2 * HALO;
  const int i0 = blockIdx.x * STAGE_TX, j0 = blockIdx.y * STAGE_TY;
  int any = 0;
  for (int k = threadIdx.x; k < PX * PY; k += blockDim.x) {
    int fx = 0, fy = 0;
    const int si = bc_source(i0 - HALO + k % PX, a.nx, a.bc[0], a.bc[1], fx);
    const int sj = bc_source(j0 - HALO + k / PX, a.ny, a.bc[2], a.bc[3], fy);
    if (a.cls[(long long)sj * a.nx + si] != CELL_FLUID) any = 1;
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) flags[blockIdx.y * gridDim.x + blockIdx.x] = any ? 1 : 0;
}

hipError_t launch_tile_body(const GridArgs& a, uint8_t* flags, hipStream_t st) {
  if (a.ndim != 2 || a.cls == nullptr) return hipErrorInvalidValue;
  const dim3 grid((a.nx + STAGE_TX - 1) / STAGE_TX, (a.ny + STAGE_TY - 1) / STAGE_TY);
  hipLaunchKernelGGL(tile_body_kernel, grid, dim3(256), 0, st, a, flags);
  return hipGetLastError();
}

// ------------------------------------------------------------ CFL kernel

// Max over fluid cells of (|u|+a)/dx + (|v|+a)/dy and min density, reduced
// exactly (max/min are order-free; the double bit patterns of non-negative
// values order like unsigned integers), then the last block turns it into
// the step: dt = cfl / max, the explicit viscous limit, and the shortening
// that lands on t_end.  Arithmetic follows the written order without
// contraction so the step is reproducible bit for bit.
template <class S>
__global__ void __launch_bounds__(256) cfl_kernel(GridArgs a, const S* __restrict__ U,
                                                  double* __restrict__ dt_out) {
  __shared__ double red_s[4], red_r[4];
  __shared__ bool is_last;
  const int b = blockIdx.y;
  const S* Ub = U + (long long)b * a.nvar * a.ncell;
  double smax = 0.0, rmin = INFINITY;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    if (a.cls != nullptr && a.cls[c] != CELL_FLUID) continue;
    double r;
    smax = fmax(smax, wave_speed_sum(a, Ub, c, &r));
    rmin = fmin(rmin, r);
  }
  smax = wave_max(smax);
  rmin = wave_min(rmin);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { red_s[wid] = smax; red_r[wid] = rmin; }
  __syncthreads();
  StepScalars* sc = a.sc + b;
  if (threadIdx.x == 0) {
    double s = red_s[0], r = red_r[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) { s = fmax(s, red_s[k]); r = fmin(r, red_r[k]); }
    atomicMax(&sc->smax_bits, (unsigned long long)__double_as_longlong(s));
    atomicMin(&sc->rmin_bits, (unsigned long long)__double_as_longlong(r));
    __threadfence();
    unsigned int prev = atomicAdd(&sc->blocks_done, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (is_last && threadIdx.x == 0) {
    __threadfence();
    const double sm = bits_to_double(atomicAdd(&sc->smax_bits, 0ull));
    const double rm = bits_to_double(atomicAdd(&sc->rmin_bits, 0ull));
    bool last;
    const double dt = step_dt(a, sc, sm, rm, &last);
    if (dt > 0.0) {
      sc->t = last ? sc->t_end : sc->t + dt;
      sc->nsteps = sc->nsteps + 1;
      if (last) sc->done = 1;
    }
    sc->dt = dt;
    a.dtbuf[b] = dt;
    if (dt_out) dt_out[b] = dt;
    atomicExch(&sc->smax_bits, 0ull);
    atomicExch(&sc->rmin_bits, (unsigned long long)__double_as_longlong(INFINITY));
    atomicExch(&sc->blocks_done, 0u);
  }
}

__global__ void init_scalars_kernel(GridArgs a, double t0, double t_end) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < a.nbatch) {
    StepScalars* sc = a.sc + b;
    sc->dt = 0.0;
    sc->t = t0;
    sc->t_end = t_end;
    sc->smax_bits = 0ull;
    sc->rmin_bits = (unsigned long long)__double_as_longlong(INFINITY);
    sc->done = t0 >= t_end ? 1 : 0;
    sc->blocks_done = 0u;
    sc->nsteps = 0;
    a.dtbuf[b] = 0.0;
    unsigned long long* xs = a.xslots + (long long)b * 2 * XSLOTS;
    for (int k = 0; k < XSLOTS; ++k) {
      xs[k] = 0ull;
      xs[XSLOTS + k] = (unsigned long long)__double_as_longlong(INFINITY);
    }
  }
  if (b == 0) {
    a.glob->fault = 0u;
    a.glob->fallbacks = 0ull;
  }
}

// E = p/(gamma-1) + rho (u^2+v^2)/2 as written (no contraction), so that a
// state built here is bit-identical to one built by any IEEE evaluation of
// the same expression.
template <class S>
__global__ void __launch_bounds__(256) prim_to_cons_kernel(GridArgs a, const S* __restrict__ W,
                                                           S* __restrict__ U) {
#pragma clang fp contract(off)
  const long long n = a.ncell;
  const long long total = n * a.nbatch;
  const double igm = a.gamma - 1.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (long long)gridDim.x * blockDim.x) {
    const long long b = k / n, c = k - b * n;
    const S* Wb = W + b * a.nvar * n;
    S* Ub = U + b * a.nvar * n;
    double r = double(Wb[c]), u = double(Wb[n + c]);
    double v = a.ndim == 2 ? double(Wb[2 * n + c]) : 0.0;
    double p = double(Wb[(a.nvar - 1) * n + c]);
    double E = p / igm + 0.5 * r * (u * u + v * v);
    Ub[c] = S(r);
    Ub[n + c] = S(r * u);
    if (a.ndim == 2) Ub[2 * n + c] = S(r * v);
    Ub[(a.nvar - 1) * n + c] = S(E);
  }
}

// Reverse mode of prim_to_cons_kernel (FP64 states): per cell, with U = (rho,
// rho u, rho v, E), E = p/(gamma-1) + rho (u^2 + v^2)/2,
//   W_bar += (dU/dW)^T U_bar:  rho: Ub0 + u Ub1 + v Ub2 + (u^2+v^2)/2 Ub3,
//   u: rho (Ub1 + u Ub3), v: rho (Ub2 + v Ub3), p: Ub3/(gamma-1);
// and the block partial of dU/dgamma . U_bar = -p/(gamma-1)^2 Ub3 summed over
// the block's cells (a fixed order: each thread's cells, then a fixed tree).
__global__ void __launch_bounds__(256) prim_to_cons_vjp_kernel(GridArgs a, const double* __restrict__ W,
                                                               const double* __restrict__ Ubar,
                                                               double* __restrict__ Wbar,
                                                               double* __restrict__ part) {
  __shared__ double red[4];
  const long long n = a.ncell;
  const int b = blockIdx.y;
  const double* Wb = W + (long long)b * a.nvar * n;
  const double* Ub = Ubar + (long long)b * a.nvar * n;
  double* Wo = Wbar ? Wbar + (long long)b * a.nvar * n : nullptr;
  const double gm1 = a.gamma - 1.0, igm = 1.0 / gm1;
  const int pv = a.nvar - 1;  // pressure / energy plane
  double s = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const double r = Wb[c], u = Wb[n + c], v = a.ndim == 2 ? Wb[2 * n + c] : 0.0, p = Wb[pv * n + c];
    const double u0 = Ub[c], u1 = Ub[n + c], u2 = a.ndim == 2 ? Ub[2 * n + c] : 0.0, u3 = Ub[pv * n + c];
    if (Wo) {
      Wo[c] += u0 + u * u1 + v * u2 + 0.5 * (u * u + v * v) * u3;
      Wo[n + c] += r * (u1 + u * u3);
      if (a.ndim == 2) Wo[2 * n + c] += r * (u2 + v * u3);
      Wo[pv * n + c] += u3 * igm;
    }
    s += -p * igm * igm * u3;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// param_bar[b][0] += the block partials of member b in block order.
__global__ void vjp_gamma_finalize_kernel(const double* __restrict__ part, int nblk, int nbatch,
                                          double* __restrict__ param_bar) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbatch) return;
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += part[(long long)b * nblk + k];
  param_bar[(long long)b * 5] += s;
}

// --------------------------------------------------------------- launchers
static inline unsigned int blocks_for(long long n, int per) {
  long long b = (n + per - 1) / per;
  if (b > 65535LL * 16) b = 65535LL * 16;
  return (unsigned int)(b < 1 ? 1 : b);
}

template <class S>
hipError_t launch_prim_to_cons(const GridArgs& a, const S* W, S* U, hipStream_t st) {
  hipLaunchKernelGGL(prim_to_cons_kernel<S>, dim3(blocks_for(a.ncell * a.nbatch, 256)), dim3(256), 0, st,
                     a, W, U);
  return hipGetLastError();
}

hipError_t launch_prim_to_cons_vjp(const GridArgs& a, const double* W, const double* Ubar, double* Wbar,
                                   double* param_bar, double* part, hipStream_t st) {
  unsigned int nb = blocks_for(a.ncell, 256 * 4);
  if (nb > VJP_BLOCKS) nb = VJP_BLOCKS;
  hipLaunchKernelGGL(prim_to_cons_vjp_kernel, dim3(nb, a.nbatch), dim3(256), 0, st, a, W, Ubar, Wbar, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !param_bar) return e;
  hipLaunchKernelGGL(vjp_gamma_finalize_kernel, dim3((a.nbatch + 63) / 64), dim3(64), 0, st, part, (int)nb,
                     a.nbatch, param_bar);
  return hipGetLastError();
}

template <class S>
hipError_t launch_cfl(const GridArgs& a, const S* U, double* dt_out, hipStream_t st) {
  // enough blocks to cover the chip, each thread then strides
  unsigned int nb = blocks_for(a.ncell, 256 * 4);
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(cfl_kernel<S>, dim3(nb, a.nbatch), dim3(256), 0, st, a, U, dt_out);
  return hipGetLastError();
}

hipError_t launch_init_scalars(const GridArgs& a, double t0, double t_end, hipStream_t st) {
  hipLaunchKernelGGL(init_scalars_kernel, dim3((a.nbatch + 63) / 64), dim3(64), 0, st, a, t0, t_end);
  return hipGetLastError();
}

// 2D tile shape (cells; one thread per cell): 32 x 8, 256 threads.  A
// 32 x 16 tile (512 threads, two workgroups per CU within the LDS) evaluates
// 2.09 faces and loads 1.56 halo cells per cell instead of 2.16 and 1.94; in
// FP64 it was 5 % faster on a 512^2 grid but 10 % slower on 4096 x 2048 and
// 1 % slower on the 1024 x 512 cylinder.
constexpr int TX2 = STAGE_TX, TY2 = STAGE_TY;
constexpr int TX1 = 256;

template <class S, class C, int MODE, bool CHAR, bool VISC>
static void launch_2d(const GridArgs& a, const S* Us, const S* Un, S* Uo, const double* dtp, const S* Lin,
                      hipStream_t st) {
  dim3 grid((a.nx + TX2 - 1) / TX2, (a.ny + TY2 - 1) / TY2, a.nbatch);
  if (a.cls != nullptr)
    hipLaunchKernelGGL((stage_kernel<S, C, 2, TX2, TY2, VISC, MODE, NET_NONE, CHAR, true>), grid, dim3(TX2 * TY2),
                       0, st, a, Us, Un, Uo, dtp, Lin, NetArgs{});
  else
    hipLaunchKernelGGL((stage_kernel<S, C, 2, TX2, TY2, VISC, MODE, NET_NONE, CHAR, false>), grid, dim3(TX2 * TY2),
                       0, st, a, Us, Un, Uo, dtp, Lin, NetArgs{});
}

template <class S, class C, int MODE, bool CHAR>
static hipError_t launch_mode_r(const GridArgs& a, const S* Us, const S* Un, S* Uo, const double* dtp,
                                const S* Lin, hipStream_t st) {
  if (a.ndim == 1) {
    dim3 grid((a.nx + TX1 - 1) / TX1, 1, a.nbatch);
    hipLaunchKernelGGL((stage_kernel<S, C, 1, TX1, 1, false, MODE, NET_NONE, CHAR>), grid, dim3(TX1), 0, st, a,
                       Us, Un, Uo, dtp, Lin, NetArgs{});
  } else if (a.viscous) {
    launch_2d<S, C, MODE, CHAR, true>(a, Us, Un, Uo, dtp, Lin, st);
  } else {
    launch_2d<S, C, MODE, CHAR, false>(a, Us, Un, Uo, dtp, Lin, st);
  }
  return hipGetLastError();
}

// The characteristic reconstruction exists for FP64 storage and arithmetic.
template <class S, class C, int MODE>
static hipError_t launch_mode(const GridArgs& a, const S* Us, const S* Un, S* Uo, const double* dtp,
                              const S* Lin, hipStream_t st) {
  if (a.weno_char) {
    if constexpr (sizeof(S) == 8 && sizeof(C) == 8)
      return launch_mode_r<S, C, MODE, true>(a, Us, Un, Uo, dtp, Lin, st);
    return hipErrorInvalidValue;
  }
  return launch_mode_r<S, C, MODE, false>(a, Us, Un, Uo, dtp, Lin, st);
}

template <class S, class C>
static hipError_t launch_stage_c(const GridArgs& a, int mode, const S* Us, const S* Un, S* Uo,
                                 const double* dtp, const S* Lin, hipStream_t st) {
  switch (mode) {
    case MODE_RHS: return launch_mode<S, C, MODE_RHS>(a, Us, Un, Uo, dtp, Lin, st);
    case MODE_STAGE1: return launch_mode<S, C, MODE_STAGE1>(a, Us, Un, Uo, dtp, Lin, st);
    case MODE_STAGE2: return launch_mode<S, C, MODE_STAGE2>(a, Us, Un, Uo, dtp, Lin, st);
    case MODE_STAGE3: return launch_mode<S, C, MODE_STAGE3>(a, Us, Un, Uo, dtp, Lin, st);
    case MODE_S1L: return launch_mode<S, C, MODE_S1L>(a, Us, Un, Uo, dtp, Lin, st);
    case MODE_S2F: return launch_mode<S, C, MODE_S2F>(a, Us, Un, Uo, dtp, Lin, st);
    case MODE_S3F: return launch_mode<S, C, MODE_S3F>(a, Us, Un, Uo, dtp, Lin, st);
    default: return hipErrorInvalidValue;
  }
}

template <int MODE, int NETK>
static hipError_t launch_net_mode(const GridArgs& a, const NetArgs& n, const double* Us, const double* Un,
                                  double* Uo, const double* dtp, hipStream_t st) {
  dim3 grid((a.nx + TX2 - 1) / TX2, (a.ny + TY2 - 1) / TY2, a.nbatch);
  // the learned-correction variants always carry the immersed-boundary
  // handling (their register use is set by the network pass)
  hipLaunchKernelGGL((stage_kernel<double, double, 2, TX2, TY2, false, MODE, NETK, false, true>), grid,
                     dim3(TX2 * TY2), 0, st, a, Us, Un, Uo, dtp, nullptr, n);
  return hipGetLastError();
}

template <int NETK>
static hipError_t launch_net_modes(const GridArgs& a, const NetArgs& n, int mode, const double* Us,
                                   const double* Un, double* Uo, const double* dtp, hipStream_t st) {
  switch (mode) {
    case MODE_RHS: return launch_net_mode<MODE_RHS, NETK>(a, n, Us, Un, Uo, dtp, st);
    case MODE_STAGE1: return launch_net_mode<MODE_STAGE1, NETK>(a, n, Us, Un, Uo, dtp, st);
    case MODE_STAGE2: return launch_net_mode<MODE_STAGE2, NETK>(a, n, Us, Un, Uo, dtp, st);
    case MODE_STAGE3: return launch_net_mode<MODE_STAGE3, NETK>(a, n, Us, Un, Uo, dtp, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage_net(const GridArgs& a, const NetArgs& n, int mode, const double* Us, const double* Un,
                            double* Uo, const double* dtp, hipStream_t st) {
  if (a.ndim != 2 || a.viscous) return hipErrorInvalidValue;
  return launch_net_modes<NET_MLP>(a, n, mode, Us, Un, Uo, dtp, st);
}

hipError_t launch_stage_ext(const GridArgs& a, int mode, const double* Us, const double* Un, double* Uo,
                            const double* dtp, hipStream_t st) {
  if (a.ndim != 2 || a.viscous || a.dFext == nullptr) return hipErrorInvalidValue;
  return launch_net_modes<NET_EXT>(a, NetArgs{}, mode, Us, Un, Uo, dtp, st);
}

// double storage: double arithmetic.  float storage: float arithmetic unless
// mixed (then double arithmetic).
hipError_t launch_stage_mixed(const GridArgs& a, int mode, const float* Us, const float* Un, float* Uo,
                              const double* dtp, const float* Lin, hipStream_t st) {
  return launch_stage_c<float, double>(a, mode, Us, Un, Uo, dtp, Lin, st);
}

template <>
hipError_t launch_stage<double>(const GridArgs& a, int mode, const double* Us, const double* Un, double* Uo,
                                const double* dtp, const double* Lin, hipStream_t st) {
  return launch_stage_c<double, double>(a, mode, Us, Un, Uo, dtp, Lin, st);
}
template <>
hipError_t launch_stage<float>(const GridArgs& a, int mode, const float* Us, const float* Un, float* Uo,
                               const double* dtp, const float* Lin, hipStream_t st) {
  return launch_stage_c<float, float>(a, mode, Us, Un, Uo, dtp, Lin, st);
}

template hipError_t launch_prim_to_cons<double>(const GridArgs&, const double*, double*, hipStream_t);
template hipError_t launch_prim_to_cons<float>(const GridArgs&, const float*, float*, hipStream_t);
template hipError_t launch_cfl<double>(const GridArgs&, const double*, double*, hipStream_t);
template hipError_t launch_cfl<float>(const GridArgs&, const float*, double*, hipStream_t);

}  // namespace shk
