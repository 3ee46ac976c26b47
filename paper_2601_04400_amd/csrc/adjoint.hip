// Discrete adjoint (reverse mode) of the right-hand side and of the SSP-RK3
// step, FP64, for gfx950.
//
// The chain rule through the unrolled solver (section 2, the gradient of the
// unrolled loss through the solver steps) needs vector-Jacobian products of
// one right-hand side, L_bar -> U_bar = (dL/dU)^T L_bar, plus the partial
// derivatives with respect to gamma and the inflow state.  They are written
// out by hand here, with every branch (Davis min/max, sign of s*, supersonic
// sides, positivity fallback, boundary rules, cell classes) fixed to the one
// the forward evaluation takes, and the WENO weights differentiated.
//
// Layout of one workgroup: a TX x TY tile of cells.  Every face whose
// stencil can reach the tile (directly or through a boundary ghost layer)
// is recomputed in the forward direction and reversed; the six stencil
// contributions of a face are added to LDS accumulators in six passes
// separated by barriers, so that within a pass no two faces touch the same
// entry.  The summation order is therefore fixed and the result is
// reproducible bit for bit, without atomics.
#include <hip/hip_runtime.h>

#include "face_dev.hpp"
#include "flux.hpp"
#include "grid.hpp"
#include "xcd.hpp"

namespace shk {

namespace {

// Boundary source (same rules as the forward loads).
__device__ __forceinline__ int adj_bc_source(int g, int n, int bc_lo, int bc_hi, int& flag) {
  if (g >= 0 && g < n) return g;
  const bool lo = g < 0;
  const int bc = lo ? bc_lo : bc_hi;
  const int depth = lo ? -g : g - (n - 1);
  int s;
  switch (bc) {
    case BC_REFL: s = lo ? depth - 1 : n - depth; flag = flag | 1; break;
    case BC_INFLOW: s = lo ? 0 : n - 1; flag = 2; break;
    case BC_PERIODIC: s = ((g % n) + n) % n; break;
    default: s = lo ? 0 : n - 1; break;
  }
  return s < 0 ? 0 : (s >= n ? n - 1 : s);
}

__device__ __forceinline__ void adj_load_cons(const GridArgs& a, const double* __restrict__ U, int gi, int gj,
                                              double q[4]) {
  int fx = 0, fy = 0;
  const int si = adj_bc_source(gi, a.nx, a.bc[0], a.bc[1], fx);
  const int sj = adj_bc_source(gj, a.ny, a.bc[2], a.bc[3], fy);
  if (fy == 2 || fx == 2) {
    for (int v = 0; v < 4; ++v) q[v] = a.inflow_cons[v];
  } else {
    const long long c = (long long)sj * a.nx + si;
    q[0] = U[c];
    q[1] = U[a.ncell + c];
    q[2] = U[2 * a.ncell + c];
    q[3] = U[3 * a.ncell + c];
    if (fx & 1) q[1] = -q[1];
  }
  if (fy & 1) q[2] = -q[2];
}

struct PB {
  double r, un, ut, p;
};

// Reverse of one HLLC bracket (side state w with energy E, wave speed s,
// contact speed ss).  Fb is the upstream gradient times the bracket weight.
__device__ __forceinline__ void hllc_side_vjp(const Prim<double>& w, double E, double s, double ss, bool sup,
                                              const double Fb[4], PB& wb, double& Eb, double& sb,
                                              double& ssb) {
  const double mn = w.r * w.un;
  double mnb = 0.0;
  if (!sup) {
    const double su = s - w.un;
    const double den = s - ss;
    const double chi = qdiv(su, den);
    const double iden = qrcp(den), isu = qrcp(su);
    const double rs = chi * w.r;
    const double d0 = rs - w.r, d1 = rs * ss - mn, d2 = rs * w.ut - w.r * w.ut;
    const double C = w.r * ss + qdiv(w.p, su);
    const double B = E + (ss - w.un) * C;
    const double d3 = chi * B - E;
    sb += Fb[0] * d0 + Fb[1] * d1 + Fb[2] * d2 + Fb[3] * d3;
    const double db0 = s * Fb[0], db1 = s * Fb[1], db2 = s * Fb[2], db3 = s * Fb[3];
    const double rsb = db0 + db1 * ss + db2 * w.ut;
    wb.r -= db0;
    ssb += db1 * rs;
    mnb -= db1;
    wb.ut += db2 * (rs - w.r);
    wb.r -= db2 * w.ut;
    double chib = db3 * B;
    const double Bb = db3 * chi;
    Eb -= db3;
    Eb += Bb;
    ssb += Bb * C;
    wb.un -= Bb * C;
    const double Cb = Bb * (ss - w.un);
    wb.r += Cb * ss;
    ssb += Cb * w.r;
    wb.p += Cb * isu;
    double sub = -Cb * w.p * (isu * isu);
    chib += rsb * w.r;
    wb.r += rsb * chi;
    sub += chib * iden;
    const double denb = -chib * chi * iden;
    sb += denb;
    ssb -= denb;
    sb += sub;
    wb.un -= sub;
  }
  // physical flux (mn, mn un + p, mn ut, un (E + p))
  mnb += Fb[0] + Fb[1] * w.un + Fb[2] * w.ut;
  wb.un += Fb[1] * mn + Fb[3] * (E + w.p);
  wb.p += Fb[1] + Fb[3] * w.un;
  wb.ut += Fb[2] * mn;
  Eb += Fb[3] * w.un;
  wb.r += mnb * w.un;
  wb.un += mnb * w.r;
}

// Reverse of the HLLC flux in the face-normal frame.
__device__ __forceinline__ void hllc_vjp(const Prim<double>& L, const Prim<double>& R, double gamma,
                                         const double Fb[4], PB& Lb, PB& Rb, double& gb) {
  const double gm1 = gamma - 1.0, igm1 = qrcp(gm1);
  const double irL = qrcp(L.r), irR = qrcp(R.r);
  // sound speeds exactly as the forward flux evaluates them
  const double zL = qdiv(gamma * L.p, L.r), zR = qdiv(gamma * R.p, R.r);
  const double aL = qsqrt(zL), aR = qsqrt(zR);
  const bool minL = (L.un - aL) <= (R.un - aR);
  const bool maxL = (L.un + aL) >= (R.un + aR);
  const double sL = minL ? L.un - aL : R.un - aR;
  const double sR = maxL ? L.un + aL : R.un + aR;
  const double dL = sL - L.un, dR = sR - R.un;
  const double num = R.p - L.p + L.r * L.un * dL - R.r * R.un * dR;
  const double den = L.r * dL - R.r * dR;
  const double ss = qdiv(num, den);
  const double iden = qrcp(den);
  const double EL = L.p * igm1 + 0.5 * L.r * (L.un * L.un + L.ut * L.ut);
  const double ER = R.p * igm1 + 0.5 * R.r * (R.un * R.un + R.ut * R.ut);
  double ELb = 0.0, ERb = 0.0, sLb = 0.0, sRb = 0.0, ssb = 0.0;
  Lb = PB{0.0, 0.0, 0.0, 0.0};
  Rb = PB{0.0, 0.0, 0.0, 0.0};
  if (ss > 0.0) {
    hllc_side_vjp(L, EL, sL, ss, sL >= 0.0, Fb, Lb, ELb, sLb, ssb);
  } else if (ss < 0.0) {
    hllc_side_vjp(R, ER, sR, ss, sR <= 0.0, Fb, Rb, ERb, sRb, ssb);
  } else {
    const double Fh[4] = {0.5 * Fb[0], 0.5 * Fb[1], 0.5 * Fb[2], 0.5 * Fb[3]};
    hllc_side_vjp(L, EL, sL, ss, sL >= 0.0, Fh, Lb, ELb, sLb, ssb);
    hllc_side_vjp(R, ER, sR, ss, sR <= 0.0, Fh, Rb, ERb, sRb, ssb);
  }
  // energies E = p/(gamma-1) + rho (un^2 + ut^2)/2
  Lb.p += ELb * igm1;
  gb -= ELb * L.p * igm1 * igm1;
  Lb.r += ELb * 0.5 * (L.un * L.un + L.ut * L.ut);
  Lb.un += ELb * L.r * L.un;
  Lb.ut += ELb * L.r * L.ut;
  Rb.p += ERb * igm1;
  gb -= ERb * R.p * igm1 * igm1;
  Rb.r += ERb * 0.5 * (R.un * R.un + R.ut * R.ut);
  Rb.un += ERb * R.r * R.un;
  Rb.ut += ERb * R.r * R.ut;
  // contact speed
  const double numb = ssb * iden;
  const double denb = -ssb * ss * iden;
  Rb.p += numb;
  Lb.p -= numb;
  Lb.r += numb * L.un * dL;
  Lb.un += numb * L.r * dL;
  double dLb = numb * L.r * L.un;
  Rb.r -= numb * R.un * dR;
  Rb.un -= numb * R.r * dR;
  double dRb = -numb * R.r * R.un;
  Lb.r += denb * dL;
  dLb += denb * L.r;
  Rb.r -= denb * dR;
  dRb -= denb * R.r;
  sLb += dLb;
  Lb.un -= dLb;
  sRb += dRb;
  Rb.un -= dRb;
  // Davis wave speeds
  double aLb = 0.0, aRb = 0.0;
  if (minL) { Lb.un += sLb; aLb -= sLb; } else { Rb.un += sLb; aRb -= sLb; }
  if (maxL) { Lb.un += sRb; aLb += sRb; } else { Rb.un += sRb; aRb += sRb; }
  // sound speeds a = sqrt(gamma p / rho)
  const double zLb = qdiv(0.5 * aLb, aL), zRb = qdiv(0.5 * aRb, aR);
  gb += zLb * L.p * irL + zRb * R.p * irR;
  Lb.p += zLb * gamma * irL;
  Lb.r -= zLb * zL * irL;
  Rb.p += zRb * gamma * irR;
  Rb.r -= zRb * zR * irR;
}

// Forward recompute and reverse of one face.  The stencil is read from LDS:
// component k of stencil cell s at q[k][s * st] (face frame: rho, normal
// velocity, tangential velocity, p).  Upstream flux gradient Fb -> stencil
// gradients sl[6][4].  The reverse re-reads the stencil and recomputes the
// WENO weights instead of keeping the forward's intermediates alive (the
// loads and inputs are hidden from common-subexpression elimination), which
// keeps the register footprint at a level that lets several waves share a
// SIMD.
__device__ __forceinline__ void face_vjp(const double* q0, const double* q1, const double* q2, const double* q3,
                                         int st, double eps, double gamma, const double Fb[4], double sl[6][4],
                                         double& gb) {
  const double* q[4] = {q0, q1, q2, q3};
  Prim<double> L, R;
  double* Lp[4] = {&L.r, &L.un, &L.ut, &L.p};
  double* Rp[4] = {&R.r, &R.un, &R.ut, &R.p};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = q[c][k * st];
    weno5_pair(v[0], v[1], v[2], v[3], v[4], v[5], eps, *Lp[c], *Rp[c]);
  }
  const bool fallback = !(L.r > 0.0) || !(L.p > 0.0) || !(R.r > 0.0) || !(R.p > 0.0);
  if (fallback) {
    L = Prim<double>{q0[2 * st], q1[2 * st], q2[2 * st], q3[2 * st]};
    R = Prim<double>{q0[3 * st], q1[3 * st], q2[3 * st], q3[3 * st]};
  }
  PB Lb, Rb;
  hllc_vjp(L, R, gamma, Fb, Lb, Rb, gb);
  const double lb[4] = {Lb.r, Lb.un, Lb.ut, Lb.p};
  const double rb[4] = {Rb.r, Rb.un, Rb.ut, Rb.p};
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int s = 0; s < 6; ++s) sl[s][c] = 0.0;
  if (fallback) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sl[2][c] = lb[c];
      sl[3][c] = rb[c];
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int off = 0;
    asm volatile("" : "+v"(off));
    double x[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = q[c][off + k * st];
    weno5_vjp(x[0], x[1], x[2], x[3], x[4], eps, lb[c], sl[0][c], sl[1][c], sl[2][c], sl[3][c], sl[4][c]);
    weno5_vjp(x[5], x[4], x[3], x[2], x[1], eps, rb[c], sl[5][c], sl[4][c], sl[3][c], sl[2][c], sl[1][c]);
  }
}

__device__ __forceinline__ double lam_at(const GridArgs& a, const double* __restrict__ lam, int v, int gi, int gj) {
  // adjoint of the right-hand side at a cell; zero outside the domain and at
  // non-fluid cells (where the right-hand side is set to zero)
  const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
  if (gi < 0 || gi >= a.nx) {
    if (!px) return 0.0;
    gi = ((gi % a.nx) + a.nx) % a.nx;
  }
  if (gj < 0 || gj >= a.ny) {
    if (!py) return 0.0;
    gj = ((gj % a.ny) + a.ny) % a.ny;
  }
  const long long c = (long long)gj * a.nx + gi;
  if (a.cls != nullptr && a.cls[c] != CELL_FLUID) return 0.0;
  return lam[v * a.ncell + c];
}

// First half of the refill transpose for ghost k of one batch member: with
// X the adjoint of the ghost's refilled conservative state, recompute the
// image-point primitives and the wall rule from the sources in Ub and
// return the adjoint of the image-point primitives, gW = (rho, u, v, p)_bar;
// *gpart receives the gamma part of the ghost energy's reverse.
__device__ __forceinline__ void ghost_reverse(const GridArgs& a, const GhostTable& gt, const double* __restrict__ Ub,
                                              int k, const double X[4], double gWk[4], double* gpart) {
  const long long n = a.ncell;
  const double gm1 = a.gamma - 1.0;
  double Wi[4] = {0.0, 0.0, 0.0, 0.0};
  // branch-free over the four corners (an unused one reads cell 0 with
  // weight 0) so that all sixteen loads are in flight together
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int s0 = gt.src[4 * k + m];
    const bool use = s0 >= 0;
    const int sm = use ? s0 : 0;
    const double wm = use ? gt.w[4 * k + m] : 0.0;
    const double r = Ub[sm];
    const double u = Ub[n + sm] / r, v = Ub[2 * n + sm] / r;
    const double p = gm1 * (Ub[3 * n + sm] - 0.5 * r * (u * u + v * v));
    Wi[0] += wm * r; Wi[1] += wm * u; Wi[2] += wm * v; Wi[3] += wm * p;
  }
  const double nxv = gt.nrm[2 * k], nyv = gt.nrm[2 * k + 1];
  double ug, vg;
  if (gt.wall == 0) {
    const double un = Wi[1] * nxv + Wi[2] * nyv;
    ug = Wi[1] - 2.0 * un * nxv;
    vg = Wi[2] - 2.0 * un * nyv;
  } else {
    ug = -Wi[1];
    vg = -Wi[2];
  }
  // reverse of U_g = (rho, rho ug, rho vg, p/(gamma-1) + rho (ug^2+vg^2)/2)
  const double rb = X[0] + X[1] * ug + X[2] * vg + X[3] * 0.5 * (ug * ug + vg * vg);
  const double ugb = X[1] * Wi[0] + X[3] * Wi[0] * ug;
  const double vgb = X[2] * Wi[0] + X[3] * Wi[0] * vg;
  *gpart = -X[3] * Wi[3] / (gm1 * gm1);
  double Wub, Wvb;
  if (gt.wall == 0) {
    const double unb = -2.0 * (ugb * nxv + vgb * nyv);
    Wub = ugb + unb * nxv;
    Wvb = vgb + unb * nyv;
  } else {
    Wub = -ugb;
    Wvb = -vgb;
  }
  gWk[0] = rb;
  gWk[1] = Wub;
  gWk[2] = Wvb;
  gWk[3] = X[3] / gm1;
}

}  // namespace

// out = J^T (clam_f dt lam) + c1 X1 + c2 X2 + c3 X3 for every cell of the
// tile, where J is the Jacobian of the right-hand side at the stage state Us.
// The X terms are read at the thread's own cell only, so out may alias one of
// them (never lam).  part receives this block's partial derivatives (gamma,
// rho_in, u_in, v_in, p_in).
template <int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) rhs_adjoint_kernel(GridArgs a, const double* __restrict__ Us,
                                                          const double* __restrict__ lam, double clam_f,
                                                          const double* __restrict__ dtp, const double* X1,
                                                          double c1, const double* X2, double c2, const double* X3,
                                                          double c3, double* out, double* __restrict__ part,
                                                          GhostTable gt, double* __restrict__ gW) {
  constexpr int M = 5;
  constexpr int PX = TX + 2 * M, PY = TY + 2 * M;
  constexpr int NFX = (TX + 5) * TY, NFY = TX * (TY + 5);
  __shared__ double w[4][PY * PX];
  __shared__ double lw[4][PY * PX];  // right-hand-side adjoint on the same cross-shaped tile
  __shared__ double ax[4][TY * PX];
  __shared__ double ay[4][PY * TX];
  __shared__ double red[5][NT / 64];

  int bx, by, b;
  xcd_tile(bx, by, b);
  const int i0 = bx * TX, j0 = by * TY;
  const long long boff = (long long)b * 4 * a.ncell;
  const double* __restrict__ Ub = Us + boff;
  const double* __restrict__ Lb = lam + boff;
  const double clam = clam_f * (dtp ? dtp[b] : 1.0);
  const double gamma = a.gamma, gm1 = gamma - 1.0;
  const bool perx = a.bc[0] == BC_PERIODIC, pery = a.bc[2] == BC_PERIODIC;

  for (int k = threadIdx.x; k < PY * PX; k += NT) {
    const int lx = k % PX, ly = k / PX;
    const bool inx = lx >= M && lx < TX + M;
    const bool iny = ly >= M && ly < TY + M;
    if (!inx && !iny) continue;
    double q[4];
    adj_load_cons(a, Ub, i0 - M + lx, j0 - M + ly, q);
    double lv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) lv[c] = lam_at(a, Lb, c, i0 - M + lx, j0 - M + ly);
    const Prim<double> p = to_prim(q[0], q[1], q[2], q[3], gm1);
    w[0][k] = p.r;
    w[1][k] = p.un;
    w[2][k] = p.ut;
    w[3][k] = p.p;
#pragma unroll
    for (int c = 0; c < 4; ++c) lw[c][k] = lv[c];
  }
  for (int k = threadIdx.x; k < TY * PX; k += NT)
    for (int c = 0; c < 4; ++c) ax[c][k] = 0.0;
  for (int k = threadIdx.x; k < PY * TX; k += NT)
    for (int c = 0; c < 4; ++c) ay[c][k] = 0.0;
  __syncthreads();

  double gacc = 0.0;
#pragma unroll 1
  for (int base = 0; base < NFX + NFY; base += NT) {
    const int k = base + threadIdx.x;
    bool act = false, isx = true, own = false;
    int row = 0, pos0 = 0;
    double sl[6][4];
    if (k < NFX + NFY) {
      isx = k < NFX;
      int s0, st, cn, ct;
      double Fb[4];
      bool valid;
      if (isx) {
        const int fl = 3 + k % (TX + 5), y = k / (TX + 5);
        const int gf = i0 - M + fl;  // left face of cell gf
        const int gj = j0 + y;
        valid = gj < a.ny && (perx || (gf >= 0 && gf <= a.nx));
        // faces near the tile edges are recomputed by two tiles; the one with
        // the face in [i0, i1) (or the right domain face) reports its gamma part
        own = (gf >= i0 && gf < min(i0 + TX, a.nx)) || (!perx && gf == a.nx && i0 + TX >= a.nx);
        s0 = (y + M) * PX + fl - 3;
        st = 1; cn = 1; ct = 2;
        row = y; pos0 = fl - 3;
        if (valid) {
          const double sc = clam * a.inv_dx;
          const int pr = (y + M) * PX + fl;  // cell gf; gf - 1 is pr - 1
          Fb[0] = sc * (lw[0][pr] - lw[0][pr - 1]);
          Fb[1] = sc * (lw[1][pr] - lw[1][pr - 1]);
          Fb[2] = sc * (lw[2][pr] - lw[2][pr - 1]);
          Fb[3] = sc * (lw[3][pr] - lw[3][pr - 1]);
        }
      } else {
        const int kk = k - NFX;
        const int x = kk % TX, gl = 3 + kk / TX;
        const int gf = j0 - M + gl;
        const int gi = i0 + x;
        valid = gi < a.nx && (pery || (gf >= 0 && gf <= a.ny));
        own = (gf >= j0 && gf < min(j0 + TY, a.ny)) || (!pery && gf == a.ny && j0 + TY >= a.ny);
        s0 = (gl - 3) * PX + x + M;
        st = PX; cn = 2; ct = 1;
        row = x; pos0 = gl - 3;
        if (valid) {
          const double sc = clam * a.inv_dy;
          const int pt = gl * PX + x + M, pb = pt - PX;  // cells gf and gf - 1
          Fb[0] = sc * (lw[0][pt] - lw[0][pb]);
          Fb[1] = sc * (lw[2][pt] - lw[2][pb]);
          Fb[2] = sc * (lw[1][pt] - lw[1][pb]);
          Fb[3] = sc * (lw[3][pt] - lw[3][pb]);
        }
      }
      if (valid && (Fb[0] != 0.0 || Fb[1] != 0.0 || Fb[2] != 0.0 || Fb[3] != 0.0)) {
        double gface = 0.0;
        face_vjp(&w[0][s0], &w[cn][s0], &w[ct][s0], &w[3][s0], st, a.eps, gamma, Fb, sl, gface);
        if (own) gacc += gface;
        if (a.dXnet != nullptr) {
          // stencil gradient of the learned correction at this face
          long long gfi;
          if (isx) {
            const int gf = i0 - M + 3 + k % (TX + 5), gj = j0 + k / (TX + 5);
            const int gw = (gf >= 0 && gf <= a.nx) ? gf : ((gf % a.nx) + a.nx) % a.nx;
            gfi = (long long)gj * (a.nx + 1) + gw;
          } else {
            const int kk = k - NFX;
            const int gi = i0 + kk % TX, gf = j0 - M + 3 + kk / TX;
            const int gw = (gf >= 0 && gf <= a.ny) ? gf : ((gf % a.ny) + a.ny) % a.ny;
            gfi = (long long)(a.nx + 1) * a.ny + (long long)gw * a.nx + gi;
          }
          const float* d = a.dXnet + ((long long)b * a.nface + gfi) * 24;
          for (int s2 = 0; s2 < 6; ++s2)
            for (int c2 = 0; c2 < 4; ++c2) sl[s2][c2] += double(d[s2 * 4 + c2]);
        }
        act = true;
      }
    }
    for (int s = 0; s < 6; ++s) {
      if (act) {
        if (isx) {
          const int p = row * PX + pos0 + s;
          ax[0][p] += sl[s][0];
          ax[1][p] += sl[s][1];
          ax[2][p] += sl[s][2];
          ax[3][p] += sl[s][3];
        } else {
          const int p = (pos0 + s) * TX + row;
          ay[0][p] += sl[s][0];
          ay[1][p] += sl[s][2];  // face frame (rho, v, u, p) -> (rho, u, v, p)
          ay[2][p] += sl[s][1];
          ay[3][p] += sl[s][3];
        }
      }
      __syncthreads();
    }
  }

  // fold boundary ghost layers, then the primitive-variable adjoint per cell
  double inb[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < TX * TY; k += NT) {
    const int x = k % TX, y = k / TX;
    const int gi = i0 + x, gj = j0 + y;
    if (gi >= a.nx || gj >= a.ny) continue;
    double Wb[4];
    for (int c = 0; c < 4; ++c) Wb[c] = ax[c][y * PX + x + M] + ay[c][(y + M) * TX + x];
    if (!perx) {
      for (int g = 1; g <= 3; ++g) {
        // left ghost -g
        const int lxl = -g - i0 + M;
        if (lxl >= 0) {
          const int p = y * PX + lxl;
          if (a.bc[0] == BC_TRANS && gi == 0) {
            for (int c = 0; c < 4; ++c) Wb[c] += ax[c][p];
          } else if (a.bc[0] == BC_REFL && gi == g - 1) {
            Wb[0] += ax[0][p]; Wb[1] -= ax[1][p]; Wb[2] += ax[2][p]; Wb[3] += ax[3][p];
          } else if (a.bc[0] == BC_INFLOW && gi == 0) {
            for (int c = 0; c < 4; ++c) inb[c] += ax[c][p];
          }
        }
        // right ghost nx-1+g
        const int lxr = a.nx - 1 + g - i0 + M;
        if (lxr < PX) {
          const int p = y * PX + lxr;
          if (a.bc[1] == BC_TRANS && gi == a.nx - 1) {
            for (int c = 0; c < 4; ++c) Wb[c] += ax[c][p];
          } else if (a.bc[1] == BC_REFL && gi == a.nx - g) {
            Wb[0] += ax[0][p]; Wb[1] -= ax[1][p]; Wb[2] += ax[2][p]; Wb[3] += ax[3][p];
          } else if (a.bc[1] == BC_INFLOW && gi == a.nx - 1) {
            for (int c = 0; c < 4; ++c) inb[c] += ax[c][p];
          }
        }
      }
    }
    if (!pery) {
      for (int g = 1; g <= 3; ++g) {
        const int lyl = -g - j0 + M;
        if (lyl >= 0) {
          const int p = lyl * TX + x;
          if (a.bc[2] == BC_TRANS && gj == 0) {
            for (int c = 0; c < 4; ++c) Wb[c] += ay[c][p];
          } else if (a.bc[2] == BC_REFL && gj == g - 1) {
            Wb[0] += ay[0][p]; Wb[1] += ay[1][p]; Wb[2] -= ay[2][p]; Wb[3] += ay[3][p];
          } else if (a.bc[2] == BC_INFLOW && gj == 0) {
            for (int c = 0; c < 4; ++c) inb[c] += ay[c][p];
          }
        }
        const int lyr = a.ny - 1 + g - j0 + M;
        if (lyr < PY) {
          const int p = lyr * TX + x;
          if (a.bc[3] == BC_TRANS && gj == a.ny - 1) {
            for (int c = 0; c < 4; ++c) Wb[c] += ay[c][p];
          } else if (a.bc[3] == BC_REFL && gj == a.ny - g) {
            Wb[0] += ay[0][p]; Wb[1] += ay[1][p]; Wb[2] -= ay[2][p]; Wb[3] += ay[3][p];
          } else if (a.bc[3] == BC_INFLOW && gj == a.ny - 1) {
            for (int c = 0; c < 4; ++c) inb[c] += ay[c][p];
          }
        }
      }
    }
    // W = (rho, m_x/rho, m_y/rho, (gamma-1)(E - (m_x^2 + m_y^2)/(2 rho))),
    // with the cell's primitives from the tile (E - rho |u|^2/2 = p/(gamma-1))
    const long long cell = (long long)gj * a.nx + gi;
    const int lc = (y + M) * PX + x + M;
    const double r = w[0][lc], u = w[1][lc], vv = w[2][lc], pc = w[3][lc];
    const double ir = qrcp(r);
    const double ke = 0.5 * (u * u + vv * vv);
    double Uo[4];
    Uo[0] = Wb[0] - Wb[1] * u * ir - Wb[2] * vv * ir + Wb[3] * gm1 * ke;
    Uo[1] = Wb[1] * ir - Wb[3] * gm1 * u;
    Uo[2] = Wb[2] * ir - Wb[3] * gm1 * vv;
    Uo[3] = Wb[3] * gm1;
    gacc += Wb[3] * qdiv(pc, gm1);
    double val[4];
    for (int c = 0; c < 4; ++c) {
      const long long o = boff + c * a.ncell + cell;
      val[c] = Uo[c];
      if (X1) val[c] += c1 * X1[o];
      if (X2) val[c] += c2 * X2[o];
      if (X3) val[c] += c3 * X3[o];
    }
    const int gk = gW != nullptr ? a.ghost_of[cell] : -1;
    if (gk >= 0) {
      // a ghost: its refilled value is overwritten by the refill, so its
      // adjoint passes to the image point (gW) and its own entry is zero
      double gWk[4], gp;
      ghost_reverse(a, gt, Ub, gk, val, gWk, &gp);
      double* g4 = gW + ((long long)b * gt.n + gk) * 4;
      g4[0] = gWk[0]; g4[1] = gWk[1]; g4[2] = gWk[2]; g4[3] = gWk[3];
      gacc += gp;
      val[0] = val[1] = val[2] = val[3] = 0.0;
    }
    for (int c = 0; c < 4; ++c) out[boff + c * a.ncell + cell] = val[c];
  }

  // block partial derivatives, reduced in a fixed order
  double vals[5] = {gacc, inb[0], inb[1], inb[2], inb[3]};
  for (int q = 0; q < 5; ++q) {
    double v = vals[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int k = 0; k < NT / 64; ++k) s += red[threadIdx.x][k];
    const long long blk = ((long long)b * gridDim.y + by) * gridDim.x + bx;
    part[blk * 5 + threadIdx.x] = s;
  }
}

// ------------------------------------------------- immersed boundary transpose
// Entries (ghost, corner) of the refill, one per valid interpolation source,
// sorted by source cell and then by entry index: rank of an entry = number of
// entries ordered before it (deterministic; the list is a few thousand long).
__global__ void __launch_bounds__(256) ibm_entries_rank_kernel(GhostTable gt, int* __restrict__ keys,
                                                               int* __restrict__ vals, int* __restrict__ nvalid) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n4 = 4 * gt.n;
  if (e >= n4) return;
  const int ke = gt.src[e];
  if (ke < 0) return;
  int rank = 0;
  for (int f = 0; f < n4; ++f) {
    const int kf = gt.src[f];
    if (kf < 0) continue;
    rank += (kf < ke || (kf == ke && f < e)) ? 1 : 0;
  }
  keys[rank] = ke;
  vals[rank] = e;
  atomicAdd(nvalid, 1);
}

// Second half of the refill transpose, one workgroup per batch member: the
// adjoint kernel has already turned the adjoint of every ghost's refilled
// state into the adjoint gW[k] = (rho, u, v, p)_bar of its image-point
// primitives (and cleared the ghost's own entry).  Here each source cell
// gathers w_m gW[k] over the ghosts k that read it, in entry order, followed
// by the primitive -> conservative transpose at the source.  The fill table
// (built when the level set is set) holds a source's cell, entry count,
// ghost indices and weights at addresses that depend on the source's number
// only, so a thread's loads wait for one round trip before the ghost
// adjoints are read, not three (run heads, entries, weights).  The
// gamma parts are summed in a fixed order into the member's partial; with
// param_bar set, the member's recorded partials of the whole reverse pass
// (slots of ps, this launch's own last) are then added to param_bar here
// instead of in a separate launch.
constexpr int FILL_NT = 1024;

__device__ __forceinline__ double block_sum_fixed(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < FILL_NT / 64; ++k) s += red[k];
  return s;
}

constexpr int FILL_SLOTS = 8;  // entry slots whose loads are issued together

__global__ void __launch_bounds__(FILL_NT) ibm_fill_adjoint_kernel(GridArgs a, GhostTable gt,
                                                                   const int* __restrict__ fsrc,
                                                                   const int* __restrict__ fcnt,
                                                                   const int* __restrict__ fk,
                                                                   const double* __restrict__ fw, int m, int nsrc,
                                                                   const double* __restrict__ Us, double* __restrict__ X,
                                                                   const double* __restrict__ gW,
                                                                   double* __restrict__ part, PartSlots ps,
                                                                   double* __restrict__ param_bar) {
  __shared__ double red[FILL_NT / 64];
  const int b = blockIdx.x;
  const long long n = a.ncell;
  const double* __restrict__ Ub = Us + (long long)b * 4 * n;
  double* __restrict__ Xb = X + (long long)b * 4 * n;
  const double* __restrict__ gWb = gW + (long long)b * 4 * gt.n;
  const double gm1 = a.gamma - 1.0;
  double gacc = 0.0;
  // the recorded partials of the earlier launches of this reverse pass are
  // summed by the last five waves (idle below unless the source list is
  // long): wave 11 + q takes quantity q
  const int qf = (int)(threadIdx.x >> 6) - (FILL_NT / 64 - 5), lanef = threadIdx.x & 63;
  double sq = 0.0;
  if (param_bar != nullptr && qf >= 0) {
    for (int slot = 0; slot < ps.n; ++slot) {
      const double* p = part - (ps.n - slot) * ps.stride;  // earlier slots precede this one
      const int nb = ps.nblk[slot];
      for (int k = lanef; k < nb; k += 64) sq += p[((long long)b * nb + k) * 5 + qf];
    }
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
  }
  for (int h = threadIdx.x; h < nsrc; h += FILL_NT) {
    const int src = fsrc[h], cnt = fcnt[h];
    double Wsb[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t0 = 0; t0 < m; t0 += FILL_SLOTS) {
      // the slots' ghost indices and weights are loaded without waiting for
      // the count (m, the most entries of any source, is uniform; unused
      // slots hold ghost 0 and weight 0 and are skipped)
      int k[FILL_SLOTS];
      double wm[FILL_SLOTS];
#pragma unroll
      for (int u = 0; u < FILL_SLOTS; ++u) {
        const int t = t0 + u;
        k[u] = t < m ? fk[(long long)t * nsrc + h] : 0;
        wm[u] = t < m ? fw[(long long)t * nsrc + h] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < FILL_SLOTS; ++u) {
        if (t0 + u >= cnt) continue;
        Wsb[0] += wm[u] * gWb[4 * k[u]];
        Wsb[1] += wm[u] * gWb[4 * k[u] + 1];
        Wsb[2] += wm[u] * gWb[4 * k[u] + 2];
        Wsb[3] += wm[u] * gWb[4 * k[u] + 3];
      }
    }
    const double r = Ub[src];
    const double u = Ub[n + src] / r, v = Ub[2 * n + src] / r;
    const double E = Ub[3 * n + src];
    const double ke = 0.5 * (u * u + v * v);
    Xb[src] += Wsb[0] - Wsb[1] * u / r - Wsb[2] * v / r + Wsb[3] * gm1 * ke;
    Xb[n + src] += Wsb[1] / r - Wsb[3] * gm1 * u;
    Xb[2 * n + src] += Wsb[2] / r - Wsb[3] * gm1 * v;
    Xb[3 * n + src] += Wsb[3] * gm1;
    gacc += Wsb[3] * (E - r * ke);
  }
  const double g = block_sum_fixed(gacc, red);
  if (param_bar == nullptr) {
    if (threadIdx.x < 5) part[(long long)b * 5 + threadIdx.x] = threadIdx.x == 0 ? g : 0.0;
    return;
  }
  // finalize: the earlier launches' partials plus this launch's gamma part
  if (qf >= 0 && lanef == 0) param_bar[b * 5 + qf] += sq + (qf == 0 ? g : 0.0);
}

// The ghost index of every cell (-1 for the others), for the adjoint kernel.
__global__ void __launch_bounds__(256) ghost_index_kernel(GridArgs a, int* __restrict__ ghost_of) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < a.ncell) ghost_of[c] = -1;
}
__global__ void __launch_bounds__(256) ghost_index_scatter_kernel(GhostTable gt, int* __restrict__ ghost_of) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < gt.n) ghost_of[gt.cell[k]] = k;
}

// param_bar[b][q] += the recorded partials of member b: one wave per q, lane
// l sums the entries l, l + 64, ... of every slot in order, then a fixed
// butterfly adds the 64 lane sums (the same order on every call).
__global__ void __launch_bounds__(320) partials_finalize_kernel(const double* __restrict__ part, PartSlots ps,
                                                                double* __restrict__ param_bar) {
  const int b = blockIdx.x;
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double s = 0.0;
  for (int slot = 0; slot < ps.n; ++slot) {
    const double* p = part + slot * ps.stride;
    const int nb = ps.nblk[slot];
    for (int k = lane; k < nb; k += 64) s += p[((long long)b * nb + k) * 5 + q];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) param_bar[b * 5 + q] += s;
}

// y = alpha x (+ y if accumulate), elementwise over n entries.
__global__ void __launch_bounds__(256) axpy_kernel(long long n, double alpha, const double* __restrict__ x,
                                                   double* __restrict__ y, int accumulate) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    y[k] = accumulate ? y[k] + alpha * x[k] : alpha * x[k];
}

// ------------------------------------------------------------------ launchers
// 32 x 8 tiles with 768 threads: the tile's 712 faces are reversed in one
// round (three waves per SIMD at <= 168 registers).  (32 x 4 tiles with 448
// threads, two workgroups per compute unit, were 1.6x slower: 22 % more
// recomputed faces and no better latency.)
constexpr int ATX = ADJ_TX, ATY = ADJ_TY, ANT = ADJ_NT;

int adjoint_blocks(const GridArgs& a) { return ((a.nx + ATX - 1) / ATX) * ((a.ny + ATY - 1) / ATY); }

hipError_t launch_rhs_adjoint(const GridArgs& a, const double* Us, const double* lam, double clam_f,
                              const double* dtp, const double* X1, double c1, const double* X2, double c2,
                              const double* X3, double c3, double* out, double* part, int* nblk,
                              const GhostTable& gt, double* gW, hipStream_t st) {
  dim3 grid((a.nx + ATX - 1) / ATX, (a.ny + ATY - 1) / ATY, a.nbatch);
  if (gW != nullptr && (a.ghost_of == nullptr || gt.n == 0)) gW = nullptr;
  hipLaunchKernelGGL((rhs_adjoint_kernel<ATX, ATY, ANT>), grid, dim3(ANT), 0, st, a, Us, lam, clam_f, dtp, X1, c1, X2,
                     c2, X3, c3, out, part, gt, gW);
  *nblk = (int)(grid.x * grid.y);
  return hipGetLastError();
}

hipError_t launch_ghost_index(const GridArgs& a, const GhostTable& gt, int* ghost_of, hipStream_t st) {
  hipLaunchKernelGGL(ghost_index_kernel, dim3((unsigned int)((a.ncell + 255) / 256)), dim3(256), 0, st, a, ghost_of);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || gt.n == 0) return e;
  hipLaunchKernelGGL(ghost_index_scatter_kernel, dim3((gt.n + 255) / 256), dim3(256), 0, st, gt, ghost_of);
  return hipGetLastError();
}

hipError_t launch_partials_finalize(const double* part, const PartSlots& ps, int nbatch, double* param_bar,
                                    hipStream_t st) {
  if (!param_bar || ps.n == 0) return hipSuccess;
  hipLaunchKernelGGL(partials_finalize_kernel, dim3(nbatch), dim3(320), 0, st, part, ps, param_bar);
  return hipGetLastError();
}

hipError_t launch_ibm_entries(const GhostTable& gt, int* keys, int* vals, int* nvalid, hipStream_t st) {
  if (gt.n == 0) return hipSuccess;
  hipLaunchKernelGGL(ibm_entries_rank_kernel, dim3((4 * gt.n + 255) / 256), dim3(256), 0, st, gt, keys, vals,
                     nvalid);
  return hipGetLastError();
}

hipError_t launch_ibm_fill_adjoint(const GridArgs& a, const GhostTable& gt, const int* fsrc, const int* fcnt,
                                   const int* fk, const double* fw, int m, int nsrc, const double* Us, double* X,
                                   const double* gW, double* part, const PartSlots& prior, double* param_bar,
                                   hipStream_t st) {
  hipLaunchKernelGGL(ibm_fill_adjoint_kernel, dim3(a.nbatch), dim3(FILL_NT), 0, st, a, gt, fsrc, fcnt, fk, fw, m, nsrc,
                     Us, X, gW, part, prior, param_bar);
  return hipGetLastError();
}

hipError_t launch_axpy(long long n, double alpha, const double* x, double* y, int accumulate, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned int)nb), dim3(256), 0, st, n, alpha, x, y, accumulate);
  return hipGetLastError();
}

}  // namespace shk
