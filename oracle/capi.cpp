// Oracle C entry points (TEST INFRASTRUCTURE ONLY): thin extern "C" wrappers
// over the templated serial solver so the Python test suite can call it
// through ctypes.  Nothing here is used by the GPU library.
#include <omp.h>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>

#include "cnn.hpp"
#include "exact_riemann.hpp"
#include "mlp.hpp"
#include "solver.hpp"
#include "training.hpp"

using namespace orc;

namespace {

bool config_ok(const Config* c) {
  if (!c) return false;
  if (c->ndim != 1 && c->ndim != 2) return false;
  if (c->nx < 1 || c->ny < 1) return false;
  if (c->ndim == 1 && c->ny != 1) return false;
  if (c->ndim == 1 && c->viscous) return false;
  if (!(c->gamma > 1.0)) return false;
  for (int k = 0; k < 4; ++k)
    if (c->bc[k] < 0 || c->bc[k] > 3) return false;
  return true;
}

// Correction handles cross the C boundary as the Correction* the create
// functions return (cast to void*).
const Correction* as_net(const void* p) { return static_cast<const Correction*>(p); }
const FluxNet* as_mlp(const void* p) { return static_cast<const FluxNet*>(as_net(p)); }
const FluxCnn* as_cnn(const void* p) { return static_cast<const FluxCnn*>(as_net(p)); }

template <class T>
void run_rhs(const Config& c, const Params<T>& P, const Ibm& ib, Field<T>& f, Field<T>& L,
             const Correction* net, long* fb) {
  ibm_fill(c, P, ib, f);
  rhs(c, P, ib, f, L, net, fb);
}

}  // namespace

extern "C" {

int orc_abi_version() { return 1; }

// Threads of the oracle's OpenMP loops (n >= 1 sets it; 0 only reads it).
// Results do not depend on it: every value is computed as in a serial run.
int orc_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

// Primitive planes (1D: rho,u,p; 2D: rho,u,v,p) -> conservative planes.
int orc_prim_to_cons(const Config* c, const double* W, double* U) {
  if (!config_ok(c)) return 1;
  const size_t n = size_t(c->nx) * c->ny;
  for (size_t k = 0; k < n; ++k) {
    double w[4], u[4];
    if (c->ndim == 1) { w[0] = W[k]; w[1] = W[n + k]; w[2] = 0.0; w[3] = W[2 * n + k]; }
    else for (int v = 0; v < 4; ++v) w[v] = W[v * n + k];
    prim_to_cons(w, c->gamma, u);
    if (c->ndim == 1) { U[k] = u[0]; U[n + k] = u[1]; U[2 * n + k] = u[3]; }
    else for (int v = 0; v < 4; ++v) U[v * n + k] = u[v];
  }
  return 0;
}

int orc_cons_to_prim(const Config* c, const double* U, double* W) {
  if (!config_ok(c)) return 1;
  const size_t n = size_t(c->nx) * c->ny;
  for (size_t k = 0; k < n; ++k) {
    double w[4], u[4];
    if (c->ndim == 1) { u[0] = U[k]; u[1] = U[n + k]; u[2] = 0.0; u[3] = U[2 * n + k]; }
    else for (int v = 0; v < 4; ++v) u[v] = U[v * n + k];
    cons_to_prim(u, c->gamma, w);
    if (c->ndim == 1) { W[k] = w[0]; W[n + k] = w[1]; W[2 * n + k] = w[3]; }
    else for (int v = 0; v < 4; ++v) W[v * n + k] = w[v];
  }
  return 0;
}

// One right-hand side.  U is not modified; when U_filled is given it receives
// U with the immersed-boundary ghost cells filled (the state the RHS saw).
int orc_rhs(const Config* c, const double* U, double* dUdt, const double* phi, int wall,
            const void* net, double* U_filled, long* fallback) {
  if (!config_ok(c)) return 1;
  Ibm ib = build_ibm(*c, phi, wall);
  Params<double> P = params_from<double>(*c);
  Field<double> f(c->nx, c->ny), L(c->nx, c->ny);
  load_state(*c, U, f);
  run_rhs(*c, P, ib, f, L, as_net(net), fallback);
  store_state(*c, L, dUdt);
  if (U_filled) store_state(*c, f, U_filled);
  return 0;
}

int orc_rk3_step(const Config* c, double* U, double dt, const double* phi, int wall, const void* net,
                 long* fallback) {
  if (!config_ok(c)) return 1;
  Ibm ib = build_ibm(*c, phi, wall);
  Params<double> P = params_from<double>(*c);
  Field<double> f(c->nx, c->ny);
  load_state(*c, U, f);
  rk3_step(*c, P, ib, f, dt, as_net(net), fallback);
  store_state(*c, f, U);
  return 0;
}

double orc_cfl_dt(const Config* c, const double* U, const double* phi, int wall) {
  if (!config_ok(c)) return -1.0;
  Ibm ib = build_ibm(*c, phi, wall);
  Field<double> f(c->nx, c->ny);
  load_state(*c, U, f);
  return cfl_dt(*c, ib, f);
}

// Advance from t0 towards t_end with the CFL step; the step that would reach
// or pass t_end is shortened to land on it exactly, and is the last one.
int orc_run(const Config* c, double* U, double t0, double t_end, int max_steps, const double* phi,
            int wall, const void* net, double* t_out, int* steps_out, long* fallback) {
  if (!config_ok(c)) return 1;
  Ibm ib = build_ibm(*c, phi, wall);
  Params<double> P = params_from<double>(*c);
  Field<double> f(c->nx, c->ny);
  load_state(*c, U, f);
  double t = t0;
  int steps = 0;
  while (steps < max_steps && t < t_end) {
    double dt = cfl_dt(*c, ib, f);
    bool last = false;
    if (t + dt >= t_end) { dt = t_end - t; last = true; }
    rk3_step(*c, P, ib, f, dt, as_net(net), fallback);
    t = last ? t_end : t + dt;
    ++steps;
  }
  store_state(*c, f, U);
  if (t_out) *t_out = t;
  if (steps_out) *steps_out = steps;
  return 0;
}

// ------------------------------------------------------------ unit pieces
double orc_weno5_left(const double* f5, double eps) { return weno5_left(f5, eps); }

void orc_hllc_x(const double* WL, const double* WR, double gamma, double* F) {
  hllc_x(WL, WR, gamma, F);
}

void orc_riemann_star(double rl, double ul, double pl, double rr, double ur, double pr, double g,
                      double* out4, int* iters) {
  RiemannStar s = riemann_star(rl, ul, pl, rr, ur, pr, g);
  out4[0] = s.p; out4[1] = s.u; out4[2] = s.rhoL; out4[3] = s.rhoR;
  if (iters) *iters = s.iterations;
}

// Exact solution (rho, u, p) at n points x, time t, diaphragm at xd.
void orc_riemann_sample(double rl, double ul, double pl, double rr, double ur, double pr, double g,
                        double xd, double t, int n, const double* x, double* rho, double* u, double* p) {
  RiemannStar s = riemann_star(rl, ul, pl, rr, ur, pr, g);
  for (int k = 0; k < n; ++k) {
    double o[3];
    riemann_sample(rl, ul, pl, rr, ur, pr, g, s, (x[k] - xd) / t, o);
    rho[k] = o[0]; u[k] = o[1]; p[k] = o[2];
  }
}

void orc_rh_post_shock(double M, double gamma, double rho1, double p1, double* out3) {
  rh_post_shock<double>(M, gamma, rho1, p1, out3);
}

// ------------------------------------------------------------------- IBM
int orc_ibm_classify(const Config* c, const double* phi, uint8_t* cls) {
  if (!config_ok(c) || !phi) return -1;
  Ibm ib = build_ibm(*c, phi, 0);
  std::memcpy(cls, ib.cls.data(), ib.cls.size());
  return int(ib.ghosts.size());
}

// Ghost table in row-major ghost order: (i, j), unit normal, 4 source cells
// (flat index or -1) and their weights.  Returns the number of ghosts.
// Ghosts of the level set whose image point is undefined (see Ibm::degenerate).
int orc_ibm_degenerate(const Config* c, const double* phi) {
  if (!config_ok(c) || !phi) return -1;
  return build_ibm(*c, phi, 0).degenerate;
}

int orc_ibm_ghosts(const Config* c, const double* phi, int cap, int* ij, double* normal, int* src,
                   double* w) {
  if (!config_ok(c) || !phi) return -1;
  Ibm ib = build_ibm(*c, phi, 0);
  int n = int(ib.ghosts.size());
  for (int k = 0; k < n && k < cap; ++k) {
    const auto& g = ib.ghosts[k];
    ij[2 * k] = g.i; ij[2 * k + 1] = g.j;
    normal[2 * k] = g.nx_; normal[2 * k + 1] = g.ny_;
    for (int m = 0; m < 4; ++m) { src[4 * k + m] = g.src[m]; w[4 * k + m] = g.w[m]; }
  }
  return n;
}

int orc_ibm_fill(const Config* c, double* U, const double* phi, int wall) {
  if (!config_ok(c) || !phi) return 1;
  Ibm ib = build_ibm(*c, phi, wall);
  Params<double> P = params_from<double>(*c);
  Field<double> f(c->nx, c->ny);
  load_state(*c, U, f);
  ibm_fill(*c, P, ib, f);
  store_state(*c, f, U);
  return 0;
}

// ------------------------------------------------------------- tangents
// Jacobian-vector product of the RHS: direction (Udot, gdot, indot[4]) over
// (state, gamma, inflow primitive state).
int orc_rhs_jvp(const Config* c, const double* U, const double* Udot, double gdot, const double* indot,
                const double* phi, int wall, double* L, double* Ldot, const void* net) {
  if (!config_ok(c)) return 1;
  using D = Dual<1>;
  Ibm ib = build_ibm(*c, phi, wall);
  Params<D> P = params_from<D>(*c);
  P.gamma.d[0] = gdot;
  for (int k = 0; k < 4; ++k) P.inflow[k].d[0] = indot ? indot[k] : 0.0;
  const size_t n = size_t(c->nx) * c->ny;
  const int ne = nvar_ext(*c);
  std::vector<D> Ud(ne * n);
  for (size_t k = 0; k < ne * n; ++k) { Ud[k] = D(U[k]); Ud[k].d[0] = Udot[k]; }
  Field<D> f(c->nx, c->ny), Lf(c->nx, c->ny);
  load_state(*c, Ud.data(), f);
  run_rhs(*c, P, ib, f, Lf, as_net(net), nullptr);
  std::vector<D> out(ne * n);
  store_state(*c, Lf, out.data());
  for (size_t k = 0; k < ne * n; ++k) { L[k] = out[k].v; Ldot[k] = out[k].d[0]; }
  return 0;
}

// Full Jacobian of the RHS by forward mode, one input direction at a time
// (small grids only): J[out][in] over the external state layout, followed by
// the columns for gamma and the four inflow primitives (ncols = n + 5).
int orc_rhs_jacobian(const Config* c, const double* U, const double* phi, int wall, double* J, const void* net) {
  if (!config_ok(c)) return 1;
  const size_t n = size_t(nvar_ext(*c)) * c->nx * c->ny;
  std::vector<double> Ud(n, 0.0), L(n), Ld(n);
  const size_t ncol = n + 5;
  for (size_t col = 0; col < ncol; ++col) {
    std::fill(Ud.begin(), Ud.end(), 0.0);
    double gd = 0.0, ind[4] = {0, 0, 0, 0};
    if (col < n) Ud[col] = 1.0;
    else if (col == n) gd = 1.0;
    else ind[col - n - 1] = 1.0;
    int rc = orc_rhs_jvp(c, U, Ud.data(), gd, ind, phi, wall, L.data(), Ld.data(), net);
    if (rc) return rc;
    for (size_t r = 0; r < n; ++r) J[r * ncol + col] = Ld[r];
  }
  return 0;
}

// Tangent of one RK3 step with fixed dt; U and Udot are advanced in place.
int orc_rk3_step_jvp(const Config* c, double* U, double* Udot, double dt, double gdot,
                     const double* indot, const double* phi, int wall, const void* net) {
  if (!config_ok(c)) return 1;
  using D = Dual<1>;
  Ibm ib = build_ibm(*c, phi, wall);
  Params<D> P = params_from<D>(*c);
  P.gamma.d[0] = gdot;
  for (int k = 0; k < 4; ++k) P.inflow[k].d[0] = indot ? indot[k] : 0.0;
  const size_t n = size_t(c->nx) * c->ny;
  const int ne = nvar_ext(*c);
  std::vector<D> Ud(ne * n);
  for (size_t k = 0; k < ne * n; ++k) { Ud[k] = D(U[k]); Ud[k].d[0] = Udot[k]; }
  Field<D> f(c->nx, c->ny);
  load_state(*c, Ud.data(), f);
  rk3_step(*c, P, ib, f, D(dt), as_net(net), nullptr);
  store_state(*c, f, Ud.data());
  for (size_t k = 0; k < ne * n; ++k) { U[k] = Ud[k].v; Udot[k] = Ud[k].d[0]; }
  return 0;
}

// Full Jacobian of one fixed-dt RK3 step (small grids), same column layout
// as orc_rhs_jacobian.
int orc_rk3_step_jacobian(const Config* c, const double* U, double dt, const double* phi, int wall,
                          double* J, const void* net) {
  if (!config_ok(c)) return 1;
  const size_t n = size_t(nvar_ext(*c)) * c->nx * c->ny;
  std::vector<double> Uc(n), Ud(n);
  const size_t ncol = n + 5;
  for (size_t col = 0; col < ncol; ++col) {
    std::copy(U, U + n, Uc.begin());
    std::fill(Ud.begin(), Ud.end(), 0.0);
    double gd = 0.0, ind[4] = {0, 0, 0, 0};
    if (col < n) Ud[col] = 1.0;
    else if (col == n) gd = 1.0;
    else ind[col - n - 1] = 1.0;
    int rc = orc_rk3_step_jvp(c, Uc.data(), Ud.data(), dt, gd, ind, phi, wall, net);
    if (rc) return rc;
    for (size_t r = 0; r < n; ++r) J[r * ncol + col] = Ud[r];
  }
  return 0;
}

// Shock-cylinder sensitivity: the initial condition is the post-shock state
// of a Mach-M normal shock (gas at rest (rho1, 0, 0, p1) ahead of it) for
// cell centres with x < xs and the pre-shock state elsewhere; an inflow
// boundary (if any) carries the post-shock state.  After nsteps RK3 steps of
// fixed dt, J = mean over fluid cells of (rho - target)^2.  Returns J and the
// exact derivatives dJ/dM, dJ/dgamma (forward mode), and the final state.
int orc_shock_tangent(const Config* c, const double* phi, int wall, double mach, double xs,
                      double rho1, double p1, int nsteps, double dt, const double* target_rho,
                      double* J, double* dJ, double* U_final) {
  if (!config_ok(c) || c->ndim != 2) return 1;
  using D = Dual<2>;
  Ibm ib = build_ibm(*c, phi, wall);
  D M(mach); M.d[0] = 1.0;
  D g(c->gamma); g.d[1] = 1.0;
  D post[3];
  rh_post_shock(M, g, rho1, p1, post);
  Params<D> P;
  P.gamma = g;
  P.inflow[0] = post[0]; P.inflow[1] = post[1]; P.inflow[2] = D(0.0); P.inflow[3] = post[2];
  Field<D> f(c->nx, c->ny);
  const double dx = dx_of(*c);
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->nx; ++i) {
      double x = c->x0 + (i + 0.5) * dx;
      D W[4], U[4];
      if (x < xs) { W[0] = post[0]; W[1] = post[1]; W[2] = D(0.0); W[3] = post[2]; }
      else { W[0] = D(rho1); W[1] = D(0.0); W[2] = D(0.0); W[3] = D(p1); }
      prim_to_cons(W, g, U);
      for (int v = 0; v < 4; ++v) f.at(v, i, j) = U[v];
    }
  for (int s = 0; s < nsteps; ++s) rk3_step(*c, P, ib, f, D(dt), nullptr, nullptr);
  D acc(0.0);
  long nf = 0;
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->nx; ++i) {
      if (ib.active && ib.cls[size_t(j) * c->nx + i] != FLUID) continue;
      D e = f.at(0, i, j) - target_rho[size_t(j) * c->nx + i];
      acc = acc + e * e;
      ++nf;
    }
  D Jd = acc / double(nf);
  *J = Jd.v; dJ[0] = Jd.d[0]; dJ[1] = Jd.d[1];
  if (U_final) {
    const size_t n = size_t(c->nx) * c->ny;
    for (int v = 0; v < 4; ++v)
      for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) U_final[v * n + size_t(j) * c->nx + i] = f.at(v, i, j).v;
  }
  return 0;
}

// Characteristic basis at the Roe average of two primitive states (face
// frame): L and R row-major 4 x 4.
void orc_char_basis(double gamma, const double* Wa, const double* Wb, double* L, double* R) {
  double Lm[4][4], Rm[4][4];
  char_basis(Wa, Wb, gamma, Lm, Rm);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) { L[i * 4 + j] = Lm[i][j]; R[i * 4 + j] = Rm[i][j]; }
}

// ------------------------------------------------------------ flux net
// Parameters in the order W0 [64][24], b0, W1 [64][64], b1, W2 [64][64], b2,
// W3 [4][64], b3 (10180 values).
void* orc_net_create(const float* params, const double* mean4, const double* inv_std4,
                     double out_scale, int emulate_bf16) {
  FluxNet* n = new (std::nothrow) FluxNet;
  if (!n) return nullptr;
  const float* p = params;
  auto take = [&](std::vector<double>& v, size_t k) { v.assign(p, p + k); p += k; };
  take(n->W0, NET_HID * NET_IN); take(n->b0, NET_HID);
  take(n->W1, NET_HID * NET_HID); take(n->b1, NET_HID);
  take(n->W2, NET_HID * NET_HID); take(n->b2, NET_HID);
  take(n->W3, NET_OUT * NET_HID); take(n->b3, NET_OUT);
  for (int k = 0; k < 4; ++k) { n->mean[k] = mean4[k]; n->inv_std[k] = inv_std4[k]; }
  n->out_scale = out_scale;
  n->emulate_bf16 = emulate_bf16 != 0;
  return static_cast<Correction*>(n);
}

void orc_net_destroy(void* n) { delete static_cast<FluxNet*>(static_cast<Correction*>(n)); }

int orc_net_param_count() {
  return NET_HID * NET_IN + NET_HID + 2 * (NET_HID * NET_HID + NET_HID) + NET_OUT * NET_HID + NET_OUT;
}

void orc_net_forward(const void* net, int nface, const double* st, double* dF) {
  for (int f = 0; f < nface; ++f) {
    double s[6][4];
    for (int a = 0; a < 6; ++a)
      for (int v = 0; v < 4; ++v) s[a][v] = st[(size_t(f) * 6 + a) * 4 + v];
    flux_net_apply(as_mlp(net), s, dF + size_t(f) * 4);
  }
}

void orc_net_backward(const void* net, int nface, const double* st, const double* dFbar, double* g,
                      double* dst) {
  for (int f = 0; f < nface; ++f) {
    double s[6][4], d[6][4];
    for (int a = 0; a < 6; ++a)
      for (int v = 0; v < 4; ++v) s[a][v] = st[(size_t(f) * 6 + a) * 4 + v];
    flux_net_backward(*as_mlp(net), s, dFbar + size_t(f) * 4, g, d);
    if (dst)
      for (int a = 0; a < 6; ++a)
        for (int v = 0; v < 4; ++v) dst[(size_t(f) * 6 + a) * 4 + v] = d[a][v];
  }
}

// ------------------------------------------------------- convolutional net
// Parameters in the order W1 [16][3][3][4], b1, W2 [32][3][3][16], b2,
// W3 [4][3][3][32], b3 (6388 values); mean4 / inv_std4 normalise the
// conservative face inputs.
void* orc_cnn_create(const float* params, const double* mean4, const double* inv_std4, double out_scale,
                     int emulate_bf16) {
  FluxCnn* n = new (std::nothrow) FluxCnn;
  if (!n) return nullptr;
  const float* p = params;
  auto take = [&](std::vector<double>& v, size_t k) { v.assign(p, p + k); p += k; };
  take(n->W1, 16 * 9 * 4); take(n->b1, 16);
  take(n->W2, 32 * 9 * 16); take(n->b2, 32);
  take(n->W3, 4 * 9 * 32); take(n->b3, 4);
  for (int k = 0; k < 4; ++k) { n->mean[k] = mean4[k]; n->inv_std[k] = inv_std4[k]; }
  n->out_scale = out_scale;
  n->emulate_bf16 = emulate_bf16 != 0;
  return static_cast<Correction*>(n);
}

void orc_cnn_destroy(void* n) { delete static_cast<FluxCnn*>(static_cast<Correction*>(n)); }

int orc_cnn_param_count() { return CNN_PARAMS; }

// The convolutional network's input images of state U (2D): Xx [ny][wx][4]
// and Xy [nx][wy][4] (y-faces transposed), normalised with net's map; wx is
// nx + 1, or nx when x is periodic (likewise wy).
int orc_cnn_images(const Config* c, const double* U, const double* phi, int wall, const void* net, double* Xx,
                   double* Xy) {
  if (!config_ok(c) || c->ndim != 2 || !net || as_net(net)->kind != CORR_CNN) return 1;
  Ibm ib = build_ibm(*c, phi, wall);
  Params<double> P = params_from<double>(*c);
  Field<double> f(c->nx, c->ny), L(c->nx, c->ny);
  load_state(*c, U, f);
  ibm_fill(*c, P, ib, f);
  std::vector<double> im[2];
  rhs(*c, P, ib, f, L, as_net(net), nullptr, im);
  std::copy(im[0].begin(), im[0].end(), Xx);
  std::copy(im[1].begin(), im[1].end(), Xy);
  return 0;
}

// One image [H][W][4] of normalised inputs -> corrections [H][W][4];
// wrap_r / wrap_c: the rows / columns are periodic.
void orc_cnn_forward(const void* net, int H, int W, int wrap_r, int wrap_c, const double* x, double* out) {
  std::vector<double> xv(x, x + size_t(H) * W * 4), o;
  const bool wrap[2] = {wrap_r != 0, wrap_c != 0};
  cnn_apply(*as_cnn(net), xv, H, W, wrap, o);
  std::copy(o.begin(), o.end(), out);
}

// Reverse of one image: g += parameter gradient, dx = input gradient.
void orc_cnn_backward(const void* net, int H, int W, int wrap_r, int wrap_c, const double* x, const double* dOut,
                      double* g, double* dx) {
  std::vector<double> xv(x, x + size_t(H) * W * 4), dv(dOut, dOut + size_t(H) * W * 4), d;
  const bool wrap[2] = {wrap_r != 0, wrap_c != 0};
  cnn_backward(*as_cnn(net), xv, H, W, wrap, dv, g, d);
  if (dx) std::copy(d.begin(), d.end(), dx);
}

// ------------------------------------------------------------ training
// Restriction d(U), unrolled-loss term and Adam step (training.hpp).
int orc_restrict(const double* fine, int nx_f, int ny_f, int factor, int nvar, int nbatch, double* coarse) {
  if (!fine || !coarse || factor < 1 || nx_f % factor || ny_f % factor || nvar < 1 || nbatch < 1) return 1;
  restrict_blocks(fine, nx_f, ny_f, factor, nvar, nbatch, coarse);
  return 0;
}

int orc_mse(const double* U, const double* T, long long per_batch, int nbatch, double scale, double* loss,
            double* G) {
  if (!U || !T || !loss || per_batch < 1 || nbatch < 1) return 1;
  mse_term(U, T, per_batch, nbatch, scale, loss, G);
  return 0;
}

int orc_adam(double* theta, const double* g, double* m, double* v, int n, double lr, double b1, double b2,
             double eps, int step) {
  if (!theta || !g || !m || !v || n < 1 || step < 1) return 1;
  adam_step(theta, g, m, v, n, lr, b1, b2, eps, step);
  return 0;
}

}  // extern "C"
