// Oracle: exact solution of the 1D Riemann problem for the ideal-gas Euler
// equations (TEST INFRASTRUCTURE ONLY).  The Sod problem of section 3 is
// compared with this exact solution; the star pressure is the root of the
// standard pressure function f_L(p) + f_R(p) + (u_R - u_L) = 0 (shock branch
// from the Rankine-Hugoniot conditions, rarefaction branch from the isentropic
// relations), found by Newton's method, and the self-similar solution is then
// sampled at x/t.
#pragma once
#include <cmath>

namespace orc {

using std::sqrt;

struct RiemannStar {
  double p, u, rhoL, rhoR;
  int iterations;
};

// Pressure function of one side and its derivative.
inline void pressure_fn(double p, double rk, double pk, double g, double* f, double* df) {
  double ak = std::sqrt(g * pk / rk);
  if (p > pk) {  // shock
    double A = 2.0 / ((g + 1.0) * rk), B = (g - 1.0) / (g + 1.0) * pk;
    double q = std::sqrt(A / (p + B));
    *f = (p - pk) * q;
    *df = q * (1.0 - 0.5 * (p - pk) / (p + B));
  } else {       // rarefaction
    double e = (g - 1.0) / (2.0 * g);
    *f = 2.0 * ak / (g - 1.0) * (std::pow(p / pk, e) - 1.0);
    *df = 1.0 / (rk * ak) * std::pow(p / pk, -(g + 1.0) / (2.0 * g));
  }
}

inline RiemannStar riemann_star(double rl, double ul, double pl, double rr, double ur, double pr,
                                double g) {
  RiemannStar s{};
  double p = 0.5 * (pl + pr);
  int it = 0;
  for (; it < 200; ++it) {
    double fl, dfl, fr, dfr;
    pressure_fn(p, rl, pl, g, &fl, &dfl);
    pressure_fn(p, rr, pr, g, &fr, &dfr);
    double pn = p - (fl + fr + (ur - ul)) / (dfl + dfr);
    if (pn < 1e-14) pn = 1e-14;
    double change = std::fabs(pn - p) / (0.5 * (pn + p));
    p = pn;
    if (change < 1e-15) break;
  }
  double fl, dfl, fr, dfr;
  pressure_fn(p, rl, pl, g, &fl, &dfl);
  pressure_fn(p, rr, pr, g, &fr, &dfr);
  s.p = p;
  s.u = 0.5 * (ul + ur) + 0.5 * (fr - fl);
  double gm = (g - 1.0) / (g + 1.0);
  s.rhoL = p > pl ? rl * (p / pl + gm) / (gm * p / pl + 1.0) : rl * std::pow(p / pl, 1.0 / g);
  s.rhoR = p > pr ? rr * (p / pr + gm) / (gm * p / pr + 1.0) : rr * std::pow(p / pr, 1.0 / g);
  s.iterations = it + 1;
  return s;
}

// Sample the self-similar solution at S = x/t; returns (rho, u, p).
inline void riemann_sample(double rl, double ul, double pl, double rr, double ur, double pr,
                           double g, const RiemannStar& st, double S, double out[3]) {
  double al = std::sqrt(g * pl / rl), ar = std::sqrt(g * pr / rr);
  double r, u, p;
  if (S <= st.u) {  // left of the contact
    if (st.p > pl) {
      double sl = ul - al * std::sqrt((g + 1.0) / (2.0 * g) * st.p / pl + (g - 1.0) / (2.0 * g));
      if (S <= sl) { r = rl; u = ul; p = pl; }
      else { r = st.rhoL; u = st.u; p = st.p; }
    } else {
      double ast = al * std::pow(st.p / pl, (g - 1.0) / (2.0 * g));
      double head = ul - al, tail = st.u - ast;
      if (S <= head) { r = rl; u = ul; p = pl; }
      else if (S >= tail) { r = st.rhoL; u = st.u; p = st.p; }
      else {
        double c = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * al) * (ul - S);
        r = rl * std::pow(c, 2.0 / (g - 1.0));
        u = 2.0 / (g + 1.0) * (al + (g - 1.0) / 2.0 * ul + S);
        p = pl * std::pow(c, 2.0 * g / (g - 1.0));
      }
    }
  } else {          // right of the contact
    if (st.p > pr) {
      double sr = ur + ar * std::sqrt((g + 1.0) / (2.0 * g) * st.p / pr + (g - 1.0) / (2.0 * g));
      if (S >= sr) { r = rr; u = ur; p = pr; }
      else { r = st.rhoR; u = st.u; p = st.p; }
    } else {
      double ast = ar * std::pow(st.p / pr, (g - 1.0) / (2.0 * g));
      double head = ur + ar, tail = st.u + ast;
      if (S >= head) { r = rr; u = ur; p = pr; }
      else if (S <= tail) { r = st.rhoR; u = st.u; p = st.p; }
      else {
        double c = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * ar) * (ur - S);
        r = rr * std::pow(c, 2.0 / (g - 1.0));
        u = 2.0 / (g + 1.0) * (-ar + (g - 1.0) / 2.0 * ur + S);
        p = pr * std::pow(c, 2.0 * g / (g - 1.0));
      }
    }
  }
  out[0] = r; out[1] = u; out[2] = p;
}

// Post-shock state behind a normal shock of Mach number M moving into gas
// at rest with (rho1, p1): density and pressure ratios of the normal-shock
// relations and the induced gas velocity M a1 (1 - rho1/rho2).  With
// (rho1, p1) = (1.4, 1) and M = 5 this is the left state of the paper's
// shock-cylinder initial condition.
template <class T>
void rh_post_shock(const T& M, const T& g, double rho1, double p1, T out[3]) {
  T a1 = sqrt(g * p1 / rho1);
  T M2 = M * M;
  T rho2 = rho1 * ((g + 1.0) * M2) / ((g - 1.0) * M2 + 2.0);
  T p2 = p1 * (1.0 + 2.0 * g / (g + 1.0) * (M2 - 1.0));
  T u2 = M * a1 * (1.0 - rho1 / rho2);
  out[0] = rho2; out[1] = u2; out[2] = p2;
}

}  // namespace orc
