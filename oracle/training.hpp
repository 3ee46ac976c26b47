// Oracle: the training pieces of the learned correction (TEST INFRASTRUCTURE
// ONLY).
//
// Section 2 trains the neural flux against data produced by the solver at a
// higher resolution:
//   - the restriction d(U) maps a fine state onto the coarse grid; on a
//     uniform grid whose coarse cells are unions of factor x factor fine
//     cells, the finite-volume restriction is the mean of the fine cell
//     averages a coarse cell contains;
//   - the loss is the mean squared difference between the coarse solver's
//     state after each of the m unrolled steps and the restricted fine state
//     at the same time (the unrolled loss equation); per batch member this
//     oracle returns one term ||U - T||^2 / N (N entries) and its gradient
//     2 (U - T) / N, times a caller scale;
//   - the parameters follow the Adam rule (Kingma & Ba, as cited in section
//     3): first and second moment estimates with bias correction.
// Everything is double precision and summed in index order.
#pragma once
#include <cmath>
#include <cstddef>

namespace orc {

// coarse[b][v][J][I] = mean over the factor x factor fine cells of block
// (I, J) of fine[b][v][.][.]; nx_f, ny_f multiples of factor.
inline void restrict_blocks(const double* fine, int nx_f, int ny_f, int factor, int nvar, int nbatch,
                            double* coarse) {
  const int nx_c = nx_f / factor, ny_c = ny_f / factor;
  for (int p = 0; p < nbatch * nvar; ++p) {
    const double* F = fine + size_t(p) * nx_f * ny_f;
    double* C = coarse + size_t(p) * nx_c * ny_c;
    for (int J = 0; J < ny_c; ++J)
      for (int I = 0; I < nx_c; ++I) {
        double s = 0.0;
        for (int jj = 0; jj < factor; ++jj)
          for (int ii = 0; ii < factor; ++ii) s += F[size_t(J * factor + jj) * nx_f + size_t(I * factor + ii)];
        C[size_t(J) * nx_c + I] = s / double(factor * factor);
      }
  }
}

// loss[b] += sum_k (U_bk - T_bk)^2 / N; if G: G_bk += scale * 2 (U_bk - T_bk) / N,
// N = per_batch entries of member b.
inline void mse_term(const double* U, const double* T, long long per_batch, int nbatch, double scale, double* loss,
                     double* G) {
  for (int b = 0; b < nbatch; ++b) {
    const size_t o = size_t(b) * size_t(per_batch);
    double s = 0.0;
    for (long long k = 0; k < per_batch; ++k) {
      const double d = U[o + k] - T[o + k];
      s += d * d;
      if (G) G[o + k] += scale * (2.0 * d / double(per_batch));
    }
    loss[b] += s / double(per_batch);
  }
}

// One Adam step (step counts from 1): m <- b1 m + (1-b1) g, v <- b2 v +
// (1-b2) g^2, theta <- theta - lr mhat / (sqrt(vhat) + eps) with mhat =
// m / (1 - b1^step), vhat = v / (1 - b2^step).
inline void adam_step(double* theta, const double* g, double* m, double* v, int n, double lr, double b1, double b2,
                      double eps, int step) {
  const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
  for (int k = 0; k < n; ++k) {
    m[k] = b1 * m[k] + (1.0 - b1) * g[k];
    v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    const double mh = m[k] / c1, vh = v[k] / c2;
    theta[k] = theta[k] - lr * mh / (std::sqrt(vh) + eps);
  }
}

}  // namespace orc
