// Ghost-cell immersed boundary on gfx950: classification of the cells of a
// signed-distance level set, a deterministic (row-major) ghost list, the
// per-ghost image-point table and the per-stage ghost refill.
//
// Section 2 adopts the ghost-cell method of Mittal & Iaccarino with a slip
// wall and fluid / solid / ghost / image classes.  Here: fluid phi >= 0,
// solid phi < 0, ghost = solid with a fluid cell within 3 cells along +-x or
// +-y (the reach of the WENO5 stencil).  The image point of a ghost G is
// x_G + 2|phi_G| n with n = grad phi/|grad phi| (central differences), i.e.
// the mirror image across the wall; the fluid state there is interpolated
// bilinearly from the enclosing cell centres that are fluid (weights
// renormalised).  The ghost takes the image density and pressure and the
// reflected normal velocity (slip) or the reversed velocity (no-slip
// adiabatic).  Geometry arithmetic is done in double without contraction so
// that the table is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>

#include "grid.hpp"
#include "ibm_dev.hpp"

namespace shk {

__global__ void __launch_bounds__(256) ibm_classify_kernel(GridArgs a, const double* __restrict__ phi,
                                                           uint8_t* __restrict__ cls, int* __restrict__ row_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= a.nx) return;
  const int nx = a.nx, ny = a.ny;
  const double* row = phi + (long long)j * nx;
  uint8_t c = CELL_FLUID;
  if (!(row[i] >= 0.0)) {
    bool near = false;
    for (int k = 1; k <= HALO; ++k) {
      if (i - k >= 0 && row[i - k] >= 0.0) near = true;
      if (i + k < nx && row[i + k] >= 0.0) near = true;
      if (j - k >= 0 && phi[(long long)(j - k) * nx + i] >= 0.0) near = true;
      if (j + k < ny && phi[(long long)(j + k) * nx + i] >= 0.0) near = true;
    }
    c = near ? CELL_GHOST : CELL_SOLID;
  }
  cls[(long long)j * nx + i] = c;
  if (c == CELL_GHOST) atomicAdd(&row_count[j], 1);
}

// Exclusive prefix sum of the per-row ghost counts (single workgroup; the
// row count is the grid height).  row_off has ny + 1 entries.
__global__ void __launch_bounds__(1024) ibm_scan_kernel(const int* __restrict__ row_count,
                                                        int* __restrict__ row_off, int ny) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (ny + 1023) / 1024;
  const int lo = t * per, hi = min(lo + per, ny);
  int s = 0;
  for (int r = lo; r < hi; ++r) s += row_count[r];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;  // exclusive
  for (int r = lo; r < hi; ++r) {
    row_off[r] = run;
    run += row_count[r];
  }
  if (t == 1023) row_off[ny] = part[1023];
}

// One workgroup (one wave) per row: ghosts get consecutive slots in
// increasing x, then each fills its table entry.
// A ghost whose image point is undefined -- the central-difference gradient
// of the signed distance is far from unit length (|grad phi| < 1/2: the
// difference straddles the solid's medial axis, as in a solid thinner than
// about two cells or a body a few cells across), or no fluid cell is found
// around the image point or along the normal -- is counted in *nbad.
__global__ void __launch_bounds__(64) ibm_table_kernel(GridArgs a, const double* __restrict__ phi,
                                                       const uint8_t* __restrict__ cls,
                                                       const int* __restrict__ row_off, GhostTable gt,
                                                       int* __restrict__ nbad) {
#pragma clang fp contract(off)
  const int j = blockIdx.x;
  const int nx = a.nx, ny = a.ny;
  const double dx = a.dx, dy = a.dy;
  int base = row_off[j];
  for (int i0 = 0; i0 < nx; i0 += 64) {
    const int i = i0 + (int)threadIdx.x;
    const bool g = i < nx && cls[(long long)j * nx + i] == CELL_GHOST;
    const unsigned long long m = __ballot(g);
    const int rank = __popcll(m & ((1ull << threadIdx.x) - 1ull));
    if (g) {
      const int slot = base + rank;
      auto P = [&](int ii, int jj) { return phi[(long long)jj * nx + ii]; };
      const int il = max(i - 1, 0), ir = min(i + 1, nx - 1);
      const int jl = max(j - 1, 0), jr = min(j + 1, ny - 1);
      const double gx = (P(ir, j) - P(il, j)) / ((ir - il) * dx);
      const double gy = (P(i, jr) - P(i, jl)) / ((jr - jl) * dy);
      const double gn = sqrt(gx * gx + gy * gy);
      const double nxv = gx / gn, nyv = gy / gn;
      const double xg = a.x0 + (i + 0.5) * dx;
      const double yg = a.y0 + (j + 0.5) * dy;
      const double dist = 2.0 * fabs(P(i, j));
      const double xi = xg + dist * nxv, yi = yg + dist * nyv;
      const double fx = (xi - a.x0) / dx - 0.5, fy = (yi - a.y0) / dy - 0.5;
      const int ci0 = (int)floor(fx), cj0 = (int)floor(fy);
      const double tx = fx - ci0, ty = fy - cj0;
      const double wb[4] = {(1.0 - tx) * (1.0 - ty), tx * (1.0 - ty), (1.0 - tx) * ty, tx * ty};
      const int ci[4] = {ci0, ci0 + 1, ci0, ci0 + 1}, cj[4] = {cj0, cj0, cj0 + 1, cj0 + 1};
      int src[4];
      double w[4];
      double wsum = 0.0;
      for (int k = 0; k < 4; ++k) {
        src[k] = -1;
        w[k] = 0.0;
        if (ci[k] < 0 || ci[k] >= nx || cj[k] < 0 || cj[k] >= ny) continue;
        if (!(P(ci[k], cj[k]) >= 0.0)) continue;
        src[k] = cj[k] * nx + ci[k];
        w[k] = wb[k];
        wsum += wb[k];
      }
      if (wsum > 0.0) {
        for (int k = 0; k < 4; ++k) w[k] = w[k] / wsum;
      } else {
        for (int k = 0; k < 4; ++k) { src[k] = -1; w[k] = 0.0; }
        const double h = 0.5 * fmin(dx, dy);
        for (int m2 = 0; m2 < 64; ++m2) {
          const double s = fabs(P(i, j)) + m2 * h;
          const double xs = xg + s * nxv, ys = yg + s * nyv;
          const int is = (int)floor((xs - a.x0) / dx), js = (int)floor((ys - a.y0) / dy);
          if (is < 0 || is >= nx || js < 0 || js >= ny) break;
          if (P(is, js) >= 0.0) { src[0] = js * nx + is; w[0] = 1.0; break; }
        }
      }
      bool resolved = false;
      for (int k = 0; k < 4; ++k) resolved = resolved || src[k] >= 0;
      if (!(gn >= 0.5) || !resolved) atomicAdd(nbad, 1);
      gt.cell[slot] = j * nx + i;
      for (int k = 0; k < 4; ++k) { gt.src[4 * slot + k] = src[k]; gt.w[4 * slot + k] = w[k]; }
      gt.nrm[2 * slot] = nxv;
      gt.nrm[2 * slot + 1] = nyv;
    }
    base += __popcll(m);
  }
}

// Per-stage refill: one thread per ghost (per batch member).  Sources are
// fluid cells only, so no ghost reads another ghost's new value.
template <class S>
__global__ void __launch_bounds__(256) ibm_fill_kernel(GridArgs a, GhostTable gt, S* __restrict__ U) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= gt.n) return;
  const long long n = a.ncell;
  S* Ub = U + (long long)blockIdx.y * 4 * n;
  double q[4];
  ghost_cons(gt, a.gamma, k, [&](int e, long long c) { return double(Ub[e * n + c]); }, q);
  const int c = gt.cell[k];
  for (int e = 0; e < 4; ++e) Ub[e * n + c] = S(q[e]);
}

hipError_t launch_ibm_classify(const GridArgs& a, const double* phi, uint8_t* cls, int* row_count,
                               hipStream_t st) {
  hipLaunchKernelGGL(ibm_classify_kernel, dim3((a.nx + 255) / 256, a.ny), dim3(256), 0, st, a, phi, cls,
                     row_count);
  return hipGetLastError();
}

hipError_t launch_ibm_table(const GridArgs& a, const double* phi, const uint8_t* cls, const int* row_count,
                            int* row_off, GhostTable gt, int* nbad, hipStream_t st) {
  hipLaunchKernelGGL(ibm_scan_kernel, dim3(1), dim3(1024), 0, st, row_count, row_off, a.ny);
  hipLaunchKernelGGL(ibm_table_kernel, dim3(a.ny), dim3(64), 0, st, a, phi, cls, row_off, gt, nbad);
  return hipGetLastError();
}

template <class S>
hipError_t launch_ibm_fill(const GridArgs& a, const GhostTable& gt, S* U, hipStream_t st) {
  if (gt.n == 0) return hipSuccess;
  hipLaunchKernelGGL(ibm_fill_kernel<S>, dim3((gt.n + 255) / 256, a.nbatch), dim3(256), 0, st, a, gt, U);
  return hipGetLastError();
}

template hipError_t launch_ibm_fill<double>(const GridArgs&, const GhostTable&, double*, hipStream_t);
template hipError_t launch_ibm_fill<float>(const GridArgs&, const GhostTable&, float*, hipStream_t);

}  // namespace shk
