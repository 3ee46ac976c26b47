// Device form of the immersed-boundary ghost value, shared by the refill
// kernel and the stage kernels' tile loads so that both give the same bits.
//
// Section 2's ghost-cell method (Mittal & Iaccarino): the primitive state at
// the ghost's image point is interpolated from the fluid cells of its table
// entry (bilinear weights renormalised over fluid cells, or the nearest fluid
// cell along the normal), then the wall rule sets the ghost's velocity:
// slip reflects the normal component, no-slip adiabatic reverses the whole
// velocity; density and pressure are the image point's.
#pragma once
#include <hip/hip_runtime.h>

#include "grid.hpp"

namespace shk {

// Conservative value q of ghost k from a state whose conservative plane e of
// interior cell c is get(e, c) (a double).  Evaluated in double with the
// divisions as IEEE quotients.
template <class Get>
__device__ __forceinline__ void ghost_cons(const GhostTable& gt, double gamma, int k, Get&& get, double q[4]) {
  const double gm1 = gamma - 1.0;
  double Wi[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int s = gt.src[4 * k + m];
    if (s < 0) continue;
    const double wm = gt.w[4 * k + m];
    const double r = get(0, s);
    const double u = get(1, s) / r;
    const double v = get(2, s) / r;
    const double p = gm1 * (get(3, s) - 0.5 * r * (u * u + v * v));
    Wi[0] = Wi[0] + wm * r;
    Wi[1] = Wi[1] + wm * u;
    Wi[2] = Wi[2] + wm * v;
    Wi[3] = Wi[3] + wm * p;
  }
  double ug, vg;
  if (gt.wall == 0) {
    const double nx = gt.nrm[2 * k], ny = gt.nrm[2 * k + 1];
    const double un = Wi[1] * nx + Wi[2] * ny;
    ug = Wi[1] - 2.0 * un * nx;
    vg = Wi[2] - 2.0 * un * ny;
  } else {
    ug = -Wi[1];
    vg = -Wi[2];
  }
  q[0] = Wi[0];
  q[1] = Wi[0] * ug;
  q[2] = Wi[0] * vg;
  q[3] = Wi[3] / gm1 + 0.5 * Wi[0] * (ug * ug + vg * vg);
}

}  // namespace shk
