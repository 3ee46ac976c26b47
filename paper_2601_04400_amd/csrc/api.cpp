// Host side of the C ABI declared in include/shk.h: argument validation,
// workspace carving and kernel sequencing on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/shk.h"
#include "cnn.hpp"
#include "grid.hpp"
#include "mlp.hpp"

using namespace shk;

// Host arithmetic here (inflow state, normal-shock relations) is evaluated as
// written, without contraction into fused multiply-adds.
#pragma clang fp contract(off)

struct WsLayout {
  size_t scalars, globals, dtbuf, xslots, u1, u2, cls, row_count, row_off, g_cell, g_src, g_w, g_nrm;
  size_t adjA, adjB, adjC, adjP, adjQ, adjPart, part_stride, adjG, ghostOf, entKeys, entVals, entCount, entHeads;
  size_t netX, netPart, cnnDF, cnnBufs, vjpPart, tileBody, tileOrder;
  size_t total;
};

struct shk_grid {
  shk_grid_desc d;
  GridArgs a;
  hipStream_t st;
  char* ws;
  size_t ws_bytes;
  WsLayout L;
  size_t esize;
  GhostTable gt;
  bool ibm_on;
  int nent = 0;  // valid (ghost, source) entries of the refill transpose
  int nsrc = 0;  // distinct source cells among them
  int fill_m = 0;  // most entries of one source (the fill table's slots per source)
  NetArgs net{};
  bool net_on = false;
  CnnArgs cnn{};
  bool cnn_on = false;
  float* net_grad = nullptr;  // parameter gradient of whichever network is set
  std::string err;
  // kernel timing (shk_profile)
  bool prof = false;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  ~shk_grid() {
    for (auto& r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

namespace {

inline size_t al(size_t x) { return (x + 255) & ~size_t(255); }

bool desc_ok(const shk_grid_desc* d, std::string* why) {
  auto bad = [&](const char* m) { if (why) *why = m; return false; };
  if (!d) return bad("null descriptor");
  if (d->ndim != 1 && d->ndim != 2) return bad("ndim must be 1 or 2");
  if (d->nx < 1 || d->ny < 1 || d->nbatch < 1) return bad("nx, ny, nbatch must be >= 1");
  if (d->ndim == 1 && d->ny != 1) return bad("ndim 1 requires ny == 1");
  if (d->nx < 3 || (d->ndim == 2 && d->ny < 3))
    return bad("nx (and ny in 2D) must be >= 3: the boundary ghost layers are three interior cells deep");
  if (d->nx > (1 << 26) || d->ny > (1 << 26)) return bad("grid too large");
  if ((long long)d->nx * d->ny * d->nbatch * 4 > (1LL << 40)) return bad("grid too large");
  if (d->prec < 0 || d->prec > 2) return bad("prec must be SHK_F64, SHK_F32 or SHK_MIXED");
  if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) return bad("gamma must be > 1");
  if (!(d->x1 > d->x0)) return bad("x1 must exceed x0");
  if (d->ndim == 2 && !(d->y1 > d->y0)) return bad("y1 must exceed y0");
  if (!(d->cfl > 0.0)) return bad("cfl must be > 0");
  for (int k = 0; k < 4; ++k)
    if (d->bc[k] < 0 || d->bc[k] > 3) return bad("unknown boundary condition");
  if ((d->bc[0] == SHK_BC_PERIODIC) != (d->bc[1] == SHK_BC_PERIODIC)) return bad("periodic x needs both sides");
  if (d->ndim == 2 && (d->bc[2] == SHK_BC_PERIODIC) != (d->bc[3] == SHK_BC_PERIODIC))
    return bad("periodic y needs both sides");
  if (d->viscous && d->ndim != 2) return bad("viscous terms need ndim 2");
  if (d->viscous && (!(d->mu >= 0.0) || !(d->prandtl > 0.0))) return bad("viscous needs mu >= 0, prandtl > 0");
  if (d->ibm && d->ndim != 2) return bad("immersed boundary needs ndim 2");
  if (d->flux_net < 0 || d->flux_net > 2) return bad("flux_net must be 0, 1 or 2");
  if (d->flux_net && (d->ndim != 2 || d->prec != SHK_F64 || d->viscous))
    return bad("flux net needs ndim 2, SHK_F64 and an inviscid grid");
  if (d->flux_net == 2 && (d->nx > 16384 || d->ny > 16384)) return bad("convolutional net: nx, ny <= 16384");
  if (d->nu_art < 0.0) return bad("nu_art must be >= 0");
  if (d->weno_char != 0 && d->weno_char != 1) return bad("weno_char must be 0 or 1");
  if (d->weno_char && (d->prec != SHK_F64 || d->flux_net || d->adjoint))
    return bad("characteristic WENO: SHK_F64, without learned correction or adjoint");
  return true;
}

size_t elem_size(const shk_grid_desc* d) { return d->prec == SHK_F64 ? 8 : 4; }

WsLayout layout(const shk_grid_desc* d) {
  WsLayout L{};
  const size_t ncell = size_t(d->nx) * d->ny;
  const int nvar = d->ndim == 1 ? 3 : 4;
  const size_t state = size_t(d->nbatch) * nvar * ncell * elem_size(d);
  size_t o = 0;
  L.scalars = o; o += al(sizeof(StepScalars) * d->nbatch);
  L.globals = o; o += al(sizeof(Globals));
  L.dtbuf = o; o += al(sizeof(double) * d->nbatch);
  L.xslots = o; o += al(sizeof(unsigned long long) * 2 * XSLOTS * d->nbatch);
  L.u1 = o; o += al(state);
  L.u2 = o; o += al(state);
  L.vjpPart = o; o += al(sizeof(double) * VJP_BLOCKS * d->nbatch);
  if (d->ibm) {
    const size_t cap = ncell;
    L.cls = o; o += al(ncell);
    L.row_count = o; o += al(sizeof(int) * (d->ny + 1));
    L.row_off = o; o += al(sizeof(int) * (d->ny + 1));
    L.g_cell = o; o += al(sizeof(int) * cap);
    L.g_src = o; o += al(sizeof(int) * 4 * cap);
    L.g_w = o; o += al(sizeof(double) * 4 * cap);
    L.g_nrm = o; o += al(sizeof(double) * 2 * cap);
    L.ghostOf = o; o += al(sizeof(int) * ncell);
    L.tileBody = o; o += al(size_t(stage_tiles(d->nx, d->ny)));
    L.tileOrder = o; o += al(sizeof(unsigned) * size_t(stage_tiles(d->nx, d->ny)));
  }
  if (d->adjoint) {
    const size_t st64 = al(size_t(d->nbatch) * 4 * ncell * sizeof(double));
    L.adjA = o; o += st64;
    L.adjB = o; o += st64;
    L.adjC = o; o += st64;
    L.adjP = o; o += st64;
    L.adjQ = o; o += st64;
    const size_t nblk = size_t((d->nx + ADJ_TX - 1) / ADJ_TX) * ((d->ny + ADJ_TY - 1) / ADJ_TY);
    L.part_stride = 5 * size_t(d->nbatch) * nblk;
    L.adjPart = o; o += al(sizeof(double) * MAX_PART_SLOTS * L.part_stride);
    if (d->ibm) {
      L.adjG = o; o += st64;  // image-point primitive adjoints, 4 per ghost
      L.entKeys = o; o += al(sizeof(int) * 4 * ncell);
      L.entVals = o; o += al(sizeof(int) * 4 * ncell);
      L.entCount = o; o += al(sizeof(int));
      L.entHeads = o; o += al(sizeof(int) * (4 * ncell + 1));
    }
  }
  if (d->flux_net) {
    const size_t nface = size_t(d->nx + 1) * d->ny + size_t(d->nx) * (d->ny + 1);
    if (d->adjoint) {
      L.netX = o; o += al(sizeof(float) * 24 * nface * d->nbatch);
      L.netPart = o; o += al(sizeof(float) * NET_NP * NET_BWD_BLOCKS);
    }
    if (d->flux_net == 2) {
      GridArgs a{};
      a.nx = d->nx; a.ny = d->ny; a.nbatch = d->nbatch;
      for (int k = 0; k < 4; ++k) a.bc[k] = d->bc[k];
      L.cnnDF = o; o += al(sizeof(float) * 4 * nface * d->nbatch);
      L.cnnBufs = o; o += al(cnn_workspace_bytes(a));
    }
  }
  L.total = o;
  return L;
}

// gamma-dependent arguments: gamma, conductivity, conservative inflow state.
static void set_physics(const shk_grid_desc& d, GridArgs& a) {
  a.gamma = d.gamma;
  a.kappa = d.viscous ? d.mu * d.gamma / ((d.gamma - 1.0) * a.prandtl) : 0.0;
  const double* w = d.inflow_prim;
  const double v = d.ndim == 2 ? w[2] : 0.0;
  a.inflow_cons[0] = w[0];
  a.inflow_cons[1] = w[0] * w[1];
  a.inflow_cons[2] = w[0] * v;
  a.inflow_cons[3] = w[3] / (d.gamma - 1.0) + 0.5 * w[0] * (w[1] * w[1] + v * v);
}

shk_status fail(shk_grid* g, shk_status s, const std::string& m) {
  if (g) g->err = m;
  return s;
}

shk_status hip_check(shk_grid* g, hipError_t e, const char* where) {
  if (e == hipSuccess) return SHK_OK;
  return fail(g, SHK_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

hipEvent_t take_event(shk_grid* g) {
  if (!g->pool.empty()) { hipEvent_t e = g->pool.back(); g->pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run f() between two events recorded on the grid's stream when profiling.
template <class F>
hipError_t timed(shk_grid* g, int cls, F&& f) {
  if (!g->prof) return f();
  hipEvent_t a = take_event(g), b = take_event(g);
  if (!a || !b) return f();
  (void)hipEventRecord(a, g->st);
  hipError_t e = f();
  (void)hipEventRecord(b, g->st);
  g->recs.push_back({cls, a, b});
  return e;
}

// Stage launch; with the per-face network on, the kernel variant that
// evaluates it inside its tile; with the convolutional network on, the
// network over the face images of Us first and the variant that adds its
// per-face output (FP64 grids only).
template <class S>
hipError_t stage_launch(shk_grid* g, const GridArgs& a, int mode, const S* Us, const S* Un, S* Uo,
                        const double* dtp, const S* Lin) {
  if (g->cnn_on) {
    GridArgs ax = a;
    ax.dFext = reinterpret_cast<float*>(g->ws + g->L.cnnDF);
    hipError_t e = launch_cnn_forward(ax, g->cnn, reinterpret_cast<const double*>(Us),
                                      const_cast<float*>(ax.dFext), cnn_bufs(ax, g->ws + g->L.cnnBufs), false,
                                      g->st);
    if (e != hipSuccess) return e;
    return launch_stage_ext(ax, mode, reinterpret_cast<const double*>(Us), reinterpret_cast<const double*>(Un),
                            reinterpret_cast<double*>(Uo), dtp, g->st);
  }
  if (g->net_on)
    return launch_stage_net(a, g->net, mode, reinterpret_cast<const double*>(Us),
                            reinterpret_cast<const double*>(Un), reinterpret_cast<double*>(Uo), dtp, g->st);
  if (g->d.prec == SHK_MIXED)
    return launch_stage_mixed(a, mode, reinterpret_cast<const float*>(Us), reinterpret_cast<const float*>(Un),
                              reinterpret_cast<float*>(Uo), dtp, reinterpret_cast<const float*>(Lin), g->st);
  return launch_stage<S>(a, mode, Us, Un, Uo, dtp, Lin, g->st);
}

// One SSP-RK3 step.  Without a fixed step, a tape or a learned correction
// the automatic step is fused into the stages (S1L, S2F, S3F); otherwise the
// stages are the plain three (after a separate reduction for the automatic
// step).  With an immersed boundary the stage kernels form the refilled
// ghost values of their stage state while loading their tiles; the refilled
// ghosts of U^n are stored back into U (stage 3 combines them, as the step's
// definition does), and with a tape each stage state's refilled ghosts are
// stored in the tape.  The convolutional network reads the stage states
// itself, so with it the ghosts are refilled by separate launches first.
// With tape != nullptr the stage-start states (U^n, U1, U2, each after the
// refill) are kept in tape[0..2] for the reverse pass.
template <class S>
shk_status stage_seq(shk_grid* g, S* U, const double* dt_in, double* dt_out, S* tape = nullptr) {
  GridArgs a = g->a;
  a.dt_out = dt_out;
  const long long nst = (long long)a.nbatch * a.nvar * a.ncell;
  S* U1 = tape ? tape + nst : reinterpret_cast<S*>(g->ws + g->L.u1);
  S* U2 = tape ? tape + 2 * nst : reinterpret_cast<S*>(g->ws + g->L.u2);
  hipError_t e;
  if (!dt_in && !g->net_on && !g->cnn_on && !tape) {
    a.ghost_back = g->ibm_on ? U : nullptr;  // refilled ghosts of U^n, read back by S2F and S3F
    if ((e = timed(g, 1, [&]() { return stage_launch<S>(g, a, MODE_S1L, U, U, U1, nullptr, nullptr); })) != hipSuccess)
      return hip_check(g, e, "stage 1");
    a.ghost_back = nullptr;  // S2F's stage state U1 is never stored
    if ((e = timed(g, 2, [&]() { return stage_launch<S>(g, a, MODE_S2F, U, U, U2, nullptr, U1); })) != hipSuccess)
      return hip_check(g, e, "stage 2");
    a.ghost_back = g->ibm_on ? U2 : nullptr;  // refilled ghosts of U2 (a work array), read back by S3F's update
    if ((e = timed(g, 3, [&]() { return stage_launch<S>(g, a, MODE_S3F, U2, U, U, nullptr, nullptr); })) != hipSuccess)
      return hip_check(g, e, "stage 3");
    return SHK_OK;
  }
  const double* dtp = dt_in;
  if (!dt_in) {
    e = timed(g, 0, [&]() { return launch_cfl<S>(a, U, dt_out, g->st); });
    if (e != hipSuccess) return hip_check(g, e, "cfl");
    dtp = a.dtbuf;
  }
  auto stage = [&](int mode, const S* Us, const S* Un, S* Uo) -> hipError_t {
    a.ghost_back = g->ibm_on ? const_cast<S*>(Us) : nullptr;
    return timed(g, mode, [&]() { return stage_launch<S>(g, a, mode, Us, Un, Uo, dtp, nullptr); });
  };
  auto fill = [&](S* X) -> hipError_t {
    if (!g->ibm_on || !g->cnn_on) return hipSuccess;
    return timed(g, 4, [&]() { return launch_ibm_fill<S>(a, g->gt, X, g->st); });
  };
  if ((e = fill(U)) != hipSuccess) return hip_check(g, e, "ibm fill");
  a.stage_in_copy = tape;  // stage 1 writes the refilled U^n to tape[0] as it reads it
  if ((e = stage(MODE_STAGE1, U, U, U1)) != hipSuccess) return hip_check(g, e, "stage 1");
  a.stage_in_copy = nullptr;
  if ((e = fill(U1)) != hipSuccess) return hip_check(g, e, "ibm fill");
  if ((e = stage(MODE_STAGE2, U1, U, U2)) != hipSuccess) return hip_check(g, e, "stage 2");
  if ((e = fill(U2)) != hipSuccess) return hip_check(g, e, "ibm fill");
  if ((e = stage(MODE_STAGE3, U2, U, U)) != hipSuccess) return hip_check(g, e, "stage 3");
  return SHK_OK;
}

}  // namespace

extern "C" {

size_t shk_workspace_bytes(const shk_grid_desc* desc) {
  if (!desc_ok(desc, nullptr)) return 0;
  return layout(desc).total;
}

shk_status shk_init_grid(const shk_grid_desc* desc, void* workspace, size_t ws_bytes, void* hip_stream,
                         shk_grid** out) {
  std::string why;
  if (!out) return SHK_EINVAL;
  *out = nullptr;
  if (!desc_ok(desc, &why)) return SHK_EINVAL;
  if (!workspace) return SHK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SHK_EINVAL;
  WsLayout L = layout(desc);
  if (ws_bytes < L.total) return SHK_ESPACE;
  shk_grid* g = new (std::nothrow) shk_grid();
  if (!g) return SHK_EINVAL;
  g->d = *desc;
  if (!(g->d.weno_eps > 0.0)) g->d.weno_eps = 1e-6;
  g->st = reinterpret_cast<hipStream_t>(hip_stream);
  g->ws = static_cast<char*>(workspace);
  g->ws_bytes = ws_bytes;
  g->L = L;
  g->esize = elem_size(desc);
  g->ibm_on = false;
  g->gt = GhostTable{0, nullptr, nullptr, nullptr, nullptr, 0};
  GridArgs& a = g->a;
  std::memset(&a, 0, sizeof(a));
  const shk_grid_desc& d = g->d;
  a.ndim = d.ndim; a.nx = d.nx; a.ny = d.ny; a.nbatch = d.nbatch; a.nvar = d.ndim == 1 ? 3 : 4;
  a.ncell = (long long)d.nx * d.ny;
  a.x0 = d.x0; a.y0 = d.ndim == 2 ? d.y0 : 0.0;
  a.dx = (d.x1 - d.x0) / d.nx;
  a.dy = d.ndim == 2 ? (d.y1 - d.y0) / d.ny : 1.0;
  a.inv_dx = 1.0 / a.dx; a.inv_dy = 1.0 / a.dy;
  a.gamma = d.gamma; a.eps = d.weno_eps; a.cfl = d.cfl;
  a.viscous = d.viscous; a.mu = d.mu; a.prandtl = d.prandtl > 0 ? d.prandtl : 1.0;
  a.nu_art = d.nu_art;
  a.weno_char = d.weno_char;
  for (int k = 0; k < 4; ++k) a.bc[k] = d.bc[k];
  set_physics(g->d, a);
  a.cls = nullptr;
  a.sc = reinterpret_cast<StepScalars*>(g->ws + L.scalars);
  a.glob = reinterpret_cast<Globals*>(g->ws + L.globals);
  a.dtbuf = reinterpret_cast<double*>(g->ws + L.dtbuf);
  a.nface = (long long)(d.nx + 1) * d.ny + (long long)d.nx * (d.ny + 1);
  a.xslots = reinterpret_cast<unsigned long long*>(g->ws + L.xslots);
  hipError_t e = launch_init_scalars(a, 0.0, std::numeric_limits<double>::infinity(), g->st);
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  if (e != hipSuccess) {
    delete g;
    return SHK_EHIP;
  }
  *out = g;
  return SHK_OK;
}

void shk_destroy(shk_grid* g) { delete g; }

shk_status shk_set_stream(shk_grid* g, void* hip_stream) {
  if (!g) return SHK_EINVAL;
  g->st = reinterpret_cast<hipStream_t>(hip_stream);
  return SHK_OK;
}

shk_status shk_prim_to_cons(shk_grid* g, const void* W, void* U) {
  if (!g) return SHK_EINVAL;
  if (!W || !U || W == U) return fail(g, SHK_EINVAL, "prim_to_cons: null or aliased arrays");
  hipError_t e = g->esize == 8
                     ? launch_prim_to_cons<double>(g->a, static_cast<const double*>(W), static_cast<double*>(U), g->st)
                     : launch_prim_to_cons<float>(g->a, static_cast<const float*>(W), static_cast<float*>(U), g->st);
  return hip_check(g, e, "prim_to_cons");
}

shk_status shk_prim_to_cons_vjp(shk_grid* g, const void* W, const void* U_bar, void* W_bar, double* param_bar) {
  if (!g) return SHK_EINVAL;
  if (g->d.prec != SHK_F64) return fail(g, SHK_EUNSUPPORTED, "prim_to_cons_vjp: SHK_F64 grids only");
  if (!W || !U_bar) return fail(g, SHK_EINVAL, "prim_to_cons_vjp: null array");
  if (!W_bar && !param_bar) return SHK_OK;
  double* part = reinterpret_cast<double*>(g->ws + g->L.vjpPart);
  return hip_check(g, launch_prim_to_cons_vjp(g->a, static_cast<const double*>(W), static_cast<const double*>(U_bar),
                                              static_cast<double*>(W_bar), param_bar, part, g->st),
                   "prim_to_cons_vjp");
}

// Byte offsets of the refill-transpose fill table within its workspace
// region: source cells and entry counts (ns each), then m slots of ghost
// indices and of weights, slot-major.
struct FillTable {
  size_t src, cnt, k, w, end;
};
static FillTable fill_table(int ns, int m) {
  FillTable f;
  f.src = 0;
  f.cnt = f.src + al(sizeof(int) * size_t(ns));
  f.k = f.cnt + al(sizeof(int) * size_t(ns));
  f.w = f.k + al(sizeof(int) * size_t(m) * ns);
  f.end = f.w + al(sizeof(double) * size_t(m) * ns);
  return f;
}

// Dispatch order of the 2D stage tiles of a grid with a body: workgroup w
// goes to XCD w % 8 (round robin), so XCD x takes the tiles of queue x in
// order.  The tiles near the body (their ghost cells chain four dependent
// loads and take longest) come first, dealt round robin, so that none of
// them is left for the launch's last round; each XCD then takes one
// contiguous run of the other tiles in row-major order, whose shared halo
// rows stay in that XCD's L2.  Each entry carries the tile's body flag in
// bit 31 (the tile count is below 2^30: at most 2^38 cells).
static std::vector<unsigned> body_first_order(int gx, int gy, const std::vector<uint8_t>& body) {
  const int n = gx * gy;
  std::vector<std::vector<int>> q(8);
  int nb = 0;
  for (int t = 0; t < n; ++t)
    if (body[t]) q[nb++ % 8].push_back(t);
  int t = 0;
  for (int x = 0; x < 8; ++x) {
    const int cnt = n > x ? (n - x + 7) / 8 : 0;  // workgroups x, x + 8, ... below n
    while (int(q[x].size()) < cnt) {  // the counts add up to the n - nb other tiles
      while (t < n - 1 && body[t]) ++t;
      q[x].push_back(t++);
    }
  }
  std::vector<unsigned> order(n);
  for (int w = 0; w < n; ++w) {
    const int tile = q[w % 8][w / 8];
    order[w] = unsigned(tile) | (body[tile] ? 0x80000000u : 0u);
  }
  return order;
}

shk_status shk_set_ib_levelset(shk_grid* g, const double* phi, int wall) {
  if (!g) return SHK_EINVAL;
  if (!phi) {
    g->ibm_on = false;
    g->a.cls = nullptr;
    g->a.ghost_of = nullptr;
    g->a.tile_order = nullptr;
    g->gt.n = 0;
    g->a.gt = g->gt;
    return SHK_OK;
  }
  if (!g->d.ibm) return fail(g, SHK_ESTATE, "set_ib_levelset: grid created without desc.ibm = 1");
  if (wall != 0 && wall != 1) return fail(g, SHK_EINVAL, "set_ib_levelset: wall must be 0 (slip) or 1 (no-slip)");
  GridArgs& a = g->a;
  uint8_t* cls = reinterpret_cast<uint8_t*>(g->ws + g->L.cls);
  int* rc = reinterpret_cast<int*>(g->ws + g->L.row_count);
  int* ro = reinterpret_cast<int*>(g->ws + g->L.row_off);
  GhostTable gt;
  gt.cell = reinterpret_cast<int*>(g->ws + g->L.g_cell);
  gt.src = reinterpret_cast<int*>(g->ws + g->L.g_src);
  gt.w = reinterpret_cast<double*>(g->ws + g->L.g_w);
  gt.nrm = reinterpret_cast<double*>(g->ws + g->L.g_nrm);
  gt.wall = wall;
  gt.n = 0;
  // rc[0..ny-1]: ghosts per row; rc[ny]: ghosts whose image point is undefined
  hipError_t e = hipMemsetAsync(rc, 0, sizeof(int) * (a.ny + 1), g->st);
  if (e == hipSuccess) e = launch_ibm_classify(a, phi, cls, rc, g->st);
  if (e == hipSuccess) e = launch_ibm_table(a, phi, cls, rc, ro, gt, rc + a.ny, g->st);
  int n = 0, nbad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&n, ro + a.ny, sizeof(int), hipMemcpyDeviceToHost, g->st);
  if (e == hipSuccess) e = hipMemcpyAsync(&nbad, rc + a.ny, sizeof(int), hipMemcpyDeviceToHost, g->st);
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  if (e != hipSuccess) return hip_check(g, e, "set_ib_levelset");
  if (nbad > 0) {
    g->ibm_on = false;
    g->a.cls = nullptr;
    g->a.ghost_of = nullptr;
    g->a.tile_order = nullptr;
    g->gt.n = 0;
    g->a.gt = g->gt;
    return fail(g, SHK_EINVAL, "set_ib_levelset: " + std::to_string(nbad) +
                                   " ghost cells have no image point (|grad phi| < 1/2 there, or no fluid cell is "
                                   "found from them); the immersed boundary is off");
  }
  gt.n = n;
  g->gt = gt;
  a.gt = gt;
  a.cls = cls;
  g->ibm_on = true;
  g->nent = 0;
  g->nsrc = 0;
  // ghost index of every cell: the stage kernels refill ghost cells while
  // loading their tiles, and the adjoint kernel runs the ghost half of the
  // refill transpose
  int* gof = reinterpret_cast<int*>(g->ws + g->L.ghostOf);
  e = launch_ghost_index(a, gt, gof, g->st);
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  if (e != hipSuccess) return hip_check(g, e, "set_ib_levelset (ghost index)");
  a.ghost_of = gof;
  // tiles whose cells and halo sources are all fluid skip the immersed-boundary
  // handling in the stage kernels
  uint8_t* tb = reinterpret_cast<uint8_t*>(g->ws + g->L.tileBody);
  unsigned* to = reinterpret_cast<unsigned*>(g->ws + g->L.tileOrder);
  a.tile_order = nullptr;
  const int tgx = (a.nx + STAGE_TX - 1) / STAGE_TX, tgy = (a.ny + STAGE_TY - 1) / STAGE_TY;
  std::vector<uint8_t> body(size_t(tgx) * tgy);
  std::vector<unsigned> order;
  e = launch_tile_body(a, tb, g->st);
  if (e == hipSuccess) e = hipMemcpyAsync(body.data(), tb, body.size(), hipMemcpyDeviceToHost, g->st);
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  if (e == hipSuccess) {
    order = body_first_order(tgx, tgy, body);
    e = hipMemcpyAsync(to, order.data(), sizeof(unsigned) * order.size(), hipMemcpyHostToDevice, g->st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  if (e != hipSuccess) return hip_check(g, e, "set_ib_levelset (tile flags)");
  a.tile_order = to;
  if (g->d.adjoint && n > 0) {
    int* keys = reinterpret_cast<int*>(g->ws + g->L.entKeys);
    int* vals = reinterpret_cast<int*>(g->ws + g->L.entVals);
    int* cnt = reinterpret_cast<int*>(g->ws + g->L.entCount);
    int nv = 0;
    e = hipMemsetAsync(cnt, 0, sizeof(int), g->st);
    if (e == hipSuccess) e = launch_ibm_entries(gt, keys, vals, cnt, g->st);
    if (e == hipSuccess) e = hipMemcpyAsync(&nv, cnt, sizeof(int), hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_check(g, e, "set_ib_levelset (adjoint entries)");
    g->nent = nv;
    // run heads of equal source keys (set-up only; host-side scan)
    std::vector<int> hk(size_t(nv > 0 ? nv : 1)), heads;
    if (nv > 0) e = hipMemcpyAsync(hk.data(), keys, sizeof(int) * nv, hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_check(g, e, "set_ib_levelset (entry keys)");
    heads.reserve(size_t(nv) + 1);
    for (int i = 0; i < nv; ++i)
      if (i == 0 || hk[i] != hk[i - 1]) heads.push_back(i);
    heads.push_back(nv);
    const int ns = int(heads.size()) - 1;
    // the fill table, source by source: source cell, entry count, and per
    // entry slot t the ghost index and weight of its t-th entry (in entry
    // order), slot-major so that a wave reads consecutive sources; it takes
    // the place of the sorted entries, which only served to build it
    std::vector<int> hv(size_t(nv > 0 ? nv : 1));
    std::vector<double> hw(size_t(4) * gt.n);
    if (nv > 0) e = hipMemcpyAsync(hv.data(), vals, sizeof(int) * nv, hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipMemcpyAsync(hw.data(), gt.w, sizeof(double) * hw.size(), hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_check(g, e, "set_ib_levelset (entries)");
    int m = 0;
    for (int h = 0; h < ns; ++h) m = std::max(m, heads[h + 1] - heads[h]);
    const FillTable ft = fill_table(ns, m);
    const size_t cap = g->L.entHeads + al(sizeof(int) * (4 * size_t(g->a.ncell) + 1)) - g->L.entKeys;
    if (ft.end > cap)
      return fail(g, SHK_EINVAL, "set_ib_levelset: the refill transpose table (" + std::to_string(ns) +
                                     " sources, up to " + std::to_string(m) + " entries each) exceeds its workspace");
    std::vector<char> tab(ft.end, 0);
    int* fsrc = reinterpret_cast<int*>(tab.data() + ft.src);
    int* fcnt = reinterpret_cast<int*>(tab.data() + ft.cnt);
    int* fk = reinterpret_cast<int*>(tab.data() + ft.k);
    double* fw = reinterpret_cast<double*>(tab.data() + ft.w);
    for (int h = 0; h < ns; ++h) {
      fsrc[h] = hk[heads[h]];
      fcnt[h] = heads[h + 1] - heads[h];
      for (int t = 0; t < fcnt[h]; ++t) {
        const int ent = hv[heads[h] + t];
        fk[size_t(t) * ns + h] = ent >> 2;
        fw[size_t(t) * ns + h] = hw[ent];
      }
    }
    e = hipMemcpyAsync(g->ws + g->L.entKeys, tab.data(), tab.size(), hipMemcpyHostToDevice, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_check(g, e, "set_ib_levelset (fill table)");
    g->nsrc = ns;
    g->fill_m = m;
  }
  return SHK_OK;
}

shk_status shk_set_params(shk_grid* g, double gamma, const double* inflow_prim) {
  if (!g) return SHK_EINVAL;
  if (!(gamma > 1.0)) return fail(g, SHK_EINVAL, "set_params: gamma must exceed 1");
  if (inflow_prim && (!(inflow_prim[0] > 0.0) || !(inflow_prim[3] > 0.0)))
    return fail(g, SHK_EINVAL, "set_params: inflow density and pressure must be positive");
  g->d.gamma = gamma;
  if (inflow_prim)
    for (int k = 0; k < 4; ++k) g->d.inflow_prim[k] = inflow_prim[k];
  set_physics(g->d, g->a);
  return SHK_OK;
}

shk_status shk_ib_ghost_count(const shk_grid* g, int* n_host) {
  if (!g || !n_host) return SHK_EINVAL;
  *n_host = g->ibm_on ? g->gt.n : 0;
  return SHK_OK;
}

shk_status shk_ib_classes(shk_grid* g, uint8_t* cls) {
  if (!g || !cls) return SHK_EINVAL;
  if (!g->ibm_on) return fail(g, SHK_ESTATE, "ib_classes: no immersed boundary set");
  return hip_check(g, hipMemcpyAsync(cls, g->a.cls, size_t(g->a.ncell), hipMemcpyDeviceToDevice, g->st),
                   "ib_classes");
}

shk_status shk_rhs(shk_grid* g, const void* U, void* dUdt) {
  if (!g) return SHK_EINVAL;
  if (!U || !dUdt || U == dUdt) return fail(g, SHK_EINVAL, "rhs: null or aliased arrays");
  hipError_t e = hipSuccess;
  if (g->esize == 8) {
    const GridArgs& a = g->a;
    const double* Us = static_cast<const double*>(U);
    if (g->ibm_on && g->cnn_on) {
      // the convolutional network reads the stage state's ghost cells: refill
      // them on a workspace copy, leaving U as it is
      double* W = reinterpret_cast<double*>(g->ws + g->L.u1);
      e = hipMemcpyAsync(W, Us, sizeof(double) * size_t(a.nbatch) * a.nvar * a.ncell, hipMemcpyDeviceToDevice,
                         g->st);
      if (e == hipSuccess) e = launch_ibm_fill<double>(a, g->gt, W, g->st);
      Us = W;
    }
    if (e == hipSuccess)
      e = stage_launch<double>(g, a, MODE_RHS, Us, Us, static_cast<double*>(dUdt), nullptr, nullptr);
  } else {
    const float* Us = static_cast<const float*>(U);
    if (g->d.prec == SHK_MIXED)
      e = launch_stage_mixed(g->a, MODE_RHS, Us, Us, static_cast<float*>(dUdt), nullptr, nullptr, g->st);
    else
      e = launch_stage<float>(g->a, MODE_RHS, Us, Us, static_cast<float*>(dUdt), nullptr, nullptr, g->st);
  }
  return hip_check(g, e, "rhs");
}

shk_status shk_ib_fill(shk_grid* g, void* U) {
  if (!g) return SHK_EINVAL;
  if (!U) return fail(g, SHK_EINVAL, "ib_fill: null state");
  if (!g->ibm_on) return fail(g, SHK_ESTATE, "ib_fill: no immersed boundary set");
  hipError_t e = g->esize == 8 ? launch_ibm_fill<double>(g->a, g->gt, static_cast<double*>(U), g->st)
                               : launch_ibm_fill<float>(g->a, g->gt, static_cast<float*>(U), g->st);
  return hip_check(g, e, "ib_fill");
}

shk_status shk_rk3_step(shk_grid* g, void* U, const double* dt_in, double* dt_out) {
  if (!g) return SHK_EINVAL;
  if (!U) return fail(g, SHK_EINVAL, "rk3_step: null state");
  if (g->esize == 8) return stage_seq<double>(g, static_cast<double*>(U), dt_in, dt_out);
  return stage_seq<float>(g, static_cast<float*>(U), dt_in, dt_out);
}

// Partial derivatives of the launches of one reverse pass, finalised once.
struct PartRec {
  double* base;
  PartSlots ps;  // ps.stride: doubles between slots
  bool finalised;  // the last refill transpose already added the partials
  double* next() const { return base + ps.n * ps.stride; }
  void add(int nblk) { ps.nblk[ps.n++] = nblk; }
};

static PartRec part_rec(shk_grid* g) {
  PartRec r{};
  r.base = reinterpret_cast<double*>(g->ws + g->L.adjPart);
  r.ps.stride = (long long)g->L.part_stride;
  return r;
}

// rhs-adjoint launch with the learned correction's reverse pass first (its
// stencil gradient is then added by the adjoint kernel face by face).
// With the immersed boundary the launch also runs the ghost half of the
// refill transpose (fillT below finishes it).
static hipError_t rhs_adj(shk_grid* g, PartRec& pr, const double* Us, const double* lam, double clam_f,
                          const double* dtp, const double* X1, double c1, const double* X2, double c2,
                          const double* X3, double c3, double* out) {
  GridArgs a = g->a;
  if (g->net_on) {
    float* dX = reinterpret_cast<float*>(g->ws + g->L.netX);
    float* np = reinterpret_cast<float*>(g->ws + g->L.netPart);
    hipError_t e = launch_net_backward(a, g->net, Us, lam, clam_f, dtp, dX, np, g->net_grad, g->st);
    if (e != hipSuccess) return e;
    a.dXnet = dX;
  } else if (g->cnn_on) {
    float* dX = reinterpret_cast<float*>(g->ws + g->L.netX);
    float* dF = reinterpret_cast<float*>(g->ws + g->L.cnnDF);
    hipError_t e = launch_cnn_backward(a, g->cnn, Us, lam, clam_f, dtp, dX, dF, cnn_bufs(a, g->ws + g->L.cnnBufs),
                                       g->net_grad, g->st);
    if (e != hipSuccess) return e;
    a.dXnet = dX;
  }
  int nb = 0;
  double* gW = g->ibm_on ? reinterpret_cast<double*>(g->ws + g->L.adjG) : nullptr;
  hipError_t e = launch_rhs_adjoint(a, Us, lam, clam_f, dtp, X1, c1, X2, c2, X3, c3, out, pr.next(), &nb, g->gt, gW,
                                    g->st);
  if (e == hipSuccess) pr.add(nb);
  return e;
}

static shk_status adjoint_ok(shk_grid* g) {
  if (!g->d.adjoint) return fail(g, SHK_ESTATE, "adjoint: grid created without desc.adjoint = 1");
  if (g->d.prec != SHK_F64 || g->d.ndim != 2 || g->d.viscous || g->d.nu_art != 0.0)
    return fail(g, SHK_EUNSUPPORTED, "adjoint: implemented for 2D inviscid FP64 without artificial viscosity");
  return SHK_OK;
}

// Ghost refill of a double state (no-op without immersed boundary).
static hipError_t fill64(shk_grid* g, double* X) {
  return g->ibm_on ? launch_ibm_fill<double>(g->a, g->gt, X, g->st) : hipSuccess;
}

// Source half of the refill transpose on an adjoint array X (w.r.t. the
// filled state Us); with param_bar set it also finalises the pass's partials.
static hipError_t fillT(shk_grid* g, PartRec& pr, const double* Us, double* X, double* param_bar = nullptr) {
  if (!g->ibm_on || g->nent == 0) return hipSuccess;
  const FillTable ft = fill_table(g->nsrc, g->fill_m);
  const char* base = g->ws + g->L.entKeys;
  const double* gW = reinterpret_cast<const double*>(g->ws + g->L.adjG);
  hipError_t e = launch_ibm_fill_adjoint(g->a, g->gt, reinterpret_cast<const int*>(base + ft.src),
                                         reinterpret_cast<const int*>(base + ft.cnt),
                                         reinterpret_cast<const int*>(base + ft.k),
                                         reinterpret_cast<const double*>(base + ft.w), g->fill_m, g->nsrc, Us, X, gW,
                                         pr.next(), pr.ps, param_bar, g->st);
  if (e == hipSuccess) {
    pr.add(1);
    if (param_bar) pr.finalised = true;
  }
  return e;
}

static hipError_t finish(shk_grid* g, const PartRec& pr, double* param_bar) {
  if (pr.finalised) return hipSuccess;
  return launch_partials_finalize(pr.base, pr.ps, g->a.nbatch, param_bar, g->st);
}

shk_status shk_rhs_adjoint(shk_grid* g, const void* U, const void* dUdt_bar, void* U_bar, double* param_bar) {
  if (!g) return SHK_EINVAL;
  shk_status s = adjoint_ok(g);
  if (s != SHK_OK) return s;
  if (!U || !dUdt_bar || !U_bar) return fail(g, SHK_EINVAL, "rhs_adjoint: null array");
  const GridArgs& a = g->a;
  const size_t bytes = size_t(a.nbatch) * 4 * a.ncell * sizeof(double);
  double* A = reinterpret_cast<double*>(g->ws + g->L.adjA);
  double* P = reinterpret_cast<double*>(g->ws + g->L.adjP);
  PartRec pr = part_rec(g);
  hipError_t e = hipMemcpyAsync(A, U, bytes, hipMemcpyDeviceToDevice, g->st);
  if (e == hipSuccess) e = fill64(g, A);
  if (e == hipSuccess)
    e = rhs_adj(g, pr, A, static_cast<const double*>(dUdt_bar), 1.0, nullptr, nullptr, 0.0, nullptr, 0.0, nullptr,
                0.0, P);
  if (e == hipSuccess) e = fillT(g, pr, A, P, param_bar);
  if (e == hipSuccess) e = launch_axpy((long long)a.nbatch * 4 * a.ncell, 1.0, P, static_cast<double*>(U_bar), 1, g->st);
  if (e == hipSuccess) e = finish(g, pr, param_bar);
  return hip_check(g, e, "rhs_adjoint");
}

// Reverse of one SSP-RK3 step from its filled stage-start states A = U^n,
// B = U1, C = U2.  With the adjoints written X3 (after the step, in Ub), X2,
// X1 (of the stage states before their refill) and R^T the transpose of the
// refill (its ghost half inside each adjoint launch):
//   X2 = R^T(2/3 X3 + 2/3 dt J(U2)^T X3)
//   X1 = R^T(1/4 X2 + 1/4 dt J(U1)^T X2)
//   X0 = R^T(X1 + dt J(U^n)^T X1 + 1/3 X3 + 3/4 X2)
static hipError_t reverse_step(shk_grid* g, const double* A, const double* B, const double* C, const double* dt,
                               double* Ub, double* param_bar) {
  double* P = reinterpret_cast<double*>(g->ws + g->L.adjP);
  double* Q = reinterpret_cast<double*>(g->ws + g->L.adjQ);
  PartRec pr = part_rec(g);
  hipError_t e = rhs_adj(g, pr, C, Ub, 2.0 / 3.0, dt, Ub, 2.0 / 3.0, nullptr, 0.0, nullptr, 0.0, P);
  if (e == hipSuccess) e = fillT(g, pr, C, P);
  if (e == hipSuccess) e = rhs_adj(g, pr, B, P, 0.25, dt, P, 0.25, nullptr, 0.0, nullptr, 0.0, Q);
  if (e == hipSuccess) e = fillT(g, pr, B, Q);
  if (e == hipSuccess) e = rhs_adj(g, pr, A, Q, 1.0, dt, Q, 1.0, Ub, 1.0 / 3.0, P, 0.75, Ub);
  if (e == hipSuccess) e = fillT(g, pr, A, Ub, param_bar);
  if (e == hipSuccess) e = finish(g, pr, param_bar);
  return e;
}

shk_status shk_rk3_step_adjoint(shk_grid* g, const void* U_n, const double* dt, void* U_bar, double* param_bar) {
  if (!g) return SHK_EINVAL;
  shk_status s = adjoint_ok(g);
  if (s != SHK_OK) return s;
  if (!U_n || !dt || !U_bar) return fail(g, SHK_EINVAL, "rk3_step_adjoint: null array");
  const GridArgs& a = g->a;
  const size_t bytes = size_t(a.nbatch) * 4 * a.ncell * sizeof(double);
  double* A = reinterpret_cast<double*>(g->ws + g->L.adjA);  // U^n filled
  double* B = reinterpret_cast<double*>(g->ws + g->L.adjB);  // U1 filled
  double* C = reinterpret_cast<double*>(g->ws + g->L.adjC);  // U2 filled
  hipError_t e = hipMemcpyAsync(A, U_n, bytes, hipMemcpyDeviceToDevice, g->st);
  // forward recompute of the stage states
  if (e == hipSuccess) e = fill64(g, A);
  if (e == hipSuccess) e = stage_launch<double>(g, a, MODE_STAGE1, A, A, B, dt, nullptr);
  if (e == hipSuccess) e = fill64(g, B);
  if (e == hipSuccess) e = stage_launch<double>(g, a, MODE_STAGE2, B, A, C, dt, nullptr);
  if (e == hipSuccess) e = fill64(g, C);
  if (e == hipSuccess) e = reverse_step(g, A, B, C, dt, static_cast<double*>(U_bar), param_bar);
  return hip_check(g, e, "rk3_step_adjoint");
}

shk_status shk_rk3_step_record(shk_grid* g, void* U, const double* dt_in, double* dt_out, void* tape) {
  if (!g) return SHK_EINVAL;
  shk_status s = adjoint_ok(g);
  if (s != SHK_OK) return s;
  if (!U || !tape) return fail(g, SHK_EINVAL, "rk3_step_record: null array");
  return stage_seq<double>(g, static_cast<double*>(U), dt_in, dt_out, static_cast<double*>(tape));
}

shk_status shk_rk3_step_adjoint_tape(shk_grid* g, const void* tape, const double* dt, void* U_bar,
                                     double* param_bar) {
  if (!g) return SHK_EINVAL;
  shk_status s = adjoint_ok(g);
  if (s != SHK_OK) return s;
  if (!tape || !dt || !U_bar) return fail(g, SHK_EINVAL, "rk3_step_adjoint_tape: null array");
  const double* A = static_cast<const double*>(tape);
  const long long nst = (long long)g->a.nbatch * 4 * g->a.ncell;
  hipError_t e = reverse_step(g, A, A + nst, A + 2 * nst, dt, static_cast<double*>(U_bar), param_bar);
  return hip_check(g, e, "rk3_step_adjoint_tape");
}

shk_status shk_rk3_steps_record(shk_grid* g, void* U, int nsteps, const double* dt, void* tapes) {
  if (!g) return SHK_EINVAL;
  shk_status s = adjoint_ok(g);
  if (s != SHK_OK) return s;
  if (!U || !dt || !tapes || nsteps < 0) return fail(g, SHK_EINVAL, "rk3_steps_record: null array or nsteps < 0");
  const long long nst = (long long)g->a.nbatch * 4 * g->a.ncell;
  for (int k = 0; k < nsteps; ++k) {
    s = stage_seq<double>(g, static_cast<double*>(U), dt, nullptr, static_cast<double*>(tapes) + 3 * nst * k);
    if (s != SHK_OK) return s;
  }
  return SHK_OK;
}

shk_status shk_rk3_steps_adjoint_tape(shk_grid* g, const void* tapes, int nsteps, const double* dt, void* U_bar,
                                      double* param_bar) {
  if (!g) return SHK_EINVAL;
  shk_status s = adjoint_ok(g);
  if (s != SHK_OK) return s;
  if (!tapes || !dt || !U_bar || nsteps < 0)
    return fail(g, SHK_EINVAL, "rk3_steps_adjoint_tape: null array or nsteps < 0");
  const long long nst = (long long)g->a.nbatch * 4 * g->a.ncell;
  for (int k = nsteps - 1; k >= 0; --k) {
    const double* A = static_cast<const double*>(tapes) + 3 * nst * k;
    hipError_t e = reverse_step(g, A, A + nst, A + 2 * nst, dt, static_cast<double*>(U_bar), param_bar);
    if (e != hipSuccess) return hip_check(g, e, "rk3_steps_adjoint_tape");
  }
  return SHK_OK;
}

shk_status shk_set_flux_net(shk_grid* g, const uint16_t* w_bf16, const float* bias, const double* norm_host,
                            float out_scale, int enable) {
  if (!g) return SHK_EINVAL;
  if (!enable) {
    g->net_on = false;
    return SHK_OK;
  }
  if (g->d.flux_net != 1) return fail(g, SHK_ESTATE, "set_flux_net: grid created without desc.flux_net = 1");
  if (!w_bf16 || !bias || !norm_host) return fail(g, SHK_EINVAL, "set_flux_net: null array");
  NetArgs n{};
  n.w = reinterpret_cast<const unsigned short*>(w_bf16);
  n.bias = bias;
  for (int k = 0; k < 4; ++k) {
    n.mean[k] = norm_host[k];
    n.inv_std[k] = norm_host[4 + k];
  }
  n.out_scale = out_scale;
  g->net = n;
  g->net_on = true;
  return SHK_OK;
}

shk_status shk_set_flux_net_grad(shk_grid* g, float* grad) {
  if (!g) return SHK_EINVAL;
  g->net_grad = grad;
  return SHK_OK;
}

shk_status shk_flux_net_eval(shk_grid* g, const void* U, float* dF) {
  if (!g || !U || !dF) return SHK_EINVAL;
  if (!g->net_on) return fail(g, SHK_ESTATE, "flux_net_eval: no flux net set");
  return hip_check(g, launch_net_forward(g->a, g->net, static_cast<const double*>(U), dF, g->st), "flux_net_eval");
}

shk_status shk_flux_net_vjp(shk_grid* g, const void* U, const void* lam, float* dX, float* grad) {
  if (!g || !U || !lam || !dX) return SHK_EINVAL;
  if (!g->net_on) return fail(g, SHK_ESTATE, "flux_net_vjp: no flux net set");
  if (!g->d.adjoint) return fail(g, SHK_ESTATE, "flux_net_vjp: grid created without desc.adjoint = 1");
  float* np = reinterpret_cast<float*>(g->ws + g->L.netPart);
  return hip_check(g,
                   launch_net_backward(g->a, g->net, static_cast<const double*>(U), static_cast<const double*>(lam),
                                       1.0, nullptr, dX, np, grad, g->st),
                   "flux_net_vjp");
}

shk_status shk_set_flux_cnn(shk_grid* g, const uint16_t* w_bf16, const float* bias, const double* norm_host,
                            float out_scale, int enable) {
  if (!g) return SHK_EINVAL;
  if (!enable) {
    g->cnn_on = false;
    return SHK_OK;
  }
  if (g->d.flux_net != 2) return fail(g, SHK_ESTATE, "set_flux_cnn: grid created without desc.flux_net = 2");
  if (!w_bf16 || !bias || !norm_host) return fail(g, SHK_EINVAL, "set_flux_cnn: null array");
  if (!(out_scale > 0.0f)) return fail(g, SHK_EINVAL, "set_flux_cnn: out_scale must be positive");
  CnnArgs n{};
  n.w = reinterpret_cast<const unsigned short*>(w_bf16);
  n.bias = bias;
  for (int k = 0; k < 4; ++k) {
    n.mean[k] = norm_host[k];
    n.inv_std[k] = norm_host[4 + k];
  }
  n.out_scale = out_scale;
  g->cnn = n;
  g->cnn_on = true;
  return SHK_OK;
}

shk_status shk_flux_cnn_eval(shk_grid* g, const void* U, float* dF) {
  if (!g || !U || !dF) return SHK_EINVAL;
  if (!g->cnn_on) return fail(g, SHK_ESTATE, "flux_cnn_eval: no convolutional net set");
  return hip_check(g,
                   launch_cnn_forward(g->a, g->cnn, static_cast<const double*>(U), dF,
                                      cnn_bufs(g->a, g->ws + g->L.cnnBufs), false, g->st),
                   "flux_cnn_eval");
}

shk_status shk_flux_cnn_vjp(shk_grid* g, const void* U, const void* lam, float* dX, float* grad) {
  if (!g || !U || !lam || !dX) return SHK_EINVAL;
  if (!g->cnn_on) return fail(g, SHK_ESTATE, "flux_cnn_vjp: no convolutional net set");
  float* dF = reinterpret_cast<float*>(g->ws + g->L.cnnDF);
  return hip_check(g,
                   launch_cnn_backward(g->a, g->cnn, static_cast<const double*>(U), static_cast<const double*>(lam),
                                       1.0, nullptr, dX, dF, cnn_bufs(g->a, g->ws + g->L.cnnBufs), grad, g->st),
                   "flux_cnn_vjp");
}

shk_status shk_flux_cnn_images(shk_grid* g, const void* U, float* images, int* npix) {
  if (!g || !npix) return SHK_EINVAL;
  *npix = cnn_geom(g->a).npix;
  if (!U && !images) return SHK_OK;  // size query
  if (!U || !images) return SHK_EINVAL;
  if (!g->cnn_on) return fail(g, SHK_ESTATE, "flux_cnn_images: no convolutional net set");
  return hip_check(g,
                   launch_cnn_images(g->a, g->cnn, static_cast<const double*>(U),
                                     cnn_bufs(g->a, g->ws + g->L.cnnBufs), images, g->st),
                   "flux_cnn_images");
}

shk_status shk_flux_cnn_pack(const float* theta, uint16_t* w_bf16, float* bias, void* hip_stream) {
  if (!theta || !w_bf16 || !bias) return SHK_EINVAL;
  return launch_cnn_pack(theta, reinterpret_cast<unsigned short*>(w_bf16), bias,
                         reinterpret_cast<hipStream_t>(hip_stream)) == hipSuccess ? SHK_OK : SHK_EHIP;
}

shk_status shk_flux_net_pack(const float* theta, uint16_t* w_bf16, float* bias, void* hip_stream) {
  if (!theta || !w_bf16 || !bias) return SHK_EINVAL;
  return launch_net_pack(theta, reinterpret_cast<unsigned short*>(w_bf16), bias,
                         reinterpret_cast<hipStream_t>(hip_stream)) == hipSuccess ? SHK_OK : SHK_EHIP;
}

shk_status shk_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float beta1, float beta2,
                    float eps, int step, void* hip_stream) {
  if (!theta || !grad || !m || !v || n <= 0 || step < 1) return SHK_EINVAL;
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f)) return SHK_EINVAL;
  return launch_adam(theta, grad, m, v, n, lr, beta1, beta2, eps, step, reinterpret_cast<hipStream_t>(hip_stream)) ==
                 hipSuccess ? SHK_OK : SHK_EHIP;
}

shk_status shk_restrict(const double* fine, double* coarse, int nx_f, int ny_f, int factor, int nvar, int nbatch,
                        void* hip_stream) {
  if (!fine || !coarse || factor < 1 || nx_f % factor || ny_f % factor || nvar < 1 || nbatch < 1) return SHK_EINVAL;
  return launch_restrict(fine, coarse, nx_f, ny_f, factor, nvar, nbatch, reinterpret_cast<hipStream_t>(hip_stream)) ==
                 hipSuccess ? SHK_OK : SHK_EHIP;
}

shk_status shk_mse(const double* U, const double* T, double* G, double scale, long long per_batch, int nbatch,
                   double* part, double* loss, void* hip_stream) {
  if (!U || !T || !part || !loss || per_batch < 1 || nbatch < 1 || nbatch > 4096) return SHK_EINVAL;
  return launch_mse(U, T, G, scale, per_batch, nbatch, part, loss, reinterpret_cast<hipStream_t>(hip_stream)) ==
                 hipSuccess ? SHK_OK : SHK_EHIP;
}

shk_status shk_mse_noalloc(const double* U, const double* T, double* G, double scale, long long per_batch,
                           int nbatch, double* loss, void* hip_stream) {
  if (!U || !T || !loss || per_batch < 1 || nbatch < 1 || nbatch > SHK_MSE_NOALLOC_MAX_BATCH) return SHK_EINVAL;
  return launch_mse_noalloc(U, T, G, scale, per_batch, nbatch, loss, reinterpret_cast<hipStream_t>(hip_stream)) ==
                 hipSuccess ? SHK_OK : SHK_EHIP;
}

shk_status shk_set_time(shk_grid* g, double t0, double t_end) {
  if (!g) return SHK_EINVAL;
  if (!(t_end >= t0)) return fail(g, SHK_EINVAL, "set_time: t_end < t0");
  return hip_check(g, launch_init_scalars(g->a, t0, t_end, g->st), "set_time");
}

shk_status shk_get_time(shk_grid* g, int b, double* t_host, int* done_host, int* steps_host) {
  if (!g || b < 0 || b >= g->d.nbatch) return SHK_EINVAL;
  StepScalars s;
  hipError_t e = hipMemcpyAsync(&s, g->a.sc + b, sizeof(s), hipMemcpyDeviceToHost, g->st);
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  if (e != hipSuccess) return hip_check(g, e, "get_time");
  if (t_host) *t_host = s.t;
  if (done_host) *done_host = s.done;
  if (steps_host) *steps_host = s.nsteps;
  return SHK_OK;
}

shk_status shk_poll_faults(shk_grid* g, uint32_t* flags_host, uint64_t* fallback_faces_host) {
  if (!g) return SHK_EINVAL;
  Globals gl;
  hipError_t e = hipMemcpyAsync(&gl, g->a.glob, sizeof(gl), hipMemcpyDeviceToHost, g->st);
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  Globals z{};
  if (e == hipSuccess) e = hipMemcpyAsync(g->a.glob, &z, sizeof(z), hipMemcpyHostToDevice, g->st);
  if (e == hipSuccess) e = hipStreamSynchronize(g->st);
  if (e != hipSuccess) return hip_check(g, e, "poll_faults");
  if (flags_host) *flags_host = gl.fault;
  if (fallback_faces_host) *fallback_faces_host = gl.fallbacks;
  return SHK_OK;
}

shk_status shk_profile(shk_grid* g, int enable) {
  if (!g) return SHK_EINVAL;
  if (!g->recs.empty()) {
    hipError_t e = hipStreamSynchronize(g->st);
    for (auto& r : g->recs) { g->pool.push_back(r.a); g->pool.push_back(r.b); }
    g->recs.clear();
    if (e != hipSuccess) return hip_check(g, e, "profile");
  }
  g->prof = enable != 0;
  return SHK_OK;
}

shk_status shk_profile_read(shk_grid* g, double* ms_host, int* count_host) {
  if (!g || !ms_host || !count_host) return SHK_EINVAL;
  for (int k = 0; k < 5; ++k) { ms_host[k] = 0.0; count_host[k] = 0; }
  hipError_t e = hipStreamSynchronize(g->st);
  if (e != hipSuccess) return hip_check(g, e, "profile_read");
  for (auto& r : g->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && r.cls >= 0 && r.cls < 5) {
      ms_host[r.cls] += ms;
      count_host[r.cls] += 1;
    }
  }
  return SHK_OK;
}

const char* shk_last_error(const shk_grid* g) { return g ? g->err.c_str() : "null handle"; }

const char* shk_status_string(int s) {
  switch (s) {
    case SHK_OK: return "SHK_OK";
    case SHK_EINVAL: return "SHK_EINVAL";
    case SHK_ESTATE: return "SHK_ESTATE";
    case SHK_EHIP: return "SHK_EHIP";
    case SHK_EFAULT: return "SHK_EFAULT";
    case SHK_EUNSUPPORTED: return "SHK_EUNSUPPORTED";
    case SHK_ESPACE: return "SHK_ESPACE";
    default: return "unknown status";
  }
}

shk_status shk_normal_shock_state(double M, double g, double r1, double p1, double* out3, double* dM3,
                                  double* dg3) {
  if (!out3 || !(g > 1.0) || !(r1 > 0.0) || !(p1 > 0.0) || !(M >= 1.0)) return SHK_EINVAL;
  const double a1 = std::sqrt(g * p1 / r1);
  const double M2 = M * M;
  const double den = (g - 1.0) * M2 + 2.0;
  const double r2 = r1 * (g + 1.0) * M2 / den;
  const double p2 = p1 * (1.0 + 2.0 * g / (g + 1.0) * (M2 - 1.0));
  const double u2 = M * a1 * (1.0 - r1 / r2);
  out3[0] = r2; out3[1] = u2; out3[2] = p2;
  // d/dM
  const double dr2_dM = r1 * (g + 1.0) * (2.0 * M * den - M2 * 2.0 * (g - 1.0) * M) / (den * den);
  const double dp2_dM = p1 * 2.0 * g / (g + 1.0) * 2.0 * M;
  const double du2_dM = a1 * (1.0 - r1 / r2) + M * a1 * (r1 / (r2 * r2)) * dr2_dM;
  // d/dgamma
  const double da1_dg = 0.5 * std::sqrt(p1 / (r1 * g));
  const double dr2_dg = r1 * (M2 * den - (g + 1.0) * M2 * M2) / (den * den);
  const double dp2_dg = p1 * 2.0 * (M2 - 1.0) / ((g + 1.0) * (g + 1.0));
  const double du2_dg = M * da1_dg * (1.0 - r1 / r2) + M * a1 * (r1 / (r2 * r2)) * dr2_dg;
  if (dM3) { dM3[0] = dr2_dM; dM3[1] = du2_dM; dM3[2] = dp2_dM; }
  if (dg3) { dg3[0] = dr2_dg; dg3[1] = du2_dg; dg3[2] = dp2_dg; }
  return SHK_OK;
}

}  // extern "C"
