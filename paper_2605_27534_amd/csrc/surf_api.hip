// surf_api.hip -- the C ABI of libsurf (declared in include/surf.h): argument
// checks, workspace carving and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/surf.h"
#include "surf_kernels.hpp"
#include "surf_step2d.hpp"
#include "surf_col2d.hpp"
#include "surf_col3d.hpp"
#include "surf_geo3d.hpp"
#include "surf_adjoint.hpp"
#include "surf_implicit.hpp"
#include "surf_bicgstab.hpp"
#include "surf_acdi.hpp"
#include "surf_capillary.hpp"
#include "surf_capillary3d.hpp"

using namespace surf;

struct surf_ctx {
  surf_grid grid;
  surf_params prm;
  Grid g;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  double* state;
  double* part;
  void* chi[2];
  void* g0;
  int chi_cur;
  bool has_chi;
  long long ncell;
  int tiles[3];
  int nblk;
  double dt;
  // 2D fused path: per-tile quiescence flags of each level-set buffer
  uint8_t* q[2];
  int tiles2d[2];
  int ntiles2d;
  // weighted-form geometry tiles (GEO_T x GEO_T) and the flag array length
  int gtiles[2];
  int ngtiles;
  int nflags;
  uint8_t* mark;  // 2D weighted-form moving geometry: live-tile marks
  // 3D moving geometry: 16^3 tiles and the live-tile list ([0] count)
  int g3tiles[3];
  int ng3;
  int* live3;


  int per_xcd;
  // 2D weighted-form transport: column-streaming waves
  int col_strips, col_groups, col_nwg;
  // 3D weighted-form transport: plane-marching workgroups (strips, row
  // blocks, plane chunks)
  int c3[3], c3_nwg;
  // implicit substep 2: FP64 work arrays and records
  ImpBuf imp{};
  int imp_nblk = 0;
  int imp_nsolves = 0;  // linear solves of the last implicit step
  void* acdi[3] = {nullptr, nullptr, nullptr};  // ACDI: phi, phi*, s (cell fields)
  unsigned long long* hprog = nullptr;  // CG progress words (pinned host memory)
  unsigned long long solve_serial = 0;
  // pipelined moving interface (2D weighted form): the next step's geometry
  // prepared on an auxiliary stream while this step's transport runs
  hipEvent_t ev_pre = nullptr;     // context stream, just before a transport
  hipEvent_t ev_geo = nullptr;     // auxiliary stream, after a prepared geometry
  bool pre_valid = false;          // ev_pre recorded since the last prepare
  const void* prepared = nullptr;  // VoF of the prepared geometry, or null
  // ACDI: the next step's phase field prepared on the auxiliary stream
  // (prepared then points at prepared_phase), with the velocity it took
  bool prepared_phase = false;
  const void* prep_u0 = nullptr;
  // 3D weighted form: the third level-set buffer, which a geometry prepared
  // while a transport reads chi[chi_cur] sweeps into (with chi[1 - chi_cur])
  // and which the step that consumes it swaps with chi[chi_cur]
  void* chi_snap = nullptr;
  uint8_t* q_snap = nullptr;  // its per-tile flags (3D moving geometry)
  bool materialized;  // chi[chi_cur] holds explicit values on every tile
  // adjoint scratch: advected state, nu, per-workgroup dtheta partials
  void* adj[4];
  double* adj_part;
  // optional per-launch event timing
  bool profile;
  struct Mark { hipEvent_t a, b; int kind; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
};

struct surf_batch {
  int n = 0;
  int prec = 0;
  std::vector<surf_grid> grids;
  std::vector<surf_params> prm;
  hipStream_t stream = nullptr;
  double* states = nullptr;
  double* part = nullptr;
  void* inst_tab = nullptr;
  int2* queue = nullptr;
  void* fargs = nullptr;
  int* first = nullptr;
  void* scratch[2] = {nullptr, nullptr};
  std::vector<void*> chi;
  std::vector<uint8_t*> q;
  std::vector<int> ntiles, tx;
  int total_tiles = 0;
  std::vector<char> host_inst;
  std::vector<int2> host_queue;
  std::vector<char> host_fargs;
  std::vector<int> host_first;
  std::vector<void*> F, P, S;
  int parity = 0;
  int nt = 512;      // tile kernel (paper-form instances): threads per workgroup
  int grid = 0;      // tile kernel: persistent workgroups
  // column kernel (weighted-form instances): row-chunk height, persistent
  // workgroups (a multiple of 8), its work-list length and record count
  int ty = 8;
  int col_grid = 0;
  int ncol_q = 0;
  int col_records = 0;  // records reserved for column entries (row chunks of 8)
  void* col_inst = nullptr;
  int2* col_queue = nullptr;
  std::vector<char> host_col_inst;
  std::vector<int2> host_col_queue;
  std::string tune_key;
  struct Graph {
    int nsteps, parity;
    double* totals;
    hipGraph_t g;
    hipGraphExec_t e;
  };
  std::vector<Graph> graphs;
};

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// tile shapes of the step kernel per (precision, dim)
void tile_shape(int prec, int dim, int* t) {
  if (dim == 2) { t[0] = 64; t[1] = 16; t[2] = 1; }
  else if (prec == SURF_F32) { t[0] = 16; t[1] = 8; t[2] = 8; }
  else { t[0] = 8; t[1] = 8; t[2] = 4; }
}

int check_grid_params(const surf_grid* gr, const surf_params* p) {
  if (!gr || !p) return SURF_EINVAL;
  if (gr->dim != 2 && gr->dim != 3) return SURF_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (d < gr->dim) {
      if (gr->n[d] < 4) return SURF_EINVAL;  // mirror ghosts need 3 interior cells
      for (int s = 0; s < 2; ++s)
        if (gr->bc[d][s] < 0 || gr->bc[d][s] > 2) return SURF_EINVAL;
      if ((gr->bc[d][0] == SURF_BC_PERIODIC) != (gr->bc[d][1] == SURF_BC_PERIODIC)) return SURF_EINVAL;
    } else if (gr->n[d] != 1) {
      return SURF_EINVAL;
    }
  }
  if (!(gr->h > 0) || !std::isfinite(gr->h)) return SURF_EINVAL;
  double ncell = (double)gr->n[0] * gr->n[1] * gr->n[2];
  if (ncell > 4.0e9) return SURF_EINVAL;
  if (p->precision != SURF_F32 && p->precision != SURF_F64) return SURF_EINVAL;
  if (p->flux_form < 0 || p->flux_form > 1) return SURF_EINVAL;
  if (p->kinetics < 0 || p->kinetics > 1) return SURF_EINVAL;
  if (p->eos < 0 || p->eos > 2) return SURF_EINVAL;
  if (!(p->eps > 0) || !(p->D_b >= 0) || !(p->D_s >= 0) || !(p->k_a >= 0) || !(p->k_d >= 0))
    return SURF_EINVAL;
  if (!(p->gamma_inf > 0)) return SURF_EINVAL;
  if (!(p->dt > 0) || !std::isfinite(p->dt)) return SURF_EINVAL;
  if (p->hj_iters_init < 0 || p->hj_iters_step < 0) return SURF_EINVAL;
  if (p->substep2 < 0 || p->substep2 > 1) return SURF_EINVAL;
  if (p->interface < 0 || p->interface > 1) return SURF_EINVAL;
  if (gr->axisym < 0 || gr->axisym > 1) return SURF_EINVAL;
  if (gr->axisym &&
      (gr->dim != 2 || gr->bc[0][0] == SURF_BC_PERIODIC || !(gr->origin[0] >= 0) ||
       !std::isfinite(gr->origin[0]) || p->adjoint))
    return SURF_EINVAL;
  if (p->interface == SURF_IFACE_ACDI &&
      (!(p->acdi_zeta > 0) || !std::isfinite(p->acdi_zeta) || !(p->acdi_vareps >= 0) ||
       p->acdi_vareps >= 0.5 || p->adjoint))
    return SURF_EINVAL;
  if (p->limiter < 0 || p->limiter > 1 || p->transverse < 0 || p->transverse > 1)
    return SURF_EINVAL;
  // the variants run in the 2D weighted-form transport, in the 3D tile
  // transport (k_step) and in the implicit path's advection (2D or 3D)
  if ((p->limiter || p->transverse) && (p->flux_form != SURF_FLUX_WEIGHTED || p->adjoint))
    return SURF_EINVAL;
  // the adjoint kernels index cells and faces in 32 bits and launch a grid of
  // (nx/64, ny/4, nz) workgroups
  if (p->adjoint && ((double)(gr->n[0] + 1) * (gr->n[1] + 1) * (gr->n[2] + 1) >= 2147483648.0 ||
                     (gr->n[1] + 3) / 4 > 65535 || gr->n[2] > 65535))
    return SURF_EINVAL;
  if (p->substep2 == SURF_SUBSTEP2_IMPLICIT &&
      (p->adjoint || p->picard_iters < 0 ||
       p->picard_iters > IMP_MAX_PICARD || p->cg_max_iters < 0 || !(p->cg_tol >= 0) ||
       ncell >= 2147483648.0))
    return SURF_EINVAL;
  return SURF_OK;
}

surf_params with_defaults(const surf_params* in, int dim) {
  surf_params p = *in;
  if (p.eta == 0) p.eta = 1e-12;
  if (p.chi_max_eps == 0) p.chi_max_eps = 12.0;
  if (p.cfl_adv == 0) p.cfl_adv = 0.5;
  if (p.cfl_diff == 0) p.cfl_diff = 0.8;
  if (p.hj_iters_step == 0) p.hj_iters_step = 8;
  if (p.picard_iters == 0) p.picard_iters = 3;
  if (p.cg_max_iters == 0) p.cg_max_iters = 400;
  if (p.cg_tol == 0) p.cg_tol = 1e-12;
  if (p.acdi_vareps == 0) p.acdi_vareps = 1e-6;
  return p;
}

int hj_init_iters(const surf_ctx* c) {
  if (c->prm.hj_iters_init > 0) return c->prm.hj_iters_init;
  double chimax = c->prm.chi_max_eps * c->prm.eps;
  double dtau = c->grid.h / c->grid.dim;
  return 2 * (int)std::ceil(chimax / dtau - 1e-9);
}

template <typename R>
Par<R> make_par(const surf_ctx* c) {
  Par<R> p;
  const surf_params& q = c->prm;
  p.h = (R)c->grid.h;
  p.inv_h = (R)(1.0 / c->grid.h);
  p.eps = (R)q.eps;
  p.inv_eps = (R)(1.0 / q.eps);
  p.Db = (R)q.D_b;
  p.Ds = (R)q.D_s;
  p.ka = (R)q.k_a;
  p.kd = (R)q.k_d;
  p.ginf = (R)q.gamma_inf;
  p.inv_ginf = (R)(1.0 / q.gamma_inf);
  p.sigma0 = (R)q.sigma0;
  p.E = (R)q.eos_E;
  p.eta = (R)q.eta;
  p.eta_eps = (R)(q.eta / q.eps);
  p.chimax = (R)(q.chi_max_eps * q.eps);
  p.form = q.flux_form;
  p.kin = q.kinetics;
  p.eos = q.eos;
  p.bulk = q.bulk_enabled ? 1 : 0;
  return p;
}

size_t esize(const surf_params* p) { return p->precision == SURF_F64 ? 8 : 4; }

int nblocks_step(const surf_grid* gr, const surf_params* p, int* tiles) {
  int t[3];
  tile_shape(p->precision, gr->dim, t);
  long long nb = 1;
  for (int d = 0; d < 3; ++d) {
    tiles[d] = d < gr->dim ? (gr->n[d] + t[d] - 1) / t[d] : 1;
    nb *= tiles[d];
  }
  return (int)nb;
}

constexpr int T2X = 64, T2Y = 16, STEP2D_THREADS = 512;

int ntiles_2d(const surf_grid* gr, int* t) {
  if (gr->dim != 2) { t[0] = t[1] = 0; return 0; }
  t[0] = (gr->n[0] + T2X - 1) / T2X;
  t[1] = (gr->n[1] + T2Y - 1) / T2Y;
  return t[0] * t[1];
}

// Column-streaming launch shape of the 2D weighted-form transport: strips of
// COL_OUT columns, row chunks of COL_TY rows (FP32) or COL_TY64 (FP64),
// COL_WAVES chunks per workgroup.  Returns the workgroup count (0 when the
// kernel does not apply).
constexpr int COL_TY = 8, COL_TY64 = 8;
int col_shape(const surf_grid* gr, const surf_params* p, int* strips, int* groups) {
  *strips = *groups = 0;
  if (gr->dim != 2 || p->flux_form != SURF_FLUX_WEIGHTED) return 0;
  // 32-bit byte offsets of the buffer-resource access
  const long long es = p->precision == SURF_F64 ? 8 : 4;
  if ((long long)(gr->n[0] + 1) * (gr->n[1] + 1) * es > 0x7fffffffll) return 0;
  int ty = p->precision == SURF_F64 ? COL_TY64 : COL_TY;
  int chunks = (gr->n[1] + ty - 1) / ty;
  *strips = (gr->n[0] + COL_OUT - 1) / COL_OUT;
  *groups = (chunks + COL_WAVES - 1) / COL_WAVES;
  return *strips * *groups;
}

// Plane-marching launch shape of the 3D weighted-form transport: strips of
// COL_OUT columns, blocks of C3_OUT_ROWS rows, chunks of C3_TZ planes (FP32)
// or C3_TZ64 (FP64).  Returns the workgroup count (0 when the kernel does not
// apply).
constexpr int C3_TZ = 16, C3_TZ64 = 8;

// the 3D pipelined moving interface keeps a third level-set buffer
bool snapshot_needed(const surf_grid* gr, const surf_params* p, int nc3) {
  return gr->dim == 3 && nc3 > 0 && p->substep2 == SURF_SUBSTEP2_EXPLICIT &&
         p->interface == SURF_IFACE_VOF;
}
int col3_shape(const surf_grid* gr, const surf_params* p, int* s) {
  s[0] = s[1] = s[2] = 0;
  if (gr->dim != 3 || p->flux_form != SURF_FLUX_WEIGHTED) return 0;
  // the substep-1 variants run in the tile transport (k_step)
  if (p->limiter || p->transverse) return 0;
  // 32-bit byte offsets of the buffer-resource access
  const long long es = p->precision == SURF_F64 ? 8 : 4;
  if ((long long)(gr->n[0] + 1) * (gr->n[1] + 1) * (gr->n[2] + 1) * es > 0x7fffffffll) return 0;
  const int tz = p->precision == SURF_F64 ? C3_TZ64 : C3_TZ;
  s[0] = (gr->n[0] + COL_OUT - 1) / COL_OUT;
  s[1] = (gr->n[1] + C3_OUT_ROWS - 1) / C3_OUT_ROWS;
  s[2] = (gr->n[2] + tz - 1) / tz;
  return s[0] * s[1] * s[2];
}

// Tiles of the weighted-form geometry kernel (0 when it does not apply).
int geo_tiles(const surf_grid* gr, const surf_params* p, int* t) {
  t[0] = t[1] = 0;
  if (gr->dim != 2 || p->flux_form != SURF_FLUX_WEIGHTED) return 0;
  t[0] = (gr->n[0] + GEO_T - 1) / GEO_T;
  t[1] = (gr->n[1] + GEO_T - 1) / GEO_T;
  return t[0] * t[1];
}

// Tiles of the 3D moving geometry (0 in 2D).
int geo3_tiles(const surf_grid* gr, int* t) {
  t[0] = t[1] = t[2] = 0;
  if (gr->dim != 3) return 0;
  for (int d = 0; d < 3; ++d) t[d] = (gr->n[d] + G3 - 1) / G3;
  return t[0] * t[1] * t[2];
}

// workgroups of the adjoint kernels (64 x 4 cells of one plane each)
long long adj_blocks(const surf_grid* gr) {
  return (long long)((gr->n[0] + ADJ_TX - 1) / ADJ_TX) * ((gr->n[1] + ADJ_TY - 1) / ADJ_TY) *
         gr->n[2];
}

int flag_count(const surf_grid* gr, const surf_params* p) {
  int t2[2], tg[2], t3[3];
  int a = ntiles_2d(gr, t2), b = geo_tiles(gr, p, tg), c = geo3_tiles(gr, t3);
  a = a > b ? a : b;
  return a > c ? a : c;
}

int status_of_launch() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SURF_OK : SURF_EDEVICE;
}

unsigned grid1d(long long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

hipEvent_t take_event(surf_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// brackets one launch with events when profiling is on
struct Timed {
  surf_ctx* c;
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(surf_ctx* cc, int k, hipStream_t s = nullptr) : c(cc), kind(k), st(s ? s : cc->stream) {
    if (c->profile) {
      a = take_event(c);
      b = take_event(c);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~Timed() {
    if (c->profile && a && b) {
      (void)hipEventRecord(b, st);
      c->marks.push_back({a, b, kind});
    }
  }
};

template <typename R>
void materialize(surf_ctx* c) {
  if (c->materialized || c->ntiles2d == 0) {
    c->materialized = true;
    return;
  }
  hipLaunchKernelGGL((k_materialize<R, T2X, T2Y>), dim3(c->ntiles2d), dim3(BLOCK), 0, c->stream,
                     c->g, (R*)c->chi[c->chi_cur], (const uint8_t*)c->q[c->chi_cur],
                     (R)(c->prm.chi_max_eps * c->prm.eps), c->tiles2d[0], c->ntiles2d);
  c->materialized = true;
}

// After a full-box level-set pass neither buffer's tiles are known to hold
// the clamp: both flag arrays say live.
void flags_live(surf_ctx* c) {
  if (c->nflags == 0) return;
  for (int b = 0; b < 3; ++b) {
    uint8_t* q = b < 2 ? c->q[b] : c->q_snap;
    if (q)
      hipLaunchKernelGGL(k_fill_u8, dim3((c->nflags + BLOCK - 1) / BLOCK), dim3(BLOCK), 0,
                         c->stream, q, (uint8_t)Q_LIVE, c->nflags);
  }
}

// ACDI: phi from the current level set
template <typename R>
void acdi_init(surf_ctx* c) {
  if (c->prm.interface != SURF_IFACE_ACDI) return;
  const long long n = c->ncell;
  hipLaunchKernelGGL(k_acdi_init<R>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g,
                     make_par<R>(c), (const R*)c->chi[c->chi_cur], (R*)c->acdi[0], n);
}

template <typename R>
int geometry_impl(surf_ctx* c, const void* vof, int full) {
  Par<R> p = make_par<R>(c);
  long long n = c->ncell;
  const R* f = (const R*)vof;
  if (!full) materialize<R>(c);
  hipLaunchKernelGGL(k_pin<R>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g, p, f,
                     (R*)c->g0, n);
  int iters;
  if (full) {
    hipLaunchKernelGGL(k_chi0<R>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g, p, f,
                       (R*)c->chi[c->chi_cur], n);
    iters = hj_init_iters(c);
  } else {
    iters = c->prm.hj_iters_step;
  }
  R dtau = (R)(c->grid.h / c->grid.dim);
  for (int it = 0; it < iters; ++it) {
    int nxt = 1 - c->chi_cur;
    Timed tm(c, 1);
    hipLaunchKernelGGL(k_hj<R>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g, p,
                       (const R*)c->chi[c->chi_cur], (const R*)c->g0, (R*)c->chi[nxt], dtau, n);
    c->chi_cur = nxt;
  }
  c->has_chi = true;
  c->materialized = true;
  flags_live(c);
  acdi_init<R>(c);
  return status_of_launch();
}

// ACDI interface: a VoF field re-initializes phi (the level set warm-started
// from the current one, then phi from it); without one phi advances by one
// ACDI step, which also writes the level set the transport reads.
// One ACDI step from the phase field: phi* and s into the context's scratch
// fields, the new phi and its level set into phi_out and chi_out.
template <typename R>
void acdi_launch(surf_ctx* c, const void* const* u, R* phi_out, R* chi_out,
                 hipStream_t st = nullptr) {
  if (!st) st = c->stream;
  AcdiArgs<R> a;
  a.g = c->g;
  a.p = make_par<R>(c);
  a.dt = (R)c->dt;
  a.cfl = (R)(c->dt / c->grid.h);
  a.zeta = (R)c->prm.acdi_zeta;
  a.ve = (R)c->prm.acdi_vareps;
  a.ncell = c->ncell;
  a.lim = c->prm.limiter;
  a.tr = c->prm.transverse;
  a.axi = c->grid.axisym ? 1 : 0;
  a.r0 = c->grid.origin[0];
  a.h = c->grid.h;
  const bool has_u = u && u[0];
  const dim3 gr(acdi_xblocks(c->grid.n[0]) * c->grid.n[1] * c->grid.n[2]);
  const R* u0 = has_u ? (const R*)u[0] : nullptr;
  const R* u1 = has_u ? (const R*)u[1] : nullptr;
  const R* u2 = (has_u && c->grid.dim == 3) ? (const R*)u[2] : nullptr;
  const bool var = c->prm.limiter || c->prm.transverse;
  if (c->grid.dim == 3) {
    if (var)
      hipLaunchKernelGGL((k_acdi_adv<R, 3, true>), gr, dim3(ACDI_TX), 0, st, a,
                         (const R*)c->acdi[0], u0, u1, u2, (R*)c->acdi[1], (R*)c->acdi[2]);
    else
      hipLaunchKernelGGL((k_acdi_adv<R, 3>), gr, dim3(ACDI_TX), 0, st, a,
                         (const R*)c->acdi[0], u0, u1, u2, (R*)c->acdi[1], (R*)c->acdi[2]);
    hipLaunchKernelGGL((k_acdi_reg<R, 3>), gr, dim3(ACDI_TX), 0, st, a,
                       (const R*)c->acdi[1], (const R*)c->acdi[2], phi_out, chi_out);
  } else {
    if (var)
      hipLaunchKernelGGL((k_acdi_adv<R, 2, true>), gr, dim3(ACDI_TX), 0, st, a,
                         (const R*)c->acdi[0], u0, u1, u2, (R*)c->acdi[1], (R*)c->acdi[2]);
    else
      hipLaunchKernelGGL((k_acdi_adv<R, 2>), gr, dim3(ACDI_TX), 0, st, a,
                         (const R*)c->acdi[0], u0, u1, u2, (R*)c->acdi[1], (R*)c->acdi[2]);
    hipLaunchKernelGGL((k_acdi_reg<R, 2>), gr, dim3(ACDI_TX), 0, st, a,
                       (const R*)c->acdi[1], (const R*)c->acdi[2], phi_out, chi_out);
  }
}

template <typename R>
int acdi_geometry(surf_ctx* c, const void* vof, const void* const* u) {
  if (vof) return geometry_impl<R>(c, vof, 0);
  {
    Timed tm(c, 1);
    acdi_launch<R>(c, u, (R*)c->acdi[0], (R*)c->chi[c->chi_cur]);
  }
  c->materialized = true;
  return status_of_launch();
}

// Measurement aid: `reps` ACDI steps back to back from the current phase
// field, the new phi and level set written to free scratch (the pin-data
// buffer and the idle level-set buffer), so the context's state is unchanged.
template <typename R>
int time_acdi_impl(surf_ctx* c, const void* const* u, int reps, double* ms_per_step) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return SURF_EDEVICE;
  }
  int rc = SURF_OK;
  if (hipEventRecord(e0, c->stream) != hipSuccess) rc = SURF_EDEVICE;
  for (int r = 0; r < reps && rc == SURF_OK; ++r)
    acdi_launch<R>(c, u, (R*)c->g0, (R*)c->chi[1 - c->chi_cur]);
  if (rc == SURF_OK) rc = status_of_launch();
  float ms = 0.f;
  if (rc == SURF_OK &&
      (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = SURF_EDEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == SURF_OK) *ms_per_step = (double)ms / reps;
  return rc;
}

template <typename R, int DIM, int TX, int TY, int TZ>
void launch_step(surf_ctx* c, const StepArgs<R>& a) {
  hipLaunchKernelGGL((k_step<R, DIM, TX, TY, TZ>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a);
}

// The fused 2D kernel handles both the static and the moving interface (the
// latter with its redistancing sweeps inside, FP32 only, up to 16 sweeps and
// grids of at least 2 (K + 2) cells per axis so mirror ghosts stay inside).
template <typename R>
bool fused_moving_ok(const surf_ctx* c) {
  if (c->grid.dim != 2 || sizeof(R) != 4) return false;
  int K = c->prm.hj_iters_step;
  if (K > 16) return false;
  int KH = K <= 8 ? 8 : 16;
  return c->grid.n[0] >= 2 * (KH + 2) && c->grid.n[1] >= 2 * (KH + 2);
}

// The standalone geometry kernel of the weighted-form path: up to 16 sweeps,
// grids of at least 2 (K + 2) cells per axis (mirror ghosts stay inside).
template <typename R>
bool geom2d_ok(const surf_ctx* c) {
  if (c->grid.dim != 2 || c->col_nwg == 0) return false;
  int K = c->prm.hj_iters_step;
  if (K > 16) return false;
  int KH = K <= 8 ? 8 : 16;
  return c->grid.n[0] >= 2 * (KH + 2) && c->grid.n[1] >= 2 * (KH + 2);
}

template <typename R, int TY>
void launch_col2d(surf_ctx* c, const ColArgs<R>& a, bool has_u, bool bulk) {
  const dim3 grid(8 * a.per_xcd), block(64 * COL_WAVES);
  if (c->grid.axisym) {
    if (has_u && (c->prm.limiter || c->prm.transverse)) {
      // substep-1 variants on the rings: Cartesian face values, ring weights
      const int v = (c->prm.limiter ? 1 : 0) + (c->prm.transverse ? 2 : 0);
      if (bulk) {
        if (v == 1) hipLaunchKernelGGL((k_col2d<R, TY, true, true, true, 1, false>), grid, block, 0, c->stream, a);
        else if (v == 2) hipLaunchKernelGGL((k_col2d<R, TY, true, true, true, 0, true>), grid, block, 0, c->stream, a);
        else hipLaunchKernelGGL((k_col2d<R, TY, true, true, true, 1, true>), grid, block, 0, c->stream, a);
      } else {
        if (v == 1) hipLaunchKernelGGL((k_col2d<R, TY, true, false, true, 1, false>), grid, block, 0, c->stream, a);
        else if (v == 2) hipLaunchKernelGGL((k_col2d<R, TY, true, false, true, 0, true>), grid, block, 0, c->stream, a);
        else hipLaunchKernelGGL((k_col2d<R, TY, true, false, true, 1, true>), grid, block, 0, c->stream, a);
      }
      return;
    }
    if (has_u && bulk) hipLaunchKernelGGL((k_col2d<R, TY, true, true, true>), grid, block, 0, c->stream, a);
    else if (has_u) hipLaunchKernelGGL((k_col2d<R, TY, true, false, true>), grid, block, 0, c->stream, a);
    else if (bulk) hipLaunchKernelGGL((k_col2d<R, TY, false, true, true>), grid, block, 0, c->stream, a);
    else hipLaunchKernelGGL((k_col2d<R, TY, false, false, true>), grid, block, 0, c->stream, a);
    return;
  }
  if (has_u && (c->prm.limiter || c->prm.transverse)) {
    // substep-1 variants (the scheme only matters with a flow)
    const int v = (c->prm.limiter ? 1 : 0) + (c->prm.transverse ? 2 : 0);
    if (bulk) {
      if (v == 1) hipLaunchKernelGGL((k_col2d<R, TY, true, true, false, 1, false>), grid, block, 0, c->stream, a);
      else if (v == 2) hipLaunchKernelGGL((k_col2d<R, TY, true, true, false, 0, true>), grid, block, 0, c->stream, a);
      else hipLaunchKernelGGL((k_col2d<R, TY, true, true, false, 1, true>), grid, block, 0, c->stream, a);
    } else {
      if (v == 1) hipLaunchKernelGGL((k_col2d<R, TY, true, false, false, 1, false>), grid, block, 0, c->stream, a);
      else if (v == 2) hipLaunchKernelGGL((k_col2d<R, TY, true, false, false, 0, true>), grid, block, 0, c->stream, a);
      else hipLaunchKernelGGL((k_col2d<R, TY, true, false, false, 1, true>), grid, block, 0, c->stream, a);
    }
    return;
  }
  if (has_u && bulk) hipLaunchKernelGGL((k_col2d<R, TY, true, true>), grid, block, 0, c->stream, a);
  else if (has_u) hipLaunchKernelGGL((k_col2d<R, TY, true, false>), grid, block, 0, c->stream, a);
  else if (bulk) hipLaunchKernelGGL((k_col2d<R, TY, false, true>), grid, block, 0, c->stream, a);
  else hipLaunchKernelGGL((k_col2d<R, TY, false, false>), grid, block, 0, c->stream, a);
}

template <typename R, int TZ>
void launch_col3d(surf_ctx* c, const Col3Args<R>& a, bool has_u, bool bulk) {
  const dim3 grid(8 * a.per_xcd), block(64 * C3_WAVES);
  if (a.Pst) {  // the instance that also stores the advected state
    if (has_u && bulk) hipLaunchKernelGGL((k_col3d<R, TZ, true, true, true>), grid, block, 0, c->stream, a);
    else if (has_u) hipLaunchKernelGGL((k_col3d<R, TZ, true, false, true>), grid, block, 0, c->stream, a);
    else if (bulk) hipLaunchKernelGGL((k_col3d<R, TZ, false, true, true>), grid, block, 0, c->stream, a);
    else hipLaunchKernelGGL((k_col3d<R, TZ, false, false, true>), grid, block, 0, c->stream, a);
    return;
  }
  if (has_u && bulk) hipLaunchKernelGGL((k_col3d<R, TZ, true, true, false>), grid, block, 0, c->stream, a);
  else if (has_u) hipLaunchKernelGGL((k_col3d<R, TZ, true, false, false>), grid, block, 0, c->stream, a);
  else if (bulk) hipLaunchKernelGGL((k_col3d<R, TZ, false, true, false>), grid, block, 0, c->stream, a);
  else hipLaunchKernelGGL((k_col3d<R, TZ, false, false, false>), grid, block, 0, c->stream, a);
}

template <typename R, int KH>
void launch_step2d(surf_ctx* c, const Step2dArgs<R>& a) {
  // the paper form on axisymmetric rings takes the instance with the ring
  // weights (the weighted form on rings runs in k_col2d)
  if (c->grid.axisym)
    hipLaunchKernelGGL((k_step2d<R, KH, STEP2D_THREADS, T2X, T2Y, true>), dim3(8 * c->per_xcd),
                       dim3(STEP2D_THREADS), 0, c->stream, a);
  else
    hipLaunchKernelGGL((k_step2d<R, KH, STEP2D_THREADS, T2X, T2Y>), dim3(8 * c->per_xcd),
                       dim3(STEP2D_THREADS), 0, c->stream, a);
}

FinalArgs final_of(const surf_grid& gr, const surf_params& q, int nblk, double dt) {
  FinalArgs f;
  f.nblk = nblk;
  f.dim = gr.dim;
  f.bulk = q.bulk_enabled ? 1 : 0;
  f.h = gr.h;
  f.ka = q.k_a;
  f.cfl_a = q.cfl_adv;
  f.cfl_d = q.cfl_diff;
  f.dt = dt;
  // explicit bound of substep 2: diffusion (with the weighted form's
  // neighbour-weight excess cosh(h/eps) - 1, or the paper form's B term) plus
  // the source's rates; the c_max term is added on the device
  const double nd = gr.dim, h = gr.h, eps = q.eps;
  const double Dmax = f.bulk ? std::fmax(q.D_b, q.D_s) : q.D_s;
  double lam = q.flux_form == SURF_FLUX_WEIGHTED
                   ? Dmax * (2.0 * nd - 1.0 + std::cosh(h / eps)) / (h * h)
                   : Dmax * (2.0 * nd / (h * h) + std::sqrt(nd) / (eps * h));
  if (f.bulk) lam += q.k_a * q.gamma_inf / eps + q.k_d;
  f.lam0 = lam;
  f.implicit = q.substep2 == SURF_SUBSTEP2_IMPLICIT ? 1 : 0;
  // ACDI: its regularization is explicit, a diffusion zeta eps plus a
  // transport at speed up to zeta (the same form as the paper-form bound)
  f.lam_acdi = q.interface == SURF_IFACE_ACDI
                   ? q.acdi_zeta * (2.0 * nd * eps / (h * h) + std::sqrt(nd) / h)
                   : 0.0;
  return f;
}

template <typename R>
void finalize(surf_ctx* c, double* totals, int nblk);

// 3D moving geometry: K warm-start sweeps over the tiles near the interface
// (even K up to the tile edge), the level set of the other tiles at the clamp.
template <typename R>
bool geo3_ok(const surf_ctx* c) {
  const int K = c->prm.hj_iters_step;
  return c->grid.dim == 3 && c->ng3 > 0 && K >= 2 && K <= G3 && (K % 2) == 0;
}

// The level set stays in chi[chi_cur] (R); chi[1 - chi_cur] (S) is the
// sweeps' partner and its flag array also carries this step's live marks.
// With third = true (a geometry prepared while a transport reads R) the
// sweeps alternate between S and chi_snap (T) and end in T, which the step
// that consumes them makes the current buffer.
template <typename R>
void geo3_impl(surf_ctx* c, const void* vof, hipStream_t st = nullptr, bool third = false) {
  if (!st) st = c->stream;
  Geo3Args ga;
  ga.g = c->g;
  for (int d = 0; d < 3; ++d) ga.tiles[d] = c->g3tiles[d];
  ga.ntiles = c->ng3;
  ga.per_xcd = (c->ng3 + 7) / 8;
  const Par<R> p = make_par<R>(c);
  R* chiR = (R*)c->chi[c->chi_cur];
  R* chiS = (R*)c->chi[1 - c->chi_cur];
  uint8_t* qR = c->q[c->chi_cur];
  uint8_t* qS = c->q[1 - c->chi_cur];
  const int K = c->prm.hj_iters_step;
  {
    Timed tm(c, 1, st);
    R* chiT = third ? (R*)c->chi_snap : nullptr;
    uint8_t* qT = third ? c->q_snap : nullptr;
    hipLaunchKernelGGL(k_geo3_classify<R>, dim3(8 * ga.per_xcd), dim3(G3_THREADS), 0, st,
                       ga, p, (const R*)vof, chiS, (R*)c->g0, (const uint8_t*)qR, qS, chiT, qT,
                       c->state);
    hipLaunchKernelGGL(k_geo3_list, dim3(1), dim3(G3_LIST_THREADS), 0, st,
                       (const uint8_t*)qS, c->ng3, c->live3);
    const R dtau = (R)(c->grid.h / 3);
    // odd sweeps R -> S (T -> S after the first with a third buffer), even
    // sweeps S -> R (S -> T)
    R* chiE = third ? chiT : chiR;
    uint8_t* qE = third ? qT : qR;
    for (int k = 1; k <= K; ++k) {
      const R* src = (k & 1) ? (k == 1 ? chiR : chiE) : chiS;
      R* dst = (k & 1) ? chiS : chiE;
      hipLaunchKernelGGL(k_geo3_sweep<R>, dim3(G3_SWEEP_GRID), dim3(G3_SWEEP_THREADS), 0,
                         st, ga, p, dtau, src, dst, (const R*)c->g0, qE,
                         (const int*)c->live3, k == K ? 1 : 0);
    }
  }
  c->materialized = true;
}

// The 2D weighted-form transport kernel alone, on the context's stream.
template <typename R>
void col2d_transport(surf_ctx* c, const void* const* u, const void* F_in, const void* psi_in,
                     void* F_out, void* psi_out, void* sigma_out) {
  ColArgs<R> a;
  a.g = c->g;
  a.p = make_par<R>(c);
  a.chi = (const R*)c->chi[c->chi_cur];
  const bool has_u = u && u[0];
  const bool bulk = c->prm.bulk_enabled != 0;
  a.u[0] = has_u ? (const R*)u[0] : nullptr;
  a.u[1] = has_u ? (const R*)u[1] : nullptr;
  a.F = (const R*)F_in;
  a.psi = (const R*)psi_in;
  a.Fo = (R*)F_out;
  a.Po = (R*)psi_out;
  a.sig = (R*)sigma_out;
  a.part = c->part;
  a.state = c->state;
  a.dt = (R)c->dt;
  a.area_dt = (R)(c->grid.h * c->dt);
  a.r0 = c->grid.origin[0];
  a.strips = c->col_strips;
  a.groups = c->col_groups;
  a.nwg = c->col_nwg;
  a.per_xcd = (c->col_nwg + 7) / 8;
  if constexpr (sizeof(R) == 4) launch_col2d<R, COL_TY>(c, a, has_u, bulk);
  else launch_col2d<R, COL_TY64>(c, a, has_u, bulk);
}

// The 3D weighted-form transport kernel alone, on the context's stream.
template <typename R>
void col3d_transport(surf_ctx* c, const void* const* u, const void* F_in, const void* psi_in,
                     void* F_out, void* psi_out, void* sigma_out, const void* chi = nullptr,
                     void* F_star = nullptr, void* psi_star = nullptr) {
  Col3Args<R> a;
  a.g = c->g;
  a.p = make_par<R>(c);
  a.chi = (const R*)(chi ? chi : c->chi[c->chi_cur]);
  const bool has_u = u && u[0];
  const bool bulk = c->prm.bulk_enabled != 0;
  for (int d = 0; d < 3; ++d) a.u[d] = has_u ? (const R*)u[d] : nullptr;
  a.F = (const R*)F_in;
  a.psi = (const R*)psi_in;
  a.Fo = (R*)F_out;
  a.Po = (R*)psi_out;
  a.sig = (R*)sigma_out;
  a.part = c->part;
  a.state = c->state;
  a.dt = (R)c->dt;
  a.area_dt = (R)(c->grid.h * c->grid.h * c->dt);
  a.strips = c->c3[0];
  a.yblocks = c->c3[1];
  a.zchunks = c->c3[2];
  a.nwg = c->c3_nwg;
  a.per_xcd = (c->c3_nwg + 7) / 8;
  a.Fst = (R*)F_star;
  a.Pst = (R*)psi_star;
  if constexpr (sizeof(R) == 4) launch_col3d<R, C3_TZ>(c, a, has_u, bulk);
  else launch_col3d<R, C3_TZ64>(c, a, has_u, bulk);
}

// Weighted-form moving geometry in 2D on `st`: the classify pass, then the
// live tiles (every tile of chi_out ends with chi^{n+1}); chi_out becomes the
// current level set.
template <typename R>
void geo2d_launch(surf_ctx* c, const void* vof_next, hipStream_t st) {
  Step2dArgs<R> a{};
  a.g = c->g;
  a.p = make_par<R>(c);
  a.vof = (const R*)vof_next;
  a.chi_in = (const R*)c->chi[c->chi_cur];
  a.chi_out = (R*)c->chi[1 - c->chi_cur];
  a.q_in = c->q[c->chi_cur];
  a.q_out = c->q[1 - c->chi_cur];
  a.mark = c->mark;
  a.state = c->state;
  a.dtau = (R)(c->grid.h / 2);
  a.ksweeps = c->prm.hj_iters_step;
  a.tiles[0] = c->gtiles[0];
  a.tiles[1] = c->gtiles[1];
  a.ntiles = c->ngtiles;
  a.per_xcd = (c->ngtiles + 7) / 8;
  a.diag = (c->gtiles[0] % 8) == 0 ? 1 : 0;
  // live-tile grid: at most GEO_LIVE_CAP tiles per workgroup even if every
  // tile is live
  int nl = GEO_LIVE_GRID;
  while ((long long)nl * GEO_LIVE_CAP < c->ngtiles) nl *= 2;
  const dim3 gc((c->ngtiles + 3) / 4), gl(nl);
  if (a.ksweeps <= 8) {
    hipLaunchKernelGGL((k_geo_classify<R, 8>), gc, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_geo_live<R, 8>), gl, dim3(GEO_WG), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_geo_classify<R, 16>), gc, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_geo_live<R, 16>), gl, dim3(GEO_WG), 0, st, a);
  }
  c->chi_cur = 1 - c->chi_cur;
  c->materialized = true;
}

// Weighted form in 2D: the moving geometry (unless a prepared one is already
// current), then the column-streaming transport on the new level set, then
// the reduction.
template <typename R>
int col2d_impl(surf_ctx* c, const void* vof_next, const void* const* u, const void* F_in,
               const void* psi_in, void* F_out, void* psi_out, void* sigma_out,
               double* totals, bool geometry_ready = false) {
  if (vof_next && !geometry_ready) {
    Timed tm(c, 1);
    geo2d_launch<R>(c, vof_next, c->stream);
  } else if (!vof_next) {
    materialize<R>(c);
  }
  // the point after which a geometry for the next step may overwrite the
  // other level-set buffer: the previous transport is done
  if (c->ev_pre) {
    (void)hipEventRecord(c->ev_pre, c->stream);
    c->pre_valid = true;
  }
  {
    Timed tm(c, 0);
    col2d_transport<R>(c, u, F_in, psi_in, F_out, psi_out, sigma_out);
  }
  finalize<R>(c, totals, c->col_nwg);
  return status_of_launch();
}

template <typename R>
int step2d_impl(surf_ctx* c, const void* vof_next, const void* const* u, const void* F_in,
                const void* psi_in, void* F_out, void* psi_out, void* sigma_out,
                double* totals) {
  Step2dArgs<R> a;
  a.g = c->g;
  a.p = make_par<R>(c);
  bool moving = vof_next != nullptr;
  if (c->col_nwg > 0) return col2d_impl<R>(c, vof_next, u, F_in, psi_in, F_out, psi_out,
                                           sigma_out, totals);
  a.vof = (const R*)vof_next;
  a.chi_in = (const R*)c->chi[c->chi_cur];
  a.chi_out = (R*)c->chi[1 - c->chi_cur];
  a.q_in = c->q[c->chi_cur];
  a.q_out = c->q[1 - c->chi_cur];
  a.mark = nullptr;
  a.has_u = (u && u[0]) ? 1 : 0;
  a.u[0] = a.has_u ? (const R*)u[0] : nullptr;
  a.u[1] = a.has_u ? (const R*)u[1] : nullptr;
  a.F = (const R*)F_in;
  a.psi = (const R*)psi_in;
  a.Fo = (R*)F_out;
  a.Po = (R*)psi_out;
  a.sig = (R*)sigma_out;
  a.part = c->part;
  a.state = c->state;
  a.dt = (R)c->dt;
  a.area_dt = (R)(c->grid.h * c->dt);
  a.dtau = (R)(c->grid.h / 2);
  a.ksweeps = c->prm.hj_iters_step;
  a.tiles[0] = c->tiles2d[0];
  a.tiles[1] = c->tiles2d[1];
  a.ntiles = c->ntiles2d;
  a.per_xcd = c->per_xcd;
  a.diag = (c->tiles2d[0] % 8) == 0 ? 1 : 0;
  a.r0 = c->grid.origin[0];
  {
    Timed tm(c, 0);
    if (!moving) {
      launch_step2d<R, 0>(c, a);
    } else if constexpr (sizeof(R) == 4) {
      if (a.ksweeps <= 8) launch_step2d<R, 8>(c, a);
      else launch_step2d<R, 16>(c, a);
    }
  }
  if (moving) {
    c->chi_cur = 1 - c->chi_cur;
    c->materialized = false;
  }
  finalize<R>(c, totals, c->ntiles2d);
  return status_of_launch();
}

// A 3D step whose geometry was prepared on the auxiliary stream (the caller
// has made the context's stream wait for it): the prepared level set, in the
// third buffer, becomes the current one (the old current buffer becomes the
// third, with its flags), the point after which the next prepared geometry
// may rewrite the two others is recorded, and the transport reads it.
template <typename R>
int col3d_prepared_step(surf_ctx* c, const void* const* u, const void* F_in, const void* psi_in,
                        void* F_out, void* psi_out, void* sigma_out, double* totals) {
  std::swap(c->chi[c->chi_cur], c->chi_snap);
  std::swap(c->q[c->chi_cur], c->q_snap);
  if (hipEventRecord(c->ev_pre, c->stream) != hipSuccess) return SURF_EDEVICE;
  c->pre_valid = true;
  {
    Timed tm(c, 0);
    col3d_transport<R>(c, u, F_in, psi_in, F_out, psi_out, sigma_out);
  }
  finalize<R>(c, totals, c->c3_nwg);
  return status_of_launch();
}

template <typename R>
int step_impl(surf_ctx* c, const void* const* u, const void* F_in, const void* psi_in,
              void* F_out, void* psi_out, void* sigma_out, double* totals) {
  if (c->grid.dim == 2)
    return step2d_impl<R>(c, nullptr, u, F_in, psi_in, F_out, psi_out, sigma_out, totals);
  materialize<R>(c);
  if (c->ev_pre && c->prm.interface == SURF_IFACE_ACDI && c->c3_nwg > 0) {
    // an ACDI step prepared next writes only the other level-set buffer: it
    // may start once the transports before this one are done
    if (hipEventRecord(c->ev_pre, c->stream) != hipSuccess) return SURF_EDEVICE;
    c->pre_valid = true;
  } else {
    c->pre_valid = false;  // this transport reads chi[chi_cur] itself
  }
  if (c->c3_nwg > 0) {
    // weighted form in 3D: plane-marching transport, then the reduction
    {
      Timed tm(c, 0);
      col3d_transport<R>(c, u, F_in, psi_in, F_out, psi_out, sigma_out);
    }
    finalize<R>(c, totals, c->c3_nwg);
    return status_of_launch();
  }
  StepArgs<R> a;
  a.g = c->g;
  a.p = make_par<R>(c);
  a.chi = (const R*)c->chi[c->chi_cur];
  a.has_u = (u && u[0]) ? 1 : 0;
  a.lim = c->prm.limiter;
  a.tr = c->prm.transverse;
  for (int d = 0; d < 3; ++d) a.u[d] = (a.has_u && d < c->grid.dim) ? (const R*)u[d] : nullptr;
  a.F = (const R*)F_in;
  a.psi = (const R*)psi_in;
  a.Fo = (R*)F_out;
  a.Po = (R*)psi_out;
  a.sig = (R*)sigma_out;
  a.part = c->part;
  a.dt = (R)c->dt;
  a.area_dt = (R)((c->grid.dim == 3 ? c->grid.h * c->grid.h : c->grid.h) * c->dt);
  for (int d = 0; d < 3; ++d) a.tiles[d] = c->tiles[d];
  {
    Timed tm(c, 0);
    if (c->grid.dim == 2) {
      launch_step<R, 2, 64, 16, 1>(c, a);
    } else {
      if constexpr (sizeof(R) == 4) launch_step<R, 3, 16, 8, 8>(c, a);
      else launch_step<R, 3, 8, 8, 4>(c, a);
    }
  }
  finalize<R>(c, totals, c->nblk);
  return status_of_launch();
}

template <typename R>
void finalize(surf_ctx* c, double* totals, int nblk) {
  FinalArgs f = final_of(c->grid, c->prm, nblk, c->dt);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_BLOCK), 0, c->stream, f, (const double*)c->part,
                     c->state, totals);
}

// Implicit substep 2 (weighted form): advection, then `picard_iters` sweeps
// of the interfacial and bulk problems, each by Jacobi-CG, then the outputs,
// the records and the reduction.
//
// CG tiling: 64 x 32-cell tiles of one z-plane; at most CG_MAXWG workgroups,
// each taking a run of per_wg consecutive tiles.
void cg_shape(const surf_grid* g, int* tiles, int* ntiles, int* nwg, int* per_wg) {
  tiles[0] = (g->n[0] + CG_TX - 1) / CG_TX;
  tiles[1] = (g->n[1] + CG_TY - 1) / CG_TY;
  tiles[2] = g->dim == 3 ? g->n[2] : 1;
  *ntiles = tiles[0] * tiles[1] * tiles[2];
  int w = *ntiles < CG_MAXWG ? *ntiles : CG_MAXWG;
  *per_wg = (*ntiles + w - 1) / w;
  *nwg = (*ntiles + *per_wg - 1) / *per_wg;
}

template <typename R>
CgArgs cg_args(surf_ctx* c, const ImpArgs<R>& a, int field) {
  CgArgs k{};
  k.g = c->g;
  const bool bulk_field = field == 1;
  k.fw = bulk_field ? c->imp.wF : c->imp.wP;
  k.kc = 0.5 * (bulk_field ? a.Db : a.Ds) * a.inv_h2;
  k.tol2 = a.tol * a.tol;
  k.x = bulk_field ? c->imp.xF : c->imp.xP;
  k.p = c->imp.p;
  for (int i = 0; i < 2; ++i) {
    k.r[i] = c->imp.r[i];
    k.w[i] = c->imp.w[i];
    k.z[i] = c->imp.z[i];
  }
  k.minv = c->imp.minv;
  k.dg = c->imp.dg;
  k.part = c->imp.part;
  k.sc = c->imp.sc;
  k.axi = a.axi;
  k.r0 = a.r0;
  k.h = a.h;
  cg_shape(&c->grid, k.tiles, &k.ntiles, &k.nwg, &k.per_wg);
  return k;
}

void cg_iter_launch(surf_ctx* c, const CgArgs& k, int it) {
  const dim3 gr(k.nwg), bl(CG_WG);
  if (c->grid.dim == 3) hipLaunchKernelGGL((k_cg_iter<3, false>), gr, bl, 0, c->stream, k, it);
  else if (k.axi) hipLaunchKernelGGL((k_cg_iter<2, true>), gr, bl, 0, c->stream, k, it);
  else hipLaunchKernelGGL((k_cg_iter<2, false>), gr, bl, 0, c->stream, k, it);
}

// Host-paced iteration launches: chunks of CG_CHUNK, enqueued once the device
// has started the launch CG_LEAD before the end of the queue.
constexpr int CG_CHUNK = 4, CG_LEAD = 8;

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// Waits until solve `id` has met its test (1) or its device progress
// reached `target` launches (0), or the stream ran dry (0: everything
// enqueued has run); SURF_EDEVICE on a stream error.
int cg_wait(surf_ctx* c, unsigned long long id, int target) {
  volatile unsigned long long* hp = c->hprog;
  for (unsigned spin = 0;; ++spin) {
    if (hp[1] >= id) return 1;
    const unsigned long long pr = hp[0];
    if ((pr >> 32) == id && (long long)(pr & 0xffffffffull) >= target) return 0;
    if ((spin & 63) == 63) {
      const hipError_t q = hipStreamQuery(c->stream);
      if (q == hipSuccess) return 0;
      if (q != hipErrorNotReady) return SURF_EDEVICE;
    }
  }
}

template <typename R>
int cg_solve(surf_ctx* c, const ImpArgs<R>& a, int field, int solve, bool paced) {
  CgArgs k = cg_args(c, a, field);
  k.hp = c->hprog;
  k.solve_id = ++c->solve_serial;
  hipLaunchKernelGGL(k_cg_setup<R>, dim3(k.nwg), dim3(CG_WG), 0, c->stream, a, k, field);
  cg_iter_launch(c, k, -1);
  const int cap = c->prm.cg_max_iters;
  if (!paced) {
    for (int it = 0; it < cap; ++it) cg_iter_launch(c, k, it);
  } else {
    int enq = 0;
    while (enq < cap) {
      const int n = cap - enq < CG_CHUNK ? cap - enq : CG_CHUNK;
      for (int j = 0; j < n; ++j) cg_iter_launch(c, k, enq + j);
      enq += n;
      if (enq >= cap) break;
      const int rc = cg_wait(c, k.solve_id, enq - CG_LEAD);
      if (rc < 0) return rc;
      if (rc == 1) break;
    }
  }
  hipLaunchKernelGGL(k_cg_end, dim3(1), dim3(CG_WG), 0, c->stream, k, cap, c->imp.rec + solve,
                     c->state);
  return SURF_OK;
}

template <typename R>
ImpArgs<R> imp_args(surf_ctx* c) {
  ImpArgs<R> a;
  a.g = c->g;
  a.p = make_par<R>(c);
  a.B = c->imp;
  const surf_params& q = c->prm;
  const bool bulk = q.bulk_enabled != 0;
  a.dt = c->dt;
  a.eta = q.eta;
  a.eta_eps = q.eta / q.eps;
  a.ka = bulk ? q.k_a : 0.0;
  a.kd = bulk ? q.k_d : 0.0;
  a.ginf = q.gamma_inf;
  a.kl = q.kinetics == SURF_KIN_LANGMUIR ? 1.0 : 0.0;
  a.tol = q.cg_tol;
  a.inv_h2 = 1.0 / (c->grid.h * c->grid.h);
  a.Db = q.D_b;
  a.Ds = q.D_s;
  a.bulk = bulk ? 1 : 0;
  a.lim = c->prm.limiter;
  a.tr = c->prm.transverse;
  a.axi = c->grid.axisym ? 1 : 0;
  a.r0 = c->grid.origin[0];
  a.h = c->grid.h;
  a.paper = q.flux_form == SURF_FLUX_PAPER ? 1 : 0;
  a.ncell = c->ncell;
  return a;
}

// One paper-form linear solve by BiCGSTAB (field 0: psi, 1: F), from the
// unknown's current values: coefficients, setup, cg_max_iters iterations of
// three launches (those after the solve stopped return at once), the end.
template <typename R>
int bicg_solve(surf_ctx* c, const ImpArgs<R>& a, int field, int solve) {
  BicgArgs k{};
  k.g = c->g;
  k.k = (field == 1 ? a.Db : a.Ds) * a.inv_h2;
  k.inv_h = 1.0 / c->grid.h;
  k.tol2 = a.tol * a.tol;
  k.x = field == 1 ? c->imp.xF : c->imp.xP;
  k.p[0] = c->imp.p;
  k.p[1] = c->imp.z[1];
  k.v[0] = c->imp.w[0];
  k.v[1] = c->imp.w[1];
  k.r = c->imp.r[0];
  k.rh = c->imp.r[1];
  k.t = c->imp.z[0];
  k.minv = c->imp.minv;
  k.dg = c->imp.dg;
  for (int d = 0; d < 3; ++d) k.B[d] = c->imp.B[d];
  k.part = c->imp.part;
  k.sc = c->imp.sc;
  k.ncell = c->ncell;
  k.axi = c->grid.axisym ? 1 : 0;
  k.r0 = c->grid.origin[0];
  k.h = c->grid.h;
  const long long nb = (c->ncell + BICG_WG - 1) / BICG_WG;
  k.nwg = (int)(nb < BICG_MAXWG ? nb : BICG_MAXWG);
  const dim3 gr(k.nwg), bl(BICG_WG);
  const bool three = c->grid.dim == 3;
  hipLaunchKernelGGL(k_bicg_coef<R>, gr, bl, 0, c->stream, a, (const R*)c->chi[c->chi_cur], field,
                     c->imp.B[0], c->imp.B[1], three ? c->imp.B[2] : c->imp.B[1]);
  if (three) hipLaunchKernelGGL((k_bicg_setup<R, 3>), gr, bl, 0, c->stream, a, k, field);
  else hipLaunchKernelGGL((k_bicg_setup<R, 2>), gr, bl, 0, c->stream, a, k, field);
  const int cap = c->prm.cg_max_iters;
  for (int it = 0; it < cap; ++it) {
    if (three) {
      hipLaunchKernelGGL(k_bicg_a<3>, gr, bl, 0, c->stream, k, it);
      hipLaunchKernelGGL(k_bicg_b<3>, gr, bl, 0, c->stream, k, it);
    } else {
      hipLaunchKernelGGL(k_bicg_a<2>, gr, bl, 0, c->stream, k, it);
      hipLaunchKernelGGL(k_bicg_b<2>, gr, bl, 0, c->stream, k, it);
    }
    hipLaunchKernelGGL(k_bicg_c, gr, bl, 0, c->stream, k, it);
  }
  hipLaunchKernelGGL(k_bicg_end, dim3(1), bl, 0, c->stream, k, cap, c->imp.rec + solve,
                     c->state);
  return SURF_OK;
}

template <typename R>
int implicit_impl(surf_ctx* c, const void* const* u, const void* F_in, const void* psi_in,
                  void* F_out, void* psi_out, void* sigma_out, double* totals) {
  materialize<R>(c);
  const ImpArgs<R> a = imp_args<R>(c);
  const surf_params& q = c->prm;
  const bool bulk = q.bulk_enabled != 0;
  const bool has_u = u && u[0];
  const R area_dt = (R)((c->grid.dim == 3 ? c->grid.h * c->grid.h : c->grid.h) * c->dt);
  const dim3 gr(c->imp_nblk), bl(IMP_BLOCK);
  {
    Timed tm(c, 0);
    hipLaunchKernelGGL(k_imp_adv<R>, gr, bl, 0, c->stream, a, (const R*)c->chi[c->chi_cur],
                       has_u ? (const R*)u[0] : nullptr, has_u ? (const R*)u[1] : nullptr,
                       (has_u && c->grid.dim == 3) ? (const R*)u[2] : nullptr,
                       (const R*)F_in, (const R*)psi_in, area_dt);
    const int sweeps = bulk ? q.picard_iters : 1;
    c->imp_nsolves = bulk ? 2 * sweeps : 1;
    // outside graph capture the host paces the iteration launches
    const bool paced = !stream_capturing(c->stream);
    if (paced && !c->hprog) {
      void* hp = nullptr;
      if (hipHostMalloc(&hp, 64, hipHostMallocCoherent) == hipSuccess) {
        std::memset(hp, 0, 64);
        c->hprog = (unsigned long long*)hp;
      }
    }
    for (int s = 0; s < sweeps; ++s) {
      int rc;
      if (a.paper) {
        // the paper form's non-symmetric problems
        rc = bicg_solve<R>(c, a, 0, 2 * s);
        if (rc == SURF_OK && bulk) rc = bicg_solve<R>(c, a, 1, 2 * s + 1);
      } else {
        rc = cg_solve<R>(c, a, 0, 2 * s, paced && c->hprog);
        if (rc == SURF_OK && bulk) rc = cg_solve<R>(c, a, 1, 2 * s + 1, paced && c->hprog);
      }
      if (rc != SURF_OK) return rc;
    }
    hipLaunchKernelGGL(k_imp_final<R>, gr, bl, 0, c->stream, a, (R*)F_out, (R*)psi_out,
                       (R*)sigma_out, c->part);
  }
  finalize<R>(c, totals, c->imp_nblk);
  return status_of_launch();
}

template <typename R>
int time_solver_impl(surf_ctx* c, int field, int reps, double* ms_per_launch) {
  const ImpArgs<R> a = imp_args<R>(c);
  CgArgs k = cg_args(c, a, field);
  k.tol2 = 0.0;  // no stop test: every launch iterates
  hipLaunchKernelGGL(k_cg_setup<R>, dim3(k.nwg), dim3(CG_WG), 0, c->stream, a, k, field);
  cg_iter_launch(c, k, -1);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return SURF_EDEVICE;
  }
  int rc = SURF_OK;
  if (hipEventRecord(e0, c->stream) != hipSuccess) rc = SURF_EDEVICE;
  for (int it = 0; it < reps && rc == SURF_OK; ++it) cg_iter_launch(c, k, it);
  if (rc == SURF_OK) rc = status_of_launch();
  float ms = 0.f;
  if (rc == SURF_OK &&
      (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = SURF_EDEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == SURF_OK) *ms_per_launch = (double)ms / reps;
  return rc;
}

template <typename R>
int init_impl(surf_ctx* c, const void* c0, double c0_const, double gamma0, void* F, void* psi) {
  materialize<R>(c);
  Par<R> p = make_par<R>(c);
  long long n = c->ncell;
  hipLaunchKernelGGL(k_init<R>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g, p,
                     (const R*)c->chi[c->chi_cur], (const R*)c0, (R)c0_const, (R)gamma0,
                     c->prm.bulk_enabled ? (R*)F : (R*)nullptr, (R*)psi, n);
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, c->stream, c->state);
  return status_of_launch();
}

template <typename R>
int force_impl(surf_ctx* c, const void* sigma, void* const* force) {
  materialize<R>(c);
  Par<R> p = make_par<R>(c);
  const R* chi = (const R*)c->chi[c->chi_cur];
  const int nx = c->grid.n[0], ny = c->grid.n[1], nz = c->grid.n[2];
  if (c->grid.dim == 2) {
    constexpr int TX = 64, TY = 8;
    const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
    hipLaunchKernelGGL((k_force2<R, TX, TY>), dim3(tx * ty), dim3(TX * TY), 0, c->stream, c->g,
                       p, chi, (const R*)sigma, (R*)force[0], (R*)force[1], tx);
  } else {
    constexpr int TX = 64, TY = 8, ZC = 16;
    const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY, tz = (nz + ZC - 1) / ZC;
    hipLaunchKernelGGL((k_force3<R, TX, TY, ZC>), dim3(tx * ty * tz), dim3(TX * TY), 0,
                       c->stream, c->g, p, chi, (const R*)sigma, (R*)force[0], (R*)force[1],
                       (R*)force[2], tx, ty);
  }
  return status_of_launch();
}

template <typename R>
int iface_force_impl(surf_ctx* c, const void* vof, const void* sigma, void* const* cap,
                     void* const* ma) {
  materialize<R>(c);
  IfaceArgs<R> a;
  a.g = c->g;
  a.p = make_par<R>(c);
  a.vof = (const R*)vof;
  a.chi = (const R*)c->chi[c->chi_cur];
  a.sig = (const R*)sigma;
  a.h = c->grid.h;
  a.axi = c->grid.axisym ? 1 : 0;
  a.r0 = c->grid.origin[0];
  const unsigned tiles =
      (unsigned)iface_tiles_x(c->grid.n[0]) * (unsigned)iface_tiles_y(c->grid.n[1]);
  R* const out[4] = {cap ? (R*)cap[0] : nullptr, cap ? (R*)cap[1] : nullptr,
                     ma ? (R*)ma[0] : nullptr, ma ? (R*)ma[1] : nullptr};
  if (a.axi)
    hipLaunchKernelGGL((k_iface_force<R, true>), dim3(tiles), dim3(IF_THREADS), 0, c->stream, a,
                       out[0], out[1], out[2], out[3]);
  else
    hipLaunchKernelGGL((k_iface_force<R, false>), dim3(tiles), dim3(IF_THREADS), 0, c->stream, a,
                       out[0], out[1], out[2], out[3]);
  return status_of_launch();
}

// 3D: the cells pass into two scratch cell arrays (the pin-data buffer and
// the idle level-set buffer), then the faces pass.  The moving geometry
// rewrites the pin data of its live tiles before it reads them, but it takes
// the idle buffer to hold the clamp wherever that buffer's flag says so: its
// flags are set live afterwards, so that the next geometry writes the clamp
// back into every tile it finds quiescent.
template <typename R>
int iface3_force_impl(surf_ctx* c, const void* vof, const void* sigma, void* const* cap,
                      void* const* ma) {
  materialize<R>(c);
  Iface3Args<R> a;
  a.g = c->g;
  a.vof = (const R*)vof;
  a.chi = (const R*)c->chi[c->chi_cur];
  a.sig = (const R*)sigma;
  a.kh = (R*)c->g0;
  a.dm = (R*)c->chi[1 - c->chi_cur];
  a.h = c->grid.h;
  for (int d = 0; d < 3; ++d) {
    a.fc[d] = cap ? (R*)cap[d] : nullptr;
    a.fm[d] = ma ? (R*)ma[d] : nullptr;
  }
  const int nx = c->grid.n[0], ny = c->grid.n[1], nz = c->grid.n[2];
  const int tx = (nx + IF3_T - 1) / IF3_T, ty = (ny + IF3_T - 1) / IF3_T;
  const long long tiles = (long long)tx * ty * ((nz + IF3_T - 1) / IF3_T);
  if (tiles >= (1ll << 31)) return SURF_EINVAL;
  for (int d = 0; d < 3; ++d) {
    const long long nf = c->ncell / c->grid.n[d] * (c->grid.n[d] + 1);
    for (R* f : {a.fc[d], a.fm[d]})
      if (f) hipLaunchKernelGGL(k_zero<R>, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0,
                                c->stream, f, nf);
  }
  hipLaunchKernelGGL(k_iface3_cells<R>, dim3((unsigned)tiles), dim3(IF3_NT), 0, c->stream, a,
                     tx, ty);
  hipLaunchKernelGGL(k_iface3_faces<R>, dim3((unsigned)tiles), dim3(IF3_NT), 0, c->stream, a,
                     tx, ty);
  if (c->nflags > 0)
    hipLaunchKernelGGL(k_fill_u8, dim3((c->nflags + BLOCK - 1) / BLOCK), dim3(BLOCK), 0,
                       c->stream, c->q[1 - c->chi_cur], (uint8_t)Q_LIVE, c->nflags);
  return status_of_launch();
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

// Work that reads or writes the level set on the context's stream outside a
// step: a geometry prepared next must wait for all of it, not only for the
// point recorded before the last transport.
void touch_levelset(surf_ctx* c) {
  if (c) c->pre_valid = false;
}

// ---------------------------------------------------------------- batches
Grid grid_of(const surf_grid& gr) {
  Grid g;
  g.dim = gr.dim;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = gr.n[d];
    g.bc[d][0] = d < gr.dim ? gr.bc[d][0] : 0;
    g.bc[d][1] = d < gr.dim ? gr.bc[d][1] : 0;
  }
  return g;
}

template <typename R>
Par<R> par_of(const surf_grid& gr, const surf_params& q) {
  surf_ctx tmp;
  tmp.grid = gr;
  tmp.prm = q;
  return make_par<R>(&tmp);
}


// the three per-cell adjoint kernels, specialized on the dimension, the bulk
// switch and the presence of a flow
template <typename R, int DIM, bool BULK>
void adj_launch(hipStream_t st, const AdjArgs<R>& a, dim3 grid, dim3 block, int which) {
  if (which == 0) hipLaunchKernelGGL((k_adv_star<R, DIM, BULK>), grid, block, 0, st, a);
  else if (which == 1) hipLaunchKernelGGL((k_adj_src<R, DIM, BULK>), grid, block, 0, st, a);
  else {
    // interior x tiles plus one workgroup of side columns per row block
    const dim3 gs(adj_xtiles(a.g.n[0]) + 1, grid.y, grid.z);
    if (a.has_u) hipLaunchKernelGGL((k_adj_adv<R, DIM, BULK, true>), gs, block, 0, st, a);
    else hipLaunchKernelGGL((k_adj_adv<R, DIM, BULK, false>), gs, block, 0, st, a);
  }
}

template <typename R>
void adj_launch(hipStream_t st, const AdjArgs<R>& a, int dim, bool bulk, dim3 grid, dim3 block,
                int which) {
  if (dim == 2) {
    if (bulk) adj_launch<R, 2, true>(st, a, grid, block, which);
    else adj_launch<R, 2, false>(st, a, grid, block, which);
  } else {
    if (bulk) adj_launch<R, 3, true>(st, a, grid, block, which);
    else adj_launch<R, 3, false>(st, a, grid, block, which);
  }
}

template <typename R>
int adjoint_step_impl(surf_ctx* c, const void* const* u, const void* F, const void* psi,
                      const void* mF, const void* mP, const double* w, void* lF, void* lP,
                      double* dtheta, const void* F_star = nullptr,
                      const void* psi_star = nullptr) {
  materialize<R>(c);
  AdjArgs<R> a;
  a.g = c->g;
  a.p = make_par<R>(c);
  a.chi = (const R*)c->chi[c->chi_cur];
  a.has_u = (u && u[0]) ? 1 : 0;
  for (int d = 0; d < 3; ++d) a.u[d] = (a.has_u && d < c->grid.dim) ? (const R*)u[d] : nullptr;
  a.F = (const R*)F;
  a.psi = (const R*)psi;
  // the advected state: given by the forward step that produced it, or
  // recomputed here
  const bool given = psi_star != nullptr;
  a.Fs = given ? (const R*)F_star : (const R*)c->adj[0];
  a.Ps = given ? (const R*)psi_star : (const R*)c->adj[1];
  a.mF = (const R*)mF;
  a.mP = (const R*)mP;
  a.nF = (R*)c->adj[2];
  a.nP = (R*)c->adj[3];
  a.lF = (R*)lF;
  a.lP = (R*)lP;
  a.w = w;
  a.part = c->adj_part;
  a.dt = (R)c->dt;
  a.ncell = c->ncell;
  const dim3 agrid((c->grid.n[0] + ADJ_TX - 1) / ADJ_TX, (c->grid.n[1] + ADJ_TY - 1) / ADJ_TY,
                   c->grid.n[2]);
  const dim3 ablock(ADJ_TX * ADJ_TY);
  const int nb = (int)(agrid.x * agrid.y * agrid.z);
  if (given) {
    // xi* from the caller
  } else if (a.has_u) {
    adj_launch<R>(c->stream, a, c->grid.dim, c->prm.bulk_enabled != 0, agrid, ablock, 0);
  } else {
    size_t bytes = (size_t)c->ncell * sizeof(R);
    if (c->prm.bulk_enabled &&
        hipMemcpyAsync(c->adj[0], F, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return SURF_EDEVICE;
    if (hipMemcpyAsync(c->adj[1], psi, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return SURF_EDEVICE;
  }
  adj_launch<R>(c->stream, a, c->grid.dim, c->prm.bulk_enabled != 0, agrid, ablock, 1);
  adj_launch<R>(c->stream, a, c->grid.dim, c->prm.bulk_enabled != 0, agrid, ablock, 2);
  hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(FIN_BLOCK), 0, c->stream,
                     (const double*)c->adj_part, nb, dtheta);
  return status_of_launch();
}

}  // namespace

extern "C" {

const char* surf_version(void) { return "surf 0.1 gfx950"; }

const char* surf_strerror(int code) {
  switch (code) {
    case SURF_OK: return "ok";
    case SURF_EINVAL: return "invalid argument";
    case SURF_ENOMEM: return "workspace too small";
    case SURF_EDEVICE: return "HIP runtime error";
    case SURF_ESTATE: return "call-order violation";
    case SURF_EUNSTABLE: return "time step above the stability bound";
    default: return "unknown error";
  }
}

int surf_workspace_bytes(const surf_grid* grid, const surf_params* params, size_t* bytes) {
  if (!bytes) return SURF_EINVAL;
  int rc = check_grid_params(grid, params);
  if (rc) return rc;
  int tiles[3], t2[2];
  int nblk = nblocks_step(grid, params, tiles);
  int n2 = ntiles_2d(grid, t2);
  int cs, cg;
  int ncol = col_shape(grid, params, &cs, &cg);
  // the weighted form on rings runs on k_col2d only (the paper form in k_step2d)
  if (grid->axisym && ncol == 0 && params->flux_form == SURF_FLUX_WEIGHTED) return SURF_EINVAL;
  // so do the explicit substep-1 variants in 2D (3D: the tile transport)
  if ((params->limiter || params->transverse) && grid->dim == 2 && ncol == 0 &&
      params->substep2 != SURF_SUBSTEP2_IMPLICIT)
    return SURF_EINVAL;
  int c3s[3];
  int nc3 = col3_shape(grid, params, c3s);
  int npart = nblk > n2 ? nblk : n2;
  npart = ncol > npart ? ncol : npart;
  npart = nc3 > npart ? nc3 : npart;
  size_t n = (size_t)grid->n[0] * grid->n[1] * grid->n[2];
  const bool imp = params->substep2 == SURF_SUBSTEP2_IMPLICIT;
  const int nimp = imp ? (int)((n + IMP_BLOCK - 1) / IMP_BLOCK) : 0;
  npart = nimp > npart ? nimp : npart;
  size_t es = esize(params);
  size_t b = align_up(NSTATE * sizeof(double));
  b += align_up((size_t)npart * NPART * sizeof(double));
  b += 3 * align_up(n * es);
  b += 3 * align_up((size_t)flag_count(grid, params) + 1);
  {
    int t3[3];
    b += align_up((size_t)(geo3_tiles(grid, t3) + 1) * sizeof(int));
  }


  if (params->adjoint) {
    b += 4 * align_up(n * es);
    b += align_up((size_t)adj_blocks(grid) * NADJ * sizeof(double));
  }
  if (params->interface == SURF_IFACE_ACDI) b += 3 * align_up(n * es);
  if (snapshot_needed(grid, params, nc3))
    b += align_up(n * es) + align_up((size_t)flag_count(grid, params) + 1);
  if (imp) {
    b += IMP_FIELDS * align_up(n * sizeof(double));
    b += align_up((size_t)nimp * 2 * sizeof(double));
    b += align_up((size_t)3 * CG_MAXWG * CT_N * sizeof(double));
    b += align_up(SC_N * sizeof(double)) + align_up(IMP_MAX_SOLVES * sizeof(double));
    // the paper form's coefficient B per cell and axis
    if (params->flux_form == SURF_FLUX_PAPER) b += grid->dim * align_up(n * sizeof(double));
  }
  *bytes = b;
  return SURF_OK;
}

int surf_init(surf_ctx** out, const surf_grid* grid, const surf_params* params, void* workspace,
              size_t ws_bytes, void* hip_stream) {
  if (!out) return SURF_EINVAL;
  *out = nullptr;
  size_t need = 0;
  int rc = surf_workspace_bytes(grid, params, &need);
  if (rc) return rc;
  if (!workspace || !aligned(workspace, ALIGN)) return SURF_EINVAL;
  if (ws_bytes < need) return SURF_ENOMEM;
  surf_ctx* c = new (std::nothrow) surf_ctx();
  if (!c) return SURF_EINVAL;
  c->grid = *grid;
  c->prm = with_defaults(params, grid->dim);
  c->g.dim = grid->dim;
  for (int d = 0; d < 3; ++d) {
    c->g.n[d] = grid->n[d];
    c->g.bc[d][0] = d < grid->dim ? grid->bc[d][0] : 0;
    c->g.bc[d][1] = d < grid->dim ? grid->bc[d][1] : 0;
  }
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;
  c->ncell = (long long)grid->n[0] * grid->n[1] * grid->n[2];
  c->nblk = nblocks_step(grid, params, c->tiles);
  c->ntiles2d = ntiles_2d(grid, c->tiles2d);
  c->per_xcd = (c->ntiles2d + 7) / 8;
  c->ngtiles = geo_tiles(grid, params, c->gtiles);
  c->ng3 = geo3_tiles(grid, c->g3tiles);
  c->nflags = flag_count(grid, params);
  c->col_nwg = col_shape(grid, params, &c->col_strips, &c->col_groups);
  c->c3_nwg = col3_shape(grid, params, c->c3);
  int npart = c->nblk > c->ntiles2d ? c->nblk : c->ntiles2d;
  npart = c->col_nwg > npart ? c->col_nwg : npart;
  npart = c->c3_nwg > npart ? c->c3_nwg : npart;
  const bool imp = params->substep2 == SURF_SUBSTEP2_IMPLICIT;
  c->imp_nblk = imp ? (int)((c->ncell + IMP_BLOCK - 1) / IMP_BLOCK) : 0;
  npart = c->imp_nblk > npart ? c->imp_nblk : npart;
  size_t es = esize(params);
  char* p = c->ws;
  c->state = (double*)p;
  p += align_up(NSTATE * sizeof(double));
  c->part = (double*)p;
  p += align_up((size_t)npart * NPART * sizeof(double));
  c->chi[0] = p;
  p += align_up(c->ncell * es);
  c->chi[1] = p;
  p += align_up(c->ncell * es);
  c->g0 = p;
  p += align_up(c->ncell * es);
  c->q[0] = (uint8_t*)p;
  p += align_up((size_t)c->nflags + 1);
  c->q[1] = (uint8_t*)p;
  p += align_up((size_t)c->nflags + 1);
  c->mark = (uint8_t*)p;
  p += align_up((size_t)c->nflags + 1);
  c->live3 = (int*)p;
  p += align_up((size_t)(c->ng3 + 1) * sizeof(int));


  for (int i = 0; i < 4; ++i) {
    c->adj[i] = params->adjoint ? (void*)p : nullptr;
    if (params->adjoint) p += align_up(c->ncell * es);
  }
  c->adj_part = params->adjoint ? (double*)p : nullptr;
  if (params->adjoint) p += align_up((size_t)adj_blocks(grid) * NADJ * sizeof(double));
  if (params->interface == SURF_IFACE_ACDI)
    for (int i = 0; i < 3; ++i) {
      c->acdi[i] = p;
      p += align_up(c->ncell * es);
    }
  if (snapshot_needed(grid, params, c->c3_nwg)) {
    c->chi_snap = p;
    p += align_up(c->ncell * es);
    c->q_snap = (uint8_t*)p;
    p += align_up((size_t)c->nflags + 1);
  }
  if (imp) {
    double** f[IMP_FIELDS] = {&c->imp.Fs,   &c->imp.Ps,   &c->imp.wF,   &c->imp.wP,
                              &c->imp.xF,   &c->imp.xP,   &c->imp.dg,   &c->imp.minv,
                              &c->imp.p,    &c->imp.r[0], &c->imp.r[1], &c->imp.w[0],
                              &c->imp.w[1], &c->imp.z[0], &c->imp.z[1]};
    for (auto a : f) {
      *a = (double*)p;
      p += align_up((size_t)c->ncell * sizeof(double));
    }
    c->imp.adv = (double*)p;
    p += align_up((size_t)c->imp_nblk * 2 * sizeof(double));
    c->imp.part = (double*)p;
    p += align_up((size_t)3 * CG_MAXWG * CT_N * sizeof(double));
    c->imp.sc = (double*)p;
    p += align_up(SC_N * sizeof(double));
    c->imp.rec = (double*)p;
    p += align_up(IMP_MAX_SOLVES * sizeof(double));
    for (int d = 0; d < 3; ++d) {
      c->imp.B[d] = nullptr;
      if (params->flux_form == SURF_FLUX_PAPER && d < grid->dim) {
        c->imp.B[d] = (double*)p;
        p += align_up((size_t)c->ncell * sizeof(double));
      }
    }
  }
  c->materialized = true;
  c->chi_cur = 0;
  c->has_chi = false;
  c->dt = params->dt;
  *out = c;
  return SURF_OK;
}

int surf_set_geometry(surf_ctx* c, const void* vof, int full_rebuild) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !vof) return SURF_EINVAL;
  if (!full_rebuild && !c->has_chi) return SURF_ESTATE;
  if (c->prm.precision == SURF_F64) return geometry_impl<double>(c, vof, full_rebuild);
  return geometry_impl<float>(c, vof, full_rebuild);
}

int surf_set_levelset(surf_ctx* c, const void* chi) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !chi) return SURF_EINVAL;
  size_t bytes = (size_t)c->ncell * esize(&c->prm);
  if (hipMemcpyAsync(c->chi[c->chi_cur], chi, bytes, hipMemcpyDeviceToDevice, c->stream) !=
      hipSuccess)
    return SURF_EDEVICE;
  c->has_chi = true;
  c->materialized = true;
  flags_live(c);
  if (c->prm.precision == SURF_F64) acdi_init<double>(c);
  else acdi_init<float>(c);
  return status_of_launch();
}

int surf_get_phase(surf_ctx* c, void* phi_out) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !phi_out) return SURF_EINVAL;
  if (c->prm.interface != SURF_IFACE_ACDI) return SURF_EINVAL;
  if (!c->has_chi) return SURF_ESTATE;
  size_t bytes = (size_t)c->ncell * esize(&c->prm);
  if (hipMemcpyAsync(phi_out, c->acdi[0], bytes, hipMemcpyDeviceToDevice, c->stream) !=
      hipSuccess)
    return SURF_EDEVICE;
  return SURF_OK;
}

int surf_get_levelset(surf_ctx* c, void* chi_out) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !chi_out) return SURF_EINVAL;
  if (!c->has_chi) return SURF_ESTATE;
  if (c->prm.precision == SURF_F64) materialize<double>(c);
  else materialize<float>(c);
  size_t bytes = (size_t)c->ncell * esize(&c->prm);
  if (hipMemcpyAsync(chi_out, c->chi[c->chi_cur], bytes, hipMemcpyDeviceToDevice, c->stream) !=
      hipSuccess)
    return SURF_EDEVICE;
  return SURF_OK;
}

int surf_init_state(surf_ctx* c, const void* c0, double c0_const, double gamma0, void* F_out,
                    void* psi_out) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !psi_out) return SURF_EINVAL;
  if (c->prm.bulk_enabled && !F_out) return SURF_EINVAL;
  if (!c->has_chi) return SURF_ESTATE;
  if (c->prm.precision == SURF_F64) return init_impl<double>(c, c0, c0_const, gamma0, F_out, psi_out);
  return init_impl<float>(c, c0, c0_const, gamma0, F_out, psi_out);
}

int surf_step(surf_ctx* c, const void* vof_next, const void* const* u, const void* F_in,
              const void* psi_in, void* F_out, void* psi_out, void* sigma_out,
              double* totals_dev) {
  if (!c || !psi_in || !psi_out) return SURF_EINVAL;
  bool bulk = c->prm.bulk_enabled != 0;
  if (bulk && (!F_in || !F_out)) return SURF_EINVAL;
  if (psi_in == psi_out || (bulk && (F_in == F_out || F_in == psi_out || psi_in == F_out)))
    return SURF_EINVAL;
  if (u && u[0])
    for (int d = 0; d < c->grid.dim; ++d)
      if (!u[d]) return SURF_EINVAL;
  size_t es = esize(&c->prm);
  if (!aligned(psi_in, es) || !aligned(psi_out, es)) return SURF_EINVAL;
  if (!c->has_chi) return SURF_ESTATE;
  if (c->prm.interface == SURF_IFACE_ACDI) {
    if (c->prepared_phase) {
      // this step's ACDI step ran on the auxiliary stream into the idle
      // level-set buffer: wait for it and read that buffer
      const void* u0 = (u && u[0]) ? u[0] : nullptr;
      if (vof_next || u0 != c->prep_u0) return SURF_ESTATE;
      c->prepared_phase = false;
      c->prepared = nullptr;
      if (hipStreamWaitEvent(c->stream, c->ev_geo, 0) != hipSuccess) return SURF_EDEVICE;
      c->chi_cur = 1 - c->chi_cur;
      c->materialized = true;
    } else {
      const int rc = c->prm.precision == SURF_F64 ? acdi_geometry<double>(c, vof_next, u)
                                                  : acdi_geometry<float>(c, vof_next, u);
      if (rc) return rc;
    }
    vof_next = nullptr;  // the transport runs on the level set just written
  }
  if (c->prm.substep2 == SURF_SUBSTEP2_IMPLICIT) {
    if (vof_next) {
      // the level set of the new interface, as in the explicit path
      if (c->grid.dim == 2 && c->col_nwg > 0 &&
          (c->prm.precision == SURF_F32 ? geom2d_ok<float>(c) : geom2d_ok<double>(c))) {
        Timed tm(c, 1);
        if (c->prm.precision == SURF_F32) geo2d_launch<float>(c, vof_next, c->stream);
        else geo2d_launch<double>(c, vof_next, c->stream);
      } else if (c->prm.precision == SURF_F32 && geo3_ok<float>(c)) {
        geo3_impl<float>(c, vof_next);
      } else if (c->prm.precision == SURF_F64 && geo3_ok<double>(c)) {
        geo3_impl<double>(c, vof_next);
      } else {
        int rc = surf_set_geometry(c, vof_next, 0);
        if (rc) return rc;
      }
    }
    if (c->prm.precision == SURF_F64)
      return implicit_impl<double>(c, u, F_in, psi_in, F_out, psi_out, sigma_out, totals_dev);
    return implicit_impl<float>(c, u, F_in, psi_in, F_out, psi_out, sigma_out, totals_dev);
  }
  if (c->prepared) {
    // the geometry of this step was prepared on the auxiliary stream
    if (vof_next != c->prepared) return SURF_ESTATE;
    c->prepared = nullptr;
    if (hipStreamWaitEvent(c->stream, c->ev_geo, 0) != hipSuccess) return SURF_EDEVICE;
    if (c->grid.dim == 3) {
      if (c->prm.precision == SURF_F32)
        return col3d_prepared_step<float>(c, u, F_in, psi_in, F_out, psi_out, sigma_out,
                                          totals_dev);
      return col3d_prepared_step<double>(c, u, F_in, psi_in, F_out, psi_out, sigma_out,
                                         totals_dev);
    }
    if (c->prm.precision == SURF_F32)
      return col2d_impl<float>(c, vof_next, u, F_in, psi_in, F_out, psi_out, sigma_out,
                               totals_dev, true);
    return col2d_impl<double>(c, vof_next, u, F_in, psi_in, F_out, psi_out, sigma_out,
                              totals_dev, true);
  }
  if (vof_next) {
    // 2D: the redistancing sweeps run inside tile kernels when they fit
    if (c->grid.dim == 2 && c->col_nwg > 0) {
      if (c->prm.precision == SURF_F32 && geom2d_ok<float>(c))
        return col2d_impl<float>(c, vof_next, u, F_in, psi_in, F_out, psi_out, sigma_out,
                                 totals_dev);
      if (c->prm.precision == SURF_F64 && geom2d_ok<double>(c))
        return col2d_impl<double>(c, vof_next, u, F_in, psi_in, F_out, psi_out, sigma_out,
                                  totals_dev);
    } else if (c->prm.precision == SURF_F32 && fused_moving_ok<float>(c)) {
      return step2d_impl<float>(c, vof_next, u, F_in, psi_in, F_out, psi_out, sigma_out,
                                totals_dev);
    }
    bool banded = false;
    if (c->prm.precision == SURF_F32 && geo3_ok<float>(c)) {
      geo3_impl<float>(c, vof_next);
      banded = true;
    } else if (c->prm.precision == SURF_F64 && geo3_ok<double>(c)) {
      geo3_impl<double>(c, vof_next);
      banded = true;
    }
    int rc = banded ? status_of_launch() : surf_set_geometry(c, vof_next, 0);
    if (rc) return rc;
  }
  if (c->prm.precision == SURF_F64)
    return step_impl<double>(c, u, F_in, psi_in, F_out, psi_out, sigma_out, totals_dev);
  return step_impl<float>(c, u, F_in, psi_in, F_out, psi_out, sigma_out, totals_dev);
}

int surf_time_transport(surf_ctx* c, const void* const* u, const void* F_in,
                        const void* psi_in, void* F_out, void* psi_out, void* sigma_out,
                        int32_t reps, double* ms_per_launch) {
  touch_levelset(c);
  if (!c || !psi_in || !psi_out || !ms_per_launch || reps < 1) return SURF_EINVAL;
  const bool bulk = c->prm.bulk_enabled != 0;
  if (bulk && (!F_in || !F_out)) return SURF_EINVAL;
  if (psi_in == psi_out || (bulk && (F_in == F_out || F_in == psi_out || psi_in == F_out)))
    return SURF_EINVAL;
  if (u && u[0])
    for (int d = 0; d < c->grid.dim; ++d)
      if (!u[d]) return SURF_EINVAL;
  const bool two = c->grid.dim == 2 && c->col_nwg > 0, three = c->grid.dim == 3 && c->c3_nwg > 0;
  if ((!two && !three) || c->prm.substep2 != SURF_SUBSTEP2_EXPLICIT) return SURF_EINVAL;
  if (!c->has_chi || c->prepared) return SURF_ESTATE;
  const bool f32 = c->prm.precision == SURF_F32;
  if (f32) materialize<float>(c);
  else materialize<double>(c);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return SURF_EDEVICE;
  }
  int rc = SURF_OK;
  if (hipEventRecord(e0, c->stream) != hipSuccess) rc = SURF_EDEVICE;
  for (int r = 0; r < reps && rc == SURF_OK; ++r) {
    if (two) {
      if (f32) col2d_transport<float>(c, u, F_in, psi_in, F_out, psi_out, sigma_out);
      else col2d_transport<double>(c, u, F_in, psi_in, F_out, psi_out, sigma_out);
    } else {
      if (f32) col3d_transport<float>(c, u, F_in, psi_in, F_out, psi_out, sigma_out);
      else col3d_transport<double>(c, u, F_in, psi_in, F_out, psi_out, sigma_out);
    }
  }
  if (rc == SURF_OK) rc = status_of_launch();
  float ms = 0.f;
  if (rc == SURF_OK &&
      (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = SURF_EDEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == SURF_OK) *ms_per_launch = (double)ms / reps;
  return rc;
}

int surf_time_acdi(surf_ctx* c, const void* const* u, int32_t reps, double* ms_per_step) {
  touch_levelset(c);
  if (!c || !ms_per_step || reps < 1) return SURF_EINVAL;
  if (c->prm.interface != SURF_IFACE_ACDI) return SURF_EINVAL;
  if (u && u[0])
    for (int d = 0; d < c->grid.dim; ++d)
      if (!u[d]) return SURF_EINVAL;
  if (!c->has_chi || c->prepared) return SURF_ESTATE;
  if (c->prm.precision == SURF_F64) return time_acdi_impl<double>(c, u, reps, ms_per_step);
  return time_acdi_impl<float>(c, u, reps, ms_per_step);
}

int surf_time_solver(surf_ctx* c, int32_t field, int32_t reps, double* ms_per_launch) {
  touch_levelset(c);
  if (!c || !ms_per_launch || reps < 1 || field < 0 || field > 1) return SURF_EINVAL;
  if (c->prm.substep2 != SURF_SUBSTEP2_IMPLICIT) return SURF_EINVAL;
  if (c->prm.flux_form != SURF_FLUX_WEIGHTED) return SURF_EINVAL;  // CG iterations only
  if (field == 1 && !c->prm.bulk_enabled) return SURF_EINVAL;
  if (c->imp_nsolves == 0 || c->prepared) return SURF_ESTATE;
  if (c->prm.precision == SURF_F64) return time_solver_impl<double>(c, field, reps, ms_per_launch);
  return time_solver_impl<float>(c, field, reps, ms_per_launch);
}

int surf_prepare_phase(surf_ctx* c, const void* const* u, void* aux_stream) {
  if (!c || !aux_stream) return SURF_EINVAL;
  if (c->prm.interface != SURF_IFACE_ACDI || c->prm.substep2 != SURF_SUBSTEP2_EXPLICIT ||
      !((c->grid.dim == 2 && c->col_nwg > 0) || (c->grid.dim == 3 && c->c3_nwg > 0)))
    return SURF_EINVAL;
  if (c->grid.dim == 3 && u && u[0] && !u[2]) return SURF_EINVAL;
  if (u && u[0] && !u[1]) return SURF_EINVAL;
  if (!c->has_chi || c->prepared) return SURF_ESTATE;
  if (!c->ev_pre) {
    if (hipEventCreateWithFlags(&c->ev_pre, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_geo, hipEventDisableTiming) != hipSuccess)
      return SURF_EDEVICE;
    c->pre_valid = false;
  }
  hipStream_t aux = (hipStream_t)aux_stream;
  // the idle level-set buffer is free once the transport that read it is
  // done: the point recorded before the latest transport, or else now; the
  // phase-field buffers are read and written by ACDI steps alone
  if (!c->pre_valid && hipEventRecord(c->ev_pre, c->stream) != hipSuccess) return SURF_EDEVICE;
  c->pre_valid = false;
  if (hipStreamWaitEvent(aux, c->ev_pre, 0) != hipSuccess) return SURF_EDEVICE;
  {
    Timed tm(c, 1, aux);
    if (c->prm.precision == SURF_F32)
      acdi_launch<float>(c, u, (float*)c->acdi[0], (float*)c->chi[1 - c->chi_cur], aux);
    else
      acdi_launch<double>(c, u, (double*)c->acdi[0], (double*)c->chi[1 - c->chi_cur], aux);
  }
  if (hipEventRecord(c->ev_geo, aux) != hipSuccess) return SURF_EDEVICE;
  c->prepared_phase = true;
  c->prepared = &c->prepared_phase;
  c->prep_u0 = (u && u[0]) ? u[0] : nullptr;
  return status_of_launch();
}

int surf_prepare_geometry(surf_ctx* c, const void* vof_next, void* aux_stream) {
  if (!c || !vof_next || !aux_stream) return SURF_EINVAL;
  if (c->prm.substep2 != SURF_SUBSTEP2_EXPLICIT || c->prm.interface != SURF_IFACE_VOF)
    return SURF_EINVAL;
  const bool three = c->grid.dim == 3;
  if (three) {
    if (!c->chi_snap || (c->prm.precision == SURF_F32 ? !geo3_ok<float>(c) : !geo3_ok<double>(c)))
      return SURF_EINVAL;
  } else if (c->col_nwg == 0 ||
             (c->prm.precision == SURF_F32 ? !geom2d_ok<float>(c) : !geom2d_ok<double>(c))) {
    return SURF_EINVAL;
  }
  if (!c->has_chi || c->prepared) return SURF_ESTATE;
  if (!aligned(vof_next, esize(&c->prm))) return SURF_EINVAL;
  if (!c->ev_pre) {
    if (hipEventCreateWithFlags(&c->ev_pre, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_geo, hipEventDisableTiming) != hipSuccess)
      return SURF_EDEVICE;
    c->pre_valid = false;
  }
  hipStream_t aux = (hipStream_t)aux_stream;
  // the other level-set buffer is free once the transport that read it is
  // done: the point recorded before the latest transport, or else now
  if (!c->pre_valid && hipEventRecord(c->ev_pre, c->stream) != hipSuccess) return SURF_EDEVICE;
  c->pre_valid = false;
  if (hipStreamWaitEvent(aux, c->ev_pre, 0) != hipSuccess) return SURF_EDEVICE;
  if (three) {
    if (c->prm.precision == SURF_F32) geo3_impl<float>(c, vof_next, aux, true);
    else geo3_impl<double>(c, vof_next, aux, true);
  } else {
    Timed tm(c, 1, aux);
    if (c->prm.precision == SURF_F32) geo2d_launch<float>(c, vof_next, aux);
    else geo2d_launch<double>(c, vof_next, aux);
  }
  if (hipEventRecord(c->ev_geo, aux) != hipSuccess) return SURF_EDEVICE;
  c->prepared = vof_next;
  return status_of_launch();
}

int surf_force(surf_ctx* c, const void* sigma, void* const* force) {
  // the force kernel reads only the current level set, which a geometry
  // prepared next leaves alone (2D: it writes the other buffer; 3D: the
  // other two)
  if (c && !c->materialized) touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !sigma || !force) return SURF_EINVAL;
  for (int d = 0; d < c->grid.dim; ++d)
    if (!force[d]) return SURF_EINVAL;
  if (!c->has_chi) return SURF_ESTATE;
  if (c->prm.precision == SURF_F64) return force_impl<double>(c, sigma, force);
  return force_impl<float>(c, sigma, force);
}

int surf_interface_force(surf_ctx* c, const void* vof, const void* sigma, void* const* f_cap,
                         void* const* f_ma) {
  // the force kernel only reads the current level set, which a geometry
  // prepared next leaves alone (it writes the other buffer); filling in the
  // current buffer from its compact form does write it
  if (c && !c->materialized) touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !vof || !sigma || (!f_cap && !f_ma)) return SURF_EINVAL;
  const int dim = c->grid.dim;
  for (int d = 0; d < dim; ++d)
    if (c->grid.n[d] < 4) return SURF_EINVAL;
  if (dim == 2 && (long long)(c->grid.n[0] + 1) * (c->grid.n[1] + 1) >= (1ll << 30))
    return SURF_EINVAL;
  for (int d = 0; d < dim; ++d)
    if ((f_cap && !f_cap[d]) || (f_ma && !f_ma[d])) return SURF_EINVAL;
  if (!c->has_chi) return SURF_ESTATE;
  if (dim == 3) {
    // the cells pass writes the idle level-set buffer: the next geometry
    // (which writes it too) must wait for it
    touch_levelset(c);
    if (c->prm.precision == SURF_F64) return iface3_force_impl<double>(c, vof, sigma, f_cap, f_ma);
    return iface3_force_impl<float>(c, vof, sigma, f_cap, f_ma);
  }
  if (c->prm.precision == SURF_F64) return iface_force_impl<double>(c, vof, sigma, f_cap, f_ma);
  return iface_force_impl<float>(c, vof, sigma, f_cap, f_ma);
}

int surf_set_dt(surf_ctx* c, double dt) {
  if (!c || !(dt > 0) || !std::isfinite(dt)) return SURF_EINVAL;
  // a prepared ACDI step has advanced the phase field with the current dt
  if (c->prepared_phase && dt != c->dt) return SURF_ESTATE;
  c->dt = dt;
  return SURF_OK;
}

int surf_set_time(surf_ctx* c, const double* time_dev) {
  if (!c) return SURF_EINVAL;
  if (c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  hipLaunchKernelGGL(k_set_time, dim3(1), dim3(64), 0, c->stream, c->state, time_dev);
  return status_of_launch();
}

int surf_get_status(surf_ctx* c, uint32_t* bits) {
  if (!c || !bits) return SURF_EINVAL;
  double s = 0;
  if (hipMemcpyAsync(&s, c->state + S_STATUS, sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return SURF_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SURF_EDEVICE;
  *bits = (uint32_t)s;
  return SURF_OK;
}

int surf_solver_iterations(surf_ctx* c, int32_t* iters, int32_t cap, int32_t* count) {
  if (!c || !count || cap < 0 || (cap > 0 && !iters)) return SURF_EINVAL;
  if (c->prm.substep2 != SURF_SUBSTEP2_IMPLICIT) return SURF_EINVAL;
  if (c->imp_nsolves == 0) return SURF_ESTATE;
  double rec[IMP_MAX_SOLVES];
  if (hipMemcpyAsync(rec, c->imp.rec, c->imp_nsolves * sizeof(double), hipMemcpyDeviceToHost,
                     c->stream) != hipSuccess)
    return SURF_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SURF_EDEVICE;
  *count = c->imp_nsolves;
  for (int i = 0; i < c->imp_nsolves && i < cap; ++i) iters[i] = (int32_t)rec[i];
  return SURF_OK;
}

int surf_clear_status(surf_ctx* c) {
  if (!c) return SURF_EINVAL;
  static const double zero[2] = {0.0, 0.0};  // S_STATUS and the S_FLAGS word
  if (hipMemcpyAsync(c->state + S_STATUS, zero, 2 * sizeof(double), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess)
    return SURF_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SURF_EDEVICE;
  return SURF_OK;
}

int surf_set_kinetics(surf_ctx* c, double k_a, double k_d, double D_b, double D_s) {
  if (!c || !(k_a >= 0) || !(k_d >= 0) || !(D_b >= 0) || !(D_s >= 0)) return SURF_EINVAL;
  c->prm.k_a = k_a;
  c->prm.k_d = k_d;
  c->prm.D_b = D_b;
  c->prm.D_s = D_s;
  return SURF_OK;
}

int surf_loss_weights(surf_ctx* c, const double* tot, int64_t stride, const double* target,
                      int32_t nsteps, double* w, double* loss) {
  if (!c || !tot || !target || !w || nsteps <= 0 || stride < 16) return SURF_EINVAL;
  double vol = c->grid.dim == 3 ? c->grid.h * c->grid.h * c->grid.h : c->grid.h * c->grid.h;
  hipLaunchKernelGGL(k_loss_w, dim3(1), dim3(BLOCK), 0, c->stream, tot, (long long)stride, target,
                     (int)nsteps, vol, w, loss);
  return status_of_launch();
}

int surf_adjoint_seed(surf_ctx* c, const void* psi, const double* w, void* lF, void* lP) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !psi || !w || !lP) return SURF_EINVAL;
  if (!c->prm.adjoint) return SURF_ESTATE;
  if (!c->has_chi) return SURF_ESTATE;
  long long n = c->ncell;
  if (c->prm.precision == SURF_F64) {
    materialize<double>(c);
    hipLaunchKernelGGL(k_loss_seed<double>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g,
                       make_par<double>(c), (const double*)c->chi[c->chi_cur], (const double*)psi,
                       w, (double*)lF, (double*)lP, n);
  } else {
    materialize<float>(c);
    hipLaunchKernelGGL(k_loss_seed<float>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g,
                       make_par<float>(c), (const float*)c->chi[c->chi_cur], (const float*)psi, w,
                       (float*)lF, (float*)lP, n);
  }
  return status_of_launch();
}

int surf_adjoint_step(surf_ctx* c, const void* const* u, const void* F, const void* psi,
                      const void* mF, const void* mP, const double* w, void* lF, void* lP,
                      double* dtheta) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !psi || !mP || !lP || !dtheta) return SURF_EINVAL;
  if (!c->prm.adjoint || c->prm.flux_form != SURF_FLUX_WEIGHTED) return SURF_ESTATE;
  if (!c->has_chi) return SURF_ESTATE;
  bool bulk = c->prm.bulk_enabled != 0;
  if (bulk && (!F || !mF || !lF)) return SURF_EINVAL;
  if (lP == mP || lP == psi || (bulk && (lF == mF || lF == F))) return SURF_EINVAL;
  if (u && u[0])
    for (int d = 0; d < c->grid.dim; ++d)
      if (!u[d]) return SURF_EINVAL;
  if (c->prm.precision == SURF_F64)
    return adjoint_step_impl<double>(c, u, F, psi, mF, mP, w, lF, lP, dtheta);
  return adjoint_step_impl<float>(c, u, F, psi, mF, mP, w, lF, lP, dtheta);
}

int surf_adjoint_step_advected(surf_ctx* c, const void* const* u, const void* F,
                               const void* psi, const void* F_star, const void* psi_star,
                               const void* mF, const void* mP, const double* w, void* lF,
                               void* lP, double* dtheta) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !psi || !psi_star || !mP || !lP || !dtheta) return SURF_EINVAL;
  if (!c->prm.adjoint || c->prm.flux_form != SURF_FLUX_WEIGHTED) return SURF_ESTATE;
  if (!c->has_chi) return SURF_ESTATE;
  bool bulk = c->prm.bulk_enabled != 0;
  if (bulk && (!F || !F_star || !mF || !lF)) return SURF_EINVAL;
  if (lP == mP || lP == psi || lP == psi_star ||
      (bulk && (lF == mF || lF == F || lF == F_star)))
    return SURF_EINVAL;
  if (u && u[0])
    for (int d = 0; d < c->grid.dim; ++d)
      if (!u[d]) return SURF_EINVAL;
  if (c->prm.precision == SURF_F64)
    return adjoint_step_impl<double>(c, u, F, psi, mF, mP, w, lF, lP, dtheta, F_star, psi_star);
  return adjoint_step_impl<float>(c, u, F, psi, mF, mP, w, lF, lP, dtheta, F_star, psi_star);
}

int surf_step_advected(surf_ctx* c, const void* const* u, const void* F_in, const void* psi_in,
                       void* F_out, void* psi_out, void* sigma_out, double* totals_dev,
                       void* F_star, void* psi_star) {
  if (!c || !psi_in || !psi_out || !psi_star) return SURF_EINVAL;
  // the 3D weighted-form plane-marching transport on a static level set
  if (c->grid.dim != 3 || c->c3_nwg == 0 || c->prm.interface != SURF_IFACE_VOF ||
      c->prm.substep2 != SURF_SUBSTEP2_EXPLICIT)
    return SURF_EINVAL;
  if (c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c->has_chi) return SURF_ESTATE;
  const bool bulk = c->prm.bulk_enabled != 0;
  if (bulk && (!F_in || !F_out || !F_star)) return SURF_EINVAL;
  // every output distinct from the inputs and from each other
  const void* ins[2] = {psi_in, bulk ? F_in : nullptr};
  const void* outs[4] = {psi_out, psi_star, bulk ? F_out : nullptr, bulk ? F_star : nullptr};
  for (int i = 0; i < 4; ++i) {
    if (!outs[i]) continue;
    for (const void* q : ins)
      if (outs[i] == q) return SURF_EINVAL;
    for (int j = i + 1; j < 4; ++j)
      if (outs[i] == outs[j]) return SURF_EINVAL;
  }
  if (u && u[0])
    for (int d = 0; d < c->grid.dim; ++d)
      if (!u[d]) return SURF_EINVAL;
  const size_t es = esize(&c->prm);
  if (!aligned(psi_in, es) || !aligned(psi_out, es) || !aligned(psi_star, es)) return SURF_EINVAL;
  touch_levelset(c);
  const bool f32 = c->prm.precision == SURF_F32;
  if (f32) materialize<float>(c);
  else materialize<double>(c);
  {
    Timed tm(c, 0);
    if (f32) col3d_transport<float>(c, u, F_in, psi_in, F_out, psi_out, sigma_out, nullptr,
                                    bulk ? F_star : nullptr, psi_star);
    else col3d_transport<double>(c, u, F_in, psi_in, F_out, psi_out, sigma_out, nullptr,
                                 bulk ? F_star : nullptr, psi_star);
  }
  if (f32) finalize<float>(c, totals_dev, c->c3_nwg);
  else finalize<double>(c, totals_dev, c->c3_nwg);
  return status_of_launch();
}

int surf_adjoint_c0(surf_ctx* c, const void* lF0, void* gc0) {
  touch_levelset(c);
  if (c && c->prepared) return SURF_ESTATE;  // only surf_step may follow a prepare
  if (!c || !lF0 || !gc0) return SURF_EINVAL;
  if (!c->has_chi) return SURF_ESTATE;
  long long n = c->ncell;
  if (c->prm.precision == SURF_F64) {
    materialize<double>(c);
    hipLaunchKernelGGL(k_adj_c0<double>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g,
                       make_par<double>(c), (const double*)c->chi[c->chi_cur],
                       (const double*)lF0, (double*)gc0, n);
  } else {
    materialize<float>(c);
    hipLaunchKernelGGL(k_adj_c0<float>, dim3(grid1d(n)), dim3(BLOCK), 0, c->stream, c->g,
                       make_par<float>(c), (const float*)c->chi[c->chi_cur], (const float*)lF0,
                       (float*)gc0, n);
  }
  return status_of_launch();
}

}  // extern "C"

namespace {

struct BatchLayout {
  size_t total = 0;
  size_t states, part, inst, col_inst, queue, col_queue, fargs, first, scratch0, scratch1;
  std::vector<size_t> chi, q;
  int total_tiles = 0;  // tile entries of the paper-form instances
  int col_records = 0;  // column entries of the weighted-form instances (row chunks of 8)
};

// Weighted-form instances run on the column-streaming kernel; the paper
// form keeps the LDS tile kernel.
bool batch_col(const surf_params& q) { return q.flux_form == SURF_FLUX_WEIGHTED; }

// workgroups of the column kernel for one instance with row chunks of ty rows
int batch_col_wgs(const surf_grid& gr, int ty) {
  const int chunks = (gr.n[1] + ty - 1) / ty;
  return ((gr.n[0] + COL_OUT - 1) / COL_OUT) * ((chunks + COL_WAVES - 1) / COL_WAVES);
}

int batch_layout(int32_t n, const surf_grid* grids, const surf_params* prm, BatchLayout* L) {
  if (n <= 0 || !grids || !prm) return SURF_EINVAL;
  size_t es = esize(&prm[0]);
  size_t maxcell = 0, off = 0;
  int tt = 0;
  L->chi.resize(n);
  L->q.resize(n);
  for (int i = 0; i < n; ++i) {
    // rings run in the column kernel only (weighted form)
    if (grids[i].axisym && !batch_col(prm[i])) return SURF_EINVAL;
    if (prm[i].limiter || prm[i].transverse) return SURF_EINVAL;  // and takes the default scheme
    int rc = check_grid_params(&grids[i], &prm[i]);
    if (rc) return rc;
    if (grids[i].dim != 2 || prm[i].precision != prm[0].precision) return SURF_EINVAL;
    int t2[2];
    if (batch_col(prm[i])) {
      // 32-bit byte offsets of the column kernel's loads
      const long long es = prm[i].precision == SURF_F64 ? 8 : 4;
      if ((long long)(grids[i].n[0] + 1) * (grids[i].n[1] + 1) * es > 0x7fffffffll)
        return SURF_EINVAL;
      L->col_records += batch_col_wgs(grids[i], 8);
    } else {
      tt += ntiles_2d(&grids[i], t2);
    }
    size_t nc = (size_t)grids[i].n[0] * grids[i].n[1];
    if (nc > maxcell) maxcell = nc;
  }
  size_t inst_bytes = prm[0].precision == SURF_F64 ? sizeof(Step2dArgs<double>) : sizeof(Step2dArgs<float>);
  size_t col_bytes = prm[0].precision == SURF_F64 ? sizeof(ColArgs<double>) : sizeof(ColArgs<float>);
  L->states = off; off += align_up((size_t)n * NSTATE * sizeof(double));
  L->part = off; off += align_up((size_t)(tt + L->col_records) * NPART * sizeof(double));
  L->inst = off; off += align_up((size_t)n * inst_bytes);
  L->col_inst = off; off += align_up((size_t)n * col_bytes);
  L->queue = off; off += align_up((size_t)(tt > 0 ? tt : 1) * sizeof(int2));
  L->col_queue = off; off += align_up((size_t)(L->col_records > 0 ? L->col_records : 1) * sizeof(int2));
  L->fargs = off; off += align_up((size_t)n * sizeof(FinalArgs));
  L->first = off; off += align_up((size_t)n * sizeof(int));
  L->scratch0 = off; off += align_up(maxcell * es);
  L->scratch1 = off; off += align_up(maxcell * es);
  for (int i = 0; i < n; ++i) {
    int t2[2];
    int nt2 = ntiles_2d(&grids[i], t2);
    L->chi[i] = off; off += align_up((size_t)grids[i].n[0] * grids[i].n[1] * es);
    L->q[i] = off; off += align_up((size_t)nt2 + 1);
  }
  L->total = off;
  L->total_tiles = tt;
  return SURF_OK;
}

// Column entries for row chunks of ty rows (ty in {8, 16}: never more
// entries than the records reserved for 8).
template <typename R>
void batch_col_tables(surf_batch* b) {
  b->host_col_queue.clear();
  int rec = 0;
  for (int i = 0; i < b->n; ++i) {
    if (!batch_col(b->prm[i])) continue;
    const int nw = batch_col_wgs(b->grids[i], b->ty);
    ColArgs<R> a;
    std::memcpy(&a, b->host_col_inst.data() + sizeof(a) * i, sizeof(a));
    a.groups = (((b->grids[i].n[1] + b->ty - 1) / b->ty) + COL_WAVES - 1) / COL_WAVES;
    a.strips = (b->grids[i].n[0] + COL_OUT - 1) / COL_OUT;
    a.nwg = nw;
    a.per_xcd = (nw + 7) / 8;
    std::memcpy(b->host_col_inst.data() + sizeof(a) * i, &a, sizeof(a));
    b->host_first[i] = rec;
    for (int w = 0; w < nw; ++w) b->host_col_queue.push_back(make_int2(i, w));
    rec += nw;
    FinalArgs f = final_of(b->grids[i], b->prm[i], nw, b->prm[i].dt);
    std::memcpy(b->host_fargs.data() + sizeof(f) * i, &f, sizeof(f));
  }
  b->ncol_q = rec;
}

template <typename R>
void batch_tables(surf_batch* b) {
  b->host_inst.resize(sizeof(Step2dArgs<R>) * b->n);
  b->host_col_inst.resize(sizeof(ColArgs<R>) * b->n);
  b->host_fargs.resize(sizeof(FinalArgs) * b->n);
  b->host_first.resize(b->n);
  b->host_queue.clear();
  for (int i = 0; i < b->n; ++i) {
    const surf_grid& gr = b->grids[i];
    const surf_params& q = b->prm[i];
    Step2dArgs<R> a{};
    a.g = grid_of(gr);
    a.p = par_of<R>(gr, q);
    a.vof = nullptr;
    a.chi_in = (const R*)b->chi[i];
    a.chi_out = nullptr;
    a.q_in = b->q[i];
    a.q_out = b->q[i];
    a.u[0] = a.u[1] = nullptr;
    a.F = (const R*)b->F[2 * i];
    a.Fo = (R*)b->F[2 * i + 1];
    a.psi = (const R*)b->P[2 * i];
    a.Po = (R*)b->P[2 * i + 1];
    a.sig = b->S.empty() ? nullptr : (R*)b->S[i];
    a.part = nullptr;
    a.state = b->states + (size_t)i * NSTATE;
    a.dt = (R)q.dt;
    a.area_dt = (R)(gr.h * q.dt);
    a.dtau = (R)(gr.h / 2);
    a.has_u = 0;
    a.ksweeps = 0;
    int t2[2];
    a.ntiles = ntiles_2d(&gr, t2);
    a.tiles[0] = t2[0];
    a.tiles[1] = t2[1];
    a.per_xcd = (a.ntiles + 7) / 8;
    a.diag = 0;
    std::memcpy(b->host_inst.data() + sizeof(a) * i, &a, sizeof(a));
    ColArgs<R> c{};
    c.g = a.g;
    c.p = a.p;
    c.chi = a.chi_in;
    c.u[0] = c.u[1] = nullptr;
    c.F = a.F;
    c.psi = a.psi;
    c.Fo = a.Fo;
    c.Po = a.Po;
    c.sig = a.sig;
    c.part = nullptr;
    c.state = b->states + (size_t)i * NSTATE;
    c.dt = a.dt;
    c.area_dt = a.area_dt;
    c.r0 = gr.axisym ? gr.origin[0] : 0.0;
    c.axi = gr.axisym ? 1 : 0;
    std::memcpy(b->host_col_inst.data() + sizeof(c) * i, &c, sizeof(c));
    if (batch_col(q)) continue;  // column entries: batch_col_tables
    // tile entries of the paper-form instances: records after the column ones
    b->host_first[i] = b->col_records + (int)b->host_queue.size();
    for (int t = 0; t < a.ntiles; ++t) b->host_queue.push_back(make_int2(i, t));
    FinalArgs f = final_of(gr, q, a.ntiles, q.dt);
    std::memcpy(b->host_fargs.data() + sizeof(f) * i, &f, sizeof(f));
  }
  batch_col_tables<R>(b);
}

template <typename R>
void batch_launch_col(surf_batch* b, int ty, int grid, int parity) {
  if (b->ncol_q == 0) return;
  bool rings = false;
  for (int i = 0; i < b->n; ++i) rings = rings || b->grids[i].axisym != 0;
  const ColArgs<R>* inst = (const ColArgs<R>*)b->col_inst;
  const int2* queue = (const int2*)b->col_queue;
  const int* first = (const int*)b->first;
  const dim3 gr(grid), bl(64 * COL_WAVES);
  if (rings) {
    if (ty == 16)
      hipLaunchKernelGGL((k_batch_col2d<R, 16, true>), gr, bl, 0, b->stream, inst, queue,
                         b->ncol_q, first, parity, b->part);
    else
      hipLaunchKernelGGL((k_batch_col2d<R, 8, true>), gr, bl, 0, b->stream, inst, queue,
                         b->ncol_q, first, parity, b->part);
  } else if (ty == 16) {
    hipLaunchKernelGGL((k_batch_col2d<R, 16>), gr, bl, 0, b->stream, inst, queue, b->ncol_q,
                       first, parity, b->part);
  } else {
    hipLaunchKernelGGL((k_batch_col2d<R, 8>), gr, bl, 0, b->stream, inst, queue, b->ncol_q,
                       first, parity, b->part);
  }
}

template <typename R>
void batch_launch_step(surf_batch* b, int nt, int grid, int parity) {
  if (b->total_tiles == 0) return;
  double* part = b->part + (size_t)b->col_records * NPART;
  if (nt == 256)
    hipLaunchKernelGGL((k_batch2d<R, 256>), dim3(grid), dim3(256), 0, b->stream,
                       (const Step2dArgs<R>*)b->inst_tab, (const int2*)b->queue, b->total_tiles,
                       parity, part);
  else
    hipLaunchKernelGGL((k_batch2d<R, 512>), dim3(grid), dim3(512), 0, b->stream,
                       (const Step2dArgs<R>*)b->inst_tab, (const int2*)b->queue, b->total_tiles,
                       parity, part);
}

void batch_step_kernels(surf_batch* b, int parity, double* totals) {
  if (b->prec == SURF_F64) {
    batch_launch_col<double>(b, b->ty, b->col_grid, parity);
    batch_launch_step<double>(b, b->nt, b->grid, parity);
  } else {
    batch_launch_col<float>(b, b->ty, b->col_grid, parity);
    batch_launch_step<float>(b, b->nt, b->grid, parity);
  }
  hipLaunchKernelGGL(k_batch_final, dim3(b->n), dim3(FIN_BLOCK), 0, b->stream,
                     (const FinalArgs*)b->fargs, (const int*)b->first, (const double*)b->part,
                     b->states, totals);
}

void batch_drop_graphs(surf_batch* b) {
  for (auto& g : b->graphs) {
    (void)hipGraphExecDestroy(g.e);
    (void)hipGraphDestroy(g.g);
  }
  b->graphs.clear();
}

// persistent grid of the column kernel: every entry in flight at once up to
// 2048 workgroups (8 per CU), a multiple of 8
int batch_col_default_grid(int nq) {
  int g = nq < 2048 ? nq : 2048;
  return ((g + 7) / 8) * 8 > 0 ? ((g + 7) / 8) * 8 : 8;
}

int batch_upload(surf_batch* b) {
  bool ok = hipMemcpyAsync(b->inst_tab, b->host_inst.data(), b->host_inst.size(),
                           hipMemcpyHostToDevice, b->stream) == hipSuccess &&
            hipMemcpyAsync(b->col_inst, b->host_col_inst.data(), b->host_col_inst.size(),
                           hipMemcpyHostToDevice, b->stream) == hipSuccess &&
            hipMemcpyAsync(b->fargs, b->host_fargs.data(), b->host_fargs.size(),
                           hipMemcpyHostToDevice, b->stream) == hipSuccess &&
            hipMemcpyAsync(b->first, b->host_first.data(), b->host_first.size() * sizeof(int),
                           hipMemcpyHostToDevice, b->stream) == hipSuccess;
  if (ok && !b->host_queue.empty())
    ok = hipMemcpyAsync(b->queue, b->host_queue.data(), b->host_queue.size() * sizeof(int2),
                        hipMemcpyHostToDevice, b->stream) == hipSuccess;
  if (ok && !b->host_col_queue.empty())
    ok = hipMemcpyAsync(b->col_queue, b->host_col_queue.data(),
                        b->host_col_queue.size() * sizeof(int2), hipMemcpyHostToDevice,
                        b->stream) == hipSuccess;
  // the host tables are pageable: wait before they may change
  if (!ok || hipStreamSynchronize(b->stream) != hipSuccess) return SURF_EDEVICE;
  return SURF_OK;
}

// Tuned launch shapes, keyed by the device and the instances' precision,
// sizes, flux forms and bulk switches; kept for the process and, when the
// environment variable SURF_TUNE_CACHE names a file, in that file (one line
// per key: the key, then ty, col_grid, nt, grid).
struct TuneChoice { int ty, col_grid, nt, grid; };
std::mutex tune_mu;
std::map<std::string, TuneChoice>& tune_cache() {
  static std::map<std::string, TuneChoice> m;
  static bool loaded = false;
  if (!loaded) {
    loaded = true;
    const char* path = std::getenv("SURF_TUNE_CACHE");
    if (path) {
      if (FILE* f = std::fopen(path, "r")) {
        char key[4096];
        TuneChoice c;
        while (std::fscanf(f, "%4095s %d %d %d %d", key, &c.ty, &c.col_grid, &c.nt, &c.grid) == 5)
          if ((c.ty == 8 || c.ty == 16) && c.col_grid > 0 && c.col_grid % 8 == 0 &&
              (c.nt == 256 || c.nt == 512) && c.grid > 0)
            m[key] = c;
        std::fclose(f);
      }
    }
  }
  return m;
}

std::string batch_tune_key(const surf_batch* b) {
  int dev = -1;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  std::string name = "gpu";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) name = prop.gcnArchName;
  for (auto& ch : name)
    if (ch == ' ' || ch == ':') ch = '_';
  std::string k = name + "/p" + std::to_string(b->prec);
  for (int i = 0; i < b->n; ++i)
    k += "/" + std::to_string(b->grids[i].n[0]) + "x" + std::to_string(b->grids[i].n[1]) +
         (batch_col(b->prm[i]) ? "w" : "p") + (b->prm[i].bulk_enabled ? "b" : "i");
  return k;
}

}  // namespace

extern "C" {

int surf_batch_workspace_bytes(int32_t n, const surf_grid* grids, const surf_params* params,
                               size_t* bytes) {
  if (!bytes) return SURF_EINVAL;
  BatchLayout L;
  int rc = batch_layout(n, grids, params, &L);
  if (rc) return rc;
  *bytes = L.total;
  return SURF_OK;
}

int surf_batch_create(surf_batch** out, int32_t n, const surf_grid* grids,
                      const surf_params* params, void* const* F, void* const* psi,
                      void* const* sigma, void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return SURF_EINVAL;
  *out = nullptr;
  BatchLayout L;
  int rc = batch_layout(n, grids, params, &L);
  if (rc) return rc;
  if (!F || !psi || !workspace || !aligned(workspace, ALIGN)) return SURF_EINVAL;
  if (ws_bytes < L.total) return SURF_ENOMEM;
  for (int i = 0; i < 2 * n; ++i)
    if (!psi[i] || (params[i / 2].bulk_enabled && !F[i])) return SURF_EINVAL;
  surf_batch* b = new (std::nothrow) surf_batch();
  if (!b) return SURF_EINVAL;
  b->n = n;
  b->prec = params[0].precision;
  b->stream = (hipStream_t)stream;
  for (int i = 0; i < n; ++i) {
    b->grids.push_back(grids[i]);
    b->prm.push_back(with_defaults(&params[i], 2));
  }
  char* base = (char*)workspace;
  b->states = (double*)(base + L.states);
  b->part = (double*)(base + L.part);
  b->inst_tab = base + L.inst;
  b->col_inst = base + L.col_inst;
  b->queue = (int2*)(base + L.queue);
  b->col_queue = (int2*)(base + L.col_queue);
  b->col_records = L.col_records;
  b->fargs = base + L.fargs;
  b->first = (int*)(base + L.first);
  b->scratch[0] = base + L.scratch0;
  b->scratch[1] = base + L.scratch1;
  for (int i = 0; i < n; ++i) {
    b->chi.push_back(base + L.chi[i]);
    b->q.push_back((uint8_t*)(base + L.q[i]));
  }
  b->total_tiles = L.total_tiles;
  for (int i = 0; i < 2 * n; ++i) {
    b->F.push_back(F[i]);
    b->P.push_back(psi[i]);
  }
  if (sigma)
    for (int i = 0; i < n; ++i) b->S.push_back(sigma[i]);
  b->tune_key = batch_tune_key(b);
  {
    // a choice tuned before for the same instances on this device
    std::lock_guard<std::mutex> lock(tune_mu);
    auto it = tune_cache().find(b->tune_key);
    if (it != tune_cache().end()) {
      b->ty = it->second.ty;
      b->col_grid = it->second.col_grid;
      b->nt = it->second.nt;
      b->grid = it->second.grid;
    }
  }
  if (b->prec == SURF_F64) batch_tables<double>(b);
  else batch_tables<float>(b);
  if (b->grid == 0) b->grid = b->total_tiles < 2048 ? b->total_tiles : 2048;
  if (b->col_grid == 0) b->col_grid = batch_col_default_grid(b->ncol_q);
  if (batch_upload(b) != SURF_OK) {
    delete b;
    return SURF_EDEVICE;
  }
  for (int i = 0; i < n; ++i)
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, b->stream, b->states + (size_t)i * NSTATE);
  *out = b;
  return status_of_launch();
}

int surf_batch_set_geometry(surf_batch* b, int32_t i, const void* vof) {
  if (!b || !vof || i < 0 || i >= b->n) return SURF_EINVAL;
  // a throw-away context over the batch's buffers drives the global sweeps
  surf_ctx c;
  c.grid = b->grids[i];
  c.prm = b->prm[i];
  c.g = grid_of(c.grid);
  c.stream = b->stream;
  c.ncell = (long long)c.grid.n[0] * c.grid.n[1];
  c.chi[0] = b->chi[i];
  c.chi[1] = b->scratch[1];
  c.g0 = b->scratch[0];
  c.chi_cur = 0;
  c.has_chi = false;
  c.materialized = true;
  c.ntiles2d = 0;
  c.ngtiles = 0;
  c.ng3 = 0;
  c.nflags = 0;
  c.col_nwg = 0;
  c.c3_nwg = 0;
  c.profile = false;
  int rc = c.prm.precision == SURF_F64 ? geometry_impl<double>(&c, vof, 1)
                                       : geometry_impl<float>(&c, vof, 1);
  if (rc) return rc;
  if (c.chi_cur != 0) {
    size_t bytes = (size_t)c.ncell * esize(&c.prm);
    if (hipMemcpyAsync(b->chi[i], b->scratch[1], bytes, hipMemcpyDeviceToDevice, b->stream) !=
        hipSuccess)
      return SURF_EDEVICE;
  }
  int t2[2];
  int nt2 = ntiles_2d(&b->grids[i], t2);
  hipLaunchKernelGGL(k_fill_u8, dim3((nt2 + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, b->stream, b->q[i],
                     (uint8_t)Q_LIVE, nt2);
  return status_of_launch();
}

int surf_batch_init_state(surf_batch* b, int32_t i, const void* c0, double c0_const,
                          double gamma0) {
  if (!b || i < 0 || i >= b->n) return SURF_EINVAL;
  long long n = (long long)b->grids[i].n[0] * b->grids[i].n[1];
  const surf_grid& gr = b->grids[i];
  const surf_params& q = b->prm[i];
  void* F = q.bulk_enabled ? b->F[2 * i] : nullptr;
  if (b->prec == SURF_F64)
    hipLaunchKernelGGL(k_init<double>, dim3(grid1d(n)), dim3(BLOCK), 0, b->stream, grid_of(gr),
                       par_of<double>(gr, q), (const double*)b->chi[i], (const double*)c0,
                       c0_const, gamma0, (double*)F, (double*)b->P[2 * i], n);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(grid1d(n)), dim3(BLOCK), 0, b->stream, grid_of(gr),
                       par_of<float>(gr, q), (const float*)b->chi[i], (const float*)c0,
                       (float)c0_const, (float)gamma0, (float*)F, (float*)b->P[2 * i], n);
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, b->stream, b->states + (size_t)i * NSTATE);
  b->parity = 0;
  return status_of_launch();
}

int surf_batch_step(surf_batch* b, int32_t nsteps, double* totals) {
  if (!b || nsteps <= 0) return SURF_EINVAL;
  if (!b->stream) {
    // no graph capture on the null stream: launch eagerly
    for (int k = 0; k < nsteps; ++k)
      batch_step_kernels(b, (b->parity + k) & 1, k == nsteps - 1 ? totals : nullptr);
    b->parity ^= nsteps & 1;
    return status_of_launch();
  }
  surf_batch::Graph* gr = nullptr;
  for (auto& g : b->graphs)
    if (g.nsteps == nsteps && g.parity == b->parity && g.totals == totals) gr = &g;
  if (!gr) {
    surf_batch::Graph g{nsteps, b->parity, totals, nullptr, nullptr};
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return SURF_EDEVICE;
    for (int k = 0; k < nsteps; ++k)
      batch_step_kernels(b, (b->parity + k) & 1, k == nsteps - 1 ? totals : nullptr);
    if (hipStreamEndCapture(b->stream, &g.g) != hipSuccess) return SURF_EDEVICE;
    if (hipGraphInstantiate(&g.e, g.g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g.g);
      return SURF_EDEVICE;
    }
    b->graphs.push_back(g);
    gr = &b->graphs.back();
  }
  if (hipGraphLaunch(gr->e, b->stream) != hipSuccess) return SURF_EDEVICE;
  b->parity ^= nsteps & 1;
  return SURF_OK;
}

int surf_batch_parity(surf_batch* b) { return b ? b->parity : SURF_EINVAL; }

int surf_batch_tune(surf_batch* b, int32_t* choice, double* times_us, int32_t max_times) {
  if (!b) return SURF_EINVAL;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SURF_EDEVICE;
  // each candidate reads the current buffers and writes the other ones: the
  // state is untouched and the next step overwrites the scratch results
  auto timed = [&](auto run) -> double {
    run();
    (void)hipEventRecord(e0, b->stream);
    for (int r = 0; r < 3; ++r) run();
    (void)hipEventRecord(e1, b->stream);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms * 1e3 / 3;
  };
  int k_out = 0, best = -1;
  // column kernel: row-chunk height (FP32 8 or 16 rows; FP64 8) by
  // persistent grid
  if (b->ncol_q > 0) {
    const int tys[2] = {8, 16};
    const int nty = b->prec == SURF_F64 ? 1 : 2;
    double best_t = 1e300;
    int best_ty = b->ty, best_grid = b->col_grid;
    for (int t = 0; t < nty; ++t) {
      b->ty = tys[t];
      if (b->prec == SURF_F64) batch_col_tables<double>(b);
      else batch_col_tables<float>(b);
      if (batch_upload(b) != SURF_OK) return SURF_EDEVICE;
      const int nq = b->ncol_q;
      const int grids[4] = {batch_col_default_grid(nq < 1024 ? nq : 1024),
                            batch_col_default_grid(nq), ((nq < 4096 ? nq : 4096) + 7) / 8 * 8,
                            (nq + 7) / 8 * 8};
      for (int g = 0; g < 4; ++g) {
        const int grid = grids[g];
        double us = timed([&]() {
          if (b->prec == SURF_F64) batch_launch_col<double>(b, b->ty, grid, b->parity);
          else batch_launch_col<float>(b, b->ty, grid, b->parity);
        });
        if (us < 0) return SURF_EDEVICE;
        if (times_us && k_out < max_times) times_us[k_out] = us;
        if (us < best_t) {
          best_t = us;
          best_ty = b->ty;
          best_grid = grid;
          best = k_out;
        }
        ++k_out;
      }
    }
    b->ty = best_ty;
    b->col_grid = best_grid;
    if (b->prec == SURF_F64) batch_col_tables<double>(b);
    else batch_col_tables<float>(b);
    if (batch_upload(b) != SURF_OK) return SURF_EDEVICE;
  }
  // tile kernel (paper-form instances): threads per workgroup by grid
  if (b->total_tiles > 0) {
    const int T = b->total_tiles;
    const int cand[][2] = {{256, T}, {512, T}, {512, T < 512 ? T : 512},
                           {512, T < 1024 ? T : 1024}, {256, T < 2048 ? T : 2048},
                           {512, T < 2048 ? T : 2048}};
    const int nc = (int)(sizeof(cand) / sizeof(cand[0]));
    double best_t = 1e300;
    int bk = 0;
    for (int k = 0; k < nc; ++k) {
      double us = timed([&]() {
        if (b->prec == SURF_F64) batch_launch_step<double>(b, cand[k][0], cand[k][1], b->parity);
        else batch_launch_step<float>(b, cand[k][0], cand[k][1], b->parity);
      });
      if (us < 0) return SURF_EDEVICE;
      if (times_us && k_out < max_times) times_us[k_out] = us;
      if (us < best_t) {
        best_t = us;
        bk = k;
      }
      if (b->ncol_q == 0 && best_t == us) best = k_out;
      ++k_out;
    }
    b->nt = cand[bk][0];
    b->grid = cand[bk][1];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  batch_drop_graphs(b);
  {
    std::lock_guard<std::mutex> lock(tune_mu);
    tune_cache()[b->tune_key] = TuneChoice{b->ty, b->col_grid, b->nt, b->grid};
    if (const char* path = std::getenv("SURF_TUNE_CACHE")) {
      if (FILE* f = std::fopen(path, "a")) {
        std::fprintf(f, "%s %d %d %d %d\n", b->tune_key.c_str(), b->ty, b->col_grid, b->nt,
                     b->grid);
        std::fclose(f);
      }
    }
  }
  if (choice) *choice = best;
  return status_of_launch();
}

int surf_batch_destroy(surf_batch* b) {
  if (!b) return SURF_OK;
  // graphs may still be in flight on the stream
  (void)hipStreamSynchronize(b->stream);
  batch_drop_graphs(b);
  delete b;
  return SURF_OK;
}

int surf_profile_enable(surf_ctx* c, int enable) {
  if (!c) return SURF_EINVAL;
  c->profile = enable != 0;
  return SURF_OK;
}

int surf_profile_read(surf_ctx* c, double* step_ms, int64_t* step_n, double* geom_ms,
                      int64_t* geom_n) {
  if (!c) return SURF_EINVAL;
  double ms[2] = {0.0, 0.0};
  int64_t cnt[2] = {0, 0};
  int rc = SURF_OK;
  for (auto& m : c->marks) {
    float t = 0.f;
    if (hipEventSynchronize(m.b) != hipSuccess || hipEventElapsedTime(&t, m.a, m.b) != hipSuccess)
      rc = SURF_EDEVICE;
    ms[m.kind] += t;
    cnt[m.kind] += 1;
    c->pool.push_back(m.a);
    c->pool.push_back(m.b);
  }
  c->marks.clear();
  if (step_ms) *step_ms = ms[0];
  if (step_n) *step_n = cnt[0];
  if (geom_ms) *geom_ms = ms[1];
  if (geom_n) *geom_n = cnt[1];
  return rc;
}

int surf_destroy(surf_ctx* c) {
  if (!c) return SURF_OK;
  for (auto& m : c->marks) {
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->ev_pre) (void)hipEventDestroy(c->ev_pre);
  if (c->ev_geo) (void)hipEventDestroy(c->ev_geo);
  if (c->hprog) {
    // the context's kernels may still write the progress words (the
    // stream itself may already be gone)
    (void)hipDeviceSynchronize();
    (void)hipHostFree(c->hprog);
  }
  delete c;
  return SURF_OK;
}

// ------------------------------------------------------------------
// Allocation-free step: the running state and the per-workgroup records of
// the reduction in a file-scope device array instead of a workspace.
// ------------------------------------------------------------------

}  // extern "C"

namespace {

// at most this many transport workgroups (2D: 58-column strips of 32-row
// groups, about 1.9 M cells per 1000; 3D: 58 x 14 x 16 blocks, about
// 13 M cells per 1000)
constexpr int STATIC_MAX_WG = 4096;
constexpr long long STATIC_DOUBLES = NSTATE + (long long)STATIC_MAX_WG * NPART;
__device__ __align__(256) double scratch[STATIC_DOUBLES];

constexpr int STATIC_MAX_DEVICES = 64;
double* scratch_dev[STATIC_MAX_DEVICES] = {};
std::mutex scratch_mu;

// The device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int static_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES)
    return SURF_EDEVICE;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SURF_EDEVICE;
    scratch_dev[dev] = (double*)p;
  }
  *out = scratch_dev[dev];
  return SURF_OK;
}

// The running state of one call: time and cumulative outflow from the
// caller's totals (zero without them), status and flags cleared.
__global__ void k_static_state(double* __restrict__ state, const double* __restrict__ totals) {
  if (threadIdx.x >= NSTATE) return;
  double v = 0.0;
  if (totals && threadIdx.x == S_TIME) v = totals[11];
  if (totals && threadIdx.x == S_OUTCUM) v = totals[3];
  state[threadIdx.x] = v;
}

}  // namespace

extern "C" {

int surf_step_static(const surf_grid* grid, const surf_params* params, double dt,
                     const void* chi, const void* const* u, const void* F_in,
                     const void* psi_in, void* F_out, void* psi_out, void* sigma_out,
                     double* totals_dev, void* hip_stream) {
  int rc = check_grid_params(grid, params);
  if (rc) return rc;
  if (!(dt > 0) || !std::isfinite(dt) || !chi || !psi_in || !psi_out) return SURF_EINVAL;
  if (params->flux_form != SURF_FLUX_WEIGHTED || params->substep2 != SURF_SUBSTEP2_EXPLICIT ||
      params->interface != SURF_IFACE_VOF)
    return SURF_EINVAL;
  const bool bulk = params->bulk_enabled != 0;
  if (bulk && (!F_in || !F_out)) return SURF_EINVAL;
  if (psi_in == psi_out || (bulk && (F_in == F_out || F_in == psi_out || psi_in == F_out)))
    return SURF_EINVAL;
  if (u && u[0])
    for (int d = 0; d < grid->dim; ++d)
      if (!u[d]) return SURF_EINVAL;
  const size_t es = esize(params);
  if (!aligned(chi, es) || !aligned(psi_in, es) || !aligned(psi_out, es)) return SURF_EINVAL;
  surf_ctx c;  // host-side description only: nothing here allocates
  c.grid = *grid;
  c.prm = with_defaults(params, grid->dim);
  c.g.dim = grid->dim;
  for (int d = 0; d < 3; ++d) {
    c.g.n[d] = grid->n[d];
    c.g.bc[d][0] = d < grid->dim ? grid->bc[d][0] : 0;
    c.g.bc[d][1] = d < grid->dim ? grid->bc[d][1] : 0;
  }
  c.stream = (hipStream_t)hip_stream;
  c.ncell = (long long)grid->n[0] * grid->n[1] * grid->n[2];
  c.col_nwg = col_shape(grid, params, &c.col_strips, &c.col_groups);
  c.c3_nwg = col3_shape(grid, params, c.c3);
  const int nwg = grid->dim == 2 ? c.col_nwg : c.c3_nwg;
  if (nwg == 0) return SURF_EINVAL;  // beyond the 32-bit offsets of the transport kernels
  if (nwg > STATIC_MAX_WG) return SURF_ENOMEM;
  double* base = nullptr;
  rc = static_scratch(&base);
  if (rc) return rc;
  c.state = base;
  c.part = base + NSTATE;
  c.chi[0] = const_cast<void*>(chi);
  c.chi[1] = nullptr;
  c.chi_cur = 0;
  c.has_chi = true;
  c.materialized = true;
  c.dt = dt;
  c.profile = false;
  hipLaunchKernelGGL(k_static_state, dim3(1), dim3(64), 0, c.stream, c.state,
                     (const double*)totals_dev);
  const bool f32 = params->precision == SURF_F32;
  if (grid->dim == 2) {
    if (f32) col2d_transport<float>(&c, u, F_in, psi_in, F_out, psi_out, sigma_out);
    else col2d_transport<double>(&c, u, F_in, psi_in, F_out, psi_out, sigma_out);
  } else {
    if (f32) col3d_transport<float>(&c, u, F_in, psi_in, F_out, psi_out, sigma_out);
    else col3d_transport<double>(&c, u, F_in, psi_in, F_out, psi_out, sigma_out);
  }
  if (f32) finalize<float>(&c, totals_dev, nwg);
  else finalize<double>(&c, totals_dev, nwg);
  return status_of_launch();
}

}  // extern "C"
