// surf_implicit.hpp -- substep 2 taken implicitly (section 3, second substep
// of the split; Appendix C), weighted flux form.
//
// After the advection of substep 1, implicit Euler for the confinement +
// diffusion + exchange step.  In terms of the carrier quotients r = xi / (w +
// eta_w) (c for the bulk, Gamma for the interface) the weighted-form flux
// divergence is -K r, K the symmetric face-weighted graph Laplacian with face
// coefficient D wbar / h^2 (wbar the face mean of w = phi or delta, no flux
// through walls and open sides).  The exchange source couples the two fields;
// Appendix C writes each equation as a linear elliptic problem whose
// reaction coefficient holds the other field at t^{n+1}.  The two problems
// are solved alternately (Picard sweeps, interface first, from c = c*):
//
//   interface:  [ (delta+eta/eps)(1/dt + kl k_a c + k_d) + K_s ] Gamma
//                   = psi*/dt + k_a c Gamma_inf delta
//   bulk:       [ (phi+eta)/dt + k_a (Gamma_inf delta - kl psi) + K_b ] c
//                   = F*/dt + k_d psi
//
// Each matrix is symmetric; it is positive definite while its reaction
// diagonal is positive (always for the interfacial one; for the bulk one
// while k_a kl psi < (phi + eta)/dt + k_a Gamma_inf delta).  Each problem is
// solved by Jacobi-preconditioned conjugate gradients in FP64, matrix-free,
// in the Chronopoulos-Gear arrangement (one global reduction per iteration,
// Chronopoulos and Gear, J. Comput. Appl. Math. 25, 1989):
//
//   r0 = b - A x0, u0 = M^-1 r0, w0 = A u0
//   iteration i:  gamma = (r, u), delta = (w, u),
//                 beta = gamma / gamma_prev (0 at i = 0),
//                 alpha = gamma / (delta - beta gamma / alpha_prev)
//                 z = w + beta z,  p = u + beta p,  x += alpha p,
//                 r -= alpha z,  u = M^-1 r,  w = A u
//
// so that one kernel launch per iteration does all vector work, including
// the matrix-vector product with the next u, which it forms at the
// neighbours from their r, w and z.  The kernels:
//   k_imp_adv    substep 1 into FP64 arrays, phi and delta, the starting
//                iterates, and per-block records of the open-side outflow
//                and the largest cell-mean velocity sum;
//   k_cg_setup   reaction diagonal, inverse Jacobi diagonal, r0 = b - A x0;
//   k_cg_iter    one iteration: every workgroup first reduces the previous
//                launch's per-workgroup partial sums (the same sums in the
//                same order, so every workgroup gets the same scalars), then
//                updates its tiles and leaves the partial sums of gamma,
//                delta, (u, u) and (x, x) for the next launch.  Launch -1 is
//                the start (alpha = beta = 0 gives u0 and w0);
//   k_cg_end     the solve's iteration count, and the status bit when it
//                ended without meeting the test;
//
// Each iteration launch also publishes its progress, and the end of the
// solve, to a word of pinned host memory.  Outside graph capture the host
// enqueues the iterations a few launches ahead of the device and stops once
// the test is met, instead of enqueuing cg_max_iters launches of which those
// after convergence return at once; which launches run is decided on the
// device either way, so the results are the same.
//   k_imp_final  F, psi, sigma and the step's reduction records.
//
// A solve ends when ||M^-1 r|| <= tol ||x|| (M the Jacobi diagonal).  The
// diagonal spans many orders of magnitude (delta + eta/eps and phi + eta
// vanish away from the interface and the liquid), so a test on ||r|| would
// leave the cells with a small diagonal unconverged; both matrices are
// strictly diagonally dominant, and then M^-1 r bounds the error cell by cell
// (|e| <= |M^-1 r| / (1 - rho), rho < 1 the largest off-diagonal row sum over
// the diagonal).  After the test is met (or on a breakdown) every later
// launch of that solve returns at once.
//
// On axisymmetric rings (Appendix B) every cell's balance is multiplied by
// its mid radius r_i (the volume 2 pi r_i h^2 up to a constant): a radial
// face's coefficient takes its radius r_face, an axial face's the ring's
// r_i, and the reaction diagonal and right-hand side r_i.  The matrix stays
// symmetric (each face has one coefficient), its solution is that of the
// divided balance, and the stop test on M^-1 r does not see the scaling.
// Substep 1 takes the radial fluxes with r_face / r_i, the outflow with the
// face areas 2 pi r h, and the records with the ring volumes.
//
// Layout: tiles of 64 x 32 cells of one z-plane, one tile row of 64 cells
// per wave lane set, four rows per lane held in registers with the rows
// above and below; x-neighbours by wave shifts, the tile's edge columns
// loaded by eight lanes and passed on; z-neighbours loaded.  Workgroups take
// contiguous runs of tiles, consecutive runs on the same XCD.
#pragma once
#include "surf_col2d.hpp"

namespace surf {

constexpr int IMP_BLOCK = 256;
constexpr int IMP_FIELDS = 15;      // FP64 cell arrays of ImpBuf
constexpr int IMP_MAX_PICARD = 32;  // Picard sweeps per step at most
constexpr int IMP_MAX_SOLVES = 2 * IMP_MAX_PICARD;

// FP64 arrays of the implicit path (one value per cell) and its records
struct ImpBuf {
  double *Fs, *Ps;          // advected state
  double *wF, *wP;          // phi and delta: face weights and carrier denominators
  double *xF, *xP;          // c and Gamma: Picard iterates and solutions
  double *dg, *minv;        // reaction diagonal, inverse Jacobi diagonal
  double *p, *r[2], *w[2], *z[2];  // CG vectors (r, w, z ping-pong by iteration)
  double* adv;              // [nblk][2]: outflow, largest velocity sum
  double* part;             // [2][CG_MAXWG][4]: CG partial sums
  double* sc;               // CG scalars and control words
  double* rec;              // [IMP_MAX_SOLVES]: iterations of the last step's solves
  double* B[3];             // paper form: the anti-diffusion coefficient per cell and axis
};

template <typename R>
struct ImpArgs {
  Grid g;
  Par<R> p;
  ImpBuf B;
  double dt, eta, eta_eps, ka, kd, ginf, kl, tol;  // FP64 coefficients
  double inv_h2, Db, Ds;
  int bulk;
  int lim, tr;  // substep-1 variants: MC limiter, BCG transverse term
  int axi;      // axisymmetric rings: x is the radius, from r0
  double r0, h; // the low radius and the cell size in FP64
  int paper;    // the paper's flux form: the unknowns are F and psi themselves
  long long ncell;
};

// Ring radii of column i (axisymmetric): low face, high face, middle
struct Rings {
  double lo, hi, mid;
};
__device__ __forceinline__ Rings rings_of(double r0, double h, int i) {
  Rings r;
  r.lo = r0 + (double)i * h;
  r.hi = r.lo + h;
  r.mid = r.lo + 0.5 * h;
  return r;
}

__device__ __forceinline__ void imp_coords(const Grid& g, long long c, int* x) {
  x[0] = (int)(c % g.n[0]);
  x[1] = (int)((c / g.n[0]) % g.n[1]);
  x[2] = (int)(c / ((long long)g.n[0] * g.n[1]));
}

template <int NT>
__device__ __forceinline__ void block_sums(double* v, int nv, double* out) {
  __shared__ double red[NT / 64][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int s = 0; s < nv; ++s) {
    const double x = wave_sum(v[s]);
    if (lane == 0) red[w][s] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    double x = red[0][threadIdx.x];
    for (int q = 1; q < NT / 64; ++q) x += red[q][threadIdx.x];
    out[threadIdx.x] = x;
  }
}

// ---------------------------------------------------------------- substep 1
template <typename R>
__global__ void __launch_bounds__(IMP_BLOCK) k_imp_adv(ImpArgs<R> a, const R* __restrict__ chi,
                                                       const R* __restrict__ u0,
                                                       const R* __restrict__ u1,
                                                       const R* __restrict__ u2,
                                                       const R* __restrict__ F,
                                                       const R* __restrict__ psi, R area_dt) {
  const long long c = (long long)blockIdx.x * IMP_BLOCK + threadIdx.x;
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  const R* u[3] = {u0, u1, u2};
  double out = 0.0, usum = 0.0;
  if (c < a.ncell) {
    int x[3];
    imp_coords(g, c, x);
    R ph, om, de;
    phase<R>(chi[c], p, ph, om, de);
    const R cfl = (R)a.dt * p.inv_h;
    R st[2] = {a.bulk ? F[c] : R(0), psi[c]};
    // axisymmetric: the radial faces' weights r_face / r_i in the balance,
    // and 2 pi r over the face areas of the outflow (Cartesian: 1)
    R wr[2] = {R(1), R(1)};
    double ar[3] = {1.0, 1.0, 1.0};  // radial low, radial high, axial
    if (a.axi) {
      const Rings r = rings_of(a.r0, a.h, x[0]);
      wr[0] = (R)(r.lo / r.mid);
      wr[1] = (R)(r.hi / r.mid);
      ar[0] = 2.0 * M_PI * r.lo;
      ar[1] = 2.0 * M_PI * r.hi;
      ar[2] = 2.0 * M_PI * r.mid;
    }
    if (u0) {
      for (int f = 0; f < 2; ++f) {
        if (f == 0 && !a.bulk) continue;
        const R* xi = f == 0 ? F : psi;
        R div = R(0);
        for (int d = 0; d < g.dim; ++d) {
          const bool per = g.bc[d][0] == BC_PERIODIC;
          const int nd = g.n[d];
          for (int s = 0; s < 2; ++s) {
            const int fidx = x[d] + s;
            const bool blo = !per && fidx == 0, bhi = !per && fidx == nd;
            int y[3] = {x[0], x[1], x[2]};
            y[d] = (per && fidx == nd) ? 0 : fidx;
            const R uf = u[d][face_index(g, d, y[0], y[1], y[2])];
            R fl;
            const double af = d == 0 ? ar[s] : ar[2];
            if (blo) {
              fl = g.bc[d][0] == BC_OPEN ? uf * xi[c] : R(0);
              out -= af * (double)(area_dt * fl);
            } else if (bhi) {
              fl = g.bc[d][1] == BC_OPEN ? uf * xi[c] : R(0);
              out += af * (double)(area_dt * fl);
            } else {
              const int off = s == 0 ? -1 : 0;
              auto at = [&](int o) {
                int w[3] = {x[0], x[1], x[2]};
                w[d] = map_axis(x[d] + o, nd, g.bc[d][0], g.bc[d][1]);
                return xi[cell_index(g, w[0], w[1], w[2])];
              };
              if (!a.lim && !a.tr) {
                fl = adv_flux<R>(uf, at(off - 1), at(off), at(off + 1), at(off + 2), cfl);
              } else {
                // the variants: the upwind cell's value, its limited slope
                // carried to the half-step foot, less dt/2h times its mean
                // transverse velocity times its upwind transverse difference
                const bool pos = uf > R(0);
                const int uo = pos ? off : off + 1;  // the upwind cell along d
                const R xm = at(uo - 1), xu = at(uo), xp = at(uo + 1);
                const R k = R(0.5) * (R(1) - fabs(uf) * cfl);
                const R sl = a.lim ? mc<R>(xu - xm, xp - xu) : minmod<R>(xu - xm, xp - xu);
                R val = xu + (pos ? k : -k) * sl;
                if (a.tr) {
                  int w[3] = {x[0], x[1], x[2]};
                  w[d] = map_axis(x[d] + uo, nd, g.bc[d][0], g.bc[d][1]);
                  for (int t = 0; t < g.dim; ++t) {
                    if (t == d) continue;
                    int hi[3] = {w[0], w[1], w[2]};
                    hi[t] = (g.bc[t][0] == BC_PERIODIC && w[t] + 1 == g.n[t]) ? 0 : w[t] + 1;
                    const R vt = R(0.5) * (u[t][face_index(g, t, w[0], w[1], w[2])] +
                                           u[t][face_index(g, t, hi[0], hi[1], hi[2])]);
                    int lo[3] = {w[0], w[1], w[2]}, up[3] = {w[0], w[1], w[2]};
                    lo[t] = map_axis(w[t] - 1, g.n[t], g.bc[t][0], g.bc[t][1]);
                    up[t] = map_axis(w[t] + 1, g.n[t], g.bc[t][0], g.bc[t][1]);
                    const R xc = xi[cell_index(g, w[0], w[1], w[2])];
                    const R dxt = vt > R(0) ? xc - xi[cell_index(g, lo[0], lo[1], lo[2])]
                                            : xi[cell_index(g, up[0], up[1], up[2])] - xc;
                    val -= R(0.5) * cfl * vt * dxt;
                  }
                }
                fl = uf * val;
              }
            }
            const R wf = d == 0 ? wr[s] : R(1);
            div += s == 0 ? -(wf * fl) : wf * fl;
          }
        }
        st[f] = xi[c] - cfl * div;
      }
      // cell-mean velocity sum (on a periodic axis the upper face of the
      // last cell is face 0, as in the fluxes)
      R s = R(0);
      for (int d = 0; d < g.dim; ++d) {
        int y[3] = {x[0], x[1], x[2]};
        const R ulo = u[d][face_index(g, d, y[0], y[1], y[2])];
        y[d] += 1;
        if (y[d] == g.n[d] && g.bc[d][1] == BC_PERIODIC) y[d] = 0;
        const R uhi = u[d][face_index(g, d, y[0], y[1], y[2])];
        // the radial mean weights each face by r_face / r_i
        s += d == 0 ? fabs(R(0.5) * (wr[0] * ulo + wr[1] * uhi)) : fabs(R(0.5) * (ulo + uhi));
      }
      usum = (double)s;
    }
    const double w0 = (double)ph, w1 = (double)de;
    a.B.wF[c] = w0;
    a.B.wP[c] = w1;
    a.B.Fs[c] = (double)st[0];
    a.B.Ps[c] = (double)st[1];
    if (a.paper) {
      a.B.xF[c] = a.bulk ? (double)st[0] : 0.0;
      a.B.xP[c] = (double)st[1];
    } else {
      a.B.xF[c] = a.bulk ? (double)st[0] / (w0 + a.eta) : 0.0;
      a.B.xP[c] = (double)st[1] / (w1 + a.eta_eps);
    }
  }
  // records: outflow (sum), largest velocity sum (max)
  __shared__ double red[IMP_BLOCK / 64][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double so = wave_sum(out), mu = wave_max(usum);
  if (lane == 0) {
    red[w][0] = so;
    red[w][1] = mu;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = 0.0, m = 0.0;
    for (int q = 0; q < IMP_BLOCK / 64; ++q) {
      o += red[q][0];
      m = fmax(m, red[q][1]);
    }
    a.B.adv[2 * blockIdx.x] = o;
    a.B.adv[2 * blockIdx.x + 1] = m;
  }
}

// ---------------------------------------------------------------- CG
constexpr int CG_WAVES = 8, CG_WG = 64 * CG_WAVES;  // 512 threads
constexpr int CG_ROWS = 4;                           // rows per lane
constexpr int CG_TX = 64, CG_TY = CG_WAVES * CG_ROWS;  // tile 64 x 32
constexpr int CG_MAXWG = 512;  // workgroups at most: each one reduces every partial
enum { CT_GAMMA = 0, CT_DELTA, CT_UU, CT_XX, CT_N = 4 };  // partial sums
// scalars: (gamma, alpha) of the last two iterations by parity, control words
enum { SC_GA = 0, SC_DONE = 4, SC_ITER = 5, SC_FAIL = 6, SC_N = 16 };
enum { STATUS_SOLVE = 16 };  // a linear solve ended without meeting its test

struct CgArgs {
  Grid g;
  const double* fw;  // face weight of the field (delta or phi)
  double kc;         // D / (2 h^2): a face's coefficient is kc (w_L + w_R)
  double tol2;
  double* x;         // the unknown (Gamma or c)
  double* p;
  double* r[2];
  double* w[2];
  double* z[2];
  double* minv;
  double* dg;
  double* part;      // [2][CG_MAXWG][CT_N]
  double* sc;        // [SC_N]
  // host-visible progress words (pinned host memory) or null: [0] the
  // solve's id << 32 | launches started, [1] the id of the last solve that
  // met its test
  unsigned long long* hp;
  unsigned long long solve_id;
  int tiles[3];      // tiles along x, y, z
  int ntiles, nwg, per_wg;
  int axi;           // axisymmetric rings: rows scaled by r_i, faces by their radius
  double r0, h;
};

__device__ __forceinline__ void cg_publish(unsigned long long* hp, int slot,
                                           unsigned long long v) {
  __hip_atomic_store(hp + slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ int cg_wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}
__device__ __forceinline__ int cg_clamp(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }
__device__ __forceinline__ int cg_map(int v, int n, bool per) {
  return per ? cg_wrap(v, n) : cg_clamp(v, n);
}

// the workgroup's run of tiles: hardware workgroup b runs on XCD b mod 8;
// the workgroups of one XCD take consecutive runs
__device__ __forceinline__ int cg_logical_wg(int b, int nwg) {
  const int q = nwg >> 3, rem = nwg & 7, k = b & 7;
  return k * q + (k < rem ? k : rem) + (b >> 3);
}

// the reaction diagonal and right-hand side of cell c (field 0: interface,
// 1: bulk), from the advected state and the other field's latest iterate
template <typename R>
__device__ __forceinline__ void cg_row(const ImpArgs<R>& a, int field, int c, double& dg,
                                       double& rhs) {
  const ImpBuf& B = a.B;
  if (field == 0) {
    const double dP = B.wP[c] + a.eta_eps, cF = a.bulk ? B.xF[c] : 0.0;
    dg = dP * (1.0 / a.dt + a.kl * a.ka * cF + a.kd);
    rhs = B.Ps[c] / a.dt + a.ka * cF * a.ginf * B.wP[c];
  } else {
    const double dF = B.wF[c] + a.eta, ps = (B.wP[c] + a.eta_eps) * B.xP[c];
    dg = dF / a.dt + a.ka * (a.ginf * B.wP[c] - a.kl * ps);
    rhs = B.Fs[c] / a.dt + a.kd * ps;
  }
}

// diagonal, inverse Jacobi diagonal and r0 = b - A x0 into r[1]; p, w[1] and
// z[0] cleared for the start launch; control words reset
template <typename R>
__global__ void __launch_bounds__(CG_WG) k_cg_setup(ImpArgs<R> a, CgArgs c, int field) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.sc[SC_DONE] = 0.0;
    c.sc[SC_ITER] = 0.0;
    c.sc[SC_FAIL] = 0.0;
  }
  const Grid& g = c.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const bool per[3] = {g.bc[0][0] == BC_PERIODIC, g.bc[1][0] == BC_PERIODIC,
                       g.dim == 3 && g.bc[2][0] == BC_PERIODIC};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int L = cg_logical_wg(blockIdx.x, c.nwg);
  const int t1 = min((L + 1) * c.per_wg, c.ntiles);
  for (int t = L * c.per_wg; t < t1; ++t) {
    const int tx = t % c.tiles[0], ty = (t / c.tiles[0]) % c.tiles[1];
    const int tz = t / (c.tiles[0] * c.tiles[1]);
    const int x = tx * CG_TX + lane;
    for (int j = 0; j < CG_ROWS; ++j) {
      const int y = ty * CG_TY + wv * CG_ROWS + j;
      if (x >= nx || y >= ny) continue;
      const int q[3] = {x, y, tz};
      const int n = x + nx * (y + ny * tz);
      double dg, rhs;
      cg_row(a, field, n, dg, rhs);
      // face radii (low, high radial face; axial faces) and the row scale
      double rf[3] = {1.0, 1.0, 1.0};
      if (c.axi) {
        const Rings r = rings_of(c.r0, c.h, x);
        rf[0] = r.lo;
        rf[1] = r.hi;
        rf[2] = r.mid;
        dg *= r.mid;
        rhs *= r.mid;
      }
      const double xc = c.x[n], wc = c.fw[n];
      double ax = dg * xc, m = dg;
      for (int d = 0; d < g.dim; ++d)
        for (int s = -1; s <= 1; s += 2) {
          const int v = q[d] + s;
          if (!per[d] && (v < 0 || v >= g.n[d])) continue;  // wall or open side
          int e[3] = {q[0], q[1], q[2]};
          e[d] = cg_wrap(v, g.n[d]);
          const int nb = e[0] + nx * (e[1] + ny * e[2]);
          const double k = c.kc * (wc + c.fw[nb]) * (d == 0 ? rf[s > 0 ? 1 : 0] : rf[2]);
          ax += k * (xc - c.x[nb]);
          m += k;
        }
      (void)nz;
      c.dg[n] = dg;
      // m > 0 unless the reaction diagonal is negative enough to make the
      // matrix indefinite; the iterations then flag a breakdown
      c.minv[n] = 1.0 / m;
      c.r[1][n] = rhs - ax;
      c.p[n] = 0.0;
      c.w[1][n] = 0.0;
      c.z[0][n] = 0.0;
    }
  }
}

// one iteration (it >= 0) or the start launch (it = -1)
template <int DIM, bool AXI>
__global__ void __launch_bounds__(CG_WG) k_cg_iter(CgArgs c, int it) {
  if (it >= 0 && c.sc[SC_DONE] != 0.0) return;  // uniform over the grid
  if (c.hp && blockIdx.x == 0 && threadIdx.x == 0)
    cg_publish(c.hp, 0, (c.solve_id << 32) | (unsigned long long)(it + 1));
  const int par = it & 1;
  double alpha = 0.0, beta = 0.0;
  if (it >= 0) {
    const double* P = c.part + (size_t)par * CG_MAXWG * CT_N;
    double v[CT_N] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < c.nwg; b += CG_WG)
      for (int k = 0; k < CT_N; ++k) v[k] += P[b * CT_N + k];
    __shared__ double tot[CT_N];
    block_sums<CG_WG>(v, CT_N, tot);
    __syncthreads();
    const double gam = tot[CT_GAMMA], del = tot[CT_DELTA];
    bool done = tot[CT_UU] <= c.tol2 * tot[CT_XX];
    bool fail = false;
    if (!done) {
      double den = del;
      if (it > 0) {
        const double* prev = c.sc + SC_GA + 2 * ((it - 1) & 1);
        beta = gam / prev[0];
        den = del - beta * gam / prev[1];
      }
      alpha = gam / den;
      fail = !(gam > 0.0) || !(den > 0.0) || !isfinite(alpha) || !isfinite(beta);
    }
    if (done || fail) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        c.sc[SC_DONE] = 1.0;
        c.sc[SC_ITER] = (double)it;
        c.sc[SC_FAIL] = fail ? 1.0 : 0.0;
        if (c.hp) cg_publish(c.hp, 1, c.solve_id);
      }
      return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c.sc[SC_GA + 2 * par] = gam;
      c.sc[SC_GA + 2 * par + 1] = alpha;
    }
  }
  const double* __restrict__ r_in = c.r[par];
  const double* __restrict__ w_in = c.w[par];
  const double* __restrict__ z_in = c.z[par ^ 1];
  double* __restrict__ r_out = c.r[par ^ 1];
  double* __restrict__ w_out = c.w[par ^ 1];
  double* __restrict__ z_out = c.z[par];
  const double* __restrict__ minv = c.minv;
  const double* __restrict__ fw = c.fw;
  const Grid& g = c.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const bool perx = g.bc[0][0] == BC_PERIODIC, pery = g.bc[1][0] == BC_PERIODIC;
  const bool perz = DIM == 3 && g.bc[2][0] == BC_PERIODIC;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double kc = c.kc;
  // u of the next iteration at cell n: M^-1 (r - alpha (w + beta z))
  auto unew = [&](int n) { return minv[n] * (r_in[n] - alpha * (w_in[n] + beta * z_in[n])); };
  double acc[CT_N] = {0.0, 0.0, 0.0, 0.0};
  const int L = cg_logical_wg(blockIdx.x, c.nwg);
  const int t1 = min((L + 1) * c.per_wg, c.ntiles);
  for (int t = L * c.per_wg; t < t1; ++t) {
    const int tx = t % c.tiles[0], ty = (t / c.tiles[0]) % c.tiles[1];
    const int zc = t / (c.tiles[0] * c.tiles[1]);
    const int x0 = tx * CG_TX, x = x0 + lane, xm = min(x, nx - 1);
    const int y0 = ty * CG_TY + wv * CG_ROWS;  // the lane's first row
    const int zoff = ny * zc;
    // face radii of the lane's column (axisymmetric; else 1)
    double rlo = 1.0, rhi = 1.0, rmid = 1.0;
    if (AXI) {
      const Rings r = rings_of(c.r0, c.h, xm);
      rlo = r.lo;
      rhi = r.hi;
      rmid = r.mid;
    }
    // register rows y0-1 .. y0+CG_ROWS (wrapped or clamped into the grid)
    double u[CG_ROWS + 2], fr[CG_ROWS + 2];
    double rold[CG_ROWS], mio[CG_ROWS], zo[CG_ROWS], ro[CG_ROWS];
#pragma unroll
    for (int k = 0; k < CG_ROWS + 2; ++k) {
      const int ym = cg_map(y0 - 1 + k, ny, pery);
      const int n = xm + nx * (ym + zoff);
      const double r_ = r_in[n], mi = minv[n];
      const double s = w_in[n] + beta * z_in[n];
      const double rn = r_ - alpha * s;
      u[k] = mi * rn;
      fr[k] = fw[n];
      if (k >= 1 && k <= CG_ROWS) {
        rold[k - 1] = r_;
        mio[k - 1] = mi;
        zo[k - 1] = s;
        ro[k - 1] = rn;
      }
    }
    // the tile's edge columns: lane 2j fetches row j's left neighbour
    // column, lane 2j + 1 its right one
    const int rl = min(63, nx - 1 - x0);  // the tile's last lane inside the grid
    const bool lex = x0 > 0 || perx, rex = x0 + CG_TX < nx || perx;
    double ue = 0.0, fe = 0.0;
    if (lane < 2 * CG_ROWS) {
      const int col = (lane & 1) ? (x0 + CG_TX < nx ? x0 + CG_TX : 0) : (x0 > 0 ? x0 - 1 : nx - 1);
      const int ym = cg_map(y0 + (lane >> 1), ny, pery);
      const int n = col + nx * (ym + zoff);
      ue = unew(n);
      fe = fw[n];
    }
#pragma unroll
    for (int j = 0; j < CG_ROWS; ++j) {
      const int k = j + 1, y = y0 + j;
      const double uc = u[k], fc = fr[k];
      double uL = from_left(uc), fL = from_left(fc);
      double uR = from_right(uc), fR = from_right(fc);
      const double ueL = __shfl(ue, 2 * j), feL = __shfl(fe, 2 * j);
      const double ueR = __shfl(ue, 2 * j + 1), feR = __shfl(fe, 2 * j + 1);
      if (lane == 0) {
        uL = ueL;
        fL = feL;
      }
      if (lane == rl) {
        uR = ueR;
        fR = feR;
      }
      const int ym = min(y, ny - 1);
      const int n = xm + nx * (ym + zoff);
      const double dgc = c.dg[n], xo = c.x[n], po = c.p[n];
      double Au = dgc * uc;
      // (the radii are 1 on a Cartesian grid: the template drops the products)
      if (lane > 0 || lex) Au += AXI ? kc * (fc + fL) * rlo * (uc - uL) : kc * (fc + fL) * (uc - uL);
      if (lane < rl || rex) Au += AXI ? kc * (fc + fR) * rhi * (uc - uR) : kc * (fc + fR) * (uc - uR);
      if (y > 0 || pery)
        Au += AXI ? kc * (fc + fr[k - 1]) * rmid * (uc - u[k - 1]) : kc * (fc + fr[k - 1]) * (uc - u[k - 1]);
      if (y + 1 < ny || pery)
        Au += AXI ? kc * (fc + fr[k + 1]) * rmid * (uc - u[k + 1]) : kc * (fc + fr[k + 1]) * (uc - u[k + 1]);
      if (DIM == 3) {
#pragma unroll
        for (int s = -1; s <= 1; s += 2) {
          const int zz = zc + s;
          const int nb = xm + nx * (ym + ny * cg_map(zz, nz, perz));
          const double un = unew(nb), fn = fw[nb];
          if ((zz >= 0 && zz < nz) || perz) Au += kc * (fc + fn) * (uc - un);
        }
      }
      const double pn = mio[j] * rold[j] + beta * po;
      const double xn = xo + alpha * pn;
      if (x < nx && y < ny) {
        c.x[n] = xn;
        c.p[n] = pn;
        r_out[n] = ro[j];
        z_out[n] = zo[j];
        w_out[n] = Au;
        acc[CT_GAMMA] += ro[j] * uc;
        acc[CT_DELTA] += Au * uc;
        acc[CT_UU] += uc * uc;
        acc[CT_XX] += xn * xn;
      }
    }
  }
  __shared__ double out[CT_N];
  block_sums<CG_WG>(acc, CT_N, out);
  if (threadIdx.x < CT_N)
    c.part[(size_t)(par ^ 1) * CG_MAXWG * CT_N + (size_t)L * CT_N + threadIdx.x] = out[threadIdx.x];
}

// after the solve's last launch: its iteration count into rec; the status
// bit when it neither met the test nor stopped on it
__global__ void __launch_bounds__(CG_WG) k_cg_end(CgArgs c, int iters, double* rec,
                                                  double* state) {
  const double done = c.sc[SC_DONE];
  double v[CT_N] = {0.0, 0.0, 0.0, 0.0};
  if (done == 0.0) {
    const double* P = c.part + (size_t)(iters & 1) * CG_MAXWG * CT_N;
    for (int b = threadIdx.x; b < c.nwg; b += CG_WG)
      for (int k = 0; k < CT_N; ++k) v[k] += P[b * CT_N + k];
  }
  __shared__ double tot[CT_N];
  block_sums<CG_WG>(v, CT_N, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  bool ok;
  if (done != 0.0) {
    *rec = c.sc[SC_ITER];
    ok = c.sc[SC_FAIL] == 0.0;
  } else {
    *rec = (double)iters;
    ok = tot[CT_UU] <= c.tol2 * tot[CT_XX];
  }
  if (!ok) atomicOr((unsigned*)(state + S_FLAGS), (unsigned)STATUS_SOLVE);
}

// ---------------------------------------------------------------- output
template <typename R>
__global__ void __launch_bounds__(IMP_BLOCK) k_imp_final(ImpArgs<R> a, R* __restrict__ Fo,
                                                         R* __restrict__ Po,
                                                         R* __restrict__ sig,
                                                         double* __restrict__ part) {
  const long long c = (long long)blockIdx.x * IMP_BLOCK + threadIdx.x;
  const Par<R>& p = a.p;
  const ImpBuf& B = a.B;
  double v[NPART];
#pragma unroll
  for (int s = 0; s < NPART; ++s) v[s] = 0.0;
  v[P_MAX_USUM] = 0.0;
  v[P_MAX_C] = -INFINITY;
  v[P_MIN_F] = INFINITY;
  v[P_MIN_PSI] = INFINITY;
  if (c < a.ncell) {
    const R ph = (R)B.wF[c], de = (R)B.wP[c];
    // the unknowns: c and Gamma (weighted form) or F and psi (paper form)
    const R Fn = a.bulk ? (R)(a.paper ? B.xF[c] : (B.wF[c] + a.eta) * B.xF[c]) : R(0);
    const R Pn = (R)(a.paper ? B.xP[c] : (B.wP[c] + a.eta_eps) * B.xP[c]);
    const R sg = eos<R>(rdiv<R>(Pn, de + p.eta_eps), p);
    if (a.bulk) Fo[c] = Fn;
    Po[c] = Pn;
    if (sig) sig[c] = sg;
    // axisymmetric: each ring counts 2 pi r_i (the finalize multiplies by h^2)
    double wv = 1.0;
    if (a.axi) {
      int x[3];
      imp_coords(a.g, c, x);
      wv = 2.0 * M_PI * rings_of(a.r0, a.h, x[0]).mid;
    }
    v[P_SUM_F] = wv * (double)Fn;
    v[P_SUM_PSI] = wv * (double)Pn;
    v[P_SUM_DELTA] = wv * (double)de;
    v[P_SUM_SIGDELTA] = wv * (double)(sg * de);
    if (a.bulk) {
      v[P_MAX_C] = (double)rdiv<R>(Fn, ph + p.eta);
      v[P_MIN_F] = (double)Fn;
    }
    v[P_MIN_PSI] = (double)Pn;
    v[P_NBAD] = isfinite(Pn + sg + Fn) ? 0.0 : 1.0;
  }
  if (threadIdx.x == 0) {
    // the advection pass's records of this block (same cells)
    v[P_OUTFLOW] = B.adv[2 * blockIdx.x];
    v[P_MAX_USUM] = B.adv[2 * blockIdx.x + 1];
  }
  block_partials<R, IMP_BLOCK>(v, part + (long long)blockIdx.x * NPART);
}

}  // namespace surf
