// surf_kernels.hpp -- HIP kernels of libsurf for gfx950.
//
//   k_pin      VoF -> redistancing pin data (section 2.5)
//   k_chi0     initial level set chi0 = (f - 1/2) h
//   k_hj       one Godunov Hamilton-Jacobi sweep (section 2.5)
//   k_step     the fused transport step: advection (section 3.1 substep 1),
//              confinement + diffusion + exchange (substep 2, sections 2.6,
//              3.2, Appendices A and C), equation of state (sections 2.3, 5,
//              6) and per-workgroup FP64 partial reductions
//   k_finalize deterministic reduction of the partials -> totals, status
//   k_init     F = c0 phi, psi = gamma0 delta
//   k_force2/3 Marangoni face force (section 2.4)
#pragma once
#include "surf_common.hpp"

namespace surf {

constexpr int BLOCK = 256;

// ---------------------------------------------------------------- geometry
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_chi0(Grid g, Par<R> p, const R* __restrict__ vof,
                                                R* __restrict__ chi, long long ncell) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= ncell) return;
  chi[c] = (vof[c] - R(0.5)) * p.h;
}

// Pin data: cells whose face neighbour has chi0 of the opposite (or zero)
// sign are pinned to the subcell distance h chi0 / Delta (Russo-Smereka);
// the others carry only the sign of chi0, stored as +-infinity.
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_pin(Grid g, Par<R> p, const R* __restrict__ vof,
                                               R* __restrict__ g0, long long ncell) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= ncell) return;
  int i = (int)(c % g.n[0]);
  int j = (int)((c / g.n[0]) % g.n[1]);
  int k = (int)(c / ((long long)g.n[0] * g.n[1]));
  int xyz[3] = {i, j, k};
  R x0 = (vof[c] - R(0.5)) * p.h;
  bool cut = false;
  R jump = R(0), grad2 = R(0);
  for (int d = 0; d < g.dim; ++d) {
    int a[3] = {i, j, k}, b[3] = {i, j, k};
    a[d] = map_axis(xyz[d] - 1, g.n[d], g.bc[d][0], g.bc[d][1]);
    b[d] = map_axis(xyz[d] + 1, g.n[d], g.bc[d][0], g.bc[d][1]);
    R xm = (vof[cell_index(g, a[0], a[1], a[2])] - R(0.5)) * p.h;
    R xp = (vof[cell_index(g, b[0], b[1], b[2])] - R(0.5)) * p.h;
    cut = cut || (x0 * xm <= R(0)) || (x0 * xp <= R(0));
    jump = fmax(jump, fabs(xm - x0));
    jump = fmax(jump, fabs(xp - x0));
    R cd = R(0.5) * (xp - xm);
    grad2 += cd * cd;
  }
  R Delta = fmax(fmax(rsqrt_<R>(grad2), jump), R(1e-30) * p.h);
  R inf = R(INFINITY);
  g0[c] = cut ? p.h * x0 / Delta : (x0 > R(0) ? inf : -inf);
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_hj(Grid g, Par<R> p, const R* __restrict__ src,
                                              const R* __restrict__ g0, R* __restrict__ dst,
                                              R dtau, long long ncell) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= ncell) return;
  R gv = g0[c];
  R v;
  if (fabs(gv) < R(INFINITY)) {
    v = gv;
  } else {
    int i = (int)(c % g.n[0]);
    int j = (int)((c / g.n[0]) % g.n[1]);
    int k = (int)(c / ((long long)g.n[0] * g.n[1]));
    int xyz[3] = {i, j, k};
    R x = src[c];
    R G2 = R(0);
    bool pos = gv > R(0);
    for (int d = 0; d < g.dim; ++d) {
      int a[3] = {i, j, k}, b[3] = {i, j, k};
      a[d] = map_axis(xyz[d] - 1, g.n[d], g.bc[d][0], g.bc[d][1]);
      b[d] = map_axis(xyz[d] + 1, g.n[d], g.bc[d][0], g.bc[d][1]);
      R bw = (x - src[cell_index(g, a[0], a[1], a[2])]) * p.inv_h;
      R fw = (src[cell_index(g, b[0], b[1], b[2])] - x) * p.inv_h;
      R t1, t2;
      if (pos) {
        t1 = bw > R(0) ? bw * bw : R(0);
        t2 = fw < R(0) ? fw * fw : R(0);
      } else {
        t1 = bw < R(0) ? bw * bw : R(0);
        t2 = fw > R(0) ? fw * fw : R(0);
      }
      G2 += t1 > t2 ? t1 : t2;
    }
    R s = pos ? R(1) : R(-1);
    v = x - dtau * s * (rsqrt_<R>(G2) - R(1));
  }
  v = v > p.chimax ? p.chimax : v;
  v = v < -p.chimax ? -p.chimax : v;
  dst[c] = v;
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_init(Grid g, Par<R> p, const R* __restrict__ chi,
                                                const R* __restrict__ c0, R c0_const, R gamma0,
                                                R* __restrict__ F, R* __restrict__ psi,
                                                long long ncell) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= ncell) return;
  R ph, om, de;
  phase<R>(chi[c], p, ph, om, de);
  if (F) F[c] = (c0 ? c0[c] : c0_const) * ph;
  psi[c] = gamma0 * de;
}

// ---------------------------------------------------------------- the step
template <typename R>
struct StepArgs {
  Grid g;
  Par<R> p;
  const R* chi;
  const R* u[3];
  const R* F;
  const R* psi;
  R* Fo;
  R* Po;
  R* sig;
  double* part;
  R dt;
  R area_dt;   // h^(dim-1) * dt, for the open-boundary budget
  int has_u;
  int tiles[3];
  int lim, tr;  // substep-1 variants: MC limiter, BCG transverse term
};

// Advective flux u xi_f through a face (section 3.1): xi_f is the upwind
// value plus the minmod-limited slope carried to the half-step foot of the
// characteristic, xi_U +- (1 - |u| dt/h)/2 minmod(dxi-, dxi+).
template <typename R>
__device__ __forceinline__ R adv_flux(R uf, R xLm, R xL, R xR, R xRp, R cfl_scale) {
  const bool pos = uf > R(0);
  const R a = pos ? xLm : xRp;  // cell behind the upwind cell
  const R b = pos ? xL : xR;    // upwind cell
  const R c = pos ? xR : xL;    // downwind cell
  const R k = R(0.5) * (R(1) - fabs(uf) * cfl_scale);
  return uf * (b + k * minmod<R>(b - a, c - b));
}

// Monotonized central slope (van Leer 1977): the centred difference bounded
// by twice each one-sided difference, 0 at extrema.
template <typename R>
__device__ __forceinline__ R mc(R a, R b) {
  const R m = fmin(fabs(R(0.5) * (a + b)), R(2) * fmin(fabs(a), fabs(b)));
  return a * b > R(0) ? copysign(m, a) : R(0);
}

// Paper-form anti-diffusion coefficient of a cell along d (section 3.2,
// Appendix C): B_F = -D_b (1-phi)/eps n_d, B_psi = -D_s (1-2 phi)/eps n_d with
// n = -grad chi/|grad chi| from centred differences read from global memory.
template <typename R>
__device__ R paper_B(const Grid& g, const Par<R>& p, const R* __restrict__ chi, const int* m,
                     int d, bool bulk_field) {
  R grad[3] = {R(0), R(0), R(0)};
  R nrm = R(0);
  for (int e = 0; e < g.dim; ++e) {
    int a[3] = {m[0], m[1], m[2]}, b[3] = {m[0], m[1], m[2]};
    a[e] = map_axis(m[e] - 1, g.n[e], g.bc[e][0], g.bc[e][1]);
    b[e] = map_axis(m[e] + 1, g.n[e], g.bc[e][0], g.bc[e][1]);
    grad[e] = (chi[cell_index(g, b[0], b[1], b[2])] - chi[cell_index(g, a[0], a[1], a[2])]) *
              (R(0.5) * p.inv_h);
    nrm += grad[e] * grad[e];
  }
  nrm = rsqrt_<R>(nrm);
  nrm = nrm < R(1e-6) ? R(1e-6) : nrm;
  R nd = -grad[d] / nrm;
  R ph, om, de;
  phase<R>(chi[cell_index(g, m[0], m[1], m[2])], p, ph, om, de);
  R w = bulk_field ? om : (om - ph);
  return -(bulk_field ? p.Db : p.Ds) * w * p.inv_eps * nd;
}

// Per-workgroup partial record: wave reductions, then the NT/64 wave results
// combined in wave order by threads 0..NPART-1.
template <typename R, int NT>
__device__ __forceinline__ void block_partials(double* v, double* out) {
  __shared__ double red[NT / 64][NPART];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NPART; ++s) {
    double x = v[s];
    if (s == P_MAX_USUM || s == P_MAX_C) x = wave_max(x);
    else if (s == P_MIN_F || s == P_MIN_PSI) x = wave_min(x);
    else x = wave_sum(x);
    if (lane == 0) red[w][s] = x;
  }
  __syncthreads();
  if (threadIdx.x < NPART) {
    int s = threadIdx.x;
    double x = red[0][s];
    for (int q = 1; q < NT / 64; ++q) {
      double y = red[q][s];
      if (s == P_MAX_USUM || s == P_MAX_C) x = fmax(x, y);
      else if (s == P_MIN_F || s == P_MIN_PSI) x = fmin(x, y);
      else x += y;
    }
    out[s] = x;
  }
}

// The advective flux through an interior face with the substep-1 variants
// (section 3.1): the upwind cell's value and its slope (MC or minmod)
// carried to the half-step foot, less dt/2h times its mean transverse
// velocity times its upwind transverse difference for each transverse axis
// (the unsplit BCG predictor).  x: a field in LDS with strides s3, lL the
// face's low cell there and gL its coordinates in the box (the high cell is
// one step along d; both are cells of the box, a periodic wrap included).
template <typename R, int DIM>
__device__ R step_flux_var(const StepArgs<R>& a, const R* x, int lL, const int* s3, int d,
                           const int* gL, R uf, R cfl) {
  const Grid& g = a.g;
  const int st = s3[d];
  const bool pos = uf > R(0);
  const int lU = pos ? lL : lL + st;  // the upwind cell
  const R xm = x[lU - st], xu = x[lU], xp = x[lU + st];
  const R k = R(0.5) * (R(1) - fabs(uf) * cfl);
  const R sl = a.lim ? mc<R>(xu - xm, xp - xu) : minmod<R>(xu - xm, xp - xu);
  R val = xu + (pos ? k : -k) * sl;
  if (a.tr) {
    int w[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int q = gL[e] + (e == d && !pos ? 1 : 0);
      w[e] = e < DIM ? map_axis(q, g.n[e], g.bc[e][0], g.bc[e][1]) : 0;
    }
#pragma unroll
    for (int t = 0; t < DIM; ++t) {
      if (t == d) continue;
      int hi[3] = {w[0], w[1], w[2]};
      hi[t] = (g.bc[t][0] == BC_PERIODIC && w[t] + 1 == g.n[t]) ? 0 : w[t] + 1;
      const R vt = R(0.5) * (a.u[t][face_index(g, t, w[0], w[1], w[2])] +
                             a.u[t][face_index(g, t, hi[0], hi[1], hi[2])]);
      const R dxt = vt > R(0) ? xu - x[lU - s3[t]] : x[lU + s3[t]] - xu;
      val -= R(0.5) * cfl * vt * dxt;
    }
  }
  return uf * val;
}

// Fused step on one tile of TX x TY (x TZ) cells.  LDS holds the old state
// with a 3-cell halo (region A), then the advected state, phi and delta on a
// 1-cell halo (region C); region A is reused for c* = F*/(phi+eta) and
// Gamma* = psi*/(delta + eta/eps).
template <typename R, int DIM, int TX, int TY, int TZ>
__global__ void __launch_bounds__(BLOCK) k_step(StepArgs<R> a) {
  constexpr int TZ_ = DIM == 3 ? TZ : 1;
  constexpr int EX3 = TX + 6, EY3 = TY + 6, EZ3 = DIM == 3 ? TZ + 6 : 1;
  constexpr int EX1 = TX + 2, EY1 = TY + 2, EZ1 = DIM == 3 ? TZ + 2 : 1;
  constexpr int N3 = EX3 * EY3 * EZ3, N1 = EX1 * EY1 * EZ1, NTILE = TX * TY * TZ_;
  static_assert(2 * N1 <= 2 * N3, "region reuse");
  __shared__ R sA[2 * N3];
  __shared__ R sC[4 * N1];
  R* sF1 = sC;
  R* sP1 = sC + N1;
  R* sPhi = sC + 2 * N1;
  R* sDel = sC + 3 * N1;

  const Grid& g = a.g;
  const Par<R>& p = a.p;
  const bool bulk = p.bulk != 0;
  int b = blockIdx.x;
  int bx = b % a.tiles[0];
  int by = (b / a.tiles[0]) % a.tiles[1];
  int bz = b / (a.tiles[0] * a.tiles[1]);
  int org[3] = {bx * TX, by * TY, DIM == 3 ? bz * TZ : 0};
  int tid = threadIdx.x;

  double acc[NPART];
#pragma unroll
  for (int s = 0; s < NPART; ++s) acc[s] = 0.0;
  acc[P_MAX_USUM] = 0.0;
  acc[P_MAX_C] = -INFINITY;
  acc[P_MIN_F] = INFINITY;
  acc[P_MIN_PSI] = INFINITY;

  // phase 1: old state into LDS
  if (a.has_u) {
    for (int l = tid; l < N3; l += BLOCK) {
      int lx = l % EX3, ly = (l / EX3) % EY3, lz = l / (EX3 * EY3);
      int mx = map_axis(org[0] + lx - 3, g.n[0], g.bc[0][0], g.bc[0][1]);
      int my = map_axis(org[1] + ly - 3, g.n[1], g.bc[1][0], g.bc[1][1]);
      int mz = DIM == 3 ? map_axis(org[2] + lz - 3, g.n[2], g.bc[2][0], g.bc[2][1]) : 0;
      long long c = cell_index(g, mx, my, mz);
      sA[l] = bulk ? a.F[c] : R(0);
      sA[N3 + l] = a.psi[c];
    }
  } else {
    for (int l = tid; l < N1; l += BLOCK) {
      int lx = l % EX1, ly = (l / EX1) % EY1, lz = l / (EX1 * EY1);
      int mx = map_axis(org[0] + lx - 1, g.n[0], g.bc[0][0], g.bc[0][1]);
      int my = map_axis(org[1] + ly - 1, g.n[1], g.bc[1][0], g.bc[1][1]);
      int mz = DIM == 3 ? map_axis(org[2] + lz - 1, g.n[2], g.bc[2][0], g.bc[2][1]) : 0;
      long long c = cell_index(g, mx, my, mz);
      sF1[l] = bulk ? a.F[c] : R(0);
      sP1[l] = a.psi[c];
    }
  }
  __syncthreads();

  // phase 2: advected state xi* and the phase field on the 1-cell halo
  const int s3[3] = {1, EX3, EX3 * EY3};
  const R cfl = a.dt * p.inv_h;
  for (int l = tid; l < N1; l += BLOCK) {
    int l1[3] = {l % EX1, (l / EX1) % EY1, l / (EX1 * EY1)};
    int gc[3], m[3];
    bool ghost = false, inside = true;
    for (int d = 0; d < 3; ++d) {
      if (d < DIM) {
        gc[d] = org[d] + l1[d] - 1;
        m[d] = map_axis(gc[d], g.n[d], g.bc[d][0], g.bc[d][1]);
        bool lo_out = gc[d] < 0, hi_out = gc[d] >= g.n[d];
        if ((lo_out && g.bc[d][0] != BC_PERIODIC) || (hi_out && g.bc[d][1] != BC_PERIODIC)) ghost = true;
        if (lo_out || hi_out) inside = false;
      } else {
        gc[d] = 0;
        m[d] = 0;
      }
    }
    long long cm = cell_index(g, m[0], m[1], m[2]);
    R ph, om, de;
    phase<R>(a.chi[cm], p, ph, om, de);
    sPhi[l] = ph;
    sDel[l] = de;
    bool interior = inside && l1[0] >= 1 && l1[0] <= TX && l1[1] >= 1 && l1[1] <= TY &&
                    (DIM == 2 || (l1[2] >= 1 && l1[2] <= TZ));
    if (a.has_u) {
      int l3 = (l1[0] + 2) + EX3 * ((l1[1] + 2) + EY3 * (DIM == 3 ? l1[2] + 2 : 0));
      R divF = R(0), divP = R(0);
      double usum = 0.0;
      if (!ghost) {
        for (int d = 0; d < DIM; ++d) {
          int st = s3[d];
          // face indices: lo face of the mapped cell, hi face (wrapped when periodic)
          int flo[3] = {m[0], m[1], m[2]}, fhi[3] = {m[0], m[1], m[2]};
          fhi[d] = m[d] + 1;
          if (fhi[d] == g.n[d] && g.bc[d][1] == BC_PERIODIC) fhi[d] = 0;
          R ulo = a.u[d][face_index(g, d, flo[0], flo[1], flo[2])];
          R uhi = a.u[d][face_index(g, d, fhi[0], fhi[1], fhi[2])];
          bool blo = gc[d] == 0 && g.bc[d][0] != BC_PERIODIC;
          bool bhi = gc[d] == g.n[d] - 1 && g.bc[d][1] != BC_PERIODIC;
          for (int f = 0; f < 2; ++f) {
            if (f == 0 && !bulk) continue;
            const R* x = sA + f * N3;
            R Flo, Fhi;
            const bool var = a.lim || a.tr;
            if (blo) {
              Flo = g.bc[d][0] == BC_OPEN ? ulo * x[l3] : R(0);
            } else if (var) {
              int gL[3] = {gc[0], gc[1], gc[2]};
              gL[d] -= 1;
              Flo = step_flux_var<R, DIM>(a, x, l3 - st, s3, d, gL, ulo, cfl);
            } else {
              Flo = adv_flux<R>(ulo, x[l3 - 2 * st], x[l3 - st], x[l3], x[l3 + st], cfl);
            }
            if (bhi) {
              Fhi = g.bc[d][1] == BC_OPEN ? uhi * x[l3] : R(0);
            } else if (var) {
              Fhi = step_flux_var<R, DIM>(a, x, l3, s3, d, gc, uhi, cfl);
            } else {
              Fhi = adv_flux<R>(uhi, x[l3 - st], x[l3], x[l3 + st], x[l3 + 2 * st], cfl);
            }
            if (f == 0) divF += Fhi - Flo; else divP += Fhi - Flo;
            if (interior) {
              if (blo && g.bc[d][0] == BC_OPEN) acc[P_OUTFLOW] -= (double)(a.area_dt * Flo);
              if (bhi && g.bc[d][1] == BC_OPEN) acc[P_OUTFLOW] += (double)(a.area_dt * Fhi);
            }
          }
          if (interior) {
            int fl[3] = {m[0], m[1], m[2]};
            fl[d] = m[d] + 1;  // upper face for the cell-mean velocity: face 0
            if (fl[d] == g.n[d] && g.bc[d][1] == BC_PERIODIC) fl[d] = 0;  // on a periodic axis
            R uup = a.u[d][face_index(g, d, fl[0], fl[1], fl[2])];
            usum += fabs((double)(R(0.5) * (ulo + uup)));
          }
        }
        if (interior) acc[P_MAX_USUM] = fmax(acc[P_MAX_USUM], usum);
        sF1[l] = bulk ? sA[l3] - cfl * divF : R(0);
        sP1[l] = sA[N3 + l3] - cfl * divP;
      } else {
        sF1[l] = R(0);
        sP1[l] = R(0);
      }
    }
  }
  __syncthreads();

  // phase 3: c* and Gamma* (weighted form) into region A
  R* sc = sA;
  R* sG = sA + N1;
  if (p.form == FORM_W) {
    for (int l = tid; l < N1; l += BLOCK) {
      sc[l] = sF1[l] / (sPhi[l] + p.eta);
      sG[l] = sP1[l] / (sDel[l] + p.eta_eps);
    }
  }
  __syncthreads();

  // phase 4: substep 2 on the tile interior, EoS, outputs, partial sums
  const int s1[3] = {1, EX1, EX1 * EY1};
  for (int t = tid; t < NTILE; t += BLOCK) {
    int it[3] = {t % TX, (t / TX) % TY, t / (TX * TY)};
    int gc[3];
    bool inside = true;
    for (int d = 0; d < 3; ++d) {
      gc[d] = d < DIM ? org[d] + it[d] : 0;
      if (d < DIM && gc[d] >= g.n[d]) inside = false;
    }
    if (!inside) continue;
    int l = (it[0] + 1) + EX1 * ((it[1] + 1) + EY1 * (DIM == 3 ? it[2] + 1 : 0));
    R divF = R(0), divP = R(0);
    for (int d = 0; d < DIM; ++d) {
      int st = s1[d];
      bool blo = gc[d] == 0 && g.bc[d][0] != BC_PERIODIC;
      bool bhi = gc[d] == g.n[d] - 1 && g.bc[d][1] != BC_PERIODIC;
      R FloF = R(0), FhiF = R(0), FloP = R(0), FhiP = R(0);
      if (p.form == FORM_W) {
        if (!blo) {
          FloF = p.Db * R(0.5) * (sPhi[l - st] + sPhi[l]) * (sc[l] - sc[l - st]) * p.inv_h;
          FloP = p.Ds * R(0.5) * (sDel[l - st] + sDel[l]) * (sG[l] - sG[l - st]) * p.inv_h;
        }
        if (!bhi) {
          FhiF = p.Db * R(0.5) * (sPhi[l] + sPhi[l + st]) * (sc[l + st] - sc[l]) * p.inv_h;
          FhiP = p.Ds * R(0.5) * (sDel[l] + sDel[l + st]) * (sG[l + st] - sG[l]) * p.inv_h;
        }
      } else {
        int m0[3], mm[3], mp[3];
        for (int e = 0; e < 3; ++e) {
          m0[e] = e < DIM ? gc[e] : 0;
          mm[e] = m0[e];
          mp[e] = m0[e];
        }
        mm[d] = map_axis(gc[d] - 1, g.n[d], g.bc[d][0], g.bc[d][1]);
        mp[d] = map_axis(gc[d] + 1, g.n[d], g.bc[d][0], g.bc[d][1]);
        for (int f = 0; f < 2; ++f) {
          if (f == 0 && !bulk) continue;
          const R* x = f == 0 ? sF1 : sP1;
          R D = f == 0 ? p.Db : p.Ds;
          R Bc = paper_B<R>(g, p, a.chi, m0, d, f == 0);
          R lo = R(0), hi = R(0);
          if (!blo) {
            R Bm = paper_B<R>(g, p, a.chi, mm, d, f == 0);
            R Bf = R(0.5) * (Bm + Bc);
            lo = D * (x[l] - x[l - st]) * p.inv_h + Bf * (Bf < R(0) ? x[l - st] : x[l]);
          }
          if (!bhi) {
            R Bp = paper_B<R>(g, p, a.chi, mp, d, f == 0);
            R Bf = R(0.5) * (Bc + Bp);
            hi = D * (x[l + st] - x[l]) * p.inv_h + Bf * (Bf < R(0) ? x[l] : x[l + st]);
          }
          if (f == 0) { FloF = lo; FhiF = hi; } else { FloP = lo; FhiP = hi; }
        }
      }
      divF += (FhiF - FloF) * p.inv_h;
      divP += (FhiP - FloP) * p.inv_h;
    }
    R Fs = sF1[l], Ps = sP1[l], ph = sPhi[l], de = sDel[l];
    R cs = Fs / (ph + p.eta);
    R q = R(0);
    if (bulk) {
      q = p.kin == KIN_LANGMUIR ? p.ka * cs * (p.ginf * de - Ps) - p.kd * Ps
                                : p.ka * cs * p.ginf * de - p.kd * Ps;
    }
    R Fn = bulk ? Fs + a.dt * (divF - q) : R(0);
    R Pn = Ps + a.dt * (divP + q);
    R G = Pn / (de + p.eta_eps);
    R sg = eos<R>(G, p);
    long long c = cell_index(g, gc[0], gc[1], gc[2]);
    if (bulk) a.Fo[c] = Fn;
    a.Po[c] = Pn;
    if (a.sig) a.sig[c] = sg;
    acc[P_SUM_F] += (double)Fn;
    acc[P_SUM_PSI] += (double)Pn;
    acc[P_SUM_DELTA] += (double)de;
    acc[P_SUM_SIGDELTA] += (double)sg * (double)de;
    if (bulk) {
      acc[P_MAX_C] = fmax(acc[P_MAX_C], (double)(Fn / (ph + p.eta)));
      acc[P_MIN_F] = fmin(acc[P_MIN_F], (double)Fn);
    }
    acc[P_MIN_PSI] = fmin(acc[P_MIN_PSI], (double)Pn);
    bool bad = !isfinite(Pn) || !isfinite(sg) || (bulk && !isfinite(Fn));
    acc[P_NBAD] += bad ? 1.0 : 0.0;
  }
  block_partials<R, BLOCK>(acc, a.part + (long long)blockIdx.x * NPART);
}

// ---------------------------------------------------------------- finalize
struct FinalArgs {
  int nblk;
  int dim, bulk;
  double h, ka, cfl_a, cfl_d, dt;
  double lam0;  // stability rate of substep 2 without the c_max term
  int implicit; // substep 2 implicit: only the advective bound applies
  double lam_acdi;  // stability rate of the ACDI regularization (0 without ACDI)
};

constexpr int FIN_BLOCK = 256;

__device__ __forceinline__ void finalize_body(const FinalArgs& f, const double* __restrict__ part,
                                              double* __restrict__ state,
                                              double* __restrict__ totals) {
  double v[NPART];
#pragma unroll
  for (int s = 0; s < NPART; ++s) v[s] = 0.0;
  v[P_MAX_USUM] = 0.0;
  v[P_MAX_C] = -INFINITY;
  v[P_MIN_F] = INFINITY;
  v[P_MIN_PSI] = INFINITY;
  // records b = tid, tid + FIN_BLOCK, ... combined in that order; four of
  // them are loaded (from valid records) before any is combined
  constexpr int U = 4;
  for (int b0 = threadIdx.x; b0 < f.nblk; b0 += U * FIN_BLOCK) {
    double r[U][NPART];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = min(b0 + u * FIN_BLOCK, f.nblk - 1);
#pragma unroll
      for (int s = 0; s < NPART; ++s) r[u][s] = part[(long long)b * NPART + s];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (b0 + u * FIN_BLOCK >= f.nblk) break;
#pragma unroll
      for (int s = 0; s < NPART; ++s) {
        if (s == P_MAX_USUM || s == P_MAX_C) v[s] = fmax(v[s], r[u][s]);
        else if (s == P_MIN_F || s == P_MIN_PSI) v[s] = fmin(v[s], r[u][s]);
        else v[s] += r[u][s];
      }
    }
  }
  __shared__ double tot[NPART];
  block_partials<double, FIN_BLOCK>(v, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  double vol = f.dim == 3 ? f.h * f.h * f.h : f.h * f.h;
  double MB = f.bulk ? tot[P_SUM_F] * vol : 0.0;
  double MS = tot[P_SUM_PSI] * vol;
  double SD = tot[P_SUM_DELTA] * vol;
  double SSD = tot[P_SUM_SIGDELTA] * vol;
  double out = tot[P_OUTFLOW];
  double outcum = state[S_OUTCUM] + out;
  double t = state[S_TIME] + f.dt;
  double su = tot[P_MAX_USUM];
  double cmax = f.bulk ? tot[P_MAX_C] : 0.0;
  double lam = f.lam0;
  if (f.bulk) lam += f.ka * (cmax > 0 ? cmax : 0.0);
  double dta = su > 0 ? f.cfl_a * f.h / su : INFINITY;
  double dtd = f.implicit ? INFINITY : f.cfl_d / lam;
  double bound = fmin(su > 0 ? f.h / su : INFINITY, f.implicit ? INFINITY : 1.0 / lam);
  if (f.lam_acdi > 0) {
    dtd = fmin(dtd, f.cfl_d / f.lam_acdi);
    bound = fmin(bound, 1.0 / f.lam_acdi);
  }
  unsigned status = (unsigned)state[S_STATUS] | *(const unsigned*)(state + S_FLAGS);
  if (tot[P_NBAD] > 0) status |= 1u;
  if ((f.bulk && tot[P_MIN_F] < 0) || tot[P_MIN_PSI] < 0) status |= 2u;
  if (f.dt > bound) status |= 4u;
  state[S_TIME] = t;
  state[S_OUTCUM] = outcum;
  state[S_STEPS] += 1.0;
  state[S_STATUS] = (double)status;
  if (totals) {
    totals[0] = MB;
    totals[1] = MS;
    totals[2] = out;
    totals[3] = outcum;
    totals[4] = SD;
    totals[5] = SSD;
    totals[6] = su;
    totals[7] = fmin(dta, dtd);
    totals[8] = f.bulk ? tot[P_MIN_F] : 0.0;
    totals[9] = tot[P_MIN_PSI];
    totals[10] = tot[P_NBAD];
    totals[11] = t;
    totals[12] = MS / SD;
    totals[13] = SSD / SD;
    totals[14] = MB + MS + outcum;
    totals[15] = cmax;
  }
}

__global__ void __launch_bounds__(FIN_BLOCK) k_finalize(FinalArgs f, const double* __restrict__ part,
                                                        double* __restrict__ state,
                                                        double* __restrict__ totals) {
  finalize_body(f, part, state, totals);
}

// one workgroup per instance: part + first[i] NPART holds instance i's records
__global__ void __launch_bounds__(FIN_BLOCK) k_batch_final(const FinalArgs* __restrict__ fa,
                                                           const int* __restrict__ first,
                                                           const double* __restrict__ part,
                                                           double* __restrict__ states,
                                                           double* __restrict__ totals) {
  const int i = blockIdx.x;
  finalize_body(fa[i], part + (long long)first[i] * NPART, states + (long long)i * NSTATE,
                totals ? totals + 16ll * i : nullptr);
}

__global__ void k_reset_state(double* state) {
  if (threadIdx.x < NSTATE) state[threadIdx.x] = 0.0;
}

// the running time from a device value (0 without one)
__global__ void k_set_time(double* state, const double* t) {
  if (threadIdx.x == 0) state[S_TIME] = t ? *t : 0.0;
}

// ---------------------------------------------------------------- force
// Marangoni face force (section 2.4), F_d = dbar (grad sigma - n (n . grad
// sigma))_d on every face, n = grad chi / max(|grad chi|, 1e-6); the face
// gradient of a cell field takes the compact difference across the face for
// its normal component and the centred transverse differences of the two
// cells, averaged, for the others; dbar is the mean delta of the two cells.
// The divisions by h and by the norm are multiplications by reciprocals.
//
// 2D work unit: a tile of TX x TY cells, one thread per cell; chi, sigma and
// delta of the tile and a one-cell halo (corners included: the transverse
// differences of the cell across the face) are staged in LDS, with mirrored
// ghosts at walls and open sides and wrapped ones on periodic axes.  3D: a
// TX x TY column tile marching along z over ZC planes, three planes (z - 1,
// z, z + 1, each with its halo ring) in an LDS ring, so that a plane is
// loaded and its delta evaluated once per chunk instead of once per tile
// layer.  Each thread writes the low face of its cell along every axis; the
// last cell along an axis also writes the high face (zero on a wall or open
// side, on a periodic axis the value of face 0, computed from the same two
// cells in the same order).  Tile and cell indices are 32-bit (no 64-bit
// division).
template <typename R>
__device__ __forceinline__ R force_finish(const R* gn, const R* gs, int dim, int d, R dbar) {
  R nrm = R(0), dot = R(0);
  for (int e = 0; e < dim; ++e) {
    nrm += gn[e] * gn[e];
    dot += gn[e] * gs[e];
  }
  nrm = rsqrt_<R>(nrm);
  const R inv = rrcp<R>(nrm < R(1e-6) ? R(1e-6) : nrm);
  return dbar * (gs[d] - gn[d] * inv * (dot * inv));
}

template <typename R, int TX, int TY>
struct ForceLds2 {
  static constexpr int HX = TX + 2, HY = TY + 2;
  R chi[HY][HX], sig[HY][HX], del[HY][HX];
};

// 2D: the face along d whose high-side cell is (lx, ly) in LDS coordinates
template <typename R, int TX, int TY>
__device__ __forceinline__ R force_face2(const ForceLds2<R, TX, TY>& L, const Par<R>& p,
                                         const int d, const int lx, const int ly) {
  const R ih = p.inv_h, iq = R(0.25) * p.inv_h;
  const int ax = lx - (d == 0), ay = ly - (d == 1);  // the low-side cell
  const int tx = d == 1, ty = d == 0;                // one step along the other axis
  R gn[2], gs[2];
  gn[d] = (L.chi[ly][lx] - L.chi[ay][ax]) * ih;
  gs[d] = (L.sig[ly][lx] - L.sig[ay][ax]) * ih;
  gn[1 - d] = ((L.chi[ay + ty][ax + tx] - L.chi[ay - ty][ax - tx]) +
               (L.chi[ly + ty][lx + tx] - L.chi[ly - ty][lx - tx])) * iq;
  gs[1 - d] = ((L.sig[ay + ty][ax + tx] - L.sig[ay - ty][ax - tx]) +
               (L.sig[ly + ty][lx + tx] - L.sig[ly - ty][lx - tx])) * iq;
  return force_finish<R>(gn, gs, 2, d, R(0.5) * (L.del[ay][ax] + L.del[ly][lx]));
}

template <typename R, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) k_force2(Grid g, Par<R> p, const R* __restrict__ chi,
                                                    const R* __restrict__ sig,
                                                    R* __restrict__ fx, R* __restrict__ fy,
                                                    int tiles_x) {
  using Lds = ForceLds2<R, TX, TY>;
  constexpr int NT = TX * TY, HX = Lds::HX, HY = Lds::HY;
  __shared__ Lds L;
  const int nx = g.n[0], ny = g.n[1];
  const int x0 = (blockIdx.x % tiles_x) * TX, y0 = (blockIdx.x / tiles_x) * TY;
  for (int l = threadIdx.x; l < HX * HY; l += NT) {
    const int lx = l % HX, ly = l / HX;
    const int gx = map_axis(x0 - 1 + lx, nx, g.bc[0][0], g.bc[0][1]);
    const int gy = map_axis(y0 - 1 + ly, ny, g.bc[1][0], g.bc[1][1]);
    const long long ci = (long long)gx + (long long)nx * gy;
    const R c = chi[ci];
    R ph, om, de;
    phase<R>(c, p, ph, om, de);
    L.chi[ly][lx] = c;
    L.sig[ly][lx] = sig[ci];
    L.del[ly][lx] = de;
  }
  __syncthreads();
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int cx = x0 + tx, cy = y0 + ty;
  if (cx >= nx || cy >= ny) return;
  const int lx = tx + 1, ly = ty + 1;
  // x faces: [ny][nx + 1]
  {
    const bool per = g.bc[0][0] == BC_PERIODIC;
    const long long row = (long long)cy * (nx + 1);
    fx[row + cx] = (cx == 0 && !per) ? R(0) : force_face2<R, TX, TY>(L, p, 0, lx, ly);
    if (cx == nx - 1) fx[row + nx] = per ? force_face2<R, TX, TY>(L, p, 0, lx + 1, ly) : R(0);
  }
  // y faces: [ny + 1][nx]
  {
    const bool per = g.bc[1][0] == BC_PERIODIC;
    fy[(long long)cy * nx + cx] = (cy == 0 && !per) ? R(0) : force_face2<R, TX, TY>(L, p, 1, lx, ly);
    if (cy == ny - 1)
      fy[(long long)ny * nx + cx] = per ? force_face2<R, TX, TY>(L, p, 1, lx, ly + 1) : R(0);
  }
}

template <typename R, int TX, int TY>
struct ForceLds3 {
  static constexpr int HX = TX + 2, HY = TY + 2;
  R chi[3][HY][HX], sig[3][HY][HX], del[3][HY][HX];
};

// 3D, a face in the plane (d = 0 or 1): its two cells in plane slot s0, the
// planes below and above in slots sm and sp; (lx, ly) is the high-side cell
template <typename R, int TX, int TY>
__device__ __forceinline__ R force_face3_xy(const ForceLds3<R, TX, TY>& L, const Par<R>& p,
                                            const int d, const int sm, const int s0,
                                            const int sp, const int lx, const int ly) {
  const R ih = p.inv_h, iq = R(0.25) * p.inv_h;
  const int ax = lx - (d == 0), ay = ly - (d == 1);
  const int tx = d == 1, ty = d == 0;
  R gn[3], gs[3];
  gn[d] = (L.chi[s0][ly][lx] - L.chi[s0][ay][ax]) * ih;
  gs[d] = (L.sig[s0][ly][lx] - L.sig[s0][ay][ax]) * ih;
  gn[1 - d] = ((L.chi[s0][ay + ty][ax + tx] - L.chi[s0][ay - ty][ax - tx]) +
               (L.chi[s0][ly + ty][lx + tx] - L.chi[s0][ly - ty][lx - tx])) * iq;
  gs[1 - d] = ((L.sig[s0][ay + ty][ax + tx] - L.sig[s0][ay - ty][ax - tx]) +
               (L.sig[s0][ly + ty][lx + tx] - L.sig[s0][ly - ty][lx - tx])) * iq;
  gn[2] = ((L.chi[sp][ay][ax] - L.chi[sm][ay][ax]) + (L.chi[sp][ly][lx] - L.chi[sm][ly][lx])) * iq;
  gs[2] = ((L.sig[sp][ay][ax] - L.sig[sm][ay][ax]) + (L.sig[sp][ly][lx] - L.sig[sm][ly][lx])) * iq;
  return force_finish<R>(gn, gs, 3, d, R(0.5) * (L.del[s0][ay][ax] + L.del[s0][ly][lx]));
}

// 3D, the face along z between the cell (lx, ly) of plane slot sl (low side)
// and of slot sh (high side)
template <typename R, int TX, int TY>
__device__ __forceinline__ R force_face3_z(const ForceLds3<R, TX, TY>& L, const Par<R>& p,
                                           const int sl, const int sh, const int lx,
                                           const int ly) {
  const R ih = p.inv_h, iq = R(0.25) * p.inv_h;
  R gn[3], gs[3];
  gn[2] = (L.chi[sh][ly][lx] - L.chi[sl][ly][lx]) * ih;
  gs[2] = (L.sig[sh][ly][lx] - L.sig[sl][ly][lx]) * ih;
  gn[0] = ((L.chi[sl][ly][lx + 1] - L.chi[sl][ly][lx - 1]) +
           (L.chi[sh][ly][lx + 1] - L.chi[sh][ly][lx - 1])) * iq;
  gs[0] = ((L.sig[sl][ly][lx + 1] - L.sig[sl][ly][lx - 1]) +
           (L.sig[sh][ly][lx + 1] - L.sig[sh][ly][lx - 1])) * iq;
  gn[1] = ((L.chi[sl][ly + 1][lx] - L.chi[sl][ly - 1][lx]) +
           (L.chi[sh][ly + 1][lx] - L.chi[sh][ly - 1][lx])) * iq;
  gs[1] = ((L.sig[sl][ly + 1][lx] - L.sig[sl][ly - 1][lx]) +
           (L.sig[sh][ly + 1][lx] - L.sig[sh][ly - 1][lx])) * iq;
  return force_finish<R>(gn, gs, 3, 2, R(0.5) * (L.del[sl][ly][lx] + L.del[sh][ly][lx]));
}

template <typename R, int TX, int TY, int ZC>
__global__ void __launch_bounds__(TX * TY) k_force3(Grid g, Par<R> p, const R* __restrict__ chi,
                                                    const R* __restrict__ sig,
                                                    R* __restrict__ fx, R* __restrict__ fy,
                                                    R* __restrict__ fz, int tiles_x,
                                                    int tiles_y) {
  using Lds = ForceLds3<R, TX, TY>;
  constexpr int NT = TX * TY, HX = Lds::HX, HY = Lds::HY;
  __shared__ Lds L;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int b = blockIdx.x;
  const int r = b / tiles_x;
  const int x0 = (b % tiles_x) * TX, y0 = (r % tiles_y) * TY, z0 = (r / tiles_y) * ZC;
  const int z1 = z0 + ZC < nz ? z0 + ZC : nz;
  // plane zq (mapped into the box) with its halo ring into slot s
  auto load = [&](int zq, int s) {
    const int gz = map_axis(zq, nz, g.bc[2][0], g.bc[2][1]);
    for (int l = threadIdx.x; l < HX * HY; l += NT) {
      const int lx = l % HX, ly = l / HX;
      const int gx = map_axis(x0 - 1 + lx, nx, g.bc[0][0], g.bc[0][1]);
      const int gy = map_axis(y0 - 1 + ly, ny, g.bc[1][0], g.bc[1][1]);
      const long long ci = (long long)gx + (long long)nx * (gy + (long long)ny * gz);
      const R c = chi[ci];
      R ph, om, de;
      phase<R>(c, p, ph, om, de);
      L.chi[s][ly][lx] = c;
      L.sig[s][ly][lx] = sig[ci];
      L.del[s][ly][lx] = de;
    }
  };
  load(z0 - 1, 0);
  load(z0, 1);
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int cx = x0 + tx, cy = y0 + ty;
  const bool in = cx < nx && cy < ny;
  const int lx = tx + 1, ly = ty + 1;
  const bool px = g.bc[0][0] == BC_PERIODIC, py = g.bc[1][0] == BC_PERIODIC,
             pz = g.bc[2][0] == BC_PERIODIC;
  for (int z = z0; z < z1; ++z) {
    const int k = z - z0;
    const int sm = k % 3, s0 = (k + 1) % 3, sp = (k + 2) % 3;
    load(z + 1, sp);
    __syncthreads();
    if (in) {
      const long long plane = (long long)z * ny;
      // x faces: [nz][ny][nx + 1]
      const long long rx = (plane + cy) * (nx + 1);
      fx[rx + cx] = (cx == 0 && !px) ? R(0) : force_face3_xy<R, TX, TY>(L, p, 0, sm, s0, sp, lx, ly);
      if (cx == nx - 1)
        fx[rx + nx] = px ? force_face3_xy<R, TX, TY>(L, p, 0, sm, s0, sp, lx + 1, ly) : R(0);
      // y faces: [nz][ny + 1][nx]
      const long long ry = (long long)z * (ny + 1);
      fy[(ry + cy) * nx + cx] =
          (cy == 0 && !py) ? R(0) : force_face3_xy<R, TX, TY>(L, p, 1, sm, s0, sp, lx, ly);
      if (cy == ny - 1)
        fy[(ry + ny) * nx + cx] = py ? force_face3_xy<R, TX, TY>(L, p, 1, sm, s0, sp, lx, ly + 1) : R(0);
      // z faces: [nz + 1][ny][nx]
      fz[(plane + cy) * nx + cx] = (z == 0 && !pz) ? R(0) : force_face3_z<R, TX, TY>(L, p, sm, s0, lx, ly);
      if (z == nz - 1)
        fz[((long long)nz * ny + cy) * nx + cx] = pz ? force_face3_z<R, TX, TY>(L, p, s0, sp, lx, ly) : R(0);
    }
    __syncthreads();  // the next plane goes into slot sm
  }
}

}  // namespace surf
