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
// Each matrix is symmetric positive definite; each problem is solved by
// Jacobi-preconditioned conjugate gradients in FP64, matrix-free, one cell
// per thread:
//   k_imp_adv    substep 1 into FP64 arrays, phi and delta, the starting
//                iterates, and per-block records of the open-side outflow
//                and the largest cell-mean velocity sum;
//   k_cg_init    reaction diagonal, right-hand side, r = b - A x, z = M^-1 r,
//                p = z, partial sums of r.z, z.z and x.x;
//   k_cg_apply   p <- z + beta p and q = A p in one pass (p ping-pongs
//                between two buffers so that neighbours read the old p),
//                partial sums of p.q;
//   k_cg_update  x += alpha p, r -= alpha q, z = M^-1 r, partial sums of r.z,
//                z.z and x.x;
//   k_cg_scal    one workgroup: the scalars alpha, beta and the convergence
//                flag, after which every later kernel of that solve returns
//                at once.
//
// The solve ends when ||M^-1 r|| <= tol ||x|| (M the Jacobi diagonal).  The
// diagonal spans many orders of magnitude (delta + eta/eps and phi + eta
// vanish away from the interface and the liquid), so a test on ||r|| would
// leave the cells with a small diagonal unconverged; both matrices are
// strictly diagonally dominant, and then M^-1 r bounds the error cell by cell
// (|e| <= |M^-1 r| / (1 - rho), rho < 1 the largest off-diagonal row sum
// over the diagonal).
//   k_imp_final  F, psi, sigma and the step's reduction records.
#pragma once
#include "surf_kernels.hpp"

namespace surf {

constexpr int IMP_BLOCK = 256;
constexpr int IMP_FIELDS = 13;  // FP64 cell arrays of ImpBuf
constexpr int CG_SCAL_THREADS = 1024;
enum { CG_RZ = 0, CG_ZZ, CG_XX, CG_PQ };                            // partial-sum slots
enum { SC_RZ = 0, SC_ZZ, SC_XX, SC_ALPHA, SC_BETA, SC_DONE, SC_ITERS, SC_N = 8 };

// FP64 arrays of the implicit path (one value per cell) and its records
struct ImpBuf {
  double *Fs, *Ps;          // advected state
  double *wF, *wP;          // phi and delta: face weights and carrier denominators
  double *xF, *xP;          // c and Gamma: Picard iterates and solutions
  double *dg, *minv;        // reaction diagonal, inverse Jacobi diagonal
  double *r, *z, *p[2], *q;
  double* adv;              // [nblk][2]: outflow, largest velocity sum
  double* cgp;              // [nblk][4]: CG partial sums
  double* sc;               // [SC_N]: CG scalars
};

template <typename R>
struct ImpArgs {
  Grid g;
  Par<R> p;
  ImpBuf B;
  double dt, eta, eta_eps, ka, kd, ginf, kl, tol;  // FP64 coefficients
  double inv_h2, Db, Ds;
  int bulk;
  long long ncell;
};

__device__ __forceinline__ void imp_coords(const Grid& g, long long c, int* x) {
  x[0] = (int)(c % g.n[0]);
  x[1] = (int)((c / g.n[0]) % g.n[1]);
  x[2] = (int)(c / ((long long)g.n[0] * g.n[1]));
}

// The neighbour across the face on side s (-1 lo, +1 hi) along d, or -1 when
// the face is a wall or open side (no diffusive flux).
__device__ __forceinline__ long long imp_nbr(const Grid& g, const int* x, int d, int s) {
  const bool per = g.bc[d][0] == BC_PERIODIC;
  int v = x[d] + s;
  if (v < 0 || v >= g.n[d]) {
    if (!per) return -1;
    v = v < 0 ? v + g.n[d] : v - g.n[d];
  }
  int y[3] = {x[0], x[1], x[2]};
  y[d] = v;
  return cell_index(g, y[0], y[1], y[2]);
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
            if (blo) {
              fl = g.bc[d][0] == BC_OPEN ? uf * xi[c] : R(0);
              out -= (double)(area_dt * fl);
            } else if (bhi) {
              fl = g.bc[d][1] == BC_OPEN ? uf * xi[c] : R(0);
              out += (double)(area_dt * fl);
            } else {
              const int off = s == 0 ? -1 : 0;
              auto at = [&](int o) {
                int w[3] = {x[0], x[1], x[2]};
                w[d] = map_axis(x[d] + o, nd, g.bc[d][0], g.bc[d][1]);
                return xi[cell_index(g, w[0], w[1], w[2])];
              };
              fl = adv_flux<R>(uf, at(off - 1), at(off), at(off + 1), at(off + 2), cfl);
            }
            div += s == 0 ? -fl : fl;
          }
        }
        st[f] = xi[c] - cfl * div;
      }
      // cell-mean velocity sum (the literal upper face on a periodic axis)
      R s = R(0);
      for (int d = 0; d < g.dim; ++d) {
        int y[3] = {x[0], x[1], x[2]};
        const R ulo = u[d][face_index(g, d, y[0], y[1], y[2])];
        y[d] += 1;
        const R uhi = u[d][face_index(g, d, y[0], y[1], y[2])];
        s += fabs(R(0.5) * (ulo + uhi));
      }
      usum = (double)s;
    }
    const double w0 = (double)ph, w1 = (double)de;
    a.B.wF[c] = w0;
    a.B.wP[c] = w1;
    a.B.Fs[c] = (double)st[0];
    a.B.Ps[c] = (double)st[1];
    a.B.xF[c] = a.bulk ? (double)st[0] / (w0 + a.eta) : 0.0;
    a.B.xP[c] = (double)st[1] / (w1 + a.eta_eps);
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
// the field's face weight, diffusivity and unknown
struct ImpField {
  const double* w;
  double D;
  double* x;
};

template <typename R>
__device__ __forceinline__ ImpField imp_field(const ImpArgs<R>& a, int field) {
  if (field == 0) return ImpField{a.B.wP, a.Ds, a.B.xP};
  return ImpField{a.B.wF, a.Db, a.B.xF};
}

// field 0: the interfacial problem, 1: the bulk problem
template <typename R>
__global__ void __launch_bounds__(IMP_BLOCK) k_cg_init(ImpArgs<R> a, int field) {
  const long long c = (long long)blockIdx.x * IMP_BLOCK + threadIdx.x;
  const Grid& g = a.g;
  const ImpField fd = imp_field(a, field);
  double v[3] = {0.0, 0.0, 0.0};
  if (c < a.ncell) {
    const ImpBuf& B = a.B;
    const double inv_h2 = a.inv_h2;
    double dg, rhs;
    if (field == 0) {
      const double dP = B.wP[c] + a.eta_eps, cF = a.bulk ? B.xF[c] : 0.0;
      dg = dP * (1.0 / a.dt + a.kl * a.ka * cF + a.kd);
      rhs = B.Ps[c] / a.dt + a.ka * cF * a.ginf * B.wP[c];
    } else {
      const double dF = B.wF[c] + a.eta, ps = (B.wP[c] + a.eta_eps) * B.xP[c];
      dg = dF / a.dt + a.ka * (a.ginf * B.wP[c] - a.kl * ps);
      rhs = B.Fs[c] / a.dt + a.kd * ps;
    }
    int x[3];
    imp_coords(g, c, x);
    const double xc = fd.x[c], wc = fd.w[c];
    double ax = dg * xc, m = dg;
    for (int d = 0; d < g.dim; ++d)
      for (int s = -1; s <= 1; s += 2) {
        const long long nb = imp_nbr(g, x, d, s);
        if (nb < 0) continue;
        const double k = fd.D * 0.5 * (wc + fd.w[nb]) * inv_h2;
        ax += k * (xc - fd.x[nb]);
        m += k;
      }
    const double r = rhs - ax, mi = 1.0 / m, z = r * mi;
    B.dg[c] = dg;
    B.minv[c] = mi;
    B.r[c] = r;
    B.z[c] = z;
    B.p[0][c] = z;
    v[CG_RZ] = r * z;
    v[CG_ZZ] = z * z;
    v[CG_XX] = xc * xc;
  }
  __shared__ double out[4];
  block_sums<IMP_BLOCK>(v, 3, out);
  if (threadIdx.x < 3) a.B.cgp[4 * blockIdx.x + threadIdx.x] = out[threadIdx.x];
}

// mode 0: after init; 1: after apply (alpha); 2: after update (beta, test)
__global__ void __launch_bounds__(CG_SCAL_THREADS) k_cg_scal(double* __restrict__ sc,
                                                            const double* __restrict__ cgp,
                                                            int nblk, int mode, double tol) {
  if (mode != 0 && sc[SC_DONE] != 0.0) return;  // uniform
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += CG_SCAL_THREADS) {
    if (mode == 1) {
      v[0] += cgp[4 * b + CG_PQ];
    } else {
      v[0] += cgp[4 * b + CG_RZ];
      v[1] += cgp[4 * b + CG_ZZ];
      v[2] += cgp[4 * b + CG_XX];
    }
  }
  __shared__ double tot[4];
  block_sums<CG_SCAL_THREADS>(v, 3, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double tol2 = tol * tol;
  if (mode == 0) {
    sc[SC_RZ] = tot[0];
    sc[SC_ZZ] = tot[1];
    sc[SC_XX] = tot[2];
    sc[SC_BETA] = 0.0;
    sc[SC_ALPHA] = 0.0;
    sc[SC_ITERS] = 0.0;
    sc[SC_DONE] = (tot[1] <= tol2 * tot[2]) ? 1.0 : 0.0;
  } else if (mode == 1) {
    if (tot[0] > 0.0) {
      sc[SC_ALPHA] = sc[SC_RZ] / tot[0];
    } else {
      sc[SC_DONE] = 1.0;  // p = 0: nothing left to reduce
    }
  } else {
    sc[SC_BETA] = sc[SC_RZ] != 0.0 ? tot[0] / sc[SC_RZ] : 0.0;
    sc[SC_RZ] = tot[0];
    sc[SC_ZZ] = tot[1];
    sc[SC_XX] = tot[2];
    sc[SC_ITERS] += 1.0;
    if (tot[1] <= tol2 * tot[2]) sc[SC_DONE] = 1.0;
  }
}

template <typename R>
__global__ void __launch_bounds__(IMP_BLOCK) k_cg_apply(ImpArgs<R> a, int field, int pin) {
  if (a.B.sc[SC_DONE] != 0.0) return;  // uniform over the grid
  const long long c = (long long)blockIdx.x * IMP_BLOCK + threadIdx.x;
  const Grid& g = a.g;
  const ImpField fd = imp_field(a, field);
  const ImpBuf& B = a.B;
  const double* po = B.p[pin];
  double* pn = B.p[pin ^ 1];
  const double beta = B.sc[SC_BETA];
  double v[1] = {0.0};
  if (c < a.ncell) {
    const double inv_h2 = a.inv_h2;
    int x[3];
    imp_coords(g, c, x);
    const double pc = B.z[c] + beta * po[c], wc = fd.w[c];
    double q = B.dg[c] * pc;
    for (int d = 0; d < g.dim; ++d)
      for (int s = -1; s <= 1; s += 2) {
        const long long nb = imp_nbr(g, x, d, s);
        if (nb < 0) continue;
        const double k = fd.D * 0.5 * (wc + fd.w[nb]) * inv_h2;
        q += k * (pc - (B.z[nb] + beta * po[nb]));
      }
    pn[c] = pc;
    B.q[c] = q;
    v[0] = pc * q;
  }
  __shared__ double out[4];
  block_sums<IMP_BLOCK>(v, 1, out);
  if (threadIdx.x == 0) B.cgp[4 * blockIdx.x + CG_PQ] = out[0];
}

template <typename R>
__global__ void __launch_bounds__(IMP_BLOCK) k_cg_update(ImpArgs<R> a, int field, int pcur) {
  if (a.B.sc[SC_DONE] != 0.0) return;  // uniform over the grid
  const long long c = (long long)blockIdx.x * IMP_BLOCK + threadIdx.x;
  const ImpField fd = imp_field(a, field);
  const ImpBuf& B = a.B;
  const double alpha = B.sc[SC_ALPHA];
  double v[3] = {0.0, 0.0, 0.0};
  if (c < a.ncell) {
    const double x = fd.x[c] + alpha * B.p[pcur][c];
    const double r = B.r[c] - alpha * B.q[c];
    const double z = r * B.minv[c];
    fd.x[c] = x;
    B.r[c] = r;
    B.z[c] = z;
    v[CG_RZ] = r * z;
    v[CG_ZZ] = z * z;
    v[CG_XX] = x * x;
  }
  __shared__ double out[4];
  block_sums<IMP_BLOCK>(v, 3, out);
  if (threadIdx.x < 3) B.cgp[4 * blockIdx.x + threadIdx.x] = out[threadIdx.x];
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
    const R Fn = a.bulk ? (R)((B.wF[c] + a.eta) * B.xF[c]) : R(0);
    const R Pn = (R)((B.wP[c] + a.eta_eps) * B.xP[c]);
    const R sg = eos<R>(rdiv<R>(Pn, de + p.eta_eps), p);
    if (a.bulk) Fo[c] = Fn;
    Po[c] = Pn;
    if (sig) sig[c] = sg;
    v[P_SUM_F] = (double)Fn;
    v[P_SUM_PSI] = (double)Pn;
    v[P_SUM_DELTA] = (double)de;
    v[P_SUM_SIGDELTA] = (double)(sg * de);
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
