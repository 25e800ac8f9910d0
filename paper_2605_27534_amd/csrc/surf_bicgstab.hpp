// surf_bicgstab.hpp -- implicit substep 2 in the paper's own flux form
// (sections 2.6, 3.2, Appendix A for the flux; Appendix C for the implicit
// step).
//
// In the paper form the unknowns are F and psi themselves, and the flux
// through a face is D (xi_R - xi_L)/h + Bbar xi_up: centred diffusion plus
// the anti-diffusive transport at velocity -B, Bbar the mean over the face's
// two cells of B_F = -D_b (1 - phi) n_d / eps (bulk) or B_psi = -D_s (1 - 2
// phi) n_d / eps (carrier), n = -grad chi / |grad chi| from centred
// differences (|grad chi| at least 1e-6), xi_up the cell upwind of -Bbar
// (the low cell when Bbar < 0).  No flux through walls and open sides.
// Minus the divergence of that flux is a matrix P that the upwind term makes
// non-symmetric, so each problem of the Picard sweeps of Appendix C,
//
//   interface:  [ 1/dt + kl k_a c + k_d + P_s ] psi = psi*/dt + k_a c Gamma_inf delta
//   bulk:       [ 1/dt + k_a (Gamma_inf delta - kl psi)/(phi + eta) + P_b ] F
//                   = F*/dt + k_d psi
//
// (c = F/(phi + eta) at its latest value), is solved by BiCGSTAB (van der
// Vorst, SIAM J. Sci. Stat. Comput. 13, 1992) with the Jacobi diagonal M as
// preconditioner, in FP64, matrix-free:
//
//   r = b - A x, rh = r, p = v = 0
//   iteration: rho = (rh, r), beta = (rho/rho_prev)(alpha/omega) (0 first),
//              p = r + beta (p - omega v), y = M^-1 p, v = A y,
//              alpha = rho / (rh, v), s = r - alpha v, z = M^-1 s, t = A z,
//              omega = (t, s)/(t, t), x += alpha y + omega z, r = s - omega t
//
// in three launches per iteration, each a persistent grid of at most
// BICG_MAXWG workgroups striding over the cells, each leaving per-workgroup
// partial sums that every workgroup of the next launch reduces in the same
// order (so all of them get the same scalars, with no device-wide atomic):
//   k_bicg_a  tests ||M^-1 r|| <= tol ||x|| and rho from the last launch's
//             sums, forms p (at the cell and, from their r, p and v, at its
//             neighbours) and v = A M^-1 p; sums (rh, v);
//   k_bicg_b  alpha; s and t = A M^-1 s the same way; sums (t, s), (t, t);
//   k_bicg_c  omega; x and r; sums (rh, r), ||M^-1 r||^2, ||x||^2.
// p and v are read at the neighbours while they are rewritten, so each has
// two buffers, by iteration parity; the partial sums take three slots, one
// per launch of an iteration.  After the test is met (or on a breakdown:
// rho, (rh, v) or (t, t) zero or not finite) every later launch of the
// solve returns at once.
//   k_bicg_coef  B_d of every cell for the solve's field;
//   k_bicg_setup reaction diagonal, M^-1, r = b - A x0, rh, p = v = 0;
//   k_bicg_end   the iteration count, and the status bit when the solve
//                neither met its test nor stopped on it.
#pragma once
#include "surf_implicit.hpp"

namespace surf {

constexpr int BICG_WG = 256, BICG_MAXWG = 512;
// scalars after the CG's: rho, alpha, omega by iteration parity
enum { BS_RHO = 8, BS_ALPHA = 10, BS_OMEGA = 12 };
static_assert(BS_OMEGA + 2 <= SC_N, "BiCGSTAB scalars fit the scalar block");
enum { BP_A = 0, BP_B = 1, BP_C = 2 };  // partial-sum slots, by launch

struct BicgArgs {
  Grid g;
  double k;          // D / h^2
  double inv_h;
  double tol2;
  double* x;         // the unknown (F or psi)
  double* p[2];      // by iteration parity
  double* v[2];
  double* r;
  double* rh;
  double* t;
  double* minv;
  double* dg;
  const double* B[3];  // B_d per cell
  double* part;      // [3][BICG_MAXWG][4]
  double* sc;
  int nwg;
  long long ncell;
  int axi;           // axisymmetric rings: radial faces weighted r_face / r_i
  double r0, h;      // rings: the radius of the low x side, the cell size
};

// rings (Appendix B): the weight of cell x's radial face on side s in its
// balance, r_face / r_i
__device__ __forceinline__ double bicg_ring_w(const BicgArgs& a, int i, int s) {
  const double rl = a.r0 + (double)i * a.h, rm = rl + 0.5 * a.h;
  return (s > 0 ? rl + a.h : rl) / rm;
}

// coordinates of cell c (32-bit: the implicit path keeps ncell < 2^31)
__device__ __forceinline__ void bicg_coords(const Grid& g, int c, int* x) {
  x[0] = c % g.n[0];
  const int r = c / g.n[0];
  x[1] = r % g.n[1];
  x[2] = r / g.n[1];
}

// the neighbour of cell c (coordinates x) at offset s = +-1 along d, or -1
// when the face between them is a wall or an open side
__device__ __forceinline__ int bicg_nb(const Grid& g, int c, const int* x, int d, int s) {
  const int stride = d == 0 ? 1 : (d == 1 ? g.n[0] : g.n[0] * g.n[1]);
  const int q = x[d] + s;
  if (q >= 0 && q < g.n[d]) return c + s * stride;
  if (g.bc[d][0] != BC_PERIODIC) return -1;
  return c + (q < 0 ? (g.n[d] - 1) : -(g.n[d] - 1)) * stride;
}

// (A y)_c for y given at the cell (yc) and by a callable at any other cell:
// dg yc plus, per face, k (yc - y_nb) and the upwind term, minus Bbar/h
// y_up on the high face and plus on the low face; on rings a radial face's
// terms take the cell's weight r_face / r_i
template <int DIM, typename Y>
__device__ __forceinline__ double bicg_apply(const BicgArgs& a, int c, const int* x, double yc,
                                             Y&& y) {
  double Ay = a.dg[c] * yc;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double Bc = a.B[d][c];
#pragma unroll
    for (int s = -1; s <= 1; s += 2) {
      const int nb = bicg_nb(a.g, c, x, d, s);
      if (nb < 0) continue;
      const double yn = y(nb);
      const double bf = 0.5 * (Bc + a.B[d][nb]) * a.inv_h;
      if (d == 0 && a.axi) {  // a radial face of a ring: the flux weighted
        const double t = s > 0 ? a.k * (yc - yn) - bf * (bf < 0.0 ? yc : yn)
                               : a.k * (yc - yn) + bf * (bf < 0.0 ? yn : yc);
        Ay += bicg_ring_w(a, x[0], s) * t;
        continue;
      }
      Ay += a.k * (yc - yn);
      if (s > 0) Ay -= bf * (bf < 0.0 ? yc : yn);  // c is the low cell
      else Ay += bf * (bf < 0.0 ? yn : yc);        // c is the high cell
    }
  }
  return Ay;
}

// the sums of the previous launch (slot), reduced by every workgroup in the
// same order
__device__ __forceinline__ void bicg_reduce(const BicgArgs& a, int slot, double* out) {
  const double* P = a.part + (size_t)slot * BICG_MAXWG * CT_N;
  double v[CT_N] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < a.nwg; b += BICG_WG)
    for (int k = 0; k < CT_N; ++k) v[k] += P[b * CT_N + k];
  __shared__ double tot[CT_N];
  block_sums<BICG_WG>(v, CT_N, tot);
  __syncthreads();
  for (int k = 0; k < CT_N; ++k) out[k] = tot[k];
  __syncthreads();  // tot is reused by the next reduction
}

__device__ __forceinline__ void bicg_leave(const BicgArgs& a, int slot, double* acc) {
  __shared__ double out[CT_N];
  block_sums<BICG_WG>(acc, CT_N, out);
  if (threadIdx.x < CT_N)
    a.part[(size_t)slot * BICG_MAXWG * CT_N + (size_t)blockIdx.x * CT_N + threadIdx.x] =
        out[threadIdx.x];
}

__device__ __forceinline__ void bicg_stop(const BicgArgs& a, int it, bool fail) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.sc[SC_DONE] = 1.0;
    a.sc[SC_ITER] = (double)it;
    a.sc[SC_FAIL] = fail ? 1.0 : 0.0;
  }
}

// B_d = -D w n_d / eps of every cell (w = 1 - phi for the bulk, 1 - 2 phi for
// the carrier), n = -grad chi / max(|grad chi|, 1e-6) from centred
// differences with mirrored or wrapped neighbours
template <typename R>
__global__ void __launch_bounds__(BICG_WG) k_bicg_coef(ImpArgs<R> a, const R* __restrict__ chi,
                                                       int field, double* B0, double* B1,
                                                       double* B2) {
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  double* B[3] = {B0, B1, B2};
  const double D = field == 1 ? a.Db : a.Ds;
  for (long long c = (long long)blockIdx.x * BICG_WG + threadIdx.x; c < a.ncell;
       c += (long long)gridDim.x * BICG_WG) {
    int x[3];
    bicg_coords(g, (int)c, x);
    double gr[3] = {0.0, 0.0, 0.0}, nrm = 0.0;
    for (int e = 0; e < g.dim; ++e) {
      int lo[3] = {x[0], x[1], x[2]}, hi[3] = {x[0], x[1], x[2]};
      lo[e] = map_axis(x[e] - 1, g.n[e], g.bc[e][0], g.bc[e][1]);
      hi[e] = map_axis(x[e] + 1, g.n[e], g.bc[e][0], g.bc[e][1]);
      gr[e] = ((double)chi[cell_index(g, hi[0], hi[1], hi[2])] -
               (double)chi[cell_index(g, lo[0], lo[1], lo[2])]) / (2.0 * a.h);
      nrm += gr[e] * gr[e];
    }
    nrm = fmax(sqrt(nrm), 1e-6);
    R ph, om, de;
    phase<R>(chi[c], p, ph, om, de);
    const double w = field == 1 ? (double)om : (double)om - (double)ph;
    for (int d = 0; d < g.dim; ++d) B[d][c] = -D * w / (double)p.eps * (-gr[d] / nrm);
  }
}

// the reaction diagonal, right-hand side, inverse Jacobi diagonal, r = b - A
// x0, rh = r, p = v = 0 (parity 0); sums (rh, r), ||M^-1 r||^2, ||x||^2
template <typename R, int DIM>
__global__ void __launch_bounds__(BICG_WG) k_bicg_setup(ImpArgs<R> ia, BicgArgs a, int field) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.sc[SC_DONE] = 0.0;
    a.sc[SC_ITER] = 0.0;
    a.sc[SC_FAIL] = 0.0;
  }
  const ImpBuf& Bf = ia.B;
  double acc[CT_N] = {0.0, 0.0, 0.0, 0.0};
  for (long long cl = (long long)blockIdx.x * BICG_WG + threadIdx.x; cl < a.ncell;
       cl += (long long)gridDim.x * BICG_WG) {
    const int c = (int)cl;
    int x[3];
    bicg_coords(a.g, c, x);
    const double dF = Bf.wF[c] + ia.eta;
    double dg, rhs;
    if (field == 0) {
      const double cF = ia.bulk ? Bf.xF[c] / dF : 0.0;
      dg = 1.0 / ia.dt + ia.kl * ia.ka * cF + ia.kd;
      rhs = Bf.Ps[c] / ia.dt + ia.ka * cF * ia.ginf * Bf.wP[c];
    } else {
      dg = 1.0 / ia.dt + ia.ka * (ia.ginf * Bf.wP[c] - ia.kl * Bf.xP[c]) / dF;
      rhs = Bf.Fs[c] / ia.dt + ia.kd * Bf.xP[c];
    }
    a.dg[c] = dg;
    // the diagonal of A: dg, k per face, |Bbar|/h per face whose upwind
    // cell is this one
    double m = dg;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int s = -1; s <= 1; s += 2) {
        const int nb = bicg_nb(a.g, c, x, d, s);
        if (nb < 0) continue;
        const double bf = 0.5 * (a.B[d][c] + a.B[d][nb]) * a.inv_h;
        if (d == 0 && a.axi) {
          double t = a.k;
          if (s > 0 && bf < 0.0) t -= bf;
          if (s < 0 && !(bf < 0.0)) t += bf;
          m += bicg_ring_w(a, x[0], s) * t;
          continue;
        }
        m += a.k;
        if (s > 0 && bf < 0.0) m -= bf;
        if (s < 0 && !(bf < 0.0)) m += bf;
      }
    const double mi = 1.0 / m;
    a.minv[c] = mi;
    const double xc = a.x[c];
    const double Ax = bicg_apply<DIM>(a, c, x, xc, [&](int n) { return a.x[n]; });
    const double r = rhs - Ax;
    a.r[c] = r;
    a.rh[c] = r;
    a.p[0][c] = 0.0;
    a.v[0][c] = 0.0;
    acc[0] += r * r;
    acc[1] += (mi * r) * (mi * r);
    acc[2] += xc * xc;
  }
  bicg_leave(a, BP_C, acc);
}

// launch A of iteration it: the stop test, rho, p, v = A M^-1 p
template <int DIM>
__global__ void __launch_bounds__(BICG_WG) k_bicg_a(BicgArgs a, int it) {
  if (a.sc[SC_DONE] != 0.0) return;  // uniform over the grid
  double tot[CT_N];
  bicg_reduce(a, BP_C, tot);
  const double rho = tot[0];
  if (tot[1] <= a.tol2 * tot[2]) {
    bicg_stop(a, it, false);
    return;
  }
  const int par = it & 1;
  double beta = 0.0, om = 0.0;
  if (it > 0) {
    const double rp = a.sc[BS_RHO + (par ^ 1)], al = a.sc[BS_ALPHA + (par ^ 1)];
    om = a.sc[BS_OMEGA + (par ^ 1)];
    beta = (rho / rp) * (al / om);
  }
  if (!(rho != 0.0) || !isfinite(rho) || !isfinite(beta)) {
    bicg_stop(a, it, true);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.sc[BS_RHO + par] = rho;
  const double* __restrict__ pin = a.p[par];
  const double* __restrict__ vin = a.v[par];
  double* __restrict__ pout = a.p[par ^ 1];
  double* __restrict__ vout = a.v[par ^ 1];
  // y = M^-1 p at any cell, from its r, p and v
  auto y = [&](int n) { return a.minv[n] * (a.r[n] + beta * (pin[n] - om * vin[n])); };
  double acc[CT_N] = {0.0, 0.0, 0.0, 0.0};
  for (long long cl = (long long)blockIdx.x * BICG_WG + threadIdx.x; cl < a.ncell;
       cl += (long long)gridDim.x * BICG_WG) {
    const int c = (int)cl;
    int x[3];
    bicg_coords(a.g, c, x);
    const double pc = a.r[c] + beta * (pin[c] - om * vin[c]);
    const double v = bicg_apply<DIM>(a, c, x, a.minv[c] * pc, y);
    pout[c] = pc;
    vout[c] = v;
    acc[0] += a.rh[c] * v;
  }
  bicg_leave(a, BP_A, acc);
}

// launch B: alpha, t = A M^-1 s with s = r - alpha v
template <int DIM>
__global__ void __launch_bounds__(BICG_WG) k_bicg_b(BicgArgs a, int it) {
  if (a.sc[SC_DONE] != 0.0) return;
  double tot[CT_N];
  bicg_reduce(a, BP_A, tot);
  const int par = it & 1;
  const double rho = a.sc[BS_RHO + par];
  const double alpha = rho / tot[0];
  if (!(tot[0] != 0.0) || !isfinite(alpha)) {
    bicg_stop(a, it, true);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.sc[BS_ALPHA + par] = alpha;
  const double* __restrict__ v = a.v[par ^ 1];
  auto z = [&](int n) { return a.minv[n] * (a.r[n] - alpha * v[n]); };
  double acc[CT_N] = {0.0, 0.0, 0.0, 0.0};
  for (long long cl = (long long)blockIdx.x * BICG_WG + threadIdx.x; cl < a.ncell;
       cl += (long long)gridDim.x * BICG_WG) {
    const int c = (int)cl;
    int x[3];
    bicg_coords(a.g, c, x);
    const double s = a.r[c] - alpha * v[c];
    const double t = bicg_apply<DIM>(a, c, x, a.minv[c] * s, z);
    a.t[c] = t;
    acc[0] += t * s;
    acc[1] += t * t;
  }
  bicg_leave(a, BP_B, acc);
}

// launch C: omega, x += alpha y + omega z, r = s - omega t
__global__ void __launch_bounds__(BICG_WG) k_bicg_c(BicgArgs a, int it) {
  if (a.sc[SC_DONE] != 0.0) return;
  double tot[CT_N];
  bicg_reduce(a, BP_B, tot);
  const int par = it & 1;
  const double omega = tot[0] / tot[1];
  if (!(tot[1] != 0.0) || !(omega != 0.0) || !isfinite(omega)) {
    bicg_stop(a, it, true);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.sc[BS_OMEGA + par] = omega;
  const double alpha = a.sc[BS_ALPHA + par];
  const double* __restrict__ p = a.p[par ^ 1];
  const double* __restrict__ v = a.v[par ^ 1];
  double acc[CT_N] = {0.0, 0.0, 0.0, 0.0};
  for (long long cl = (long long)blockIdx.x * BICG_WG + threadIdx.x; cl < a.ncell;
       cl += (long long)gridDim.x * BICG_WG) {
    const int c = (int)cl;
    const double mi = a.minv[c];
    const double s = a.r[c] - alpha * v[c];
    const double xn = a.x[c] + alpha * (mi * p[c]) + omega * (mi * s);
    const double rn = s - omega * a.t[c];
    a.x[c] = xn;
    a.r[c] = rn;
    acc[0] += a.rh[c] * rn;
    acc[1] += (mi * rn) * (mi * rn);
    acc[2] += xn * xn;
  }
  bicg_leave(a, BP_C, acc);
}

// after the solve's last launch: its iteration count into rec; the status
// bit when it neither met the test nor stopped on it
__global__ void __launch_bounds__(BICG_WG) k_bicg_end(BicgArgs a, int iters, double* rec,
                                                      double* state) {
  double tot[CT_N];
  bicg_reduce(a, BP_C, tot);
  if (threadIdx.x != 0) return;
  bool ok;
  if (a.sc[SC_DONE] != 0.0) {
    *rec = a.sc[SC_ITER];
    ok = a.sc[SC_FAIL] == 0.0;
  } else {
    *rec = (double)iters;
    ok = tot[1] <= a.tol2 * tot[2];
  }
  if (!ok) atomicOr((unsigned*)(state + S_FLAGS), (unsigned)STATUS_SOLVE);
}

}  // namespace surf
