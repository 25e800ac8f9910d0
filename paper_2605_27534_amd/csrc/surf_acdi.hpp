// surf_acdi.hpp -- the phase field phi evolved by ACDI (section 2.5, the
// Phase-Field method) instead of a level set rebuilt from the VoF at every
// step.  The paper's ACDI equation, in this library's notation:
//
//   d phi/dt + div(u phi) = div( zeta [ eps grad phi
//                                       - 1/4 (1 - tanh^2(s/(2 eps))) grad s/|grad s| ] )
//   s = eps ln((phi + ve)/(1 - phi + ve))   (the paper's auxiliary field; psi here
//                                            is the interfacial carrier)
//
// One step takes the Lie split of the surfactant fields:
//   k_acdi_adv  phi* = the substep-1 advection of phi (BCG face values with
//               the minmod limiter, flux form), and s(phi*);
//   k_acdi_reg  phi = phi* + dt div G(phi*), with the face flux
//               G = zeta [eps (phi_R - phi_L)/h - 1/4 (1 - T^2) n_d],
//               T = tanh(s_f / (2 eps)), s_f the mean of s over the face's two
//               cells, n the unit face gradient of s (normal component
//               (s_R - s_L)/h, transverse components the mean of the two
//               cells' centred differences) with |grad s| bounded below by
//               1/2, no flux through walls and open sides; and the level set
//               the transport kernels read, chi = -s(phi), clamped to
//               |chi| <= chi_max.
// Since phi (1 - phi) grad s = eps grad phi, the flux is zeta eps grad phi
// (1 - 1/|grad s|): anti-diffusion where the profile is too wide.  In the
// tails s flattens and a unit normal would make that anti-diffusion
// unbounded; bounded below by 1/2, it is at most zeta eps |grad phi|, and
// every profile up to twice the equilibrium width keeps the unit normal.
// Each face flux is evaluated by both of its cells with the same arithmetic
// in the same order, so the update conserves sum(phi) exactly.  s is taken of
// phi clamped into [0, 1]; re-initialization from a VoF field (k_acdi_init)
// sets phi = 1/(1 + e^{chi/eps}) from the level set.  On axisymmetric rings
// (Appendix B) the fluxes are the same expressions in (r, z), and a radial
// face's flux enters ring i with the weight r_face / r_i (both substeps).
#pragma once
#include "surf_kernels.hpp"
#include "surf_col2d.hpp"  // mc()

namespace surf {

template <typename R>
struct AcdiArgs {
  Grid g;
  Par<R> p;
  R dt, cfl, zeta, ve;  // time step, dt/h, velocity scale, regularization of s
  long long ncell;
  int lim, tr;          // substep-1 variants: MC limiter, BCG transverse term
  int axi;              // axisymmetric rings: x is the radius, from r0
  double r0, h;
};

// the weights of ring x0's low and high radial faces, r_face / r_i (1, 1 on
// a Cartesian grid)
template <typename R>
__device__ __forceinline__ void acdi_ring_weights(const AcdiArgs<R>& a, int x0, R& wlo, R& whi) {
  wlo = R(1);
  whi = R(1);
  if (a.axi) {
    const double rl = a.r0 + (double)x0 * a.h, rm = rl + 0.5 * a.h;
    wlo = (R)(rl / rm);
    whi = (R)((rl + a.h) / rm);
  }
}

// The advective flux through the face along d on side sd (0 low, 1 high) of
// cell x with the substep-1 variants: the upwind cell's value and limited
// slope (v: phi at x[d]-2 .. x[d]+2), less dt/2h times its mean transverse
// velocity times its upwind transverse difference per transverse axis.
template <typename R, int DIM>
__device__ R acdi_flux_var(const AcdiArgs<R>& a, const R* __restrict__ phi,
                           const R* const* u, const int* x, int d, int sd, R uf, const R* v) {
  const Grid& g = a.g;
  const bool pos = uf > R(0);
  const int k0 = sd == 0 ? (pos ? 1 : 2) : (pos ? 2 : 3);  // the upwind cell in v
  const R xm = v[k0 - 1], xu = v[k0], xp = v[k0 + 1];
  const R k = R(0.5) * (R(1) - fabs(uf) * a.cfl);
  const R sl = a.lim ? mc<R>(xu - xm, xp - xu) : minmod<R>(xu - xm, xp - xu);
  R val = xu + (pos ? k : -k) * sl;
  if (a.tr) {
    int w[3] = {x[0], x[1], x[2]};
    w[d] = map_axis(x[d] + k0 - 2, g.n[d], g.bc[d][0], g.bc[d][1]);
#pragma unroll
    for (int t = 0; t < DIM; ++t) {
      if (t == d) continue;
      int hi[3] = {w[0], w[1], w[2]};
      hi[t] = (g.bc[t][0] == BC_PERIODIC && w[t] + 1 == g.n[t]) ? 0 : w[t] + 1;
      const R vt = R(0.5) * (u[t][face_index(g, t, w[0], w[1], w[2])] +
                             u[t][face_index(g, t, hi[0], hi[1], hi[2])]);
      int lo[3] = {w[0], w[1], w[2]}, up[3] = {w[0], w[1], w[2]};
      lo[t] = map_axis(w[t] - 1, g.n[t], g.bc[t][0], g.bc[t][1]);
      up[t] = map_axis(w[t] + 1, g.n[t], g.bc[t][0], g.bc[t][1]);
      const R xc = phi[cell_index(g, w[0], w[1], w[2])];
      const R dxt = vt > R(0) ? xc - phi[cell_index(g, lo[0], lo[1], lo[2])]
                              : phi[cell_index(g, up[0], up[1], up[2])] - xc;
      val -= R(0.5) * a.cfl * vt * dxt;
    }
  }
  return uf * val;
}

template <typename R>
__device__ __forceinline__ R acdi_s(R phi, R eps, R ve) {
  const R q = fmin(fmax(phi, R(0)), R(1));
  return eps * rlog<R>(rdiv<R>(q + ve, R(1) - q + ve));
}

// Launch shape of the per-cell ACDI kernels: each workgroup takes ACDI_TX
// cells of one row (y, z); the row and the offset in it come from the
// workgroup index by scalar arithmetic, so no thread divides.
constexpr int ACDI_TX = 256;

__host__ __device__ __forceinline__ int acdi_xblocks(int nx) { return (nx + ACDI_TX - 1) / ACDI_TX; }

// the cell of this thread; false past the end of its row
__device__ __forceinline__ bool acdi_cell(const Grid& g, int* x, long long& c) {
  const int xb = acdi_xblocks(g.n[0]);
  const int row = (int)blockIdx.x / xb;  // uniform: y + ny z
  x[0] = ((int)blockIdx.x - row * xb) * ACDI_TX + (int)threadIdx.x;
  x[1] = row % g.n[1];
  x[2] = row / g.n[1];
  c = (long long)row * g.n[0] + x[0];
  return x[0] < g.n[0];
}

// phi from the level set (initial state and re-initialization)
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_acdi_init(Grid g, Par<R> p, const R* __restrict__ chi,
                                                     R* __restrict__ phi, long long n) {
  const long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= n) return;
  R ph, om, de;
  phase<R>(chi[c], p, ph, om, de);
  phi[c] = ph;
}

// substep 1 for phi, and s of the result.  Every load (the 5-cell stencil
// along each axis, both face velocities) is issued up front from indices
// mapped into the grid; the boundary cases only select among the results.
template <typename R, int DIM, bool VAR = false>
__global__ void __launch_bounds__(ACDI_TX) k_acdi_adv(AcdiArgs<R> a, const R* __restrict__ phi,
                                                      const R* __restrict__ u0,
                                                      const R* __restrict__ u1,
                                                      const R* __restrict__ u2,
                                                      R* __restrict__ phs, R* __restrict__ s) {
  const Grid& g = a.g;
  int x[3];
  long long c;
  if (!acdi_cell(g, x, c)) return;
  const R pc = phi[c];
  R st = pc;
  if (u0) {
    const R* u[3] = {u0, u1, u2};
    R v[DIM][5], ul[DIM], uh[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int nd = g.n[d];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        int w[3] = {x[0], x[1], x[2]};
        w[d] = map_axis(x[d] + k - 2, nd, g.bc[d][0], g.bc[d][1]);
        v[d][k] = phi[cell_index(g, w[0], w[1], w[2])];
      }
      int y[3] = {x[0], x[1], x[2]};
      ul[d] = u[d][face_index(g, d, y[0], y[1], y[2])];
      const bool per = g.bc[d][0] == BC_PERIODIC;
      y[d] = (per && x[d] + 1 == nd) ? 0 : x[d] + 1;
      uh[d] = u[d][face_index(g, d, y[0], y[1], y[2])];
    }
    R wlo, whi;
    acdi_ring_weights(a, x[0], wlo, whi);
    R div = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const bool per = g.bc[d][0] == BC_PERIODIC;
      const bool blo = !per && x[d] == 0, bhi = !per && x[d] + 1 == g.n[d];
      R flo_i, fhi_i;
      if constexpr (VAR) {  // the substep-1 variants (a separate instantiation)
        flo_i = acdi_flux_var<R, DIM>(a, phi, u, x, d, 0, ul[d], v[d]);
        fhi_i = acdi_flux_var<R, DIM>(a, phi, u, x, d, 1, uh[d], v[d]);
      } else {
        flo_i = adv_flux<R>(ul[d], v[d][0], v[d][1], v[d][2], v[d][3], a.cfl);
        fhi_i = adv_flux<R>(uh[d], v[d][1], v[d][2], v[d][3], v[d][4], a.cfl);
      }
      const R flo = blo ? (g.bc[d][0] == BC_OPEN ? ul[d] * pc : R(0)) : flo_i;
      const R fhi = bhi ? (g.bc[d][1] == BC_OPEN ? uh[d] * pc : R(0)) : fhi_i;
      div += -((d == 0 ? wlo : R(1)) * flo);
      div += (d == 0 ? whi : R(1)) * fhi;
    }
    st = pc - a.cfl * div;
  }
  phs[c] = st;
  s[c] = acdi_s<R>(st, a.p.eps, a.ve);
}

// The regularization substep, then the level set of the new phi.  s on the
// 3^DIM block around the cell and phi* on the cell and its face neighbours
// are loaded up front (indices mapped into the grid); each face flux is then
// formed from registers.  A face's flux is computed by both of its cells from
// the same values in the same order.
template <typename R, int DIM>
__global__ void __launch_bounds__(ACDI_TX) k_acdi_reg(AcdiArgs<R> a, const R* __restrict__ phs,
                                                      const R* __restrict__ s,
                                                      R* __restrict__ phi_out,
                                                      R* __restrict__ chi_out) {
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  int x[3];
  long long c;
  if (!acdi_cell(g, x, c)) return;
  constexpr int NZ = DIM == 3 ? 3 : 1;
  int m[3][3];  // m[d][k]: the cell coordinate x[d] + k - 1, mapped
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      m[d][k] = d < DIM ? map_axis(x[d] + k - 1, g.n[d], g.bc[d][0], g.bc[d][1]) : x[d];
  R S[NZ][3][3];
#pragma unroll
  for (int kz = 0; kz < NZ; ++kz)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx)
        S[kz][ky][kx] = s[cell_index(g, m[0][kx], m[1][ky], DIM == 3 ? m[2][kz] : x[2])];
  R P[DIM][3];  // phi* at offsets -1, 0, +1 along each axis
  const R pc = phs[c];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int lo[3] = {x[0], x[1], x[2]}, hi[3] = {x[0], x[1], x[2]};
    lo[d] = m[d][0];
    hi[d] = m[d][2];
    P[d][0] = phs[cell_index(g, lo[0], lo[1], lo[2])];
    P[d][1] = pc;
    P[d][2] = phs[cell_index(g, hi[0], hi[1], hi[2])];
  }
  // s at the block offsets (k0, k1, k2) along axes 0, 1, 2 (each 0..2)
  auto sat = [&](int k0, int k1, int k2) { return S[DIM == 3 ? k2 : 0][k1][k0]; };
  R wlo, whi;
  acdi_ring_weights(a, x[0], wlo, whi);
  R acc = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const bool per = g.bc[d][0] == BC_PERIODIC;
    R G[2];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int kL = sd, kR = sd + 1;  // the face's cells along d
      int oL[3] = {1, 1, 1}, oR[3] = {1, 1, 1};
      oL[d] = kL;
      oR[d] = kR;
      const R sL = sat(oL[0], oL[1], oL[2]), sR = sat(oR[0], oR[1], oR[2]);
      const R gn = (sR - sL) * p.inv_h;
      R g2 = gn * gn;
#pragma unroll
      for (int t = 0; t < DIM; ++t) {
        if (t == d) continue;
        int lp[3] = {oL[0], oL[1], oL[2]}, lm[3] = {oL[0], oL[1], oL[2]};
        int rp[3] = {oR[0], oR[1], oR[2]}, rm[3] = {oR[0], oR[1], oR[2]};
        lp[t] = 2;
        lm[t] = 0;
        rp[t] = 2;
        rm[t] = 0;
        const R cdL = (sat(lp[0], lp[1], lp[2]) - sat(lm[0], lm[1], lm[2])) * (R(0.5) * p.inv_h);
        const R cdR = (sat(rp[0], rp[1], rp[2]) - sat(rm[0], rm[1], rm[2])) * (R(0.5) * p.inv_h);
        const R gt = R(0.5) * (cdL + cdR);
        g2 += gt * gt;
      }
      const R nd = rdiv<R>(gn, fmax(rsqrt_<R>(g2), R(0.5)));
      const R T = rtanh<R>(R(0.5) * (sL + sR) * (R(0.5) * p.inv_eps));
      const R f = a.zeta * (p.eps * (P[d][kR] - P[d][kL]) * p.inv_h - R(0.25) * (R(1) - T * T) * nd);
      const bool has = per || (sd == 0 ? x[d] > 0 : x[d] + 1 < g.n[d]);
      G[sd] = has ? f : R(0);
    }
    acc += d == 0 ? whi * G[1] - wlo * G[0] : G[1] - G[0];
  }
  const R phn = pc + a.cfl * acc;
  phi_out[c] = phn;
  const R chi = -acdi_s<R>(phn, a.p.eps, a.ve);
  chi_out[c] = fmin(fmax(chi, -a.p.chimax), a.p.chimax);
}

}  // namespace surf
