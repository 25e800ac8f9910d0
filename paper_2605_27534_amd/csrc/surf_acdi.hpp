// surf_acdi.hpp -- the phase field phi evolved by ACDI (section 2.5, the
// Phase-Field method) instead of a level set rebuilt from the VoF at every
// step.  The paper's ACDI equation, in the build's notation:
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
// sets phi = 1/(1 + e^{chi/eps}) from the level set.
#pragma once
#include "surf_kernels.hpp"

namespace surf {

template <typename R>
struct AcdiArgs {
  Grid g;
  Par<R> p;
  R dt, cfl, zeta, ve;  // time step, dt/h, velocity scale, regularization of s
  long long ncell;
};

template <typename R>
__device__ __forceinline__ R acdi_s(R phi, R eps, R ve) {
  const R q = fmin(fmax(phi, R(0)), R(1));
  return eps * rlog<R>(rdiv<R>(q + ve, R(1) - q + ve));
}

template <typename R>
__device__ __forceinline__ void acdi_coords(const Grid& g, long long c, int* x) {
  x[0] = (int)(c % g.n[0]);
  x[1] = (int)((c / g.n[0]) % g.n[1]);
  x[2] = (int)(c / ((long long)g.n[0] * g.n[1]));
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

// substep 1 for phi, and s of the result
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_acdi_adv(AcdiArgs<R> a, const R* __restrict__ phi,
                                                    const R* __restrict__ u0,
                                                    const R* __restrict__ u1,
                                                    const R* __restrict__ u2,
                                                    R* __restrict__ phs, R* __restrict__ s) {
  const long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= a.ncell) return;
  const Grid& g = a.g;
  R st = phi[c];
  if (u0) {
    const R* u[3] = {u0, u1, u2};
    int x[3];
    acdi_coords<R>(g, c, x);
    R div = R(0);
    for (int d = 0; d < g.dim; ++d) {
      const bool per = g.bc[d][0] == BC_PERIODIC;
      const int nd = g.n[d];
      for (int sd = 0; sd < 2; ++sd) {
        const int fidx = x[d] + sd;
        const bool blo = !per && fidx == 0, bhi = !per && fidx == nd;
        int y[3] = {x[0], x[1], x[2]};
        y[d] = (per && fidx == nd) ? 0 : fidx;
        const R uf = u[d][face_index(g, d, y[0], y[1], y[2])];
        R fl;
        if (blo) {
          fl = g.bc[d][0] == BC_OPEN ? uf * phi[c] : R(0);
        } else if (bhi) {
          fl = g.bc[d][1] == BC_OPEN ? uf * phi[c] : R(0);
        } else {
          const int off = sd == 0 ? -1 : 0;
          auto at = [&](int o) {
            int w[3] = {x[0], x[1], x[2]};
            w[d] = map_axis(x[d] + o, nd, g.bc[d][0], g.bc[d][1]);
            return phi[cell_index(g, w[0], w[1], w[2])];
          };
          fl = adv_flux<R>(uf, at(off - 1), at(off), at(off + 1), at(off + 2), a.cfl);
        }
        div += sd == 0 ? -fl : fl;
      }
    }
    st = phi[c] - a.cfl * div;
  }
  phs[c] = st;
  s[c] = acdi_s<R>(st, a.p.eps, a.ve);
}

// G through the face between cell xl and its neighbour along +d (wrapped on
// a periodic axis); the caller checks that the face carries flux
template <typename R>
__device__ __forceinline__ R acdi_face(const AcdiArgs<R>& a, const R* __restrict__ phs,
                                       const R* __restrict__ s, const int* xl, int d) {
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  int xr[3] = {xl[0], xl[1], xl[2]};
  xr[d] = xl[d] + 1 == g.n[d] ? 0 : xl[d] + 1;
  const long long L = cell_index(g, xl[0], xl[1], xl[2]);
  const long long Rc = cell_index(g, xr[0], xr[1], xr[2]);
  const R sL = s[L], sR = s[Rc];
  const R gn = (sR - sL) * p.inv_h;
  R g2 = gn * gn;
  for (int t = 0; t < g.dim; ++t) {
    if (t == d) continue;
    R cd[2];
    for (int k = 0; k < 2; ++k) {
      const int* q = k == 0 ? xl : xr;
      int hi[3] = {q[0], q[1], q[2]}, lo[3] = {q[0], q[1], q[2]};
      hi[t] = map_axis(q[t] + 1, g.n[t], g.bc[t][0], g.bc[t][1]);
      lo[t] = map_axis(q[t] - 1, g.n[t], g.bc[t][0], g.bc[t][1]);
      cd[k] = (s[cell_index(g, hi[0], hi[1], hi[2])] - s[cell_index(g, lo[0], lo[1], lo[2])]) *
              (R(0.5) * p.inv_h);
    }
    const R gt = R(0.5) * (cd[0] + cd[1]);
    g2 += gt * gt;
  }
  const R nd = rdiv<R>(gn, fmax(rsqrt_<R>(g2), R(0.5)));
  const R T = rtanh<R>(R(0.5) * (sL + sR) * (R(0.5) * p.inv_eps));
  return a.zeta * (p.eps * (phs[Rc] - phs[L]) * p.inv_h - R(0.25) * (R(1) - T * T) * nd);
}

// the regularization substep, then the level set of the new phi
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_acdi_reg(AcdiArgs<R> a, const R* __restrict__ phs,
                                                    const R* __restrict__ s,
                                                    R* __restrict__ phi_out,
                                                    R* __restrict__ chi_out) {
  const long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= a.ncell) return;
  const Grid& g = a.g;
  int x[3];
  acdi_coords<R>(g, c, x);
  R acc = R(0);
  for (int d = 0; d < g.dim; ++d) {
    const bool per = g.bc[d][0] == BC_PERIODIC;
    R Ghi = R(0), Glo = R(0);
    if (per || x[d] + 1 < g.n[d]) Ghi = acdi_face<R>(a, phs, s, x, d);
    if (per || x[d] > 0) {
      int xl[3] = {x[0], x[1], x[2]};
      xl[d] = x[d] > 0 ? x[d] - 1 : g.n[d] - 1;
      Glo = acdi_face<R>(a, phs, s, xl, d);
    }
    acc += Ghi - Glo;
  }
  const R phn = phs[c] + a.cfl * acc;
  phi_out[c] = phn;
  const R chi = -acdi_s<R>(phn, a.p.eps, a.ve);
  chi_out[c] = fmin(fmax(chi, -a.p.chimax), a.p.chimax);
}

}  // namespace surf
