// surf_adjoint.hpp -- discrete adjoint of one step (weighted flux form) for
// gfx950, in gather form (no atomics): each cell collects the transposed
// contributions of the faces whose stencils reach it.
//
//   k_adv_star   recompute the advected state xi* = A(xi^n) (section 3.1)
//   k_adj_src    nu = J_R^T mu: transpose of substep 2 (confinement +
//                diffusion, sections 2.6, 3.2) and of the exchange source
//                (Appendix C), plus per-workgroup partials of dL/dtheta
//   k_adj_adv    lambda^n = J_A^T nu (+ the loss term of t^n): transpose of
//                the advection with the minmod branches frozen at xi^n
//   k_loss_seed  lambda^N from the loss term of the last step
//   k_loss_w     loss weights w_n and the loss from the forward totals
//   k_adj_c0     dL/dc0 = lambda_F^0 phi
#pragma once
#include "surf_kernels.hpp"

namespace surf {

constexpr int NADJ = 4;  // dL/d(k_a, k_d, D_b, D_s)

template <typename R>
struct AdjArgs {
  Grid g;
  Par<R> p;
  const R* chi;
  const R* u[3];
  const R* F;     // state at t^n
  const R* psi;
  const R* Fs;    // advected state xi*
  const R* Ps;
  const R* mF;    // lambda^{n+1}
  const R* mP;
  R* nF;          // nu = J_R^T lambda^{n+1}
  R* nP;
  R* lF;          // lambda^n
  R* lP;
  const double* w;  // loss weight of t^n or nullptr
  double* part;     // [nblk][NADJ]
  R dt;
  int has_u;
  long long ncell;
};

__device__ __forceinline__ void cell_coords(const Grid& g, long long c, int* x) {
  x[0] = (int)(c % g.n[0]);
  long long r = c / g.n[0];
  x[1] = (int)(r % g.n[1]);
  x[2] = (int)(r / g.n[1]);
}

template <typename R>
__device__ __forceinline__ long long nb_index(const Grid& g, const int* x, int d, int s) {
  int y[3] = {x[0], x[1], x[2]};
  y[d] = map_axis(x[d] + s, g.n[d], g.bc[d][0], g.bc[d][1]);
  return cell_index(g, y[0], y[1], y[2]);
}

// advective face value slope-limited as in the forward step, per cell
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_adv_star(AdjArgs<R> a) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= a.ncell) return;
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  int x[3];
  cell_coords(g, c, x);
  const R cfl = a.dt * p.inv_h;
  for (int f = 0; f < 2; ++f) {
    if (f == 0 && !p.bulk) continue;
    const R* xi = f == 0 ? a.F : a.psi;
    R div = R(0);
    for (int d = 0; d < g.dim; ++d) {
      const bool per = g.bc[d][0] == BC_PERIODIC;
      const int nd = g.n[d];
      // lo face (index x[d]) and hi face (index x[d] + 1)
      for (int s = 0; s < 2; ++s) {
        int fidx = x[d] + s;
        bool blo = !per && fidx == 0, bhi = !per && fidx == nd;
        int fw = (per && fidx == nd) ? 0 : fidx;
        int y[3] = {x[0], x[1], x[2]};
        y[d] = fw;
        R uf = a.u[d][face_index(g, d, y[0], y[1], y[2])];
        R fl;
        if (blo) {
          fl = g.bc[d][0] == BC_OPEN ? uf * xi[c] : R(0);
        } else if (bhi) {
          fl = g.bc[d][1] == BC_OPEN ? uf * xi[c] : R(0);
        } else {
          // cells L = fidx - 1 and R = fidx along d (mapped), and their outer neighbours
          int off = s == 0 ? -1 : 0;  // offset of L from this cell
          R xLm = xi[nb_index<R>(g, x, d, off - 1)], xL = xi[nb_index<R>(g, x, d, off)];
          R xR = xi[nb_index<R>(g, x, d, off + 1)], xRp = xi[nb_index<R>(g, x, d, off + 2)];
          fl = adv_flux<R>(uf, xLm, xL, xR, xRp, cfl);
        }
        div += s == 0 ? -fl : fl;
      }
    }
    R v = xi[c] - cfl * div;
    if (f == 0) ((R*)a.Fs)[c] = v; else ((R*)a.Ps)[c] = v;
  }
}

template <int NT>
__device__ __forceinline__ void block_sum4(double* v, double* out) {
  __shared__ double red[NT / 64][NADJ];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NADJ; ++s) {
    double x = wave_sum(v[s]);
    if (lane == 0) red[w][s] = x;
  }
  __syncthreads();
  if (threadIdx.x < NADJ) {
    double x = red[0][threadIdx.x];
    for (int q = 1; q < NT / 64; ++q) x += red[q][threadIdx.x];
    out[threadIdx.x] = x;
  }
}

// nu = mu + dt (L^T mu + dq/dxi* (mu_psi - mu_F)); the weighted operator is
// D M diag(1/w) with M the symmetric face-weighted graph Laplacian, so
// (L^T mu)_i = D sum_f wbar_f (mu_nb - mu_i) / (w_i h^2).
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_adj_src(AdjArgs<R> a) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  double acc[NADJ] = {0.0, 0.0, 0.0, 0.0};
  if (c < a.ncell) {
    const Grid& g = a.g;
    const Par<R>& p = a.p;
    int x[3];
    cell_coords(g, c, x);
    R ph, om, de;
    phase<R>(a.chi[c], p, ph, om, de);
    const R wF = ph + p.eta, wP = de + p.eta_eps;
    const R muF = a.mF[c], muP = a.mP[c];
    const R cF = p.bulk ? a.Fs[c] / wF : R(0), cP = a.Ps[c] / wP;
    R LtF = R(0), LtP = R(0), SF = R(0), SP = R(0);
    for (int d = 0; d < g.dim; ++d) {
      for (int s = -1; s <= 1; s += 2) {
        bool bnd = (s < 0 && x[d] == 0 && g.bc[d][0] != BC_PERIODIC) ||
                   (s > 0 && x[d] == g.n[d] - 1 && g.bc[d][1] != BC_PERIODIC);
        if (bnd) continue;
        long long o = nb_index<R>(g, x, d, s);
        R pho, omo, deo;
        phase<R>(a.chi[o], p, pho, omo, deo);
        R fbar = R(0.5) * (ph + pho), dbar = R(0.5) * (de + deo);
        if (p.bulk) {
          LtF += fbar * (a.mF[o] - muF);
          SF += fbar * (a.Fs[o] / (pho + p.eta) - cF);
        }
        LtP += dbar * (a.mP[o] - muP);
        SP += dbar * (a.Ps[o] / (deo + p.eta_eps) - cP);
      }
    }
    const R ih2 = p.inv_h * p.inv_h;
    LtF *= p.Db * ih2 / wF;
    LtP *= p.Ds * ih2 / wP;
    SF *= ih2;
    SP *= ih2;
    const R diff = muP - muF;
    R nuF = muF, nuP = muP + a.dt * LtP;
    if (p.bulk) {
      const R Psv = a.Ps[c];
      R dqdF, dqdP, dqdka;
      if (p.kin == KIN_LANGMUIR) {
        dqdF = p.ka * (p.ginf * de - Psv) / wF;
        dqdP = -p.ka * cF - p.kd;
        dqdka = cF * (p.ginf * de - Psv);
      } else {
        dqdF = p.ka * p.ginf * de / wF;
        dqdP = -p.kd;
        dqdka = cF * p.ginf * de;
      }
      nuF = muF + a.dt * (LtF + dqdF * diff);
      nuP += a.dt * dqdP * diff;
      acc[0] = (double)(a.dt * dqdka * diff);
      acc[1] = (double)(a.dt * (-Psv) * diff);
      acc[2] = (double)(a.dt * SF * muF);
    }
    acc[3] = (double)(a.dt * SP * muP);
    a.nF[c] = nuF;
    a.nP[c] = nuP;
  }
  block_sum4<BLOCK>(acc, a.part + (long long)blockIdx.x * NADJ);
}

// derivative of the equation of state
template <typename R>
__device__ __forceinline__ R eos_prime(R G, const Par<R>& p) {
  R x = G * p.inv_ginf;
  if (p.eos == EOS_LIN) return -p.sigma0 * p.E * p.inv_ginf;
  if (p.eos == EOS_LANG) {
    if (x <= R(0) || x >= R(1) - R(1e-6)) return R(0);
    return -p.sigma0 * p.E * p.inv_ginf / (R(1) - x);
  }
  R t = rtanh<R>(p.E * x);
  return -p.sigma0 * p.E * p.inv_ginf * (R(1) - t * t);
}

// lambda_j = nu_j + (dt/h) sum_f dflux_f/dxi_j (nu_R(f) - nu_L(f)), over the
// faces f whose (mirrored or wrapped) stencil holds j: along each axis the
// faces j-3/2 .. j+3/2
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_adj_adv(AdjArgs<R> a) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= a.ncell) return;
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  int x[3];
  cell_coords(g, c, x);
  R lamF = a.nF[c], lamP = a.nP[c];
  if (a.has_u) {
    const R cfl = a.dt * p.inv_h;
    for (int d = 0; d < g.dim; ++d) {
      const bool per = g.bc[d][0] == BC_PERIODIC;
      const int nd = g.n[d];
      for (int k = -1; k <= 2; ++k) {
        int fidx = x[d] + k;  // face between cells fidx-1 and fidx
        if (per) {
          fidx = ((fidx % nd) + nd) % nd;  // face nd is face 0
        } else if (fidx < 0 || fidx > nd) {
          continue;
        }
        int y[3] = {x[0], x[1], x[2]};
        y[d] = fidx;
        R uf = a.u[d][face_index(g, d, y[0], y[1], y[2])];
        bool blo = !per && fidx == 0, bhi = !per && fidx == nd;
        // the face's left/right cells relative to this cell: offsets k-1, k
        for (int f = 0; f < 2; ++f) {
          if (f == 0 && !p.bulk) continue;
          const R* xi = f == 0 ? a.F : a.psi;
          const R* nu = f == 0 ? a.nF : a.nP;
          R gsum = R(0);
          if (blo || bhi) {
            // open boundary: flux = u xi_interior, interior cell is this one only
            int bc = blo ? g.bc[d][0] : g.bc[d][1];
            if (bc == BC_OPEN && ((blo && x[d] == 0) || (bhi && x[d] == nd - 1))) {
              R gdiff = blo ? nu[c] : -nu[c];
              gsum = uf * gdiff;
            }
          } else {
            long long L = nb_index<R>(g, x, d, k - 1), Rr = nb_index<R>(g, x, d, k);
            bool pos = uf > R(0);
            // upwind cell b and its neighbours along d (mapped)
            int ob = pos ? k - 1 : k;
            long long ib = nb_index<R>(g, x, d, ob);
            int yb[3] = {x[0], x[1], x[2]};
            yb[d] = map_axis(x[d] + ob, nd, g.bc[d][0], g.bc[d][1]);
            long long im = nb_index<R>(g, yb, d, -1), iq = nb_index<R>(g, yb, d, +1);
            R s1 = xi[ib] - xi[im], s2 = xi[iq] - xi[ib];
            R sel1 = R(0), sel2 = R(0);
            bool same = (s1 > R(0) && s2 > R(0)) || (s1 < R(0) && s2 < R(0));
            if (same) {
              if (fabs(s1) < fabs(s2)) sel1 = R(1); else sel2 = R(1);
            }
            R kk = (pos ? R(1) : R(-1)) * R(0.5) * (R(1) - fabs(uf) * cfl);
            R wm = uf * (-kk * sel1), wb = uf * (R(1) + kk * sel1 - kk * sel2), wq = uf * kk * sel2;
            R w = R(0);
            if (im == c) w += wm;
            if (ib == c) w += wb;
            if (iq == c) w += wq;
            gsum = w * (nu[Rr] - nu[L]);
          }
          if (f == 0) lamF += cfl * gsum; else lamP += cfl * gsum;
        }
      }
    }
  }
  if (a.w) {
    R ph, om, de;
    phase<R>(a.chi[c], p, ph, om, de);
    R e = de + p.eta_eps;
    lamP += (R)(*a.w) * eos_prime<R>(a.psi[c] / e, p) * de / e;
  }
  a.lF[c] = p.bulk ? lamF : a.mF[c];
  a.lP[c] = lamP;
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_loss_seed(Grid g, Par<R> p, const R* __restrict__ chi,
                                                     const R* __restrict__ psi,
                                                     const double* __restrict__ w, R* lF, R* lP,
                                                     long long ncell) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= ncell) return;
  R ph, om, de;
  phase<R>(chi[c], p, ph, om, de);
  R e = de + p.eta_eps;
  if (lF) lF[c] = R(0);
  lP[c] = (R)(*w) * eos_prime<R>(psi[c] / e, p) * de / e;
}

// w_n = (2/N)(<sigma>^n - target^n) vol / sum(delta vol) for n = 1..N (row
// n-1 of the forward totals) and L = mean (<sigma>^n - target^n)^2
__global__ void k_loss_w(const double* __restrict__ tot, long long stride,
                         const double* __restrict__ target, int N, double vol,
                         double* __restrict__ w, double* __restrict__ loss) {
  __shared__ double part[BLOCK];
  double s = 0.0;
  for (int n = threadIdx.x; n < N; n += BLOCK) {
    const double* t = tot + (long long)n * stride;
    double r = t[13] - target[n];
    w[n] = 2.0 / N * r * vol / t[4];
    s += r * r;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int i = 0; i < BLOCK; ++i) acc += part[i];
    if (loss) *loss = acc / N;
  }
}

__global__ void k_adj_final(const double* __restrict__ part, int nblk, double* __restrict__ dtheta) {
  double v[NADJ] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += FIN_BLOCK)
    for (int s = 0; s < NADJ; ++s) v[s] += part[(long long)b * NADJ + s];
  __shared__ double tot[NADJ];
  block_sum4<FIN_BLOCK>(v, tot);
  __syncthreads();
  if (threadIdx.x < NADJ) dtheta[threadIdx.x] += tot[threadIdx.x];
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_adj_c0(Grid g, Par<R> p, const R* __restrict__ chi,
                                                  const R* __restrict__ lF, R* __restrict__ gc0,
                                                  long long ncell) {
  long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= ncell) return;
  R ph, om, de;
  phase<R>(chi[c], p, ph, om, de);
  gc0[c] = lF[c] * ph;
}

}  // namespace surf
