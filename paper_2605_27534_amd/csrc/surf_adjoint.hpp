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

// Launch shape of the three per-cell adjoint kernels: 32 x 8 cells of one
// plane per 256-thread workgroup (a wave holds two rows of 32), grid
// (ceil(nx/32), ceil(ny/8), nz), so that a cell's coordinates come from the
// workgroup and thread indices (no integer division); cell indices are
// 32-bit (grids under 2^31 cells).  The 32-wide rows keep the waves whose
// stencils reach an x side (and take the general path there) to the first
// and last tile of each row.
constexpr int ADJ_TX = 32, ADJ_TY = 8;

__device__ __forceinline__ bool adj_cell(const Grid& g, int* x) {
  x[0] = blockIdx.x * ADJ_TX + (int)(threadIdx.x % ADJ_TX);
  x[1] = blockIdx.y * ADJ_TY + (int)(threadIdx.x / ADJ_TX);
  x[2] = blockIdx.z;
  return x[0] < g.n[0] && x[1] < g.n[1];
}

// The advection adjoint's launch: the columns whose x stencils stay inside
// the box (3 <= x <= nx - 4) in 32 x 8 tiles, workgroups 0 .. adj_xtiles - 1
// along x, and the six x-side columns (all columns when nx < 7) of the same
// 8 rows in one more workgroup, so that the general (mapped) path along x
// runs only in the waves of that workgroup.
__host__ __device__ __forceinline__ int adj_xtiles(int nx) {
  return nx >= 7 ? (nx - 6 + ADJ_TX - 1) / ADJ_TX : 0;
}

__device__ __forceinline__ bool adj_cell_split(const Grid& g, int* x) {
  const int nx = g.n[0], ntx = adj_xtiles(nx);
  x[2] = blockIdx.z;
  if ((int)blockIdx.x < ntx) {
    x[0] = 3 + blockIdx.x * ADJ_TX + (int)(threadIdx.x % ADJ_TX);
    x[1] = blockIdx.y * ADJ_TY + (int)(threadIdx.x / ADJ_TX);
    return x[0] <= nx - 4 && x[1] < g.n[1];
  }
  const int ne = nx >= 7 ? 6 : nx;  // side columns
  const int e = (int)threadIdx.x % ne, r = (int)threadIdx.x / ne;
  x[0] = (nx >= 7 && e >= 3) ? nx - 6 + e : e;
  x[1] = blockIdx.y * ADJ_TY + r;
  return r < ADJ_TY && x[1] < g.n[1];
}

// stride of axis d in the cell layout
__device__ __forceinline__ int axis_stride(const Grid& g, int d) {
  return d == 0 ? 1 : (d == 1 ? g.n[0] : g.n[0] * g.n[1]);
}

// 32-bit face index along d (the d coordinate runs 0..n_d)
__device__ __forceinline__ int face_index32(const Grid& g, int d, const int* y) {
  const int mx = g.n[0] + (d == 0), my = g.n[1] + (d == 1);
  return y[0] + mx * (y[1] + my * y[2]);
}

// the advected state xi* = xi - dt/h sum_d (flux_hi - flux_lo), fluxes as in
// the forward step (BCG-minmod face values); per axis the five cells c-2 ..
// c+2 (mapped) are loaded once and serve both faces
template <typename R, int DIM, bool BULK>
__device__ __forceinline__ void adv_star_cell(const AdjArgs<R>& a, const int* x) {
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  const int c = x[0] + g.n[0] * (x[1] + g.n[1] * x[2]);
  const R cfl = a.dt * p.inv_h;
  R divF = R(0), divP = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const bool per = g.bc[d][0] == BC_PERIODIC;
    const int nd = g.n[d], st = axis_stride(g, d);
    // inside along d (2 <= x_d <= n_d - 3) the stencil needs no mapping and
    // neither face lies on a side
    const bool in = x[d] >= 2 && x[d] <= nd - 3;
    int idx[5];
    int ylo[3] = {x[0], x[1], x[2]};
    const int flo_i = face_index32(g, d, ylo);
    int fhi_i = flo_i + st;
    if (in) {
#pragma unroll
      for (int o = -2; o <= 2; ++o) idx[o + 2] = c + o * st;
    } else {
#pragma unroll
      for (int o = -2; o <= 2; ++o)
        idx[o + 2] = c + (map_axis(x[d] + o, nd, g.bc[d][0], g.bc[d][1]) - x[d]) * st;
      int yhi[3] = {x[0], x[1], x[2]};
      yhi[d] = (per && x[d] + 1 == nd) ? 0 : x[d] + 1;
      fhi_i = face_index32(g, d, yhi);
    }
    const R ulo = a.u[d][flo_i], uhi = a.u[d][fhi_i];
    const bool blo = !per && x[d] == 0, bhi = !per && x[d] == nd - 1;
#pragma unroll
    for (int f = BULK ? 0 : 1; f < 2; ++f) {
      const R* xi = f == 0 ? a.F : a.psi;
      const R v0 = xi[idx[0]], v1 = xi[idx[1]], v2 = xi[idx[2]], v3 = xi[idx[3]],
              v4 = xi[idx[4]];
      const R flo = blo ? (g.bc[d][0] == BC_OPEN ? ulo * v2 : R(0))
                        : adv_flux<R>(ulo, v0, v1, v2, v3, cfl);
      const R fhi = bhi ? (g.bc[d][1] == BC_OPEN ? uhi * v2 : R(0))
                        : adv_flux<R>(uhi, v1, v2, v3, v4, cfl);
      if (f == 0) {
        divF += -flo;
        divF += fhi;
      } else {
        divP += -flo;
        divP += fhi;
      }
    }
  }
  if (BULK) ((R*)a.Fs)[c] = a.F[c] - cfl * divF;
  ((R*)a.Ps)[c] = a.psi[c] - cfl * divP;
}

template <typename R, int DIM, bool BULK>
__global__ void __launch_bounds__(ADJ_TX * ADJ_TY) k_adv_star(AdjArgs<R> a) {
  int x[3];
  if (adj_cell(a.g, x)) adv_star_cell<R, DIM, BULK>(a, x);
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
// (L^T mu)_i = D sum_f wbar_f (mu_nb - mu_i) / (w_i h^2).  The divisions by
// the weights are multiplications by their reciprocals, as in the forward
// step.
template <typename R, int DIM, bool BULK>
__device__ __forceinline__ void adj_src_cell(const AdjArgs<R>& a, const int* x, double* acc) {
  {
    const Grid& g = a.g;
    const Par<R>& p = a.p;
    const int c = x[0] + g.n[0] * (x[1] + g.n[1] * x[2]);
    R ph, om, de;
    phase<R>(a.chi[c], p, ph, om, de);
    const R wF = ph + p.eta, wP = de + p.eta_eps;
    const R iwF = rrcp<R>(wF), iwP = rrcp<R>(wP);
    const R muF = a.mF[c], muP = a.mP[c];
    const R cF = BULK ? a.Fs[c] * iwF : R(0), cP = a.Ps[c] * iwP;
    R LtF = R(0), LtP = R(0), SF = R(0), SP = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int st = axis_stride(g, d);
#pragma unroll
      for (int s = -1; s <= 1; s += 2) {
        bool bnd = (s < 0 && x[d] == 0 && g.bc[d][0] != BC_PERIODIC) ||
                   (s > 0 && x[d] == g.n[d] - 1 && g.bc[d][1] != BC_PERIODIC);
        if (bnd) continue;
        const int o = c + (map_axis(x[d] + s, g.n[d], g.bc[d][0], g.bc[d][1]) - x[d]) * st;
        R pho, omo, deo;
        phase<R>(a.chi[o], p, pho, omo, deo);
        R fbar = R(0.5) * (ph + pho), dbar = R(0.5) * (de + deo);
        if (BULK) {
          LtF += fbar * (a.mF[o] - muF);
          SF += fbar * (a.Fs[o] * rrcp<R>(pho + p.eta) - cF);
        }
        LtP += dbar * (a.mP[o] - muP);
        SP += dbar * (a.Ps[o] * rrcp<R>(deo + p.eta_eps) - cP);
      }
    }
    const R ih2 = p.inv_h * p.inv_h;
    LtF *= p.Db * ih2 * iwF;
    LtP *= p.Ds * ih2 * iwP;
    SF *= ih2;
    SP *= ih2;
    const R diff = muP - muF;
    R nuF = muF, nuP = muP + a.dt * LtP;
    if (BULK) {
      const R Psv = a.Ps[c];
      R dqdF, dqdP, dqdka;
      if (p.kin == KIN_LANGMUIR) {
        dqdF = p.ka * (p.ginf * de - Psv) * iwF;
        dqdP = -p.ka * cF - p.kd;
        dqdka = cF * (p.ginf * de - Psv);
      } else {
        dqdF = p.ka * p.ginf * de * iwF;
        dqdP = -p.kd;
        dqdka = cF * p.ginf * de;
      }
      nuF = muF + a.dt * (LtF + dqdF * diff);
      nuP += a.dt * dqdP * diff;
      acc[0] += (double)(a.dt * dqdka * diff);
      acc[1] += (double)(a.dt * (-Psv) * diff);
      acc[2] += (double)(a.dt * SF * muF);
    }
    acc[3] += (double)(a.dt * SP * muP);
    a.nF[c] = nuF;
    a.nP[c] = nuP;
  }
}

template <typename R, int DIM, bool BULK>
__global__ void __launch_bounds__(ADJ_TX * ADJ_TY) k_adj_src(AdjArgs<R> a) {
  double acc[NADJ] = {0.0, 0.0, 0.0, 0.0};
  int x[3];
  if (adj_cell(a.g, x)) adj_src_cell<R, DIM, BULK>(a, x, acc);
  const int blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  block_sum4<ADJ_TX * ADJ_TY>(acc, a.part + (long long)blk * NADJ);
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
// faces j-1/2 .. j+5/2 (face k lies between cells j+k-1 and j+k), whose
// stencils reach the cells j-3 .. j+3; per axis those cells' xi (7), their
// nu (5 of them) and the four face velocities are loaded once
// The same sum along axis d for a cell whose stencils along d stay inside
// the box (3 <= x_d <= n_d - 4): no mapped or boundary faces, and each face
// reaches the cell in one role.  Face k (between offsets k-1 and k) has the
// upwind cell b at k-1 (u > 0) or k and the stencil b-1, b, b+1; the cell is
// q of face -1 (u < 0), q or b of face 0, b or m of face 1 and m of face 2
// (u > 0).  The arithmetic of each weight, its sum from zero and the order
// of the terms are those of the general path, bit for bit.
template <typename R, bool BULK>
__device__ __forceinline__ void adj_adv_interior(const AdjArgs<R>& a, int c, int st, int d,
                                                 const int* x, R cfl, R& lamF, R& lamP) {
  int fy[3] = {x[0], x[1], x[2]};
  fy[d] = x[d] - 1;
  const int fb = face_index32(a.g, d, fy);  // face -1; faces step by st along d
  R uf[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) uf[k] = a.u[d][fb + k * st];
#pragma unroll
  for (int f = BULK ? 0 : 1; f < 2; ++f) {
    const R* xi = f == 0 ? a.F : a.psi;
    const R* nu = f == 0 ? a.nF : a.nP;
    R v[7], w5[5];
#pragma unroll
    for (int o = 0; o < 7; ++o) v[o] = xi[c + (o - 3) * st];
#pragma unroll
    for (int o = 0; o < 5; ++o) w5[o] = nu[c + (o - 2) * st];
    R lam = f == 0 ? lamF : lamP;
#pragma unroll
    for (int k = -1; k <= 2; ++k) {
      const R u = uf[k + 1];
      const bool pos = u > R(0);
      const int ob = pos ? k - 1 : k;
      // v[ob + 2 .. ob + 4] with ob in {k - 1, k}
      const R xm = pos ? v[k + 1] : v[k + 2], xb = pos ? v[k + 2] : v[k + 3],
              xq = pos ? v[k + 3] : v[k + 4];
      (void)ob;
      const R s1 = xb - xm, s2 = xq - xb;
      R sel1 = R(0), sel2 = R(0);
      const bool same = (s1 > R(0) && s2 > R(0)) || (s1 < R(0) && s2 < R(0));
      if (same) {
        if (fabs(s1) < fabs(s2)) sel1 = R(1); else sel2 = R(1);
      }
      const R kk = (pos ? R(1) : R(-1)) * R(0.5) * (R(1) - fabs(u) * cfl);
      const R wm = u * (-kk * sel1), wb = u * (R(1) + kk * sel1 - kk * sel2),
              wq = u * kk * sel2;
      R w;
      if (k == -1) w = pos ? R(0) : R(0) + wq;
      else if (k == 0) w = R(0) + (pos ? wq : wb);
      else if (k == 1) w = R(0) + (pos ? wb : wm);
      else w = pos ? R(0) + wm : R(0);
      const R gsum = w * (w5[k + 2] - w5[k + 1]);
      lam += cfl * gsum;
    }
    if (f == 0) lamF = lam; else lamP = lam;
  }
}

template <typename R, int DIM, bool BULK, bool HU>
__device__ __forceinline__ void adj_adv_cell(const AdjArgs<R>& a, const int* x) {
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  const int c = x[0] + g.n[0] * (x[1] + g.n[1] * x[2]);
  R lamF = a.nF[c], lamP = a.nP[c];
  if (HU) {
    const R cfl = a.dt * p.inv_h;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const bool per = g.bc[d][0] == BC_PERIODIC;
      const int nd = g.n[d], st = axis_stride(g, d);
      if (x[d] >= 3 && x[d] <= nd - 4) {
        adj_adv_interior<R, BULK>(a, c, st, d, x, cfl, lamF, lamP);
        continue;
      }
      // mapped neighbours along d at offsets -3 .. 3: index and whether it is
      // this cell (a mirrored stencil can reach it twice)
      int idx[7];
      bool me[7];
#pragma unroll
      for (int o = -3; o <= 3; ++o) {
        const int m = map_axis(x[d] + o, nd, g.bc[d][0], g.bc[d][1]);
        idx[o + 3] = c + (m - x[d]) * st;
        me[o + 3] = m == x[d];
      }
      R uf[4];
      bool skip[4], blo[4], bhi[4];
#pragma unroll
      for (int k = -1; k <= 2; ++k) {
        int fidx = x[d] + k;  // face between cells fidx-1 and fidx
        skip[k + 1] = false;
        if (per) {
          fidx = fidx < 0 ? fidx + nd : (fidx >= nd ? fidx - nd : fidx);  // face nd is face 0
        } else if (fidx < 0 || fidx > nd) {
          skip[k + 1] = true;
          fidx = 0;
        }
        int y[3] = {x[0], x[1], x[2]};
        y[d] = fidx;
        uf[k + 1] = a.u[d][face_index32(g, d, y)];
        blo[k + 1] = !per && fidx == 0;
        bhi[k + 1] = !per && fidx == nd;
      }
#pragma unroll
      for (int f = BULK ? 0 : 1; f < 2; ++f) {
        const R* xi = f == 0 ? a.F : a.psi;
        const R* nu = f == 0 ? a.nF : a.nP;
        R v[7], w5[5];
#pragma unroll
        for (int o = 0; o < 7; ++o) v[o] = xi[idx[o]];
#pragma unroll
        for (int o = 0; o < 5; ++o) w5[o] = nu[idx[o + 1]];  // offsets -2 .. 2
#pragma unroll
        for (int k = -1; k <= 2; ++k) {
          if (skip[k + 1]) continue;
          const R u = uf[k + 1];
          R gsum = R(0);
          if (blo[k + 1] || bhi[k + 1]) {
            // open boundary: flux = u xi_interior, the interior cell only
            const int bc = blo[k + 1] ? g.bc[d][0] : g.bc[d][1];
            if (bc == BC_OPEN && ((blo[k + 1] && x[d] == 0) || (bhi[k + 1] && x[d] == nd - 1))) {
              const R gdiff = blo[k + 1] ? nu[c] : -nu[c];
              gsum = u * gdiff;
            }
          } else {
            // L at offset k-1, R at k; the upwind cell b and its neighbours
            const bool pos = u > R(0);
            const int ob = pos ? k - 1 : k;
            const R xb = v[ob + 3], xm = v[ob + 2], xq = v[ob + 4];
            const R s1 = xb - xm, s2 = xq - xb;
            R sel1 = R(0), sel2 = R(0);
            const bool same = (s1 > R(0) && s2 > R(0)) || (s1 < R(0) && s2 < R(0));
            if (same) {
              if (fabs(s1) < fabs(s2)) sel1 = R(1); else sel2 = R(1);
            }
            const R kk = (pos ? R(1) : R(-1)) * R(0.5) * (R(1) - fabs(u) * cfl);
            const R wm = u * (-kk * sel1), wb = u * (R(1) + kk * sel1 - kk * sel2),
                    wq = u * kk * sel2;
            R w = R(0);
            if (me[ob + 2]) w += wm;
            if (me[ob + 3]) w += wb;
            if (me[ob + 4]) w += wq;
            gsum = w * (w5[k + 2] - w5[k + 1]);
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
  a.lF[c] = BULK ? lamF : a.mF[c];
  a.lP[c] = lamP;
}

template <typename R, int DIM, bool BULK, bool HU>
__global__ void __launch_bounds__(ADJ_TX * ADJ_TY) k_adj_adv(AdjArgs<R> a) {
  int x[3];
  if (adj_cell_split(a.g, x)) adj_adv_cell<R, DIM, BULK, HU>(a, x);
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
#pragma unroll 8
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
