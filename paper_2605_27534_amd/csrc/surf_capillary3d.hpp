// surf_capillary3d.hpp -- the interfacial forces for the coupling to a flow
// solver (section 2.4) in 3D: the capillary force sigma kappa delta_s n and
// the Marangoni force delta_m grad_s sigma with delta_m = A_f / V_c, on the
// faces of the velocity grid.  The rules are those of the 2D kernel
// (surf_capillary.hpp), carried to 3D:
//   * a cell is interfacial when 1e-6 < c < 1 - 1e-6;
//   * the Youngs normal m = -grad c from the 3x3x3 stencil (along each axis
//     the difference of the two neighbouring planes, each summed over its
//     3x3 cells with the weights (1, 2, 1) x (1, 2, 1));
//   * kappa by height functions (Cummins, Francois and Kothe 2005): along an
//     axis a, the fluid-1 heights H(p, q) of the nine columns of nine cells
//     through the cell and its neighbours in the other two axes b < c, and
//     kappa = (H_bb (1 + H_c^2) + H_cc (1 + H_b^2) - 2 H_bc H_b H_c)
//             / (1 + H_b^2 + H_c^2)^(3/2)
//     (centred differences; H_bb, H_cc over h, H_bc over 4h).  The axes are
//     tried in the order of m's components, largest first (ties to the
//     higher axis), zero ones skipped; the first whose columns all close
//     (end cells full on the fluid-1 side and empty on the other) gives
//     kappa.  Where none closes the cell takes the mean of the height
//     curvatures of the interfacial cells of its 3x3x3 block (in the order
//     dz, dy, dx from -1 to 1), or where there is none the level set's
//     curvature moved to the interface, kappa / (1 - chi kappa / 2);
//   * delta_m = A_f / h: the plane m.x = alpha leaving the fraction c of the
//     unit cube on its side m.x <= alpha, A_f its area inside the cube.  With
//     the axes reflected so that n = |m| / |m|_1 >= 0 and k the axis of n's
//     largest component, the plane is z_k = (alpha - L)/n_k over the unit
//     square of the other two axes, L = n_i x_i + n_j x_j.  With G(t) the
//     area of {L <= t} in the square (piecewise quadratic in t) and I(t) its
//     integral from 0 (piecewise cubic), the volume below the plane is
//     (I(alpha) - I(alpha - n_k)) / n_k and A_f = (G(alpha) - G(alpha - n_k))
//     |n| / n_k: no division by a small component (n_k >= 1/3, and the
//     pieces of G and I that divide by n_i or n_j are taken only on their
//     own intervals).  alpha by Newton's method on that volume inside a
//     shrinking bracket, bisecting when a step leaves it.
// On a face kappa is the mean over its interfacial cells, delta_m and sigma
// the means of both; grad_s sigma is the face gradient of sigma (compact
// normal difference, the two cells' centred transverse differences averaged)
// minus its part along the same face gradient of chi.  Faces on walls and
// open sides carry no force; on a periodic axis the last face repeats the
// first.  The geometry runs in FP64 in both precisions.
//
// Two launches.  k_iface3_cells takes a 64 x 4 x 2 tile per workgroup, lists
// the tile's interfacial cells in LDS and gives them to its first threads (a
// sphere's surface leaves a few dozen per tile, so the heavy work packs into
// one wave instead of one per row of the tile); it writes each listed cell's
// height curvature (NaN where no axis closes) and delta_m into two scratch
// cell arrays, and nothing for the other cells.  k_iface3_faces, one thread
// per cell, writes the cell's low face along each axis (and the last cell
// its high face), reading the scratch arrays only at interfacial cells and
// filling in the curvature of a cell without heights from the first array,
// which no thread writes.  A face with neither cell interfacial has both
// forces zero and reads nothing past the two fractions.
#pragma once
#include "surf_capillary.hpp"

namespace surf {

constexpr int IF3_HL = 4;  // height columns reach IF3_HL cells each side

template <typename R>
struct Iface3Args {
  Grid g;
  const R* vof;
  const R* chi;
  const R* sig;
  R* kh;     // height curvature per cell
  R* dm;     // delta_m per cell
  double h;
};

__device__ __forceinline__ bool if3_cut(double c) { return c > IFACE_CUT && c < 1.0 - IFACE_CUT; }

template <typename R>
__device__ __forceinline__ double if3_at(const R* a, const Grid& g, int x, int y, int z) {
  const int i = map_axis(x, g.n[0], g.bc[0][0], g.bc[0][1]);
  const int j = map_axis(y, g.n[1], g.bc[1][0], g.bc[1][1]);
  const int k = map_axis(z, g.n[2], g.bc[2][0], g.bc[2][1]);
  return (double)a[cell_index(g, i, j, k)];
}

// ---- PLIC area in the unit cube
// G(t) = area of {a x + b y <= t} in the unit square and I(t) = its integral
// over [0, t], for 0 <= a <= b: with s = a + b, G is t^2 / (2ab) on [0, a],
// (t - a/2) / b on [a, b] and symmetric about (s/2, 1/2) (the square's
// centre), so I(t) = t - s/2 + I(s - t) past s/2.
__device__ __forceinline__ double plic_G(double a, double b, double t) {
  const double s = a + b;
  if (t <= 0.0) return 0.0;
  if (t >= s) return 1.0;
  const bool flip = t > 0.5 * s;
  const double u = flip ? s - t : t;  // in (0, s/2], so u <= b
  const double g = u <= a ? u * u / (2.0 * a * b) : (u - 0.5 * a) / b;
  return flip ? 1.0 - g : g;
}

__device__ __forceinline__ double plic_I(double a, double b, double t) {
  const double s = a + b;
  if (t <= 0.0) return 0.0;
  if (t >= s) return t - 0.5 * s;
  const bool flip = t > 0.5 * s;
  const double u = flip ? s - t : t;
  const double v =
      u <= a ? u * u * u / (6.0 * a * b) : a * a / (6.0 * b) + (u * u - a * u) / (2.0 * b);
  return flip ? t - 0.5 * s + v : v;
}

__device__ double plic_area3(double m0, double m1, double m2, double c) {
  if (!if3_cut(c)) return 0.0;
  double n[3] = {fabs(m0), fabs(m1), fabs(m2)};
  const double s = n[0] + n[1] + n[2];
  if (!(s > 0.0)) return 0.0;
  n[0] /= s;
  n[1] /= s;
  n[2] /= s;
  int k = 2;
  if (n[1] > n[k]) k = 1;
  if (n[0] > n[k]) k = 0;
  const double nk = n[k], p = n[k == 0 ? 1 : 0], q = n[k == 2 ? 1 : 2];
  const double a = fmin(p, q), b = fmax(p, q);
  // the plane leaves the same area cutting off 1 - c from the opposite
  // corner: solve for the smaller volume, where V and G carry no cancellation
  if (c > 0.5) c = 1.0 - c;
  // V(alpha) = (I(alpha) - I(alpha - nk)) / nk rises from 0 to 1 on [0, 1]
  double lo = 0.0, hi = 1.0, al = c;
  for (int it = 0; it < 200; ++it) {
    const double f = (plic_I(a, b, al) - plic_I(a, b, al - nk)) / nk - c;
    if (f == 0.0) break;
    if (f < 0.0) lo = al;
    else hi = al;
    const double dv = (plic_G(a, b, al) - plic_G(a, b, al - nk)) / nk;
    double nx = dv > 0.0 ? al - f / dv : 0.5 * (lo + hi);
    if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
    if (nx == al) break;
    al = nx;
  }
  const double band = plic_G(a, b, al) - plic_G(a, b, al - nk);
  return band * sqrt(nk * nk + a * a + b * b) / nk;
}

// ---- the cells pass
template <typename R>
__device__ void if3_youngs(const Iface3Args<R>& a, int x, int y, int z, double* m) {
  const double w[3] = {1.0, 2.0, 1.0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int b = d == 0 ? 1 : 0, cc = d == 2 ? 1 : 2;
    double s = 0.0;
    for (int p = -1; p <= 1; ++p)
      for (int r = -1; r <= 1; ++r) {
        int o[3] = {0, 0, 0};
        o[b] = p;
        o[cc] = r;
        o[d] = 1;
        const double hi = if3_at(a.vof, a.g, x + o[0], y + o[1], z + o[2]);
        o[d] = -1;
        const double lo = if3_at(a.vof, a.g, x + o[0], y + o[1], z + o[2]);
        s += w[p + 1] * w[r + 1] * (hi - lo);
      }
    m[d] = -s;
  }
}

// kappa by height functions; false when no axis closes
template <typename R>
__device__ bool if3_heights(const Iface3Args<R>& a, int x, int y, int z, const double* m,
                            double& kappa) {
  // axes by |m| descending, ties to the higher axis
  int ord[3] = {2, 1, 0};
  for (int u = 0; u < 3; ++u)
    for (int v = u + 1; v < 3; ++v)
      if (fabs(m[ord[v]]) > fabs(m[ord[u]])) {
        const int t = ord[u];
        ord[u] = ord[v];
        ord[v] = t;
      }
  for (int q = 0; q < 3; ++q) {
    const int ax = ord[q];
    if (m[ax] == 0.0) continue;
    const int b = ax == 0 ? 1 : 0, cc = ax == 2 ? 1 : 2;
    double H[3][3];
    bool ok = true;
    for (int p = -1; p <= 1; ++p)
      for (int r = -1; r <= 1; ++r) {
        double sum = 0.0, lo = 0.0, hi = 0.0;
        for (int l = -IF3_HL; l <= IF3_HL; ++l) {
          int o[3] = {0, 0, 0};
          o[ax] = l;
          o[b] = p;
          o[cc] = r;
          const double c = if3_at(a.vof, a.g, x + o[0], y + o[1], z + o[2]);
          sum += c;
          if (l == -IF3_HL) lo = c;
          if (l == IF3_HL) hi = c;
        }
        const double full = m[ax] > 0.0 ? lo : hi, empty = m[ax] > 0.0 ? hi : lo;
        if (!(full >= 1.0 - IFACE_CUT && empty <= IFACE_CUT)) ok = false;
        H[p + 1][r + 1] = sum;
      }
    if (!ok) continue;
    const double h = a.h;
    const double Hb = 0.5 * (H[2][1] - H[0][1]);
    const double Hc = 0.5 * (H[1][2] - H[1][0]);
    const double Hbb = (H[2][1] - 2.0 * H[1][1] + H[0][1]) / h;
    const double Hcc = (H[1][2] - 2.0 * H[1][1] + H[1][0]) / h;
    const double Hbc = (H[2][2] - H[2][0] - H[0][2] + H[0][0]) / (4.0 * h);
    const double qq = 1.0 + Hb * Hb + Hc * Hc;
    kappa = (Hbb * (1.0 + Hc * Hc) + Hcc * (1.0 + Hb * Hb) - 2.0 * Hbc * Hb * Hc) / (qq * sqrt(qq));
    return true;
  }
  return false;
}

constexpr int IF3_TX = 64, IF3_TY = 4, IF3_TZ = 2, IF3_NT = IF3_TX * IF3_TY * IF3_TZ;

template <typename R>
__global__ void __launch_bounds__(IF3_NT) k_iface3_cells(Iface3Args<R> a, int tiles_x,
                                                        int tiles_y) {
  __shared__ int sList[IF3_NT];
  __shared__ int sWave[IF3_NT / 64];
  const Grid& g = a.g;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int bx = blockIdx.x % tiles_x, r = blockIdx.x / tiles_x;
  const int x0 = bx * IF3_TX, y0 = (r % tiles_y) * IF3_TY, z0 = (r / tiles_y) * IF3_TZ;
  int x = x0 + t % IF3_TX, y = y0 + (t / IF3_TX) % IF3_TY, z = z0 + t / (IF3_TX * IF3_TY);
  const bool cut = x < g.n[0] && y < g.n[1] && z < g.n[2] &&
                   if3_cut((double)a.vof[cell_index(g, x, y, z)]);
  // the tile's interfacial cells, in thread order
  const unsigned long long bal = __ballot(cut);
  if (lane == 0) sWave[w] = __popcll(bal);
  __syncthreads();
  int base = 0, total = 0;
#pragma unroll
  for (int v = 0; v < IF3_NT / 64; ++v) {
    const int cnt = sWave[v];
    base += v < w ? cnt : 0;
    total += cnt;
  }
  if (cut) sList[base + __popcll(bal & ((1ull << lane) - 1ull))] = t;
  __syncthreads();
  if (t >= total) return;
  const int u = sList[t];
  x = x0 + u % IF3_TX;
  y = y0 + (u / IF3_TX) % IF3_TY;
  z = z0 + u / (IF3_TX * IF3_TY);
  const long long cl = cell_index(g, x, y, z);
  const double c = (double)a.vof[cl];
  double m[3], kap = 0.0;
  if3_youngs(a, x, y, z, m);
  if (!if3_heights(a, x, y, z, m, kap)) kap = (double)NAN;
  a.kh[cl] = (R)kap;
  a.dm[cl] = (R)(plic_area3(m[0], m[1], m[2], c) / a.h);
}

// ---- the faces pass
// the level set's curvature at cell (x, y, z), moved to the interface
template <typename R>
__device__ double if3_levelset_kappa(const Iface3Args<R>& a, int x, int y, int z) {
  const double h = a.h;
  auto C = [&](int dx, int dy, int dz) { return if3_at(a.chi, a.g, x + dx, y + dy, z + dz); };
  const double c0 = C(0, 0, 0);
  const double gx = (C(1, 0, 0) - C(-1, 0, 0)) / (2.0 * h);
  const double gy = (C(0, 1, 0) - C(0, -1, 0)) / (2.0 * h);
  const double gz = (C(0, 0, 1) - C(0, 0, -1)) / (2.0 * h);
  const double hxx = (C(1, 0, 0) - 2.0 * c0 + C(-1, 0, 0)) / (h * h);
  const double hyy = (C(0, 1, 0) - 2.0 * c0 + C(0, -1, 0)) / (h * h);
  const double hzz = (C(0, 0, 1) - 2.0 * c0 + C(0, 0, -1)) / (h * h);
  const double hxy = (C(1, 1, 0) - C(1, -1, 0) - C(-1, 1, 0) + C(-1, -1, 0)) / (4.0 * h * h);
  const double hxz = (C(1, 0, 1) - C(1, 0, -1) - C(-1, 0, 1) + C(-1, 0, -1)) / (4.0 * h * h);
  const double hyz = (C(0, 1, 1) - C(0, 1, -1) - C(0, -1, 1) + C(0, -1, -1)) / (4.0 * h * h);
  const double gm = fmax(sqrt(gx * gx + gy * gy + gz * gz), 1e-6);
  const double num = hxx * (gy * gy + gz * gz) + hyy * (gx * gx + gz * gz) +
                     hzz * (gx * gx + gy * gy) -
                     2.0 * (gx * gy * hxy + gx * gz * hxz + gy * gz * hyz);
  const double kc = num / (gm * gm * gm);
  return kc / (1.0 - c0 * kc / 2.0);
}

// kappa of an interfacial cell (mapped coordinates)
template <typename R>
__device__ double if3_kappa(const Iface3Args<R>& a, int x, int y, int z) {
  const double kh = (double)a.kh[cell_index(a.g, x, y, z)];
  if (!isnan(kh)) return kh;
  double s = 0.0;
  int cnt = 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        if (!if3_cut(if3_at(a.vof, a.g, x + dx, y + dy, z + dz))) continue;
        const double v = if3_at(a.kh, a.g, x + dx, y + dy, z + dz);
        if (!isnan(v)) {
          s += v;
          ++cnt;
        }
      }
  return cnt ? s / cnt : if3_levelset_kappa(a, x, y, z);
}

// the face gradient of a cell field across the face between cells L and R
// (R = L + e_d, both mapped into the box)
template <typename R>
__device__ void if3_face_grad(const Iface3Args<R>& a, const R* f, int d, const int* L,
                              const int* Rc, double* gr) {
  const double h = a.h;
  gr[d] = (if3_at(f, a.g, Rc[0], Rc[1], Rc[2]) - if3_at(f, a.g, L[0], L[1], L[2])) / h;
  for (int t = 0; t < 3; ++t) {
    if (t == d) continue;
    double s = 0.0;
    for (int side = 0; side < 2; ++side) {
      const int* X = side == 0 ? L : Rc;
      int p[3] = {X[0], X[1], X[2]}, q[3] = {X[0], X[1], X[2]};
      p[t] += 1;
      q[t] -= 1;
      s += 0.5 * (if3_at(f, a.g, p[0], p[1], p[2]) - if3_at(f, a.g, q[0], q[1], q[2])) / (2.0 * h);
    }
    gr[t] = s;
  }
}

// the two forces on the face along d between cells L and R
template <typename R>
__device__ void if3_face(const Iface3Args<R>& a, int d, const int* L, const int* Rc, double& cap,
                         double& ma) {
  const long long iL = cell_index(a.g, L[0], L[1], L[2]), iR = cell_index(a.g, Rc[0], Rc[1], Rc[2]);
  const double cL = (double)a.vof[iL], cR = (double)a.vof[iR];
  const bool cutL = if3_cut(cL), cutR = if3_cut(cR);
  cap = ma = 0.0;
  // kappa and delta_m vanish on both sides: so do both forces
  if (!cutL && !cutR) return;
  const double kL = cutL ? if3_kappa(a, L[0], L[1], L[2]) : 0.0;
  const double kR = cutR ? if3_kappa(a, Rc[0], Rc[1], Rc[2]) : 0.0;
  const double kf = cutL && cutR ? 0.5 * (kL + kR) : (cutL ? kL : (cutR ? kR : 0.0));
  const double sf = 0.5 * ((double)a.sig[iL] + (double)a.sig[iR]);
  cap = -sf * kf * (cR - cL) / a.h;
  double gs[3], gc[3];
  if3_face_grad(a, a.sig, d, L, Rc, gs);
  if3_face_grad(a, a.chi, d, L, Rc, gc);
  const double nrm = fmax(sqrt(gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2]), 1e-6);
  const double n0 = gc[0] / nrm, n1 = gc[1] / nrm, n2 = gc[2] / nrm;
  const double nd = d == 0 ? n0 : (d == 1 ? n1 : n2);
  const double ndot = n0 * gs[0] + n1 * gs[1] + n2 * gs[2];
  const double dmf = 0.5 * ((cutL ? (double)a.dm[iL] : 0.0) + (cutR ? (double)a.dm[iR] : 0.0));
  ma = dmf * (gs[d] - nd * ndot);
}

// one thread per cell: rows of the box along x in chunks of 256, a workgroup
// per (chunk, y, z)
template <typename R>
__global__ void __launch_bounds__(256) k_iface3_faces(Iface3Args<R> a, int chunks_x, R* cx,
                                                      R* cy, R* cz, R* mx, R* my, R* mz) {
  const Grid& g = a.g;
  R* cap[3] = {cx, cy, cz};
  R* ma[3] = {mx, my, mz};
  const int row = blockIdx.x / chunks_x;
  const int x = (blockIdx.x % chunks_x) * 256 + threadIdx.x;
  const int y = row % g.n[1], z = row / g.n[1];
  if (x >= g.n[0]) return;
  const int X[3] = {x, y, z};
  for (int d = 0; d < 3; ++d) {
    const bool per = g.bc[d][0] == BC_PERIODIC;
    // the low face of the cell, and the high face for the last cell
    for (int side = 0; side < (X[d] + 1 == g.n[d] ? 2 : 1); ++side) {
      const int f = X[d] + side;  // face coordinate along d
      double fc = 0.0, fm = 0.0;
      if (per || (f > 0 && f < g.n[d])) {
        int Rc[3] = {x, y, z}, L[3] = {x, y, z};
        Rc[d] = f % g.n[d];
        L[d] = (f - 1 + g.n[d]) % g.n[d];
        if3_face(a, d, L, Rc, fc, fm);
      }
      int F[3] = {x, y, z};
      F[d] = f;
      const long long fi = face_index(g, d, F[0], F[1], F[2]);
      if (cap[d]) cap[d][fi] = (R)fc;
      if (ma[d]) ma[d][fi] = (R)fm;
    }
  }
}

}  // namespace surf
