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
// The face arrays are zeroed (k_zero), then two launches over 16^3 tiles (a
// thread per z-column).  k_iface3_cells lists the tile's interfacial
// cells in LDS and gives them to its first threads (a sphere's surface
// leaves a few dozen to a few hundred per tile, so the heavy work packs into
// a wave or two); it writes each listed cell's height curvature (NaN where
// no axis closes) and delta_m into two scratch cell arrays, and nothing for
// the other cells.  k_iface3_faces lists the faces of all three axes with an
// interfacial cell on either side and computes those, reading the scratch
// arrays only at interfacial cells and filling in the curvature of a cell
// without heights from the first array, which no thread writes.
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
  R* fc[3];  // capillary force per face set (or null)
  R* fm[3];  // Marangoni force per face set (or null)
  double h;
};

__device__ __forceinline__ bool if3_cut(double c) { return c > IFACE_CUT && c < 1.0 - IFACE_CUT; }

// the cell index of (x, y, z) mapped into the box (mirrored or wrapped ghosts)
__device__ __forceinline__ long long if3_index(const Grid& g, int x, int y, int z) {
  const int i = map_axis(x, g.n[0], g.bc[0][0], g.bc[0][1]);
  const int j = map_axis(y, g.n[1], g.bc[1][0], g.bc[1][1]);
  const int k = map_axis(z, g.n[2], g.bc[2][0], g.bc[2][1]);
  return cell_index(g, i, j, k);
}

template <typename R>
__device__ __forceinline__ double if3_at(const R* a, const Grid& g, int x, int y, int z) {
  return (double)a[if3_index(g, x, y, z)];
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
// fv(x, y, z): the fraction of cell (x, y, z), ghosts mapped
template <typename FV>
__device__ __forceinline__ void if3_youngs(const FV& fv, int x, int y, int z, double* m) {
  const double w[3] = {1.0, 2.0, 1.0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int b = d == 0 ? 1 : 0, cc = d == 2 ? 1 : 2;
    double s = 0.0;
#pragma unroll
    for (int p = -1; p <= 1; ++p)
#pragma unroll
      for (int r = -1; r <= 1; ++r) {
        int o[3] = {0, 0, 0};
        o[b] = p;
        o[cc] = r;
        o[d] = 1;
        const double hi = fv(x + o[0], y + o[1], z + o[2]);
        o[d] = -1;
        const double lo = fv(x + o[0], y + o[1], z + o[2]);
        s += w[p + 1] * w[r + 1] * (hi - lo);
      }
    m[d] = -s;
  }
}

// kappa by height functions; false when no axis closes
template <typename FV>
__device__ __forceinline__ bool if3_heights(const FV& fv, double h, int x, int y, int z,
                                            const double* m, double& kappa) {
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
    const int b = ax == 0 ? 1 : 0;
    // the offset along axis e of cell l of column (p, r): l along ax, p along
    // b, r along the third axis (no indexed arrays, so that the 81 loads are
    // issued together)
    auto off = [&](int e, int p, int r, int l) { return e == ax ? l : (e == b ? p : r); };
    double H[9];
    bool ok = true;
    for (int pr = 0; pr < 9; ++pr) {  // column (p, r) = (pr / 3 - 1, pr % 3 - 1)
      const int p = pr / 3 - 1, r = pr % 3 - 1;
      double col[2 * IF3_HL + 1];  // the column's nine values gathered together
#pragma unroll
      for (int l = -IF3_HL; l <= IF3_HL; ++l)
        col[l + IF3_HL] = fv(x + off(0, p, r, l), y + off(1, p, r, l), z + off(2, p, r, l));
      double sum = 0.0;
#pragma unroll
      for (int l = 0; l <= 2 * IF3_HL; ++l) sum += col[l];
      const double lo = col[0], hi = col[2 * IF3_HL];
      const double full = m[ax] > 0.0 ? lo : hi, empty = m[ax] > 0.0 ? hi : lo;
      if (!(full >= 1.0 - IFACE_CUT && empty <= IFACE_CUT)) ok = false;
      H[pr] = sum;
    }
    if (!ok) continue;
    // H[3 (p + 1) + (r + 1)]
    const double Hb = 0.5 * (H[7] - H[1]);
    const double Hc = 0.5 * (H[5] - H[3]);
    const double Hbb = (H[7] - 2.0 * H[4] + H[1]) / h;
    const double Hcc = (H[5] - 2.0 * H[4] + H[3]) / h;
    const double Hbc = (H[8] - H[6] - H[2] + H[0]) / (4.0 * h);
    const double qq = 1.0 + Hb * Hb + Hc * Hc;
    kappa = (Hbb * (1.0 + Hc * Hc) + Hcc * (1.0 + Hb * Hb) - 2.0 * Hbc * Hb * Hc) / (qq * sqrt(qq));
    return true;
  }
  return false;
}

constexpr int IF3_T = 16, IF3_NT = IF3_T * IF3_T;  // 16^3 tiles, a thread per z-column
constexpr int IF3_S = IF3_T + 2 * IF3_HL;           // the staged region's edge

// The workgroup's list of this thread's entries (the set bits k of mask,
// stored as (k << 8) | t | tag, tag above bit 11) after those of the
// threads before it, in sList; returns the list length.  Two barriers.
__device__ __forceinline__ int if3_list(unsigned mask, unsigned short* sList, int* sWave,
                                        unsigned tag = 0) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int cnt = __popc(mask);
  int inc = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int up = __shfl_up(inc, o);
    if (lane >= o) inc += up;
  }
  if (lane == 63) sWave[w] = inc;
  __syncthreads();
  int pos = inc - cnt, total = 0;
#pragma unroll
  for (int v = 0; v < IF3_NT / 64; ++v) {
    pos += v < w ? sWave[v] : 0;
    total += sWave[v];
  }
  for (unsigned m = mask; m; m &= m - 1u)
    sList[pos++] = (unsigned short)((((__ffs(m) - 1) << 8) | t) | tag);
  __syncthreads();
  return total;
}

// the face index of cell (x, y, z) with coordinate d replaced by f
__device__ __forceinline__ long long if3_face_index(const Grid& g, int d, int x, int y, int z,
                                                    int f) {
  return face_index(g, d, d == 0 ? f : x, d == 1 ? f : y, d == 2 ? f : z);
}

template <typename R>
__global__ void __launch_bounds__(IF3_NT) k_iface3_cells(Iface3Args<R> a, int tiles_x,
                                                        int tiles_y) {
  __shared__ unsigned short sList[IF3_T * IF3_T * IF3_T];
  __shared__ int sWave[IF3_NT / 64];
  __shared__ float sV[IF3_S][IF3_S][IF3_S];  // FP32 fractions of the tile and its halo
  const Grid& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int t = threadIdx.x;
  const int r = blockIdx.x / tiles_x;
  const int x0 = (blockIdx.x % tiles_x) * IF3_T, y0 = (r % tiles_y) * IF3_T,
            z0 = (r / tiles_y) * IF3_T;
  const int x = x0 + t % IF3_T, y = y0 + t / IF3_T;
  const long long pl = (long long)nx * ny;
  // this column's interfacial cells as a bit mask, every load issued first
  unsigned mask = 0;
  if (x < nx && y < ny) {
    const long long cxy = (long long)x + (long long)nx * y;
    R v[IF3_T];
#pragma unroll
    for (int k = 0; k < IF3_T; ++k) v[k] = z0 + k < nz ? a.vof[cxy + pl * (z0 + k)] : R(0);
#pragma unroll
    for (int k = 0; k < IF3_T; ++k) mask |= if3_cut((double)v[k]) ? (1u << k) : 0u;
  }
  const int total = if3_list(mask, sList, sWave);
  if (total == 0) return;
  auto cell = [&](const auto& fv) {
    for (int i = t; i < total; i += IF3_NT) {
      const int e = sList[i];
      const int cx = x0 + (e & 15), cy = y0 + ((e >> 4) & 15), cz = z0 + (e >> 8);
      const long long cl = (long long)cx + (long long)nx * cy + pl * cz;
      const double c = (double)a.vof[cl];
      double m3[3], kap = 0.0;
      if3_youngs(fv, cx, cy, cz, m3);
      if (!if3_heights(fv, a.h, cx, cy, cz, m3, kap)) kap = (double)NAN;
      a.kh[cl] = (R)kap;
      a.dm[cl] = (R)(plic_area3(m3[0], m3[1], m3[2], c) / a.h);
    }
  };
  if constexpr (sizeof(R) == 4) {
    // FP32: the tile and IF3_HL cells around it (mapped) staged in LDS, a
    // column of 24 per thread with its loads issued together
    for (int q = t; q < IF3_S * IF3_S; q += IF3_NT) {
      const int sx = q % IF3_S, sy = q / IF3_S;
      R v[IF3_S];
#pragma unroll
      for (int k = 0; k < IF3_S; ++k)
        v[k] = a.vof[if3_index(g, x0 - IF3_HL + sx, y0 - IF3_HL + sy, z0 - IF3_HL + k)];
#pragma unroll
      for (int k = 0; k < IF3_S; ++k) sV[k][sy][sx] = v[k];
    }
    __syncthreads();
    cell([&](int X, int Y, int Z) {
      return (double)sV[Z - z0 + IF3_HL][Y - y0 + IF3_HL][X - x0 + IF3_HL];
    });
  } else {
    cell([&](int X, int Y, int Z) { return if3_at(a.vof, g, X, Y, Z); });
  }
}

// ---- the faces pass
// the level set's curvature at cell (x, y, z), moved to the interface
template <typename R>
__device__ __forceinline__ double if3_levelset_kappa(const Iface3Args<R>& a, int x, int y, int z) {
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
__device__ __forceinline__ double if3_kappa(const Iface3Args<R>& a, int x, int y, int z) {
  const double kh = (double)a.kh[cell_index(a.g, x, y, z)];
  if (!isnan(kh)) return kh;
  // every neighbour's fraction and scratch curvature loaded first (the
  // curvature is used only where the neighbour is interfacial)
  R fv[27], kv[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const long long i = if3_index(a.g, x + q % 3 - 1, y + (q / 3) % 3 - 1, z + q / 9 - 1);
    fv[q] = a.vof[i];
    kv[q] = a.kh[i];
  }
  double s = 0.0;
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < 27; ++q) {  // dz, dy, dx from -1 to 1
    if (q == 13 || !if3_cut((double)fv[q])) continue;
    const double v = (double)kv[q];
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
__device__ __forceinline__ void if3_face_grad(const Iface3Args<R>& a, const R* f, int d, const int* L,
                              const int* Rc, double* gr) {
  const double h = a.h;
  const double nrm = (if3_at(f, a.g, Rc[0], Rc[1], Rc[2]) - if3_at(f, a.g, L[0], L[1], L[2])) / h;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    double s = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int* X = side == 0 ? L : Rc;
      const int px = X[0] + (t == 0), py = X[1] + (t == 1), pz = X[2] + (t == 2);
      const int qx = X[0] - (t == 0), qy = X[1] - (t == 1), qz = X[2] - (t == 2);
      s += 0.5 * (if3_at(f, a.g, px, py, pz) - if3_at(f, a.g, qx, qy, qz)) / (2.0 * h);
    }
    gr[t] = t == d ? nrm : s;
  }
}

// the two forces on the face along d between cells L and R
template <typename R>
__device__ __forceinline__ void if3_face(const Iface3Args<R>& a, int d, const int* L, const int* Rc, double& cap,
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
  const double gsd = d == 0 ? gs[0] : (d == 1 ? gs[1] : gs[2]);
  ma = dmf * (gsd - nd * ndot);
}

// The faces next to interfacial cells, over 16^3 tiles: the low face of a
// cell along d is computed when the cell or its low neighbour along d is
// interfacial (on a periodic axis the last cell also its high face, the
// same two cells as face 0), the other faces keep the zero the cells pass
// wrote.  Per axis the tile lists its faces in LDS and its threads take them
// in turn, so the interfacial work of a tile packs into a wave or two.
template <typename R>
__global__ void __launch_bounds__(IF3_NT) k_iface3_faces(Iface3Args<R> a, int tiles_x,
                                                        int tiles_y) {
  __shared__ unsigned short sList[3 * (IF3_T * IF3_T * IF3_T + IF3_NT)];
  __shared__ int sWave[IF3_NT / 64];
  const Grid& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int t = threadIdx.x;
  const int r = blockIdx.x / tiles_x;
  const int x0 = (blockIdx.x % tiles_x) * IF3_T, y0 = (r % tiles_y) * IF3_T,
            z0 = (r / tiles_y) * IF3_T;
  const int x = x0 + t % IF3_T, y = y0 + t / IF3_T;
  const bool colin = x < nx && y < ny;
  const long long pl = (long long)nx * ny;
  // cut bits of the column (bit k: cell z0 + k) and of the column's low
  // neighbours along x and y, the cell below the column and, for the last
  // cells along an axis, the first cell along it
  unsigned cc = 0, cxm = 0, cym = 0;
  bool czm = false, cz0 = false;
  if (colin) {
    const long long cxy = (long long)x + (long long)nx * y;
    const long long xm = (long long)(x == 0 ? nx - 1 : x - 1) + (long long)nx * y;
    const long long ym = (long long)x + (long long)nx * (y == 0 ? ny - 1 : y - 1);
    R v[IF3_T], vx[IF3_T], vy[IF3_T];
#pragma unroll
    for (int k = 0; k < IF3_T; ++k) {
      const long long z = (long long)min(z0 + k, nz - 1);
      v[k] = a.vof[cxy + pl * z];
      vx[k] = a.vof[xm + pl * z];
      vy[k] = a.vof[ym + pl * z];
    }
    const R vz = a.vof[cxy + pl * (z0 == 0 ? nz - 1 : z0 - 1)];  // the cell below
    const R vz0 = a.vof[cxy];                                     // z = 0
#pragma unroll
    for (int k = 0; k < IF3_T; ++k) {
      const unsigned b = z0 + k < nz ? (1u << k) : 0u;
      cc |= if3_cut((double)v[k]) ? b : 0u;
      cxm |= if3_cut((double)vx[k]) ? b : 0u;
      cym |= if3_cut((double)vy[k]) ? b : 0u;
    }
    czm = if3_cut((double)vz);
    cz0 = if3_cut((double)vz0);
  }
  // per axis the low faces (bit k when the face exists, interior or
  // periodic, and a side is interfacial) and the high faces of the last
  // cells on a periodic axis (the cell or the first one along the axis)
  int n = 0;
  for (int d = 0; d < 3; ++d) {
    const bool per = g.bc[d][0] == BC_PERIODIC;
    unsigned lo = 0, hi = 0;
    if (colin) {
      if (d == 0) {
        lo = (x > 0 || per) ? (cc | cxm) : 0u;
      } else if (d == 1) {
        lo = (y > 0 || per) ? (cc | cym) : 0u;
      } else {
        const unsigned below = (cc << 1) | (czm ? 1u : 0u);  // bit k: cell z0 + k - 1
        lo = (cc | below) & ((1u << IF3_T) - 1u);
        if (z0 == 0 && !per) lo &= ~1u;
      }
      if (per) {
        if (d == 0 && x == nx - 1) {
          unsigned first = 0;  // the row's first cells
          for (int k = 0; k < IF3_T; ++k)
            if (z0 + k < nz && if3_cut((double)a.vof[(long long)nx * y + pl * (z0 + k)]))
              first |= 1u << k;
          hi = cc | first;
        } else if (d == 1 && y == ny - 1) {
          unsigned first = 0;  // the column's first cells
          for (int k = 0; k < IF3_T; ++k)
            if (z0 + k < nz && if3_cut((double)a.vof[(long long)x + pl * (z0 + k)])) first |= 1u << k;
          hi = cc | first;
        } else if (d == 2 && nz - 1 >= z0 && nz - 1 < z0 + IF3_T) {
          const int k = nz - 1 - z0;
          if (((cc >> k) & 1u) || cz0) hi = 1u << k;
        }
      }
      const unsigned inbox = z0 + IF3_T <= nz ? 0xffffu : ((1u << (nz - z0)) - 1u);
      lo &= inbox;
      hi &= inbox;
    }
    // tag: the axis in bits 12-13, a high face in bit 14
    n += if3_list(lo, sList + n, sWave, (unsigned)d << 12);
    n += if3_list(hi, sList + n, sWave, ((unsigned)d << 12) | (1u << 14));
  }
  for (int i = t; i < n; i += IF3_NT) {
    const int e = sList[i];
    const int d = (e >> 12) & 3;
    const bool high = (e >> 14) & 1;
    const int cx = x0 + (e & 15), cy = y0 + ((e >> 4) & 15), cz = z0 + ((e >> 8) & 15);
    const int X[3] = {cx, cy, cz};
    const int nd = g.n[d], xd = d == 0 ? cx : (d == 1 ? cy : cz);
    const int f = high ? nd : xd;  // face coordinate along d
    const int rd = f == nd ? 0 : f, ld = f == 0 ? nd - 1 : f - 1;
    const int Rc[3] = {d == 0 ? rd : X[0], d == 1 ? rd : X[1], d == 2 ? rd : X[2]};
    const int L[3] = {d == 0 ? ld : X[0], d == 1 ? ld : X[1], d == 2 ? ld : X[2]};
    double fc = 0.0, fm = 0.0;
    if3_face(a, d, L, Rc, fc, fm);
    const long long fi = if3_face_index(g, d, cx, cy, cz, f);
    R* cap = d == 0 ? a.fc[0] : (d == 1 ? a.fc[1] : a.fc[2]);
    R* ma = d == 0 ? a.fm[0] : (d == 1 ? a.fm[1] : a.fm[2]);
    if (cap) cap[fi] = (R)fc;
    if (ma) ma[fi] = (R)fm;
  }
}

// zero over n values (the face arrays, before the interfacial faces are
// written)
template <typename R>
__global__ void __launch_bounds__(256) k_zero(R* __restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = R(0);
}

}  // namespace surf
