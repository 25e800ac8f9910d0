// surf_capillary.hpp -- the interfacial forces for the coupling to a flow
// solver (section 2.4), 2D: the capillary force sigma kappa delta_s n and the
// Marangoni force delta_m grad_s sigma with delta_m = A_f / V_c, on the faces
// of the velocity grid.
//
// n points out of fluid 1 (n = grad phi / |grad phi|), so delta_s n =
// |grad c| n = -grad c and the capillary force on a face is
// -sigma_f kappa_f (c_R - c_L) / h.  A cell is interfacial when
// 1e-6 < c < 1 - 1e-6.  Per interfacial cell:
//   * the Youngs normal m = -grad c from the 3x3 stencil (weights 1, 2, 1);
//   * kappa by height functions (Cummins, Francois and Kothe 2005): along the
//     axis of m's larger component, the fluid-1 heights of the three columns
//     of seven cells through the cell and its two neighbours,
//     kappa = H'' / (1 + H'^2)^(3/2); a column whose end cells are not full
//     on the fluid-1 side and empty on the other falls back to the curvature
//     of the level set, div(grad chi / |grad chi|) moved to the interface
//     with kappa / (1 - chi kappa);
//   * delta_m = chord / h, the chord of the PLIC line inside the cell from
//     the closed-form plane constant of a line in a square (Scardovelli and
//     Zaleski, J. Comput. Phys. 164, 2000) with |m| normalized to
//     |m_1| + |m_2| = 1.
// On a face kappa is the mean over its interfacial cells, delta_m and sigma
// the means over both; grad_s sigma is the face gradient of sigma (compact
// normal difference, the two cells' centred transverse differences
// averaged) minus its part along the face gradient of chi.  Faces on walls
// and open sides carry no force; on a periodic axis the last face repeats
// the first.  On axisymmetric rings (Appendix B; x the radius, ring i at
// r_i = r0 + (i + 1/2) h) the interface is a surface of revolution: kappa
// adds the azimuthal curvature -n_r / r_i (n the unit Youngs normal; the
// level-set fallback adds (d chi / dr) / (|grad chi| r_i) and moves the sum
// with kappa / (1 - chi kappa / 2)), and delta_m = A_f / V_c is the chord's
// swept area over the ring's volume, (|chord| / h^2) r_m / r_i with r_m the
// radius of the chord's midpoint.
#pragma once
#include "surf_kernels.hpp"

namespace surf {

constexpr double IFACE_CUT = 1e-6;

template <typename R>
struct IfaceArgs {
  Grid g;
  Par<R> p;
  const R* vof;
  const R* chi;
  const R* sig;
  double h;   // the cell size in FP64 for the geometry
  int axi;    // axisymmetric rings: x is the radius, from r0
  double r0;
};

template <typename R>
__device__ __forceinline__ bool iface_cut(R c) {
  return c > R(IFACE_CUT) && c < R(1) - R(IFACE_CUT);
}

// The interface geometry (Youngs normal, heights, curvature, PLIC chord) is
// evaluated in FP64 in both precisions: the inputs are exact there, sums of
// seven fractions stay exact, and the second difference of the heights,
// about kappa h cells, would otherwise lose four digits to cancellation in
// FP32 at h = 1/1024.  The functions read the fields through accessors
// f(dj, di) that return the value at the cell offset (di, dj) as a double.
template <typename V>
__device__ __forceinline__ void youngs(const V& f, double& mx, double& my) {
  const double a = f(1, 1), b = f(0, 1), cc = f(-1, 1);
  const double d = f(1, -1), e = f(0, -1), w1 = f(-1, -1);
  const double u = f(1, 0), w = f(-1, 0);
  mx = -((a + 2.0 * b + cc) - (d + 2.0 * e + w1));
  my = -((a + 2.0 * u + d) - (cc + 2.0 * w + w1));
}

// the chord of the PLIC line (normal m, fraction c) inside the unit square
__device__ __forceinline__ double plic_chord(double mx, double my, double c) {
  double n1 = fabs(mx), n2 = fabs(my);
  const double s = n1 + n2;
  if (!(s > 0.0)) return 0.0;
  n1 /= s;
  n2 /= s;
  if (n1 > n2) {
    const double t = n1;
    n1 = n2;
    n2 = t;
  }
  // n1 <= n2, n1 + n2 = 1: the area below the line n1 x + n2 y = alpha is
  // alpha^2/(2 n1 n2) up to alpha = n1, then (alpha - n1/2)/n2 up to n2, then
  // 1 - (1 - alpha)^2/(2 n1 n2); the chord is the hypotenuse of the corner
  // triangle in the outer ranges and sqrt(1 + (n1/n2)^2) between them
  const double c1 = n1 / (2.0 * n2);
  if (c > c1 && c < 1.0 - c1) return sqrt(1.0 + (n1 / n2) * (n1 / n2));
  const double al = sqrt(2.0 * n1 * n2 * (c <= c1 ? c : 1.0 - c));
  return sqrt((al / n1) * (al / n1) + (al / n2) * (al / n2));
}

// The chord of the PLIC line and the x coordinate of its midpoint (0 .. 1
// across the cell), for the rings' swept area.  In the frame (u, v) of the
// normal's smaller and larger components, reflected so that both are >= 0,
// the chord runs between the axes (fraction up to c1 = n_u / (2 n_v)) or
// across the cell from u = 0 to 1 at mean height c; a fraction above 1/2 is
// the point reflection through the centre of the complement's chord.
__device__ __forceinline__ double plic_chord_mid(double mx, double my, double c, double& xmid) {
  xmid = 0.5;
  const double a1 = fabs(mx), a2 = fabs(my), s = a1 + a2;
  if (!(s > 0.0)) return 0.0;
  const bool swap = a1 > a2;  // u along y when the x component is the larger
  const double nu = (swap ? a2 : a1) / s, nv = (swap ? a1 : a2) / s;
  const bool flip = c > 0.5;
  const double cc = flip ? 1.0 - c : c;
  const double c1 = nu / (2.0 * nv);
  double um, vm, chord;
  if (cc > c1) {
    um = 0.5;
    vm = cc;
    chord = sqrt(1.0 + (nu / nv) * (nu / nv));
  } else {
    const double al = sqrt(2.0 * nu * nv * cc);
    um = al / (2.0 * nu);
    vm = al / (2.0 * nv);
    chord = sqrt((al / nu) * (al / nu) + (al / nv) * (al / nv));
  }
  if (flip) {
    um = 1.0 - um;
    vm = 1.0 - vm;
  }
  const double xr = swap ? vm : um;  // along x in the reflected frame
  xmid = mx >= 0.0 ? xr : 1.0 - xr;
  return chord;
}

// div(grad chi / |grad chi|) by central differences, moved to the interface
// (on rings r > 0: with the azimuthal part (d chi / dr) / (|grad chi| r),
// moved with kappa / (1 - chi kappa / 2), exact on a sphere)
template <typename X>
__device__ double levelset_curvature_axi(const X& x, double h, double r) {
  const double c00 = x(0, 0);
  const double cxp = x(0, 1), cxm = x(0, -1), cyp = x(1, 0), cym = x(-1, 0);
  const double cx = (cxp - cxm) / (2.0 * h), cy = (cyp - cym) / (2.0 * h);
  const double cxx = (cxp - 2.0 * c00 + cxm) / (h * h), cyy = (cyp - 2.0 * c00 + cym) / (h * h);
  const double cxy = (x(1, 1) - x(1, -1) - x(-1, 1) + x(-1, -1)) / (4.0 * h * h);
  const double gm = fmax(sqrt(cx * cx + cy * cy), 1e-6);
  double kc = (cxx * cy * cy - 2.0 * cx * cy * cxy + cyy * cx * cx) / (gm * gm * gm);
  kc += cx / (gm * r);
  return kc / (1.0 - c00 * kc / 2.0);
}

// div(grad chi / |grad chi|) by central differences, moved to the interface
template <typename X>
__device__ double levelset_curvature(const X& x, double h) {
  const double c00 = x(0, 0);
  const double cxp = x(0, 1), cxm = x(0, -1), cyp = x(1, 0), cym = x(-1, 0);
  const double cx = (cxp - cxm) / (2.0 * h), cy = (cyp - cym) / (2.0 * h);
  const double cxx = (cxp - 2.0 * c00 + cxm) / (h * h), cyy = (cyp - 2.0 * c00 + cym) / (h * h);
  const double cxy = (x(1, 1) - x(1, -1) - x(-1, 1) + x(-1, -1)) / (4.0 * h * h);
  const double gm = fmax(sqrt(cx * cx + cy * cy), 1e-6);
  const double kc = (cxx * cy * cy - 2.0 * cx * cy * cxy + cyy * cx * cx) / (gm * gm * gm);
  return kc / (1.0 - c00 * kc);
}

// kappa of an interfacial cell by height functions; false when a column does
// not close (full on the fluid-1 side and empty on the other), and the cell
// then takes the level set's curvature
template <typename V>
__device__ bool height_curvature(const V& f, double h, double& kappa) {
  double mx, my;
  youngs(f, mx, my);
  const bool vert = fabs(my) >= fabs(mx);  // columns along y
  const double out = vert ? my : mx;       // the normal's component along the columns
  double H[3];
  bool ok = true;
#pragma unroll
  for (int k = -1; k <= 1; ++k) {
    double sum = 0.0, lo = 0.0, hi = 0.0;
#pragma unroll
    for (int l = -3; l <= 3; ++l) {
      const double c = vert ? f(l, k) : f(k, l);
      sum += c;
      if (l == -3) lo = c;
      if (l == 3) hi = c;
    }
    // fluid 1 lies against the normal: the low end is full when it points to +
    const double full = out > 0.0 ? lo : hi, empty = out > 0.0 ? hi : lo;
    if (!(full >= 1.0 - IFACE_CUT && empty <= IFACE_CUT)) ok = false;
    H[k + 1] = sum;
  }
  const double d1 = 0.5 * (H[2] - H[0]);
  const double d2 = (H[2] - 2.0 * H[1] + H[0]) / h;
  const double q = 1.0 + d1 * d1;
  kappa = d2 / (q * sqrt(q));
  return ok;
}

template <typename V>
__device__ __forceinline__ double cell_delta_m(const V& f, double h) {
  double mx, my;
  youngs(f, mx, my);
  return plic_chord(mx, my, f(0, 0)) / h;
}

// Launch shape: a workgroup takes a tile of IF_TX x IF_TY cells (i, j); each
// cell owns its low x face (i, j) and low y face (i, j), and the cells of the
// last column and row also own the faces at i = nx and j = ny.  The faces'
// cells are the (IF_TX+2) x (IF_TY+2) cells from (x0-1, y0-1); their
// stencils reach three cells further for the heights and one for the level
// set, so the workgroup stages the VoF with a halo of 4 and the level set and
// sigma with a halo of 2 in LDS, at coordinates mapped into the box as the
// per-cell kernels map them.  A tile with no interfacial face cell writes
// zeros after one pass over the VoF.  Otherwise the interfacial cells are
// gathered into a list so that their FP64 geometry runs on consecutive
// lanes, the level set and sigma are loaded into registers before that
// geometry and stored to LDS after it.
constexpr int IF_TX = 64, IF_TY = 8, IF_THREADS = 256;
constexpr int IF_GX = IF_TX + 2, IF_GY = IF_TY + 2;  // the faces' cells, from (x0-1, y0-1)
constexpr int IF_VX = IF_TX + 8, IF_VY = IF_TY + 8;  // VoF tile from (x0-4, y0-4)
constexpr int IF_CX = IF_TX + 4, IF_CY = IF_TY + 4;  // chi and sigma from (x0-2, y0-2)
constexpr int IF_CPT = (IF_CX * IF_CY + IF_THREADS - 1) / IF_THREADS;  // per thread

__host__ __device__ __forceinline__ int iface_tiles_x(int nx) { return (nx + IF_TX - 1) / IF_TX; }
__host__ __device__ __forceinline__ int iface_tiles_y(int ny) { return (ny + IF_TY - 1) / IF_TY; }

// AXI: the ring terms, compiled only into the instance for rings
template <typename R, bool AXI>
__global__ void __launch_bounds__(IF_THREADS) k_iface_force(IfaceArgs<R> a, R* __restrict__ cap_x,
                                                            R* __restrict__ cap_y,
                                                            R* __restrict__ ma_x,
                                                            R* __restrict__ ma_y) {
  const Grid& g = a.g;
  const int nx = g.n[0], ny = g.n[1];
  const int tiles_x = iface_tiles_x(nx);
  const int ty_blk = (int)blockIdx.x / tiles_x;
  const int x0 = ((int)blockIdx.x - ty_blk * tiles_x) * IF_TX, y0 = ty_blk * IF_TY;
  const int tid = (int)threadIdx.x;
  __shared__ R sv[IF_VY][IF_VX];
  __shared__ R sx[IF_CY][IF_CX];
  __shared__ R ss[IF_CY][IF_CX];
  __shared__ double sk[IF_GY][IF_GX];
  __shared__ double sd[IF_GY][IF_GX];
  __shared__ short list[IF_GX * IF_GY];
  __shared__ int count;
  const int bx0 = g.bc[0][0], bx1 = g.bc[0][1], by0 = g.bc[1][0], by1 = g.bc[1][1];
  // the faces use the cells x0-1 .. min(x0+TX-1, nx-1) + 1 (cell nx: the
  // right cell of the last face, cell 0 on a periodic axis), y likewise
  const int gx_end = min(IF_GX, nx - x0 + 2), gy_end = min(IF_GY, ny - y0 + 2);

  // 1. the VoF tile, then the list of interfacial face cells
  if (tid == 0) count = 0;
  for (int l = tid; l < IF_VX * IF_VY; l += IF_THREADS) {
    const int vy = l / IF_VX, vx = l - vy * IF_VX;
    const int ci = map_axis(x0 - 4 + vx, nx, bx0, bx1), cj = map_axis(y0 - 4 + vy, ny, by0, by1);
    sv[vy][vx] = a.vof[cell_index(g, ci, cj, 0)];
  }
  __syncthreads();
  for (int l = tid; l < IF_GX * IF_GY; l += IF_THREADS) {
    const int gy = l / IF_GX, gx = l - gy * IF_GX;
    if (gx < gx_end && gy < gy_end && iface_cut(sv[gy + 3][gx + 3]))
      list[atomicAdd(&count, 1)] = (short)l;
  }
  __syncthreads();
  const int ncut = count;

  if (ncut > 0) {
    // 2. level set and sigma into registers; kappa (heights) and delta_m of
    // the listed cells meanwhile; then the tiles to LDS and the level-set
    // curvature of the cells whose columns do not close
    R rx[IF_CPT], rs[IF_CPT];
#pragma unroll
    for (int k = 0; k < IF_CPT; ++k) {
      const int l = min(tid + k * IF_THREADS, IF_CX * IF_CY - 1);
      const int cy = l / IF_CX, cx = l - cy * IF_CX;
      const int ci = map_axis(x0 - 2 + cx, nx, bx0, bx1), cj = map_axis(y0 - 2 + cy, ny, by0, by1);
      const long long c = cell_index(g, ci, cj, 0);
      rx[k] = a.chi[c];
      rs[k] = a.sig[c];
    }
    bool fallback = false;
    for (int k = tid; k < ncut; k += IF_THREADS) {
      const int l = list[k];
      const int gy = l / IF_GX, gx = l - gy * IF_GX;
      const auto f = [&](int dj, int di) { return (double)sv[gy + 3 + dj][gx + 3 + di]; };
      double kap;
      if (!height_curvature(f, a.h, kap)) {
        fallback = true;
        kap = __builtin_nan("");  // replaced below
      }
      if constexpr (!AXI) {
        sd[gy][gx] = cell_delta_m(f, a.h);
      } else {
        // the ring's radius at the cell's geometric position (a mirrored
        // ghost beyond the axis has r < 0 and its normal mirrored)
        const int i = x0 - 1 + gx;
        const double r = a.r0 + (i + 0.5) * a.h;
        double mx, my, xm;
        youngs(f, mx, my);
        const double chord = plic_chord_mid(mx, my, f(0, 0), xm);
        sd[gy][gx] = r != 0.0 ? chord / a.h * (a.r0 + (i + xm) * a.h) / r : 0.0;
        const double nm = sqrt(mx * mx + my * my);
        if (!isnan(kap) && nm > 0.0 && r != 0.0) kap -= mx / nm / r;  // -n_r / r
      }
      sk[gy][gx] = kap;
    }
#pragma unroll
    for (int k = 0; k < IF_CPT; ++k) {
      const int l = tid + k * IF_THREADS;
      if (l < IF_CX * IF_CY) {
        const int cy = l / IF_CX, cx = l - cy * IF_CX;
        sx[cy][cx] = rx[k];
        ss[cy][cx] = rs[k];
      }
    }
    if (__syncthreads_or(fallback)) {
      for (int k = tid; k < ncut; k += IF_THREADS) {
        const int l = list[k];
        const int gy = l / IF_GX, gx = l - gy * IF_GX;
        if (isnan(sk[gy][gx])) {
          const auto x = [&](int dj, int di) { return (double)sx[gy + 1 + dj][gx + 1 + di]; };
          const double r = a.r0 + (x0 - 1 + gx + 0.5) * a.h;
          sk[gy][gx] = (AXI && r != 0.0) ? levelset_curvature_axi(x, a.h, r)
                                           : levelset_curvature(x, a.h);
        }
      }
      __syncthreads();
    }
  }

  // 3. the faces of this thread's cells
  const Par<R>& p = a.p;
  const int tx = tid % IF_TX;
  for (int ty = tid / IF_TX; ty < IF_TY; ty += IF_THREADS / IF_TX) {
    const int i0 = x0 + tx, j0 = y0 + ty;
    if (i0 >= nx || j0 >= ny) continue;
    // faces: x at (i0, j0) [and (nx, j0)], y at (i0, j0) [and (i0, ny)]
    const int nf = 2 + (i0 == nx - 1) + (j0 == ny - 1);
    for (int q = 0; q < nf; ++q) {
      const int D = q == 0 ? 0 : q == 1 ? 1 : (q == 2 && i0 == nx - 1) ? 0 : 1;
      const int i = (q >= 2 && D == 0) ? nx : i0, j = (q >= 2 && D == 1) ? ny : j0;
      R fc = R(0), fm = R(0);
      const int f = D == 0 ? i : j, nd = D == 0 ? nx : ny;
      const bool open = g.bc[D][0] == BC_PERIODIC || (f > 0 && f < nd);
      // geometry coordinates of the face's cells
      const int gxR = i - x0 + 1, gyR = j - y0 + 1;
      const int gxL = D == 0 ? gxR - 1 : gxR, gyL = D == 0 ? gyR : gyR - 1;
      if (ncut > 0 && open) {
        const R cL = sv[gyL + 3][gxL + 3], cR = sv[gyR + 3][gxR + 3];
        const bool uL = iface_cut(cL), uR = iface_cut(cR);
        if (uL || uR) {
          const R sL = ss[gyL + 1][gxL + 1], sR = ss[gyR + 1][gxR + 1];
          const double kL = uL ? sk[gyL][gxL] : 0.0, kR = uR ? sk[gyR][gxR] : 0.0;
          const R kf = (R)((uL && uR) ? 0.5 * (kL + kR) : (uL ? kL : kR));
          fc = -(R(0.5) * (sL + sR)) * kf * (cR - cL) * p.inv_h;
          const R dmf = (R)(0.5 * ((uL ? sd[gyL][gxL] : 0.0) + (uR ? sd[gyR][gxR] : 0.0)));
          // face gradients: compact along D, averaged centred differences across
          const int di = D == 0 ? 0 : 1, dj = D == 0 ? 1 : 0;
          const R gsD = (sR - sL) * p.inv_h;
          const R gcD = (sx[gyR + 1][gxR + 1] - sx[gyL + 1][gxL + 1]) * p.inv_h;
          const R qL = ss[gyL + 1 + dj][gxL + 1 + di] - ss[gyL + 1 - dj][gxL + 1 - di];
          const R qR = ss[gyR + 1 + dj][gxR + 1 + di] - ss[gyR + 1 - dj][gxR + 1 - di];
          const R gsT = R(0.5) * (qL + qR) * (R(0.5) * p.inv_h);
          const R xL = sx[gyL + 1 + dj][gxL + 1 + di] - sx[gyL + 1 - dj][gxL + 1 - di];
          const R xR = sx[gyR + 1 + dj][gxR + 1 + di] - sx[gyR + 1 - dj][gxR + 1 - di];
          const R gcT = R(0.5) * (xL + xR) * (R(0.5) * p.inv_h);
          const R gc0 = D == 0 ? gcD : gcT, gc1 = D == 0 ? gcT : gcD;
          const R gs0 = D == 0 ? gsD : gsT, gs1 = D == 0 ? gsT : gsD;
          const R nrm = fmax(sqrt(gc0 * gc0 + gc1 * gc1), R(1e-6));
          const R n0 = gc0 / nrm, n1 = gc1 / nrm;
          const R ndot = n0 * gs0 + n1 * gs1;
          fm = dmf * (gsD - (D == 0 ? n0 : n1) * ndot);
        }
      }
      if (D == 0) {
        const int o = j * (nx + 1) + i;
        if (cap_x) cap_x[o] = fc;
        if (ma_x) ma_x[o] = fm;
      } else {
        const int o = j * nx + i;
        if (cap_y) cap_y[o] = fc;
        if (ma_y) ma_y[o] = fm;
      }
    }
  }
}

}  // namespace surf
