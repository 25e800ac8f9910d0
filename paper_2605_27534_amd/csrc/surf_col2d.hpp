// surf_col2d.hpp -- the 2D transport step (substeps 1 and 2, the source, the
// equation of state and the reduction record) for the weighted flux form, as
// column-streaming waves.
//
// Work unit: one wave owns a strip of 64 consecutive columns, x0 - 3 .. x0 +
// 60 (lane L holds column x0 - 3 + L), and a chunk of TY rows y0 .. y0 + TY - 1.
// Lanes 3 .. 60 produce the strip's 58 output columns; the three lanes on
// each side are the halo that the advective stencil (upwind cell plus its
// limited slope) and the flux difference of substep 2 need.  The wave loads
// every row it reads up front (independent loads, many in flight) and then
// marches down the rows with a lag:
//   row s:   x-face advective fluxes (neighbour columns by wave-wide DPP
//            shifts), the y-face advective flux between rows s and s+1, the
//            advected state (F*, psi*), phi and delta, c* and Gamma*
//            (section 3.1, substep 1; section 2.6 for the carrier forms),
//            the weighted diffusion/confinement fluxes of the faces right of
//            and below s (section 3.2, read in the weighted form);
//   row s-1: the update with the delta-localised source, sigma(Gamma) and
//            the reduction terms (sections 2.3, 2.6).
// Every face flux is computed once (by the lane and row on its low side) and
// handed to the other side through a DPP shift or a register.
//
// Boundaries: walls and open sides mirror ghost values, periodic sides wrap;
// the advective flux through a wall is zero, through an open side it carries
// the interior value (accounted in the outflow budget), the diffusive and
// confinement fluxes through both are zero.  Waves whose strip and rows
// touch no side run a variant without any of this logic.  A workgroup holds
// four waves: four consecutive row chunks of one strip.
#pragma once
#include "surf_common.hpp"
#include "surf_kernels.hpp"

namespace surf {

constexpr int COL_OUT = 58;   // output columns per wave
constexpr int COL_WAVES = 4;  // waves per workgroup (consecutive row chunks)
constexpr int COL_LOOKAHEAD = 4;  // rows of loads in flight ahead of the arithmetic

template <typename R>
struct ColArgs {
  Grid g;
  Par<R> p;
  const R* chi;     // level set, explicit values everywhere
  const R* u[2];    // face velocities (x: [ny][nx+1], y: [ny+1][nx]) or nullptr
  const R* F;
  const R* psi;
  R* Fo;
  R* Po;
  R* sig;           // may be nullptr
  double* part;     // [workgroups][NPART]
  R dt;
  R area_dt;        // h dt: face length times the step
  int strips;       // ceil(nx / 58)
  int groups;       // ceil(chunks / 4): row-chunk groups per strip
  int nwg;          // strips * groups
  int per_xcd;      // ceil(nwg / 8)
};

// wave-wide lane shifts: from_right gives lane L the value of lane L + 1,
// from_left the value of lane L - 1; lanes without a source read 0
constexpr int DPP_WF_SL1 = 0x130, DPP_WF_SR1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float wshift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double wshift(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename R> __device__ __forceinline__ R from_right(R v) { return wshift<DPP_WF_SL1>(v); }
template <typename R> __device__ __forceinline__ R from_left(R v) { return wshift<DPP_WF_SR1>(v); }

// minmod(a, b) is the median of (a, b, 0): 0 for opposite signs, else the
// argument of smaller magnitude
template <typename R> __device__ __forceinline__ R mm(R a, R b) { return minmod<R>(a, b); }
template <> __device__ __forceinline__ float mm<float>(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}

// a / b given r = 1/b in FP32 (reciprocal-multiply), a true division in FP64
template <typename R> __device__ __forceinline__ R quot(R a, R b, R r) { return a * r; }
template <> __device__ __forceinline__ double quot<double>(double a, double b, double) { return a / b; }

// u times the BCG face value between cells x (low side) and xr (high side):
// the upwind cell plus (1 - |u| dt/h)/2 times its minmod slope; dl = x - (the
// cell below x), d = xr - x, dr = (the cell above xr) - xr
template <typename R>
__device__ __forceinline__ R bcg_face(R uf, R x, R xr, R dl, R d, R dr, R half_cfl) {
  const bool pos = uf > R(0);
  const R k = R(0.5) - fabs(uf) * half_cfl;
  const R m = mm<R>(pos ? dl : dr, d);
  return uf * ((pos ? x : xr) + (pos ? k : -k) * m);
}

template <typename R>
struct ColAcc {
  double sF, sP, sD, sSD, out;
  R usum, mxC, mnF, mnP;
  int nbad;
};

// One wave: strip x0, rows y0 .. y0 + TY - 1 (y0 < ny).  INT: the strip and
// every row it reads lie inside the box, away from all sides.
template <typename R, int TY, bool HU, bool BULK, bool INT>
__device__ __forceinline__ void col2d_wave(const ColArgs<R>& a, const int x0, const int y0,
                                           const int lane, ColAcc<R>& acc) {
  constexpr int NR3 = TY + 6;  // state rows y0-3 .. y0+TY+2
  constexpr int NR1 = TY + 2;  // rows of the advected state y0-1 .. y0+TY
  constexpr int NFY = TY + 3;  // y faces y0-1 .. y0+TY+1 (face j lies below row j)
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  const int nx = g.n[0], ny = g.n[1];
  const bool px = g.bc[0][0] == BC_PERIODIC, py = g.bc[1][0] == BC_PERIODIC;
  const bool ox_lo = g.bc[0][0] == BC_OPEN, ox_hi = g.bc[0][1] == BC_OPEN;
  const bool oy_lo = g.bc[1][0] == BC_OPEN, oy_hi = g.bc[1][1] == BC_OPEN;
  const R cfl = a.dt * p.inv_h, hcfl = R(0.5) * cfl;
  const R dcoef = p.Db * R(0.5) * p.inv_h * p.inv_h, scoef = p.Ds * R(0.5) * p.inv_h * p.inv_h;

  // ---- the lane's column
  const int xs = x0 - 3 + lane;
  int mx = xs, fxm = xs + 1;
  bool gcell_x = false, xf_lo = false, xf_hi = false, xf_out = false;
  if constexpr (!INT) {
    mx = map_axis(xs, nx, g.bc[0][0], g.bc[0][1]);
    gcell_x = !px && (xs < 0 || xs >= nx);
    const int fx = xs + 1;  // the lane's right face
    xf_lo = !px && fx == 0;
    xf_hi = !px && fx == nx;
    xf_out = !px && (fx < 0 || fx > nx);
    if (px) fxm = ((fx % nx) + nx) % nx;
  }
  const bool out_lane = lane >= 3 && lane < 3 + COL_OUT && (INT || xs < nx);

  // ---- loads, in the order of use: group k holds state row k (F, psi),
  // y face k-3 and level-set / x-face row k-4; iteration i consumes group i,
  // and group i + LOOKAHEAD is issued before iteration i computes
  R rF[NR3], rP[NR3], rC[NR1], rUx[NR1], rUy[NFY];
  auto load_group = [&](const int k) {
    if (k < NR3) {
      const int my = INT ? y0 - 3 + k : map_axis(y0 - 3 + k, ny, g.bc[1][0], g.bc[1][1]);
      const long long row = (long long)nx * my;
      rF[k] = BULK ? a.F[row + mx] : R(0);
      rP[k] = a.psi[row + mx];
    }
    if (k >= 3 && k - 3 < NFY) {
      const int i = k - 3;
      rUy[i] = R(0);
      if (HU) {
        int j = y0 - 1 + i;
        bool ok = true;
        if (!INT) {
          ok = !gcell_x;
          if (py) j = ((j % ny) + ny) % ny;
          else ok = ok && j >= 0 && j <= ny;
        }
        if (ok) rUy[i] = a.u[1][(long long)nx * j + mx];
      }
    }
    if (k >= 4 && k - 4 < NR1) {
      const int i = k - 4;
      const int ys = y0 - 1 + i;
      const int my = INT ? ys : map_axis(ys, ny, g.bc[1][0], g.bc[1][1]);
      rC[i] = a.chi[(long long)nx * my + mx];
      rUx[i] = R(0);
      if (HU) {
        const bool ok = INT || (!xf_out && !(!py && (ys < 0 || ys >= ny)));
        if (ok) rUx[i] = a.u[0][(long long)(nx + 1) * my + fxm];
      }
    }
  };
#pragma unroll
  for (int k = 0; k < 3 + COL_LOOKAHEAD && k < NR3; ++k) load_group(k);

  // ---- values carried from row to row
  R dF2 = rF[1] - rF[0], dP2 = rP[1] - rP[0];  // y differences below rows s-1 and s
  R dF1 = rF[2] - rF[1], dP1 = rP[2] - rP[1];
  R gyF = R(0), gyP = R(0);    // advective flux through face s (below row s)
  R pGyF = R(0), pGyP = R(0);  // advective flux through face s-1
  R pFs = R(0), pPs = R(0), pC = R(0), pPh = R(0), pDe = R(0), pIF = R(1), pIP = R(1);
  R pG = R(0);
  R pAxF = R(0), pAxP = R(0);  // x part of the weighted divergence of row s-1
  R pWyF = R(0), pWyP = R(0);  // weighted flux through face s-1
  R pFxF = R(0), pFxP = R(0), pFxLF = R(0), pFxLP = R(0);  // advective x fluxes of row s-1
  R pUx = R(0), pUxL = R(0);

#pragma unroll
  for (int i = 3; i < NR3; ++i) {
    if (i + COL_LOOKAHEAD < NR3) load_group(i + COL_LOOKAHEAD);
    // keep the issue order: this iteration's loads, then its arithmetic
    __builtin_amdgcn_sched_barrier(0);
    // ---- advective flux through face j = s+1 between rows s = y0-5+i (index
    // i-2) and s+1 (index i-1)
    const int j = y0 - 4 + i;
    const R dF0 = rF[i] - rF[i - 1], dP0 = rP[i] - rP[i - 1];
    R nyF = R(0), nyP = R(0);
    if (HU) {
      const R uf = rUy[i - 3];
      nyF = BULK ? bcg_face<R>(uf, rF[i - 2], rF[i - 1], dF2, dF1, dF0, hcfl) : R(0);
      nyP = bcg_face<R>(uf, rP[i - 2], rP[i - 1], dP2, dP1, dP0, hcfl);
      if (!INT) {
        if (!py && j == 0) {
          nyF = (BULK && oy_lo) ? uf * rF[i - 1] : R(0);
          nyP = oy_lo ? uf * rP[i - 1] : R(0);
        } else if (!py && j == ny) {
          nyF = (BULK && oy_hi) ? uf * rF[i - 2] : R(0);
          nyP = oy_hi ? uf * rP[i - 2] : R(0);
        } else if (!py && (j < 0 || j > ny)) {
          nyF = R(0);
          nyP = R(0);
        }
        if (gcell_x) { nyF = R(0); nyP = R(0); }
      }
    }
    dF2 = dF1; dP2 = dP1;
    dF1 = dF0; dP1 = dP0;

    if (i >= 4) {
      // ---- row s: advected state, phase field, c*, Gamma*
      const int s = y0 - 5 + i;
      const int k1 = i - 4;
      const bool grow = !INT && !py && (s < 0 || s >= ny);
      const R xF = rF[i - 2], xP = rP[i - 2];
      R Fs = xF, Ps = xP;
      R fxF = R(0), fxP = R(0), fxLF = R(0), fxLP = R(0);
      const R ux = rUx[k1];
      if (HU) {
        // the right-face flux of this lane's cell; the left face is the
        // right face of the lane to the left (every shift runs on all lanes)
        const R xFr = from_right(xF), xPr = from_right(xP);
        const R eF = xFr - xF, eP = xPr - xP;
        const R eFl = from_left(eF), eFr = from_right(eF);
        const R ePl = from_left(eP), ePr = from_right(eP);
        fxF = BULK ? bcg_face<R>(ux, xF, xFr, eFl, eF, eFr, hcfl) : R(0);
        fxP = bcg_face<R>(ux, xP, xPr, ePl, eP, ePr, hcfl);
        if (!INT) {
          if (xf_lo) {
            fxF = (BULK && ox_lo) ? ux * xFr : R(0);
            fxP = ox_lo ? ux * xPr : R(0);
          }
          if (xf_hi) {
            fxF = (BULK && ox_hi) ? ux * xF : R(0);
            fxP = ox_hi ? ux * xP : R(0);
          }
          if (xf_out || grow) { fxF = R(0); fxP = R(0); }
        }
        fxLF = from_left(fxF);
        fxLP = from_left(fxP);
        Fs = xF - cfl * ((fxF - fxLF) + (nyF - gyF));
        Ps = xP - cfl * ((fxP - fxLP) + (nyP - gyP));
      }
      if (!INT && (gcell_x || grow)) { Fs = R(0); Ps = R(0); }
      if (!BULK) Fs = R(0);
      R ph, om, de;
      phase<R>(rC[k1], p, ph, om, de);
      const R dnF = ph + p.eta, dnP = de + p.eta_eps;
      const R iF = rrcp<R>(dnF), iP = rrcp<R>(dnP);
      const R cs = quot<R>(Fs, dnF, iF);
      const R Gs = quot<R>(Ps, dnP, iP);
      // weighted fluxes through the right face of this lane and face s
      const R phr = from_right(ph), der = from_right(de);
      const R csr = from_right(cs), Gsr = from_right(Gs);
      R wxF = (ph + phr) * (csr - cs), wxP = (de + der) * (Gsr - Gs);
      if (!INT && (xf_lo || xf_hi)) { wxF = R(0); wxP = R(0); }
      const R axF = wxF - from_left(wxF), axP = wxP - from_left(wxP);
      R wyF = (pPh + ph) * (cs - pC), wyP = (pDe + de) * (Gs - pG);
      if (!INT && !py && (s == 0 || s == ny)) { wyF = R(0); wyP = R(0); }
      const R uxL = from_left(ux);

      if (i >= 6) {
        // ---- row o = s-1: update, source, sigma, reduction terms
        const int o = s - 1;
        if (out_lane && (INT || o < ny)) {
          const R divF = dcoef * (pAxF + (wyF - pWyF));
          const R divP = scoef * (pAxP + (wyP - pWyP));
          R q = R(0);
          if (BULK)
            q = p.kin == KIN_LANGMUIR ? p.ka * pC * (p.ginf * pDe - pPs) - p.kd * pPs
                                      : p.ka * pC * p.ginf * pDe - p.kd * pPs;
          const R Fn = BULK ? pFs + a.dt * (divF - q) : R(0);
          const R Pn = pPs + a.dt * (divP + q);
          const R sg = eos<R>(quot<R>(Pn, pDe + p.eta_eps, pIP), p);
          const long long row = (long long)nx * o;
          if (BULK) a.Fo[row + xs] = Fn;
          a.Po[row + xs] = Pn;
          if (a.sig) a.sig[row + xs] = sg;
          acc.sF += (double)Fn;
          acc.sP += (double)Pn;
          acc.sD += (double)pDe;
          acc.sSD += (double)(sg * pDe);
          if (BULK) {
            acc.mxC = fmax(acc.mxC, quot<R>(Fn, pPh + p.eta, pIF));
            acc.mnF = fmin(acc.mnF, Fn);
          }
          acc.mnP = fmin(acc.mnP, Pn);
          acc.nbad += isfinite(Pn + sg + Fn) ? 0 : 1;
          if (HU) {
            // cell-mean velocities (the literal upper face of a periodic axis)
            R uxh = pUx, uyl = rUy[i - 5], uyh = rUy[i - 4];
            if (!INT) {
              if (px && xs == nx - 1) uxh = a.u[0][(long long)(nx + 1) * o + nx];
              if (py && o == ny - 1) uyh = a.u[1][(long long)nx * ny + xs];
            }
            acc.usum = fmax(acc.usum, fabs(R(0.5) * (pUxL + uxh)) + fabs(R(0.5) * (uyl + uyh)));
            if (!INT) {
              // open-side budget of the faces of this cell
              if (!px && xs == 0 && ox_lo) acc.out -= (double)(a.area_dt * (pFxLF + pFxLP));
              if (!px && xs == nx - 1 && ox_hi) acc.out += (double)(a.area_dt * (pFxF + pFxP));
              if (!py && o == 0 && oy_lo) acc.out -= (double)(a.area_dt * (pGyF + pGyP));
              if (!py && o == ny - 1 && oy_hi) acc.out += (double)(a.area_dt * (gyF + gyP));
            }
          }
        }
      }
      pFs = Fs; pPs = Ps; pC = cs; pG = Gs; pPh = ph; pDe = de; pIF = iF; pIP = iP;
      pAxF = axF; pAxP = axP; pWyF = wyF; pWyP = wyP;
      pFxF = fxF; pFxP = fxP; pFxLF = fxLF; pFxLP = fxLP;
      pUx = ux; pUxL = uxL;
    }
    pGyF = gyF; pGyP = gyP;
    gyF = nyF; gyP = nyP;
  }
}

template <typename R, int TY, bool HU, bool BULK>
__global__ void __launch_bounds__(64 * COL_WAVES) k_col2d(ColArgs<R> a) {
  const int b = blockIdx.x;
  const int wg = (b & 7) * a.per_xcd + (b >> 3);  // banded over the XCDs
  if (wg >= a.nwg) return;  // uniform per workgroup: no barrier is skipped by part of it
  const int nx = a.g.n[0], ny = a.g.n[1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sx = wg / a.groups, cg = wg - sx * a.groups;
  const int x0 = sx * COL_OUT, y0 = (cg * COL_WAVES + wv) * TY;
  ColAcc<R> acc{0.0, 0.0, 0.0, 0.0, 0.0, R(0), R(-INFINITY), R(INFINITY), R(INFINITY), 0};
  if (y0 < ny) {  // chunks past the last row only join the reduction
    const bool interior = x0 >= 3 && x0 + 62 <= nx && y0 >= 3 && y0 + TY + 3 <= ny;
    if (interior) col2d_wave<R, TY, HU, BULK, true>(a, x0, y0, lane, acc);
    else col2d_wave<R, TY, HU, BULK, false>(a, x0, y0, lane, acc);
  }
  double v[NPART];
  v[P_SUM_F] = acc.sF;
  v[P_SUM_PSI] = acc.sP;
  v[P_SUM_DELTA] = acc.sD;
  v[P_SUM_SIGDELTA] = acc.sSD;
  v[P_OUTFLOW] = acc.out;
  v[P_MAX_USUM] = (double)acc.usum;
  v[P_MAX_C] = (double)acc.mxC;
  v[P_MIN_F] = (double)acc.mnF;
  v[P_MIN_PSI] = (double)acc.mnP;
  v[P_NBAD] = (double)acc.nbad;
  block_partials<R, 64 * COL_WAVES>(v, a.part + (long long)wg * NPART);
}

}  // namespace surf
