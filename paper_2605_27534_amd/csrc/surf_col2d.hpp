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
  const double* state;  // running state: the time keys the FP32 stochastic rounding
  R dt;
  R area_dt;        // h dt: face length times the step
  double r0;        // axisymmetric: the radius of the low x side
  int axi;          // batched form: 1 for an instance on axisymmetric rings
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

// Plain global access: a 64-bit scalar base and a 32-bit byte offset.  Every
// index passed here is mapped into its array by the caller.
template <typename R>
__device__ __forceinline__ R gld(const R* base, int voff, int soff) {
  return *(const R*)((const char*)base + (unsigned)(voff + soff));
}
template <typename R>
__device__ __forceinline__ void gst(R v, R* base, int voff, int soff) {
  *(R*)((char*)base + (unsigned)(voff + soff)) = v;
}

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

// The face value of the substep-1 variants: the slope limiter LIM (0 minmod,
// 1 MC), plus tl or tr, the transverse term of the upwind cell (low or high
// side), when the unsplit predictor is on.
template <typename R, int LIM>
__device__ __forceinline__ R bcg_face_v(R uf, R x, R xr, R dl, R d, R dr, R half_cfl, R tl,
                                        R tr) {
  const bool pos = uf > R(0);
  const R k = R(0.5) - fabs(uf) * half_cfl;
  const R m = LIM == 1 ? mc<R>(pos ? dl : dr, d) : mm<R>(pos ? dl : dr, d);
  return uf * ((pos ? x : xr) + (pos ? k : -k) * m + (pos ? tl : tr));
}

template <typename R>
struct ColAcc {
  double sF, sP, sD, sSD, out;
  R usum, mxC, mnF, mnP;
  int nbad;
};

// One wave: strip x0, rows y0 .. y0 + TY - 1 (y0 < ny).  IX: every column
// the strip reads lies inside the box away from the x sides; IY: the same
// for the rows and the y sides.
// LIM and TR select the substep-1 variants (2D Cartesian only): the slope
// limiter and the transverse term of the unsplit BCG predictor, which needs
// the x-face velocities of one more row below and above the advected rows.
template <typename R, int TY, bool HU, bool BULK, bool IX, bool IY, bool AXI, int LIM = 0,
          bool TR = false>
__device__ __forceinline__ void col2d_wave(const ColArgs<R>& a, const int x0, const int y0,
                                           const int lane, ColAcc<R>& acc, const unsigned tkey) {
  constexpr bool SRND = sizeof(R) == 4;  // FP32: stochastically rounded state
  constexpr bool VAR = LIM != 0 || TR;
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
  if constexpr (!IX) {
    mx = map_axis(xs, nx, g.bc[0][0], g.bc[0][1]);
    gcell_x = !px && (xs < 0 || xs >= nx);
    const int fx = xs + 1;  // the lane's right face
    xf_lo = !px && fx == 0;
    xf_hi = !px && fx == nx;
    xf_out = !px && (fx < 0 || fx > nx);
    // the face column read by the lane, always inside the face array (the
    // value of a face beyond a side is discarded below)
    fxm = px ? ((fx % nx) + nx) % nx : (xf_out ? 0 : fx);
  }
  const bool out_lane = lane >= 3 && lane < 3 + COL_OUT && (IX || xs < nx);
  // lane constants of the x sides
  const bool x_side = xf_lo || xf_hi;
  const bool x_lo_open = xf_lo && ox_lo, x_hi_open = xf_hi && ox_hi;
  double wlo = (!IX && !px && xs == 0 && ox_lo) ? -1.0 : 0.0;
  double whi = (!IX && !px && xs == nx - 1 && ox_hi) ? 1.0 : 0.0;
  // axisymmetric rings (Appendix B): the lane's column is the ring between
  // r_lo and r_hi (the mapped column for ghost lanes, whose values are never
  // used); radial face fluxes enter its balance with r_face / r_mid, its
  // volume is 2 pi r_mid h^2 (the reduction counts 2 pi r_mid per cell, the
  // finalize multiplies by h^2) and its faces' areas 2 pi r h
  R a_lo = R(1), a_hi = R(1);
  double w_mid = 1.0;
  if constexpr (AXI) {
    const double rl = a.r0 + (double)mx * (double)p.h, rh = rl + (double)p.h;
    const double rm = rl + 0.5 * (double)p.h;
    a_lo = (R)(rl / rm);
    a_hi = (R)(rh / rm);
    w_mid = 2.0 * M_PI * rm;
    wlo *= 2.0 * M_PI * rl;
    whi *= 2.0 * M_PI * rh;
  }

  // ---- loads, in the order of use: group k holds state row k (F, psi),
  // y face k-3 and level-set / x-face row k-4; iteration i consumes group i,
  // and group i + LOOKAHEAD is issued before iteration i computes
  constexpr int ES = (int)sizeof(R);
  const R* const bF = a.F;
  const R* const bP = a.psi;
  const R* const bC = a.chi;
  const R* const bUx = a.u[0];
  const R* const bUy = a.u[1];
  const int vmx = mx * ES, vfx = fxm * ES;  // per-lane byte offsets
  // TR: x-face velocities of rows y0-2 .. y0+TY+1 (rUxT[m] is row y0-2+m,
  // loaded with group m+2); else rows y0-1 .. y0+TY in rUx
  constexpr int NUX = TR ? TY + 4 : 1;
  R rF[NR3], rP[NR3], rC[NR1], rUx[TR ? 1 : NR1], rUy[NFY], rUxT[NUX];
  auto load_group = [&](const int k) {
    if (k < NR3) {
      const int my = IY ? y0 - 3 + k : map_axis(y0 - 3 + k, ny, g.bc[1][0], g.bc[1][1]);
      const int row = nx * my * ES;
      rF[k] = BULK ? gld<R>(bF, vmx, row) : R(0);
      rP[k] = gld<R>(bP, vmx, row);
    }
    if (k >= 3 && k - 3 < NFY) {
      const int i = k - 3;
      rUy[i] = R(0);
      if (HU) {
        int j = y0 - 1 + i;
        bool ok = IX || !gcell_x;
        if (!IY) {
          if (py) {
            while (j < 0) j += ny;
            while (j >= ny) j -= ny;
          } else if (j < 0 || j > ny) {
            j = 0;
            ok = false;
          }
        }
        const R v = gld<R>(bUy, vmx, nx * j * ES);
        rUy[i] = ok ? v : R(0);
      }
    }
    if (k >= 4 && k - 4 < NR1) {
      const int i = k - 4;
      const int ys = y0 - 1 + i;
      const int my = IY ? ys : map_axis(ys, ny, g.bc[1][0], g.bc[1][1]);
      rC[i] = gld<R>(bC, vmx, nx * my * ES);
      if constexpr (!TR) {
        rUx[i] = R(0);
        if (HU) {
          const bool ok = (IX || !xf_out) && (IY || py || (ys >= 0 && ys < ny));
          const R v = gld<R>(bUx, vfx, (nx + 1) * my * ES);
          rUx[i] = ok ? v : R(0);
        }
      }
    }
    if constexpr (TR) {
      if (k >= 2 && k - 2 < NUX) {
        const int m = k - 2;
        const int ys = y0 - 2 + m;
        const int my = IY ? ys : map_axis(ys, ny, g.bc[1][0], g.bc[1][1]);
        const bool ok = (IX || !xf_out) && (IY || py || (ys >= 0 && ys < ny));
        const R v = gld<R>(bUx, vfx, (nx + 1) * my * ES);
        rUxT[m] = ok ? v : R(0);
      }
    }
  };
#pragma unroll
  for (int k = 0; k < 3 + COL_LOOKAHEAD && k < NR3; ++k) load_group(k);

  R* const bFo = a.Fo;
  R* const bPo = a.Po;
  R* const bS = a.sig;
  const int vxs = xs * ES;
  const R kl = p.kin == KIN_LANGMUIR ? R(1) : R(0);

  // ---- values carried from row to row
  R dF2 = rF[1] - rF[0], dP2 = rP[1] - rP[0];  // y differences below rows s-1 and s
  R dF1 = rF[2] - rF[1], dP1 = rP[2] - rP[1];
  R gyF = R(0), gyP = R(0);    // advective flux through face s (below row s)
  R pGyF = R(0), pGyP = R(0);  // advective flux through face s-1
  R pFs = R(0), pPs = R(0), pC = R(0), pPh = R(0), pDe = R(0), pIF = R(1), pIP = R(1);
  R pG = R(0);
  // FP32: the old state and the advective increment of row s-1, added to
  // the substep-2 increment in one stochastically rounded update
  R pXF = R(0), pXP = R(0), pAF = R(0), pAP = R(0);
  R pAxF = R(0), pAxP = R(0);  // x part of the weighted divergence of row s-1
  R pWyF = R(0), pWyP = R(0);  // weighted flux through face s-1
  R pFxF = R(0), pFxP = R(0), pFxLF = R(0), pFxLP = R(0);  // advective x fluxes of row s-1
  R pUx = R(0), pUxL = R(0);
  // TR: the transverse term of the y faces' upwind cells in the row below
  // the current face (carried from the previous iteration)
  R tyF = R(0), tyP = R(0);
  // the y-face transverse term of row r (rF / rP index kr, x-face velocities
  // rUxT[mr]): minus dt/2h times the cell-mean x velocity times the upwind
  // x difference
  auto ty_row = [&](const int kr, const int mr, R& tF, R& tP) {
    const R uc = R(0.5) * (from_left(rUxT[mr]) + rUxT[mr]);
    const R eF = from_right(rF[kr]) - rF[kr], eP = from_right(rP[kr]) - rP[kr];
    const R lF = from_left(eF), lP = from_left(eP);
    const bool up = uc > R(0);
    tF = BULK ? -hcfl * uc * (up ? lF : eF) : R(0);
    tP = -hcfl * uc * (up ? lP : eP);
  };

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
      if constexpr (VAR) {
        // rows s (index i-2, x velocities rUxT[i-3]) and s+1 (i-1, rUxT[i-2])
        R tF1 = R(0), tP1 = R(0);
        if constexpr (TR) {
          if (i == 3) ty_row(i - 2, i - 3, tyF, tyP);
          ty_row(i - 1, i - 2, tF1, tP1);
        }
        nyF = BULK ? bcg_face_v<R, LIM>(uf, rF[i - 2], rF[i - 1], dF2, dF1, dF0, hcfl, tyF, tF1)
                   : R(0);
        nyP = bcg_face_v<R, LIM>(uf, rP[i - 2], rP[i - 1], dP2, dP1, dP0, hcfl, tyP, tP1);
        tyF = tF1;
        tyP = tP1;
      } else {
        nyF = BULK ? bcg_face<R>(uf, rF[i - 2], rF[i - 1], dF2, dF1, dF0, hcfl) : R(0);
        nyP = bcg_face<R>(uf, rP[i - 2], rP[i - 1], dP2, dP1, dP0, hcfl);
      }
      if (!IY) {
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
      }
      if (!IX) {
        nyF = gcell_x ? R(0) : nyF;
        nyP = gcell_x ? R(0) : nyP;
      }
    }
    dF2 = dF1; dP2 = dP1;
    dF1 = dF0; dP1 = dP0;

    if (i >= 4) {
      // ---- row s: advected state, phase field, c*, Gamma*
      const int s = y0 - 5 + i;
      const int k1 = i - 4;
      const bool grow = !IY && !py && (s < 0 || s >= ny);
      const R xF = rF[i - 2], xP = rP[i - 2];
      R Fs = xF, Ps = xP;
      R aF = R(0), aP = R(0);  // FP32: the advective increments
      R fxF = R(0), fxP = R(0), fxLF = R(0), fxLP = R(0);
      R ux;
      if constexpr (TR) ux = rUxT[k1 + 1];
      else ux = rUx[k1];
      if (HU) {
        // the right-face flux of this lane's cell; the left face is the
        // right face of the lane to the left (every shift runs on all lanes)
        const R xFr = from_right(xF), xPr = from_right(xP);
        const R eF = xFr - xF, eP = xPr - xP;
        const R eFl = from_left(eF), eFr = from_right(eF);
        const R ePl = from_left(eP), ePr = from_right(eP);
        if constexpr (VAR) {
          // the transverse term of this lane's cell from its own column:
          // minus dt/2h times the mean of its y faces s and s+1 times the
          // upwind y difference; the right neighbour's by one shift
          R txF = R(0), txP = R(0);
          if constexpr (TR) {
            const R vc = R(0.5) * (rUy[i - 4] + rUy[i - 3]);
            const bool up = vc > R(0);
            txF = BULK ? -hcfl * vc * (up ? rF[i - 2] - rF[i - 3] : rF[i - 1] - rF[i - 2]) : R(0);
            txP = -hcfl * vc * (up ? rP[i - 2] - rP[i - 3] : rP[i - 1] - rP[i - 2]);
          }
          const R txFr = TR ? from_right(txF) : R(0), txPr = TR ? from_right(txP) : R(0);
          fxF = BULK ? bcg_face_v<R, LIM>(ux, xF, xFr, eFl, eF, eFr, hcfl, txF, txFr) : R(0);
          fxP = bcg_face_v<R, LIM>(ux, xP, xPr, ePl, eP, ePr, hcfl, txP, txPr);
        } else {
          fxF = BULK ? bcg_face<R>(ux, xF, xFr, eFl, eF, eFr, hcfl) : R(0);
          fxP = bcg_face<R>(ux, xP, xPr, ePl, eP, ePr, hcfl);
        }
        if (!IX || !IY) {
          // lane-constant selects: an open side carries the interior cell,
          // a wall nothing, faces beyond a side and rows outside nothing
          const R oF = x_lo_open ? ux * xFr : (x_hi_open ? ux * xF : R(0));
          const R oP = x_lo_open ? ux * xPr : (x_hi_open ? ux * xP : R(0));
          fxF = x_side ? (BULK ? oF : R(0)) : fxF;
          fxP = x_side ? oP : fxP;
          fxF = (xf_out || grow) ? R(0) : fxF;
          fxP = (xf_out || grow) ? R(0) : fxP;
        }
        fxLF = from_left(fxF);
        fxLP = from_left(fxP);
        if constexpr (SRND) {
          if constexpr (AXI) {
            aF = -cfl * ((a_hi * fxF - a_lo * fxLF) + (nyF - gyF));
            aP = -cfl * ((a_hi * fxP - a_lo * fxLP) + (nyP - gyP));
          } else {
            aF = -cfl * ((fxF - fxLF) + (nyF - gyF));
            aP = -cfl * ((fxP - fxLP) + (nyP - gyP));
          }
          Fs = xF + aF;
          Ps = xP + aP;
        } else if constexpr (AXI) {
          Fs = xF - cfl * ((a_hi * fxF - a_lo * fxLF) + (nyF - gyF));
          Ps = xP - cfl * ((a_hi * fxP - a_lo * fxLP) + (nyP - gyP));
        } else {
          Fs = xF - cfl * ((fxF - fxLF) + (nyF - gyF));
          Ps = xP - cfl * ((fxP - fxLP) + (nyP - gyP));
        }
      }
      if (!IX || !IY) {
        const bool ghost = gcell_x || grow;
        Fs = ghost ? R(0) : Fs;
        Ps = ghost ? R(0) : Ps;
      }
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
      if (!IX) {
        wxF = x_side ? R(0) : wxF;
        wxP = x_side ? R(0) : wxP;
      }
      R axF, axP;
      if constexpr (AXI) {
        axF = a_hi * wxF - a_lo * from_left(wxF);
        axP = a_hi * wxP - a_lo * from_left(wxP);
      } else {
        axF = wxF - from_left(wxF);
        axP = wxP - from_left(wxP);
      }
      R wyF = (pPh + ph) * (cs - pC), wyP = (pDe + de) * (Gs - pG);
      if (!IY && !py && (s == 0 || s == ny)) { wyF = R(0); wyP = R(0); }
      const R uxL = from_left(ux);

      if (i >= 6) {
        // ---- row o = s-1: update, source, sigma, reduction terms
        const int o = s - 1;
        if (out_lane && (IY || o < ny)) {
          const R divF = dcoef * (pAxF + (wyF - pWyF));
          const R divP = scoef * (pAxP + (wyP - pWyP));
          // Langmuir k_a c (Gamma_inf delta - psi) - k_d psi; Henry drops the
          // psi in the adsorption term (kl = 0)
          const R q = BULK ? p.ka * pC * (p.ginf * pDe - kl * pPs) - p.kd * pPs : R(0);
          R Fn, Pn;
          if constexpr (SRND) {
            // one random word per cell and step: 16 bits for each field
            const unsigned rk = fmix32((unsigned)(nx * o + xs) ^ tkey);
            Fn = BULK ? upd<R>(pXF, pAF + a.dt * (divF - q), rk) : R(0);
            Pn = upd<R>(pXP, pAP + a.dt * (divP + q), rk >> 16);
          } else {
            Fn = BULK ? pFs + a.dt * (divF - q) : R(0);
            Pn = pPs + a.dt * (divP + q);
          }
          const R sg = eos<R>(quot<R>(Pn, pDe + p.eta_eps, pIP), p);
          const int row = nx * o * ES;
          if (BULK) gst(Fn, bFo, vxs, row);
          gst(Pn, bPo, vxs, row);
          if (a.sig) gst(sg, bS, vxs, row);
          if constexpr (AXI) {
            acc.sF += w_mid * (double)Fn;
            acc.sP += w_mid * (double)Pn;
            acc.sD += w_mid * (double)pDe;
            acc.sSD += w_mid * (double)(sg * pDe);
          } else {
            acc.sF += (double)Fn;
            acc.sP += (double)Pn;
            acc.sD += (double)pDe;
            acc.sSD += (double)(sg * pDe);
          }
          if (BULK) {
            acc.mxC = fmax(acc.mxC, quot<R>(Fn, pPh + p.eta, pIF));
            acc.mnF = fmin(acc.mnF, Fn);
          }
          acc.mnP = fmin(acc.mnP, Pn);
          acc.nbad += isfinite(Pn + sg + Fn) ? 0 : 1;
          if (HU) {
            // cell-mean velocities (on a periodic axis the upper face of the
            // last cell is face 0, as in the fluxes)
            R uxh = pUx, uyl = rUy[i - 5], uyh = rUy[i - 4];
            if constexpr (AXI)
              acc.usum = fmax(acc.usum, fabs(R(0.5) * (a_lo * pUxL + a_hi * uxh)) +
                                            fabs(R(0.5) * (uyl + uyh)));
            else
              acc.usum = fmax(acc.usum, fabs(R(0.5) * (pUxL + uxh)) + fabs(R(0.5) * (uyl + uyh)));
            // open-side budget of the faces of this cell (lane weights
            // -1 / 0 / +1 for the x sides, uniform branches for the y sides)
            if (!IX)
              acc.out += wlo * (double)(a.area_dt * (pFxLF + pFxLP)) +
                         whi * (double)(a.area_dt * (pFxF + pFxP));
            if (!IY) {
              if (!py && o == 0 && oy_lo) acc.out -= w_mid * (double)(a.area_dt * (pGyF + pGyP));
              if (!py && o == ny - 1 && oy_hi) acc.out += w_mid * (double)(a.area_dt * (gyF + gyP));
            }
          }
        }
      }
      pFs = Fs; pPs = Ps; pC = cs; pG = Gs; pPh = ph; pDe = de; pIF = iF; pIP = iP;
      if constexpr (SRND) { pXF = xF; pXP = xP; pAF = aF; pAP = aP; }
      pAxF = axF; pAxP = axP; pWyF = wyF; pWyP = wyP;
      pFxF = fxF; pFxP = fxP; pFxLF = fxLF; pFxLP = fxLP;
      pUx = ux; pUxL = uxL;
    }
    pGyF = gyF; pGyP = gyP;
    gyF = nyF; gyP = nyP;
  }
}

template <typename R, int TY, bool HU, bool BULK, bool AXI = false, int LIM = 0, bool TR = false>
__global__ void __launch_bounds__(64 * COL_WAVES) k_col2d(ColArgs<R> a) {
  const int b = blockIdx.x;
  const int wg = (b & 7) * a.per_xcd + (b >> 3);  // banded over the XCDs
  if (wg >= a.nwg) return;  // uniform per workgroup: no barrier is skipped by part of it
  const int nx = a.g.n[0], ny = a.g.n[1];
  // the wave index is uniform over the wave: say so, so that row offsets
  // stay in scalar registers
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sx = wg / a.groups, cg = wg - sx * a.groups;
  const int x0 = sx * COL_OUT, y0 = (cg * COL_WAVES + wv) * TY;
  ColAcc<R> acc{0.0, 0.0, 0.0, 0.0, 0.0, R(0), R(-INFINITY), R(INFINITY), R(INFINITY), 0};
  const unsigned tk = sizeof(R) == 4 ? step_key(a.state[S_TIME]) : 0u;
  if (y0 < ny) {  // chunks past the last row only join the reduction
    const bool ix = x0 >= 3 && x0 + 62 <= nx, iy = y0 >= 3 && y0 + TY + 3 <= ny;
    if (ix && iy) col2d_wave<R, TY, HU, BULK, true, true, AXI, LIM, TR>(a, x0, y0, lane, acc, tk);
    else if (iy) col2d_wave<R, TY, HU, BULK, false, true, AXI, LIM, TR>(a, x0, y0, lane, acc, tk);
    else if (ix) col2d_wave<R, TY, HU, BULK, true, false, AXI, LIM, TR>(a, x0, y0, lane, acc, tk);
    else col2d_wave<R, TY, HU, BULK, false, false, AXI, LIM, TR>(a, x0, y0, lane, acc, tk);
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

// Batched form on the column-streaming transport: one persistent launch over
// the flattened work list of every weighted-form instance of a batch, one
// entry per workgroup of that instance's single-problem launch (a strip and
// a group of COL_WAVES row chunks of TY rows).  inst[i] holds instance i's
// arguments for parity 0 (reading F, psi and writing Fo, Po); parity 1
// swaps the two buffers.  Entry (i, w) leaves its record in
// part[first[i] + w], so each instance's records are contiguous and in the
// order of the single-problem launch.  The entries are dealt to the eight
// XCDs in contiguous bands (workgroup b runs on XCD b mod 8), so that the
// vertically adjacent chunks of a strip, which share halo rows, meet in one
// L2.  The grid is a multiple of 8.  RINGS: the instance for batches that
// hold instances on axisymmetric rings (Appendix B), which run the ring
// variant of the column waves; Cartesian-only batches keep the kernel
// without it.
template <typename R, int TY, bool RINGS = false>
__global__ void __launch_bounds__(64 * COL_WAVES) k_batch_col2d(
    const ColArgs<R>* __restrict__ inst, const int2* __restrict__ queue, int nqueue,
    const int* __restrict__ first, int parity, double* __restrict__ part) {
  const int b = blockIdx.x;
  const int per_xcd = (nqueue + 7) / 8;
  const int stride = gridDim.x >> 3;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int k = b >> 3; k < per_xcd; k += stride) {
    const int q = (b & 7) * per_xcd + k;
    if (q >= nqueue) break;  // uniform over the workgroup; later k only grow
    const int2 e = queue[q];
    ColArgs<R> a = inst[e.x];
    if (parity) {
      const R* f = a.F;
      a.F = a.Fo;
      a.Fo = (R*)f;
      const R* ps = a.psi;
      a.psi = a.Po;
      a.Po = (R*)ps;
    }
    const int wg = e.y;
    const int nx = a.g.n[0], ny = a.g.n[1];
    const int sx = wg / a.groups, cg = wg - sx * a.groups;
    const int x0 = sx * COL_OUT, y0 = (cg * COL_WAVES + wv) * TY;
    ColAcc<R> acc{0.0, 0.0, 0.0, 0.0, 0.0, R(0), R(-INFINITY), R(INFINITY), R(INFINITY), 0};
    const unsigned tk = sizeof(R) == 4 ? step_key(a.state[S_TIME]) : 0u;
    if (y0 < ny) {
      const bool ix = x0 >= 3 && x0 + 62 <= nx, iy = y0 >= 3 && y0 + TY + 3 <= ny;
      if (RINGS && a.axi) {
        if (a.p.bulk) {
          if (ix && iy) col2d_wave<R, TY, false, true, true, true, true>(a, x0, y0, lane, acc, tk);
          else if (iy) col2d_wave<R, TY, false, true, false, true, true>(a, x0, y0, lane, acc, tk);
          else if (ix) col2d_wave<R, TY, false, true, true, false, true>(a, x0, y0, lane, acc, tk);
          else col2d_wave<R, TY, false, true, false, false, true>(a, x0, y0, lane, acc, tk);
        } else {
          if (ix && iy) col2d_wave<R, TY, false, false, true, true, true>(a, x0, y0, lane, acc, tk);
          else if (iy) col2d_wave<R, TY, false, false, false, true, true>(a, x0, y0, lane, acc, tk);
          else if (ix) col2d_wave<R, TY, false, false, true, false, true>(a, x0, y0, lane, acc, tk);
          else col2d_wave<R, TY, false, false, false, false, true>(a, x0, y0, lane, acc, tk);
        }
      } else if (a.p.bulk) {
        if (ix && iy) col2d_wave<R, TY, false, true, true, true, false>(a, x0, y0, lane, acc, tk);
        else if (iy) col2d_wave<R, TY, false, true, false, true, false>(a, x0, y0, lane, acc, tk);
        else if (ix) col2d_wave<R, TY, false, true, true, false, false>(a, x0, y0, lane, acc, tk);
        else col2d_wave<R, TY, false, true, false, false, false>(a, x0, y0, lane, acc, tk);
      } else {
        if (ix && iy) col2d_wave<R, TY, false, false, true, true, false>(a, x0, y0, lane, acc, tk);
        else if (iy) col2d_wave<R, TY, false, false, false, true, false>(a, x0, y0, lane, acc, tk);
        else if (ix) col2d_wave<R, TY, false, false, true, false, false>(a, x0, y0, lane, acc, tk);
        else col2d_wave<R, TY, false, false, false, false, false>(a, x0, y0, lane, acc, tk);
      }
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
    block_partials<R, 64 * COL_WAVES>(v, part + (long long)(first[e.x] + wg) * NPART);
    __syncthreads();  // the record's LDS is reused by the next entry
  }
}

}  // namespace surf
