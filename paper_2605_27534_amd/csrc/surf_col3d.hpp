// surf_col3d.hpp -- the 3D transport step (substeps 1 and 2, the source,
// the equation of state and the reduction record) for the weighted flux
// form, as plane-marching workgroups.
//
// Work unit: a workgroup of 16 waves owns a strip of 64 columns along x
// (lane L holds column x0 - 3 + L, lanes 3 .. 60 produce output), the rows
// y0 - 1 .. y0 + 14 (wave w holds row y0 - 1 + w; waves 1 .. 14 produce
// output) and a chunk of TZ planes z0 .. z0 + TZ - 1.  It marches along z:
//   plane s:   the advected state on its 16 rows (x-face fluxes through
//              wave-wide DPP shifts, y-face fluxes from the neighbour rows in
//              LDS, z-face fluxes from registers), then phi, delta, c* and
//              Gamma* (sections 3.1, 2.6), then the weighted fluxes of the
//              x and y faces (section 3.2, Appendix A);
//   plane s-1: the z-face weighted fluxes, the update with the source,
//              sigma(Gamma) and the reduction terms (sections 2.3, 2.6).
// Two barriers per plane: after the rows' advected inputs are in LDS, and
// after their c*, Gamma*, phi, delta are.  Rows y0 - 3, y0 - 2, y0 + 15,
// y0 + 16 are loaded (by waves 0, 1, 14, 15) for the y stencil only.
// Boundaries as in the 2D kernel: walls and open sides mirror ghost values,
// periodic sides wrap; advective flux zero through walls, the interior value
// through open sides (accounted in the outflow budget); diffusive and
// confinement fluxes zero through both.  Workgroups whose strip and rows touch
// no x or y side run a variant without the side logic (z sides are uniform
// per plane and cost nothing).  Loads are plain global accesses: a scalar
// base and a 32-bit lane offset, which keeps the scalar register budget for
// the side variant.
#pragma once
#include "surf_col2d.hpp"

namespace surf {

constexpr int C3_WAVES = 16;          // waves (rows) per workgroup
constexpr int C3_OUT_ROWS = 14;       // output rows per workgroup
constexpr int C3_XI_ROWS = C3_WAVES + 4;
constexpr int C3_LOOKAHEAD = 2;       // planes of loads in flight ahead of the arithmetic

template <typename R>
struct Col3Lds {
  R xF[C3_XI_ROWS][64], xP[C3_XI_ROWS][64];  // advected inputs of plane s, rows y0-3 .. y0+16
  R ph[C3_WAVES][64], de[C3_WAVES][64];      // phi, delta of plane s, rows y0-1 .. y0+14
  R cs[C3_WAVES][64], gs[C3_WAVES][64];      // c*, Gamma* of plane s
};

template <typename R>
struct Col3Args {
  Grid g;
  Par<R> p;
  const R* chi;
  const R* u[3];
  const R* F;
  const R* psi;
  R* Fo;
  R* Po;
  R* sig;
  double* part;
  const double* state;  // running state: the time keys the FP32 stochastic rounding
  R dt;
  R area_dt;   // h^2 dt
  int strips;  // ceil(nx / 58)
  int yblocks; // ceil(ny / 14)
  int zchunks; // ceil(nz / TZ)
  int nwg;
  int per_xcd;
  // optional: the advected state xi* (F*, psi*) of every cell, the input of
  // the adjoint step's substep-2 and advection transposes
  R* Fst = nullptr;
  R* Pst = nullptr;
};

// One workgroup: strip x0, rows y0 - 1 .. y0 + 14, planes z0 .. z0 + TZ - 1.
// IX: every column the strip reads lies inside the box away from the x
// sides; IY: the same for the rows the workgroup reads and the y sides.
template <typename R, int TZ, bool HU, bool BULK, bool IX, bool IY, bool ST>
__device__ __forceinline__ void col3d_wg(const Col3Args<R>& a, Col3Lds<R>& L, const int x0,
                                         const int y0, const int z0, const int lane,
                                         const int wv, ColAcc<R>& acc, const unsigned tkey) {
  constexpr bool SRND = sizeof(R) == 4;  // FP32: stochastically rounded state
  R (&sXF)[C3_XI_ROWS][64] = L.xF;
  R (&sXP)[C3_XI_ROWS][64] = L.xP;
  R (&sPh)[C3_WAVES][64] = L.ph;
  R (&sDe)[C3_WAVES][64] = L.de;
  R (&sCs)[C3_WAVES][64] = L.cs;
  R (&sGs)[C3_WAVES][64] = L.gs;
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const bool px = !IX && g.bc[0][0] == BC_PERIODIC, py = !IY && g.bc[1][0] == BC_PERIODIC;
  const bool pz = g.bc[2][0] == BC_PERIODIC;
  const R cfl = a.dt * p.inv_h, hcfl = R(0.5) * cfl;
  const R dcoef = p.Db * R(0.5) * p.inv_h * p.inv_h, scoef = p.Ds * R(0.5) * p.inv_h * p.inv_h;
  const R kl = p.kin == KIN_LANGMUIR ? R(1) : R(0);
  constexpr int ES = (int)sizeof(R);

  // ---- the lane's column (x) and the wave's row (y)
  const int xs = x0 - 3 + lane;
  int mx = xs, fxm = xs + 1;
  bool gx = false, xf_lo = false, xf_hi = false, xf_out = false;
  if constexpr (!IX) {
    mx = map_axis(xs, nx, g.bc[0][0], g.bc[0][1]);
    gx = !px && (xs < 0 || xs >= nx);                           // ghost column
    const int fx = xs + 1;                                      // the lane's right face
    xf_lo = !px && fx == 0;
    xf_hi = !px && fx == nx;
    xf_out = !px && (fx < 0 || fx > nx);
    fxm = px ? ((fx % nx) + nx) % nx : (xf_out ? 0 : fx);
  }
  const bool x_side = xf_lo || xf_hi;
  const bool x_lo_open = xf_lo && g.bc[0][0] == BC_OPEN, x_hi_open = xf_hi && g.bc[0][1] == BC_OPEN;
  const int ys = y0 - 1 + wv;                                   // the wave's row
  int my = ys, fylo = ys, fyhi = ys + 1;
  bool gy = false, yf_lo_side = false, yf_hi_side = false, yf_lo_out = false, yf_hi_out = false;
  if constexpr (!IY) {
    my = map_axis(ys, ny, g.bc[1][0], g.bc[1][1]);
    gy = !py && (ys < 0 || ys >= ny);                           // ghost row
    // y faces of the row: lo = ys (between ys-1 and ys), hi = ys + 1
    yf_lo_side = !py && ys == 0;
    yf_hi_side = !py && ys + 1 == ny;
    yf_lo_out = !py && (ys < 0 || ys > ny);
    yf_hi_out = !py && (ys + 1 < 0 || ys + 1 > ny);
    fylo = py ? ((ys % ny) + ny) % ny : (yf_lo_out ? 0 : ys);
    fyhi = py ? (((ys + 1) % ny) + ny) % ny : (yf_hi_out ? 0 : ys + 1);
  }
  const bool out_lane = lane >= 3 && lane < 3 + COL_OUT && (IX || xs < nx);
  const bool out_row = wv >= 1 && wv <= C3_OUT_ROWS && (IY || ys < ny);
  // extra rows of the y stencil loaded by waves 0, 1 (rows y0-3, y0-2) and
  // 14, 15 (rows y0+15, y0+16)
  const bool extra = wv <= 1 || wv >= C3_WAVES - 2;
  const int ye = wv <= 1 ? y0 - 3 + wv : y0 + 1 + wv;
  const int mye = IY ? ye : map_axis(ye, ny, g.bc[1][0], g.bc[1][1]);
  const int xrow = wv <= 1 ? wv : wv + 4;                       // LDS row of the extra row

  // every index below is mapped into its array: plain global accesses with
  // a 64-bit scalar base and a 32-bit byte offset
  const R* const bF = a.F;
  const R* const bP = a.psi;
  const R* const bC = a.chi;
  const R* const bUx = a.u[0];
  const R* const bUy = a.u[1];
  const R* const bUz = a.u[2];
  R* const bFo = a.Fo;
  R* const bPo = a.Po;
  R* const bS = a.sig;
  const int vmx = mx * ES, vfx = fxm * ES, vxs = xs * ES;

  // ---- per-plane loads: plane index k = 0 .. NZ3-1 is z = z0 - 3 + k
  constexpr int NZ3 = TZ + 6;
  R rF[NZ3], rP[NZ3], rFe[NZ3], rPe[NZ3];  // own row, extra row
  R rC[TZ + 2], rUx[TZ + 2], rUyl[TZ + 2], rUyh[TZ + 2], rUz[TZ + 3];
  auto load_plane = [&](const int k) {
    if (k < NZ3) {
      const int mz = map_axis(z0 - 3 + k, nz, g.bc[2][0], g.bc[2][1]);
      const int pl = nx * ny * mz;
      rF[k] = BULK ? gld<R>(bF, vmx, (pl + nx * my) * ES) : R(0);
      rP[k] = gld<R>(bP, vmx, (pl + nx * my) * ES);
      if (extra) {  // uniform per wave
        rFe[k] = BULK ? gld<R>(bF, vmx, (pl + nx * mye) * ES) : R(0);
        rPe[k] = gld<R>(bP, vmx, (pl + nx * mye) * ES);
      }
    }
    if (k >= 3 && k - 3 < TZ + 3) {
      // z face j = z0 - 1 + i (below plane j)
      const int i = k - 3;
      rUz[i] = R(0);
      if (HU) {
        int j = z0 - 1 + i;
        bool ok = !gx && !gy;  // gx, gy are false in the interior variants
        if (pz) {
          while (j < 0) j += nz;
          while (j >= nz) j -= nz;
        } else if (j < 0 || j > nz) {
          j = 0;
          ok = false;
        }
        const R v = gld<R>(bUz, vmx, (nx * ny * j + nx * my) * ES);
        rUz[i] = ok ? v : R(0);
      }
    }
    if (k >= 4 && k - 4 < TZ + 2) {
      // plane z0 - 1 + i of the advected state
      const int i = k - 4;
      const int zs = z0 - 1 + i;
      const int mz = map_axis(zs, nz, g.bc[2][0], g.bc[2][1]);
      const bool gz = !pz && (zs < 0 || zs >= nz);
      rC[i] = gld<R>(bC, vmx, (nx * ny * mz + nx * my) * ES);
      rUx[i] = R(0);
      rUyl[i] = R(0);
      rUyh[i] = R(0);
      if (HU) {
        const R vx = gld<R>(bUx, vfx, ((nx + 1) * ny * mz + (nx + 1) * my) * ES);
        rUx[i] = (!xf_out && !gy && !gz) ? vx : R(0);  // ghost faces carry nothing
        const R vl = gld<R>(bUy, vmx, (nx * (ny + 1) * mz + nx * fylo) * ES);
        const R vh = gld<R>(bUy, vmx, (nx * (ny + 1) * mz + nx * fyhi) * ES);
        rUyl[i] = (!yf_lo_out && !gx && !gz) ? vl : R(0);
        rUyh[i] = (!yf_hi_out && !gx && !gz) ? vh : R(0);
      }
    }
  };
#pragma unroll
  for (int k = 0; k < 3 + C3_LOOKAHEAD && k < NZ3; ++k) load_plane(k);

  const bool y_lo_open = !IY && ys == 0 && !py && g.bc[1][0] == BC_OPEN;
  const bool y_hi_open = !IY && ys == ny - 1 && !py && g.bc[1][1] == BC_OPEN;

  // values carried from plane to plane
  R dF2 = rF[1] - rF[0], dP2 = rP[1] - rP[0], dF1 = rF[2] - rF[1], dP1 = rP[2] - rP[1];
  R gzF = R(0), gzP = R(0);       // advective z flux below plane s
  R pFs = R(0), pPs = R(0), pC = R(0), pG = R(0), pPh = R(0), pDe = R(0), pIF = R(1), pIP = R(1);
  R pDivF = R(0), pDivP = R(0);   // x + y weighted divergence of plane s-1
  // FP32: the old state and the advective increment of plane s-1, added to
  // the substep-2 increment in one stochastically rounded update
  R pXF = R(0), pXP = R(0), pAF = R(0), pAP = R(0);
  R pWzF = R(0), pWzP = R(0);     // weighted flux through z face s-1

#pragma unroll
  for (int i = 3; i < NZ3; ++i) {
    if (i + C3_LOOKAHEAD < NZ3) load_plane(i + C3_LOOKAHEAD);
    __builtin_amdgcn_sched_barrier(0);
    // ---- advective flux through z face j = s + 1 (planes s = z0-5+i, s+1)
    const int j = z0 - 4 + i;
    const R dF0 = rF[i] - rF[i - 1], dP0 = rP[i] - rP[i - 1];
    R nzF = R(0), nzP = R(0);
    if (HU) {
      const R uf = rUz[i - 3];
      nzF = BULK ? bcg_face<R>(uf, rF[i - 2], rF[i - 1], dF2, dF1, dF0, hcfl) : R(0);
      nzP = bcg_face<R>(uf, rP[i - 2], rP[i - 1], dP2, dP1, dP0, hcfl);
      if (!pz && j == 0) {
        nzF = (BULK && g.bc[2][0] == BC_OPEN) ? uf * rF[i - 1] : R(0);
        nzP = g.bc[2][0] == BC_OPEN ? uf * rP[i - 1] : R(0);
      } else if (!pz && j == nz) {
        nzF = (BULK && g.bc[2][1] == BC_OPEN) ? uf * rF[i - 2] : R(0);
        nzP = g.bc[2][1] == BC_OPEN ? uf * rP[i - 2] : R(0);
      } else if (!pz && (j < 0 || j > nz)) {
        nzF = R(0);
        nzP = R(0);
      }
    }
    dF2 = dF1; dP2 = dP1;
    dF1 = dF0; dP1 = dP0;
    if (i >= 4) {
      const int s = z0 - 5 + i;
      const int k1 = i - 4;
      const bool gz = !pz && (s < 0 || s >= nz);
      const R xF = rF[i - 2], xP = rP[i - 2];
      // ---- the advected inputs of plane s into LDS
      sXF[wv + 2][lane] = xF;
      sXP[wv + 2][lane] = xP;
      if (extra) {
        sXF[xrow][lane] = rFe[i - 2];
        sXP[xrow][lane] = rPe[i - 2];
      }
      __syncthreads();
      R Fs = xF, Ps = xP;
      R aF = R(0), aP = R(0);  // FP32: the advective increments
      R fxF = R(0), fxP = R(0), fxLF = R(0), fxLP = R(0);
      R fyLF = R(0), fyLP = R(0), fyHF = R(0), fyHP = R(0);
      const R ux = rUx[k1];
      if (HU) {
        // x faces (right face of this lane; the left face from the lane to the left)
        const R xFr = from_right(xF), xPr = from_right(xP);
        const R eF = xFr - xF, eP = xPr - xP;
        const R eFl = from_left(eF), eFr = from_right(eF), ePl = from_left(eP), ePr = from_right(eP);
        fxF = BULK ? bcg_face<R>(ux, xF, xFr, eFl, eF, eFr, hcfl) : R(0);
        fxP = bcg_face<R>(ux, xP, xPr, ePl, eP, ePr, hcfl);
        if constexpr (!IX) {
          const R oF = x_lo_open ? ux * xFr : (x_hi_open ? ux * xF : R(0));
          const R oP = x_lo_open ? ux * xPr : (x_hi_open ? ux * xP : R(0));
          fxF = x_side ? (BULK ? oF : R(0)) : fxF;
          fxP = x_side ? oP : fxP;
          fxF = xf_out ? R(0) : fxF;
          fxP = xf_out ? R(0) : fxP;
        }
        if (gy || gz) {  // uniform
          fxF = R(0);
          fxP = R(0);
        }
        fxLF = from_left(fxF);
        fxLP = from_left(fxP);
        // y faces of this row from the rows in LDS (row r of LDS is y0 - 3 + r)
        const int r0 = wv + 2;
        const R Fm2 = sXF[r0 - 2][lane], Fm1 = sXF[r0 - 1][lane], Fp1 = sXF[r0 + 1][lane],
                Fp2 = sXF[r0 + 2][lane];
        const R Pm2 = sXP[r0 - 2][lane], Pm1 = sXP[r0 - 1][lane], Pp1 = sXP[r0 + 1][lane],
                Pp2 = sXP[r0 + 2][lane];
        const R ul = rUyl[k1], uh = rUyh[k1];
        // lo face (rows ys-1 | ys), hi face (rows ys | ys+1)
        fyLF = BULK ? bcg_face<R>(ul, Fm1, xF, Fm1 - Fm2, xF - Fm1, Fp1 - xF, hcfl) : R(0);
        fyLP = bcg_face<R>(ul, Pm1, xP, Pm1 - Pm2, xP - Pm1, Pp1 - xP, hcfl);
        fyHF = BULK ? bcg_face<R>(uh, xF, Fp1, xF - Fm1, Fp1 - xF, Fp2 - Fp1, hcfl) : R(0);
        fyHP = bcg_face<R>(uh, xP, Pp1, xP - Pm1, Pp1 - xP, Pp2 - Pp1, hcfl);
        if constexpr (!IY) {
          if (yf_lo_side) {
            fyLF = (BULK && g.bc[1][0] == BC_OPEN) ? ul * xF : R(0);
            fyLP = g.bc[1][0] == BC_OPEN ? ul * xP : R(0);
          }
          if (yf_hi_side) {
            fyHF = (BULK && g.bc[1][1] == BC_OPEN) ? uh * xF : R(0);
            fyHP = g.bc[1][1] == BC_OPEN ? uh * xP : R(0);
          }
          if (yf_lo_out) { fyLF = R(0); fyLP = R(0); }
          if (yf_hi_out) { fyHF = R(0); fyHP = R(0); }
        }
        if constexpr (!IX) {
          fyLF = gx ? R(0) : fyLF;
          fyLP = gx ? R(0) : fyLP;
          fyHF = gx ? R(0) : fyHF;
          fyHP = gx ? R(0) : fyHP;
        }
        if (gz) { fyLF = R(0); fyLP = R(0); fyHF = R(0); fyHP = R(0); }
        if constexpr (SRND) {
          aF = -cfl * (((fxF - fxLF) + (fyHF - fyLF)) + (nzF - gzF));
          aP = -cfl * (((fxP - fxLP) + (fyHP - fyLP)) + (nzP - gzP));
          Fs = xF + aF;
          Ps = xP + aP;
        } else {
          Fs = xF - cfl * (((fxF - fxLF) + (fyHF - fyLF)) + (nzF - gzF));
          Ps = xP - cfl * (((fxP - fxLP) + (fyHP - fyLP)) + (nzP - gzP));
        }
      }
      if constexpr (!IX) {
        Fs = gx ? R(0) : Fs;
        Ps = gx ? R(0) : Ps;
      }
      if (gy || gz) {  // uniform
        Fs = R(0);
        Ps = R(0);
      }
      if (!BULK) Fs = R(0);
      R ph, om, de;
      phase<R>(rC[k1], p, ph, om, de);
      const R dnF = ph + p.eta, dnP = de + p.eta_eps;
      const R iF = rrcp<R>(dnF), iP = rrcp<R>(dnP);
      const R cs = quot<R>(Fs, dnF, iF);
      const R Gs = quot<R>(Ps, dnP, iP);
      sPh[wv][lane] = ph;
      sDe[wv][lane] = de;
      sCs[wv][lane] = cs;
      sGs[wv][lane] = Gs;
      __syncthreads();
      // ---- weighted fluxes of plane s: x (right face, DPP), y (both faces, LDS)
      const R phr = from_right(ph), der = from_right(de);
      const R csr = from_right(cs), Gsr = from_right(Gs);
      R wxF = (ph + phr) * (csr - cs), wxP = (de + der) * (Gsr - Gs);
      if constexpr (!IX) {
        wxF = x_side ? R(0) : wxF;
        wxP = x_side ? R(0) : wxP;
      }
      const R axF = wxF - from_left(wxF), axP = wxP - from_left(wxP);
      R ayF = R(0), ayP = R(0);
      if (wv >= 1 && wv <= C3_WAVES - 2) {
        const R phm = sPh[wv - 1][lane], dem = sDe[wv - 1][lane], csm = sCs[wv - 1][lane],
                Gsm = sGs[wv - 1][lane];
        const R php = sPh[wv + 1][lane], dep = sDe[wv + 1][lane], csp = sCs[wv + 1][lane],
                Gsp = sGs[wv + 1][lane];
        R hF = (ph + php) * (csp - cs), hP = (de + dep) * (Gsp - Gs);
        R lF = (phm + ph) * (cs - csm), lP = (dem + de) * (Gs - Gsm);
        if (!IY && yf_hi_side) { hF = R(0); hP = R(0); }
        if (!IY && yf_lo_side) { lF = R(0); lP = R(0); }
        ayF = hF - lF;
        ayP = hP - lP;
      }
      // z face s (below plane s), from plane s-1 in registers
      R wzF = (pPh + ph) * (cs - pC), wzP = (pDe + de) * (Gs - pG);
      if (!pz && (s == 0 || s == nz)) { wzF = R(0); wzP = R(0); }
      if (ST && out_lane && out_row && s >= z0 && s < z0 + TZ && s < nz) {
        const int off = (nx * ny * s + nx * ys) * ES;
        if (BULK) gst(Fs, a.Fst, vxs, off);
        gst(Ps, a.Pst, vxs, off);
      }
      const R uxL = from_left(ux);  // every lane takes part in the shift
      if (HU && out_lane && out_row && s >= z0 && s < z0 + TZ && s < nz) {
        // cell-mean velocities of the output cells of plane s (on a periodic
        // axis the upper face of the last cell is face 0, as in the fluxes)
        // and the open-side budget of their faces
        R uxh = ux, uyh = rUyh[k1], uzl = rUz[i - 4], uzh = rUz[i - 3];
        acc.usum = fmax(acc.usum, fabs(R(0.5) * (uxL + uxh)) + fabs(R(0.5) * (rUyl[k1] + uyh)) +
                                      fabs(R(0.5) * (uzl + uzh)));
        if constexpr (!IX) {
          if (!px && xs == 0 && g.bc[0][0] == BC_OPEN) acc.out -= (double)(a.area_dt * (fxLF + fxLP));
          if (!px && xs == nx - 1 && g.bc[0][1] == BC_OPEN) acc.out += (double)(a.area_dt * (fxF + fxP));
        }
        if (y_lo_open) acc.out -= (double)(a.area_dt * (fyLF + fyLP));
        if (y_hi_open) acc.out += (double)(a.area_dt * (fyHF + fyHP));
        if (!pz && s == 0 && g.bc[2][0] == BC_OPEN) acc.out -= (double)(a.area_dt * (gzF + gzP));
        if (!pz && s == nz - 1 && g.bc[2][1] == BC_OPEN) acc.out += (double)(a.area_dt * (nzF + nzP));
      }

      if (i >= 6) {
        // ---- plane o = s-1: update, source, sigma, reduction terms
        const int o = s - 1;
        if (out_lane && out_row && o < nz) {
          const R divF = dcoef * (pDivF + (wzF - pWzF));
          const R divP = scoef * (pDivP + (wzP - pWzP));
          const R q = BULK ? p.ka * pC * (p.ginf * pDe - kl * pPs) - p.kd * pPs : R(0);
          R Fn, Pn;
          if constexpr (SRND) {
            // one random word per cell and step: 16 bits for each field
            const unsigned rk = fmix32((unsigned)(nx * (ny * o + ys) + xs) ^ tkey);
            Fn = BULK ? upd<R>(pXF, pAF + a.dt * (divF - q), rk) : R(0);
            Pn = upd<R>(pXP, pAP + a.dt * (divP + q), rk >> 16);
          } else {
            Fn = BULK ? pFs + a.dt * (divF - q) : R(0);
            Pn = pPs + a.dt * (divP + q);
          }
          const R sg = eos<R>(quot<R>(Pn, pDe + p.eta_eps, pIP), p);
          const int off = (nx * ny * o + nx * ys) * ES;
          if (BULK) gst(Fn, bFo, vxs, off);
          gst(Pn, bPo, vxs, off);
          if (a.sig) gst(sg, bS, vxs, off);
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
        }
      }
      pFs = Fs; pPs = Ps; pC = cs; pG = Gs; pPh = ph; pDe = de; pIF = iF; pIP = iP;
      if constexpr (SRND) { pXF = xF; pXP = xP; pAF = aF; pAP = aP; }
      pDivF = axF + ayF; pDivP = axP + ayP; pWzF = wzF; pWzP = wzP;
    }
    gzF = nzF; gzP = nzP;
  }
}

template <typename R, int TZ, bool HU, bool BULK, bool ST>
__global__ void __launch_bounds__(64 * C3_WAVES) k_col3d(Col3Args<R> a) {
  __shared__ Col3Lds<R> L;
  const int b = blockIdx.x;
  const int wg = (b & 7) * a.per_xcd + (b >> 3);  // banded over the XCDs
  if (wg >= a.nwg) return;  // uniform per workgroup: no barrier is skipped by part of it
  const int nx = a.g.n[0], ny = a.g.n[1];
  // the wave index is uniform over the wave: say so, so that row offsets
  // stay in scalar registers
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sx = wg % a.strips, rest = wg / a.strips;
  const int yb = rest % a.yblocks, zc = rest / a.yblocks;
  const int x0 = sx * COL_OUT, y0 = yb * C3_OUT_ROWS, z0 = zc * TZ;
  ColAcc<R> acc{0.0, 0.0, 0.0, 0.0, 0.0, R(0), R(-INFINITY), R(INFINITY), R(INFINITY), 0};
  const bool ix = x0 >= 3 && x0 + 62 <= nx, iy = y0 >= 3 && y0 + 17 <= ny;
  const unsigned tk = sizeof(R) == 4 ? step_key(a.state[S_TIME]) : 0u;
  if (ix && iy) col3d_wg<R, TZ, HU, BULK, true, true, ST>(a, L, x0, y0, z0, lane, wv, acc, tk);
  else col3d_wg<R, TZ, HU, BULK, false, false, ST>(a, L, x0, y0, z0, lane, wv, acc, tk);
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
  block_partials<R, 64 * C3_WAVES>(v, a.part + (long long)wg * NPART);
}

}  // namespace surf
