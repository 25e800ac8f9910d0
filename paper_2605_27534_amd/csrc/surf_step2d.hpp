// surf_step2d.hpp -- the fused 2D step for gfx950: warm-started redistancing
// of the moving interface (section 2.5), advection (section 3.1 substep 1),
// confinement + diffusion + exchange (substep 2, sections 2.6 and 3.2,
// Appendix C), equation of state (sections 2.3, 5, 6) and FP64 partial sums,
// in one launch over 64 x 16 tiles.
//
// Far-field tiles.  Beyond the clamp |chi| <= chi_max the signed distance is
// the constant s chi_max; a tile all of whose cells hold that value is
// "quiescent" and is stored only as a per-tile flag (1: +chi_max inside fluid
// 1, 2: -chi_max in the liquid, 0: field values live in the chi buffer).  A
// tile whose own VoF is uniform and whose neighbour tiles were quiescent with
// the same sign stays quiescent: K Jacobi sweeps cannot reach it from any
// interface cell, since the warm start assumes the interface moved less than
// the clamp distance in one step (a violation raises status bit 8).  Only the
// other tiles run the K redistancing sweeps, temporally blocked in LDS on the
// tile plus a (K + 2)-cell halo, which gives chi exactly (as K global Jacobi
// sweeps would) on the tile plus the 2-cell halo the transport needs.
#pragma once
#include "surf_kernels.hpp"

namespace surf {

enum { Q_LIVE = 0, Q_POS = 1, Q_NEG = 2, Q_TODO = 3 };  // Q_TODO: live, not yet rebuilt
enum { STATUS_GEOM_JUMP = 8 };

template <typename R>
struct Step2dArgs {
  Grid g;
  Par<R> p;
  const R* vof;      // VoF at t^{n+1} or nullptr (static geometry)
  const R* chi_in;   // level set buffer of the current geometry
  R* chi_out;        // moving geometry: buffer receiving chi^{n+1}
  const uint8_t* q_in;
  uint8_t* q_out;
  uint8_t* mark;     // weighted-form moving geometry: 1 for the live tiles of
                     // this step (read by every live-tile workgroup; never
                     // rewritten while they scan it), 0 otherwise
  const R* u[2];
  const R* F;
  const R* psi;
  R* Fo;
  R* Po;
  R* sig;
  double* part;      // [ntiles][NPART]
  double* state;     // status bits for the jump flag
  R dt;
  R area_dt;
  R dtau;
  int has_u;
  int ksweeps;       // sweeps this step (<= KH)
  int tiles[2];
  int ntiles;
  int per_xcd;       // tiles per XCD chunk
  int diag;          // 1: diagonal XCD mapping (tiles[0] % 8 == 0), 0: banded
  double r0;         // axisymmetric rings: the radius of the low x side
};

// Workgroup -> tile.  Consecutive workgroups land on consecutive XCDs
// (b % 8).  Banded: XCD x walks the contiguous tile range [x per_xcd,
// (x + 1) per_xcd), which keeps vertical halos in one L2 but puts a band of
// tile rows on one XCD.  Diagonal: in tile row ty, XCD x takes the tiles whose
// column is (x + 3 ty) mod 8 in every group of 8 columns, so any localized
// feature (the interface band, where the tiles do redistancing work) spreads
// over all eight XCDs.
__device__ __forceinline__ int tile_of_block(int b, int ntx, int per_xcd, int diag) {
  const int x = b & 7, j = b >> 3;
  if (!diag) return x * per_xcd + j;
  const int m = ntx >> 3;
  const int ty = j / m, k = j - ty * m;
  return 8 * k + ((x + 3 * ty) & 7) + ntx * ty;
}

// Paper-form anti-diffusion coefficient of halo-1 cell (cx, cy) along d
// (section 3.2, Appendix C): B_F = -D_b (1-phi)/eps n_d, B_psi = -D_s
// (1-2 phi)/eps n_d, n = -grad chi/|grad chi| by centred differences of the
// level set held in LDS with a halo of at least 2.
template <typename R>
__device__ __forceinline__ R paper_B_lds(const R* chiL, int EXC, int HC, int cx, int cy, int d,
                                         bool bulk_field, const Par<R>& p) {
  int lc = (cx + HC - 1) + EXC * (cy + HC - 1);
  R gx = (chiL[lc + 1] - chiL[lc - 1]) * (R(0.5) * p.inv_h);
  R gy = (chiL[lc + EXC] - chiL[lc - EXC]) * (R(0.5) * p.inv_h);
  R nrm = rsqrt_<R>(gx * gx + gy * gy);
  nrm = nrm < R(1e-6) ? R(1e-6) : nrm;
  R nd = -(d == 0 ? gx : gy) / nrm;
  R ph, om, de;
  phase<R>(chiL[lc], p, ph, om, de);
  R w = bulk_field ? om : (om - ph);
  return -(bulk_field ? p.Db : p.Ds) * w * p.inv_eps * nd;
}

template <int TX, int TY>
__device__ __forceinline__ int tile_of(const Grid& g, int tilesx, int x, int y) {
  return (x / TX) + tilesx * (y / TY);
}

// Sizes of the per-tile LDS arrays of the 2D tile kernels.
template <int KH, int TX, int TY>
struct Tile2 {
  static constexpr int HC = KH > 0 ? KH + 2 : 2;        // chi halo held in LDS
  static constexpr int EXC = TX + 2 * HC, EYC = TY + 2 * HC, NC = EXC * EYC;
  static constexpr int RX = (HC + TX - 1) / TX, RY = (HC + TY - 1) / TY;  // flag neighbourhood
  static constexpr int QW = 2 * RX + 1, QN = QW * (2 * RY + 1);
};

// Level set of the (mapped) cell (gx, gy) for tile (tx, ty): the clamp value
// on tiles flagged quiescent in sQ (the flag neighbourhood), else the buffer.
template <typename R, int KH, int TX, int TY>
__device__ __forceinline__ R chi_at_tile(const Step2dArgs<R>& a, const uint8_t* sQ, int tx, int ty,
                                         int gx, int gy) {
  using T = Tile2<KH, TX, TY>;
  const Grid& g = a.g;
  const int nx = g.n[0], ny = g.n[1];
  int mx = map_axis(gx, nx, g.bc[0][0], g.bc[0][1]);
  int my = map_axis(gy, ny, g.bc[1][0], g.bc[1][1]);
  int dx = mx / TX - tx, dy = my / TY - ty;
  if (dx > T::RX) dx -= a.tiles[0];
  if (dx < -T::RX) dx += a.tiles[0];
  if (dy > T::RY) dy -= a.tiles[1];
  if (dy < -T::RY) dy += a.tiles[1];
  uint8_t q = sQ[(dx + T::RX) + T::QW * (dy + T::RY)];
  if (q == Q_POS) return a.p.chimax;
  if (q == Q_NEG) return -a.p.chimax;
  return a.chi_in[(long long)mx + (long long)nx * my];
}

// Quiescence flags of the neighbour tiles into sQ (255: outside a
// non-periodic side).  Ends with a barrier.
template <typename R, int KH, int NT, int TX, int TY>
__device__ __forceinline__ void load_flags(const Step2dArgs<R>& a, uint8_t* sQ, int tx, int ty) {
  using T = Tile2<KH, TX, TY>;
  const Grid& g = a.g;
  const int tid = threadIdx.x;
  if (tid < T::QN) {
    int ux = tx + tid % T::QW - T::RX, uy = ty + tid / T::QW - T::RY;
    bool ok = true;
    if (ux < 0 || ux >= a.tiles[0]) {
      if (g.bc[0][ux < 0 ? 0 : 1] == BC_PERIODIC) ux = (ux + a.tiles[0]) % a.tiles[0]; else ok = false;
    }
    if (uy < 0 || uy >= a.tiles[1]) {
      if (g.bc[1][uy < 0 ? 0 : 1] == BC_PERIODIC) uy = (uy + a.tiles[1]) % a.tiles[1]; else ok = false;
    }
    sQ[tid] = ok ? a.q_in[ux + a.tiles[0] * uy] : (uint8_t)255;
  }
  __syncthreads();
}

// The moving-interface geometry of tile t (section 2.5): decides from the
// tile's VoF and the neighbour flags whether the tile stays quiescent (level
// set at the clamp); otherwise rebuilds it with K warm-start Jacobi sweeps
// (Russo-Smereka pinned cut cells, Godunov elsewhere) on the tile plus a
// halo that shrinks by one cell per sweep, all in LDS.  Each thread keeps
// the pin data and the current value of its cells in registers; LDS holds
// the two sweep buffers (the second one first holds the VoF).  On return
// sChi holds chi^{n+1} on the tile and its halo of 2 (HC - K) for live
// tiles (and, unless write_quiet, the clamp value on quiescent ones),
// chi_out the tile's values of live tiles (and, with write_quiet, of
// quiescent tiles too), q_out[t] the new flag.  Returns whether the tile was
// live.  sQ must hold the flags (load_flags) and all1 / all0 the VoF
// uniformity of the tile (block-wide); sB has NC elements.  DECIDED: the
// tile is known to be live and chi_in holds explicit values everywhere (sQ
// and all1 / all0 are not used).
// Whether the VoF of tile t is uniformly 1 / uniformly 0 (block-wide).
template <typename R, int NT, int TX, int TY>
__device__ __forceinline__ void tile_vof_uniform(const Step2dArgs<R>& a, const int t, bool& all1,
                                                 bool& all0) {
  constexpr int IT = (TX * TY + NT - 1) / NT;
  const int nx = a.g.n[0], ny = a.g.n[1];
  const int x0 = (t % a.tiles[0]) * TX, y0 = (t / a.tiles[0]) * TY;
  all1 = true;
  all0 = true;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    int l = threadIdx.x + it * NT;
    int gx = x0 + l % TX, gy = y0 + l / TX;
    if (l < TX * TY && gx < nx && gy < ny) {
      R f = a.vof[(long long)gx + (long long)nx * gy];
      all1 = all1 && f == R(1);
      all0 = all0 && f == R(0);
    }
  }
  all1 = __syncthreads_and(all1);
  all0 = __syncthreads_and(all0);
}

template <typename R, int KH, int NT, int TX, int TY, bool DECIDED = false>
__device__ __forceinline__ bool tile_geometry(const Step2dArgs<R>& a, const int t, R* sChi,
                                              R* sB, const uint8_t* sQ, bool write_quiet,
                                              const bool all1, const bool all0) {
  using T = Tile2<KH, TX, TY>;
  constexpr int HC = T::HC, EXC = T::EXC, EYC = T::EYC, NC = T::NC;
  constexpr int IC = (NC + NT - 1) / NT, IT = (TX * TY + NT - 1) / NT;
  const Grid& g = a.g;
  const Par<R>& p = a.p;
  const int tid = threadIdx.x;
  const int nx = g.n[0], ny = g.n[1];
  const int tx = t % a.tiles[0], ty = t / a.tiles[0];
  const int x0 = tx * TX, y0 = ty * TY;
  if constexpr (!DECIDED) {
    int want = all1 ? Q_POS : (all0 ? Q_NEG : -1);
    bool quiet = true, nb_quiet = true;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        uint8_t q = sQ[(dx + T::RX) + T::QW * (dy + T::RY)];
        if (q == 255) continue;
        if ((int)q != want) quiet = false;
        if (q == Q_LIVE) nb_quiet = false;
      }
    const bool active = !quiet;
    // the VoF changed under a tile whose whole neighbourhood was quiescent:
    // the interface moved farther than the clamp distance in one step
    if (tid == 0 && active && nb_quiet)
      atomicOr((unsigned*)(a.state + S_FLAGS), (unsigned)STATUS_GEOM_JUMP);
    if (!active) {
      R v = want == Q_POS ? p.chimax : -p.chimax;
      if (write_quiet) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
          int l = tid + it * NT;
          int gx = x0 + l % TX, gy = y0 + l / TX;
          if (l < TX * TY && gx < nx && gy < ny) a.chi_out[(long long)gx + (long long)nx * gy] = v;
        }
      } else {
        for (int l = tid; l < NC; l += NT) sChi[l] = v;
      }
      if (tid == 0) a.q_out[t] = (uint8_t)want;
      return false;
    }
  }
  R* sV = sB;  // the VoF until the pin data is in registers
  // this thread's cells of the tile + HC region
  int cl[IC], cx[IC], cy[IC];
#pragma unroll
  for (int it = 0; it < IC; ++it) {
    cl[it] = tid + it * NT;
    cx[it] = cl[it] % EXC;
    cy[it] = cl[it] / EXC;
  }
  {
    R rv[IC], rc[IC];
    // every load goes to a mapped (valid) cell, also for the threads past the
    // region, so that none waits behind a branch
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      int gx = x0 + cx[it] - HC, gy = y0 + cy[it] - HC;
      int mx = map_axis(gx, nx, g.bc[0][0], g.bc[0][1]);
      int my = map_axis(gy, ny, g.bc[1][0], g.bc[1][1]);
      rv[it] = a.vof[(long long)mx + (long long)nx * my];
      if constexpr (DECIDED) rc[it] = a.chi_in[(long long)mx + (long long)nx * my];
      else if (cl[it] < NC) rc[it] = chi_at_tile<R, KH, TX, TY>(a, sQ, tx, ty, gx, gy);
    }
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      if (cl[it] < NC) {
        sV[cl[it]] = rv[it];
        sChi[cl[it]] = rc[it];
      }
    }
  }
  __syncthreads();
  // pin data on the tile + (HC - 1) halo: subcell distance of cut cells
  // (Russo-Smereka), +-infinity carrying the sign elsewhere
  R G[IC], cur[IC];
#pragma unroll
  for (int it = 0; it < IC; ++it) {
    const int l = cl[it];
    G[it] = R(0);
    cur[it] = R(0);
    if (l >= NC) continue;
    cur[it] = sChi[l];
    if (cx[it] < 1 || cx[it] >= EXC - 1 || cy[it] < 1 || cy[it] >= EYC - 1) continue;
    R c0 = (sV[l] - R(0.5)) * p.h;
    R xm = (sV[l - 1] - R(0.5)) * p.h, xp = (sV[l + 1] - R(0.5)) * p.h;
    R ym = (sV[l - EXC] - R(0.5)) * p.h, yp = (sV[l + EXC] - R(0.5)) * p.h;
    bool cut = (c0 * xm <= R(0)) || (c0 * xp <= R(0)) || (c0 * ym <= R(0)) || (c0 * yp <= R(0));
    R jump = fmax(fmax(fabs(xm - c0), fabs(xp - c0)), fmax(fabs(ym - c0), fabs(yp - c0)));
    R ccx = R(0.5) * (xp - xm), ccy = R(0.5) * (yp - ym);
    R Delta = fmax(fmax(rsqrt_<R>(ccx * ccx + ccy * ccy), jump), R(1e-30) * p.h);
    G[it] = cut ? p.h * c0 / Delta : (c0 > R(0) ? R(INFINITY) : R(-INFINITY));
  }
  __syncthreads();  // sV is read; sB becomes the second sweep buffer
  // K Jacobi sweeps on shrinking regions: the cell at depth d (distance to
  // the edge of the tile + HC region) is updated by sweeps 1 .. d, so the
  // next sweep never reads a value this one did not write
  int dep[IC];
#pragma unroll
  for (int it = 0; it < IC; ++it) {
    const int dx = min(cx[it], EXC - 1 - cx[it]), dy = min(cy[it], EYC - 1 - cy[it]);
    dep[it] = cl[it] < NC ? min(dx, dy) : -1;
  }
  int par = 0;
  for (int k = 1; k <= a.ksweeps; ++k) {
    const R* src = par ? sB : sChi;
    R* dst = par ? sChi : sB;
    R xm[IC], xp[IC], ym[IC], yp[IC];
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      // neighbour reads first (an in-range index for cells off this sweep)
      const int l = dep[it] >= k ? cl[it] : EXC + 1;
      xm[it] = src[l - 1];
      xp[it] = src[l + 1];
      ym[it] = src[l - EXC];
      yp[it] = src[l + EXC];
    }
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      if (dep[it] < k) continue;
      const R gv = G[it];
      R v = gv;
      if (!(fabs(gv) < R(INFINITY))) {
        const R x = cur[it];
        const R bwx = (x - xm[it]) * p.inv_h, fwx = (xp[it] - x) * p.inv_h;
        const R bwy = (x - ym[it]) * p.inv_h, fwy = (yp[it] - x) * p.inv_h;
        const R sgn = gv > R(0) ? R(1) : R(-1);
        // Godunov: upwind one-sided differences for the sign of chi0
        const R a1 = sgn * bwx, b1 = sgn * fwx, a2 = sgn * bwy, b2 = sgn * fwy;
        R t1 = a1 > R(0) ? a1 * a1 : R(0), t2 = b1 < R(0) ? b1 * b1 : R(0);
        R G2 = t1 > t2 ? t1 : t2;
        t1 = a2 > R(0) ? a2 * a2 : R(0);
        t2 = b2 < R(0) ? b2 * b2 : R(0);
        G2 += t1 > t2 ? t1 : t2;
        v = x - a.dtau * sgn * (rsqrt_<R>(G2) - R(1));
      }
      v = v > p.chimax ? p.chimax : v;
      v = v < -p.chimax ? -p.chimax : v;
      cur[it] = v;
      dst[cl[it]] = v;
    }
    __syncthreads();
    par ^= 1;
  }
  if (par != 0) {
    // the last sweep wrote sB: bring the result back into sChi
#pragma unroll
    for (int it = 0; it < IC; ++it)
      if (cl[it] < NC) sChi[cl[it]] = sB[cl[it]];
    __syncthreads();
  }
  // chi^{n+1} of the tile interior and its quiescence flag
  bool allpos = true, allneg = true;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    int l = tid + it * NT;
    int ix = l % TX, iy = l / TX;
    int gx = x0 + ix, gy = y0 + iy;
    if (l < TX * TY && gx < nx && gy < ny) {
      R v = sChi[(ix + HC) + EXC * (iy + HC)];
      a.chi_out[(long long)gx + (long long)nx * gy] = v;
      allpos = allpos && v == p.chimax;
      allneg = allneg && v == -p.chimax;
    }
  }
  // both votes with one barrier: per-wave votes through LDS (the sweep
  // buffer sB is free again)
  {
    int* sVote = reinterpret_cast<int*>(sB);
    const bool wp = __all(allpos), wn = __all(allneg);
    if ((tid & 63) == 0) sVote[tid >> 6] = (wp ? 1 : 0) | (wn ? 2 : 0);
    __syncthreads();
    if (tid == 0) {
      int m = 3;
      for (int w = 0; w < (NT + 63) / 64; ++w) m &= sVote[w];
      a.q_out[t] = (m & 1) ? Q_POS : ((m & 2) ? Q_NEG : Q_LIVE);
    }
  }
  return true;
}

// One tile of the step; its FP64 partial record goes to a.part[t].
// AXI (paper form on axisymmetric rings, Appendix B; x is the radius): the
// radial face fluxes of both substeps enter a cell's balance with weights
// r_face / r_mid, the reductions count each cell with 2 pi r_mid (the
// finalize multiplies by h^2) and the open-side budget each face with its
// area 2 pi r h.
template <typename R, int KH, int NT, int TX, int TY, bool AXI = false>
__device__ __forceinline__ void step2d_tile(const Step2dArgs<R>& a, const int t) {
  // K sweeps reach K cells: within the 3 x 3 tile neighbourhood used to
  // decide which tiles stay quiescent
  static_assert(KH <= TY && KH <= TX, "sweeps must stay within the neighbour tiles");
  using T = Tile2<KH, TX, TY>;
  constexpr int HC = T::HC, EXC = T::EXC, NC = T::NC;
  constexpr int EX3 = TX + 6, EY3 = TY + 6, N3 = EX3 * EY3;
  constexpr int EX1 = TX + 2, EY1 = TY + 2, N1 = EX1 * EY1;
  constexpr int NUX = (TX + 3) * EY1, NUY = EX1 * (TY + 3);
  constexpr int I3 = (N3 + NT - 1) / NT, IUX = (NUX + NT - 1) / NT;
  constexpr int IUY = (NUY + NT - 1) / NT, IC = (NC + NT - 1) / NT;
  constexpr int IT = (TX * TY + NT - 1) / NT;
  // LDS: the final level set (tile + HC halo) stays live throughout; the
  // redistancing scratch (second sweep buffer, VoF, pin data) and the
  // transport arrays share one pool
  constexpr int NTR = 2 * N3 + 3 * (NUX + NUY) + 4 * N1;
  constexpr int NGEO = KH > 0 ? NC : 0;
  constexpr int NPOOL = NGEO > NTR ? NGEO : NTR;
  __shared__ R sChi[NC];
  __shared__ R sPool[NPOOL];
  __shared__ uint8_t sQ[T::QN];
  R* sF3 = sPool;              // old F (halo 3), later c* in place
  R* sP3 = sPool + N3;         // old psi (halo 3), later Gamma* in place
  R* sUx = sPool + 2 * N3;     // x-face velocities of the halo-1 cells
  R* sUy = sUx + NUX;          // y-face velocities
  R* sFlx = sUy + NUY;         // x-face advective fluxes (F, psi)
  R* sFly = sFlx + 2 * NUX;    // y-face advective fluxes (F, psi)
  R* sC = sFly + 2 * NUY;      // F*, psi*, phi, delta (halo 1)

  const Grid& g = a.g;
  const Par<R>& p = a.p;
  const bool bulk = p.bulk != 0;
  const bool has_u = a.has_u != 0;
  const int tid = threadIdx.x;
  const int nx = g.n[0], ny = g.n[1];

  const int tx = t % a.tiles[0], ty = t / a.tiles[0];
  const int x0 = tx * TX, y0 = ty * TY;
  const bool moving = KH > 0 && a.vof != nullptr;

  // ---------------------------------------------------------- prefetch
  // every input of the transport, loaded up front with independent loads
  R rF[I3], rP[I3], rUx[IUX], rUy[IUY];
#pragma unroll
  for (int it = 0; it < I3; ++it) {
    int l = tid + it * NT;
    rF[it] = R(0);
    rP[it] = R(0);
    if (l < N3) {
      int mx = map_axis(x0 + l % EX3 - 3, nx, g.bc[0][0], g.bc[0][1]);
      int my = map_axis(y0 + l / EX3 - 3, ny, g.bc[1][0], g.bc[1][1]);
      long long c = (long long)mx + (long long)nx * my;
      if (bulk) rF[it] = a.F[c];
      rP[it] = a.psi[c];
    }
  }
  // face velocities: wrapped on periodic axes (the last face is face 0),
  // zero on faces of ghost cells
#pragma unroll
  for (int it = 0; it < IUX; ++it) {
    int l = tid + it * NT;
    rUx[it] = R(0);
    if (has_u && l < NUX) {
      int gx = x0 + l % (TX + 3) - 1, gy = y0 + l / (TX + 3) - 1;
      bool ok = true;
      if (gx < 0) { if (g.bc[0][0] == BC_PERIODIC) gx += nx; else ok = false; }
      if (gx > nx) { if (g.bc[0][1] == BC_PERIODIC) gx -= nx; else ok = false; }
      if (gx == nx && g.bc[0][1] == BC_PERIODIC) gx = 0;
      if (gy < 0 || gy >= ny) {
        if (g.bc[1][gy < 0 ? 0 : 1] == BC_PERIODIC) gy = gy < 0 ? gy + ny : gy - ny; else ok = false;
      }
      if (ok) rUx[it] = a.u[0][(long long)gx + (long long)(nx + 1) * gy];
    }
  }
#pragma unroll
  for (int it = 0; it < IUY; ++it) {
    int l = tid + it * NT;
    rUy[it] = R(0);
    if (has_u && l < NUY) {
      int gx = x0 + l % EX1 - 1, gy = y0 + l / EX1 - 1;
      bool ok = true;
      if (gy < 0) { if (g.bc[1][0] == BC_PERIODIC) gy += ny; else ok = false; }
      if (gy > ny) { if (g.bc[1][1] == BC_PERIODIC) gy -= ny; else ok = false; }
      if (gy == ny && g.bc[1][1] == BC_PERIODIC) gy = 0;
      if (gx < 0 || gx >= nx) {
        if (g.bc[0][gx < 0 ? 0 : 1] == BC_PERIODIC) gx = gx < 0 ? gx + nx : gx - nx; else ok = false;
      }
      if (ok) rUy[it] = a.u[1][(long long)gx + (long long)nx * gy];
    }
  }
  load_flags<R, KH, NT, TX, TY>(a, sQ, tx, ty);

  // ---------------------------------------------------------- geometry
  if constexpr (KH > 0) {
    if (moving) {
      bool all1, all0;
      tile_vof_uniform<R, NT, TX, TY>(a, t, all1, all0);
      tile_geometry<R, KH, NT, TX, TY>(a, t, sChi, sPool, sQ, false, all1, all0);
    }
  }
  if (!moving) {
    // static geometry: the current level set on tile + 2 halo
    R rc[IC];
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      int l = tid + it * NT;
      rc[it] = R(0);
      int lx = l % EXC, ly = l / EXC;
      if (l < NC && lx >= HC - 2 && lx < HC + TX + 2 && ly >= HC - 2 && ly < HC + TY + 2)
        rc[it] = chi_at_tile<R, KH, TX, TY>(a, sQ, tx, ty, x0 + lx - HC, y0 + ly - HC);
    }
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      int l = tid + it * NT;
      if (l < NC) sChi[l] = rc[it];
    }
  }
  __syncthreads();

  // ---------------------------------------------------------- transport
#pragma unroll
  for (int it = 0; it < I3; ++it) {
    int l = tid + it * NT;
    if (l < N3) {
      sF3[l] = rF[it];
      sP3[l] = rP[it];
    }
  }
#pragma unroll
  for (int it = 0; it < IUX; ++it) {
    int l = tid + it * NT;
    if (l < NUX) sUx[l] = rUx[it];
  }
#pragma unroll
  for (int it = 0; it < IUY; ++it) {
    int l = tid + it * NT;
    if (l < NUY) sUy[l] = rUy[it];
  }
  __syncthreads();

  double acc[NPART];
#pragma unroll
  for (int s = 0; s < NPART; ++s) acc[s] = 0.0;
  acc[P_MAX_C] = -INFINITY;
  acc[P_MIN_F] = INFINITY;
  acc[P_MIN_PSI] = INFINITY;

  R* sF1 = sC;
  R* sP1 = sC + N1;
  R* sPhi = sC + 2 * N1;
  R* sDel = sC + 3 * N1;
  const R cfl = a.dt * p.inv_h;
  const bool px = g.bc[0][0] == BC_PERIODIC, py = g.bc[1][0] == BC_PERIODIC;

  // substep 1: the advective flux through every face of the halo-1 cells,
  // once per face.  x-face fi (0..TX+2) of row fj lies between halo-1 cells
  // fi-1 and fi; the cell on its + side is global (x0+fi-1, y0+fj-1).
  if (has_u) {
    for (int m = tid; m < NUX + NUY; m += NT) {
      const bool xf = m < NUX;
      const int mm = xf ? m : m - NUX;
      const int fi = xf ? mm % (TX + 3) : mm % EX1;
      const int fj = xf ? mm / (TX + 3) : mm / EX1;
      const int gx = x0 + fi - 1, gy = y0 + fj - 1;
      const int gd = xf ? gx : gy, nd = xf ? nx : ny;
      const int gt = xf ? gy : gx, nt = xf ? ny : nx;
      const bool per = xf ? px : py, pert = xf ? py : px;
      const bool blo = !per && gd == 0, bhi = !per && gd == nd;
      const bool ghost = (!per && (gd < 0 || gd > nd)) || (!pert && (gt < 0 || gt >= nt));
      const R uf = xf ? sUx[mm] : sUy[mm];
      const int st = xf ? 1 : EX3;
      const int lp = (fi + 2) + EX3 * (fj + 2);
      const int dd = xf ? 0 : 1;
      R fF = R(0), fP = R(0);
      if (!ghost) {
        if (blo) {
          if (g.bc[dd][0] == BC_OPEN) { fF = uf * sF3[lp]; fP = uf * sP3[lp]; }
        } else if (bhi) {
          if (g.bc[dd][1] == BC_OPEN) { fF = uf * sF3[lp - st]; fP = uf * sP3[lp - st]; }
        } else {
          fF = adv_flux<R>(uf, sF3[lp - 2 * st], sF3[lp - st], sF3[lp], sF3[lp + st], cfl);
          fP = adv_flux<R>(uf, sP3[lp - 2 * st], sP3[lp - st], sP3[lp], sP3[lp + st], cfl);
        }
        if (!bulk) fF = R(0);
        // open-boundary budget, counted by the tile owning the interior cell
        const int fa = xf ? fi : fj, ta = xf ? TX : TY;
        const bool own_t = xf ? (fj >= 1 && fj <= TY && gy < ny) : (fi >= 1 && fi <= TX && gx < nx);
        if (own_t) {
          double wa = 1.0;  // rings: the face's area over h
          if constexpr (AXI)
            wa = 2.0 * M_PI * (a.r0 + (xf ? (double)gd : (double)gx + 0.5) * (double)p.h);
          if (blo && g.bc[dd][0] == BC_OPEN && fa >= 1 && fa <= ta)
            acc[P_OUTFLOW] -= wa * (double)(a.area_dt * (fF + fP));
          if (bhi && g.bc[dd][1] == BC_OPEN && fa >= 2 && fa <= ta + 1)
            acc[P_OUTFLOW] += wa * (double)(a.area_dt * (fF + fP));
        }
      }
      if (xf) { sFlx[mm] = fF; sFlx[NUX + mm] = fP; }
      else { sFly[mm] = fF; sFly[NUY + mm] = fP; }
    }
    __syncthreads();
  }

  // advected state and phase field on the halo-1 cells; c* and Gamma* are
  // written over the old state of the same cell (only that cell reads it)
  for (int l = tid; l < N1; l += NT) {
    const int lx = l % EX1, ly = l / EX1;
    const int gx = x0 + lx - 1, gy = y0 + ly - 1;
    R ph, om, de;
    phase<R>(sChi[(lx + HC - 1) + EXC * (ly + HC - 1)], p, ph, om, de);
    const int l3 = (lx + 2) + EX3 * (ly + 2);
    const bool ghost = (!px && (gx < 0 || gx >= nx)) || (!py && (gy < 0 || gy >= ny));
    R Fs = R(0), Ps = R(0);
    if (!ghost) {
      Fs = bulk ? sF3[l3] : R(0);
      Ps = sP3[l3];
      if (has_u) {
        const int xl = lx + (TX + 3) * ly, yl = lx + EX1 * ly;
        R alo = R(1), ahi = R(1);
        if constexpr (AXI) {
          const double rl = a.r0 + (double)gx * (double)p.h, rm = rl + 0.5 * (double)p.h;
          alo = (R)(rl / rm);
          ahi = (R)((rl + (double)p.h) / rm);
        }
        const R dF = (ahi * sFlx[xl + 1] - alo * sFlx[xl]) + (sFly[yl + EX1] - sFly[yl]);
        const R dP = (ahi * sFlx[NUX + xl + 1] - alo * sFlx[NUX + xl]) +
                     (sFly[NUY + yl + EX1] - sFly[NUY + yl]);
        Fs = Fs - cfl * dF;
        Ps = Ps - cfl * dP;
        if (lx >= 1 && lx <= TX && ly >= 1 && ly <= TY && gx < nx && gy < ny) {
          // cell-mean velocity magnitudes (on a periodic axis the upper
          // face of the last cell is face 0, as in the fluxes)
          R uxl = sUx[xl], uxh = sUx[xl + 1], uyl = sUy[yl], uyh = sUy[yl + EX1];
          double us = fabs((double)(R(0.5) * (alo * uxl + ahi * uxh))) +
                      fabs((double)(R(0.5) * (uyl + uyh)));
          acc[P_MAX_USUM] = fmax(acc[P_MAX_USUM], us);
        }
      }
    }
    sF1[l] = bulk ? Fs : R(0);
    sP1[l] = Ps;
    sPhi[l] = ph;
    sDel[l] = de;
    sF3[l3] = rdiv<R>(Fs, ph + p.eta);
    sP3[l3] = rdiv<R>(Ps, de + p.eta_eps);
  }
  __syncthreads();

  // per-thread sums and extrema in the working precision (at most IT cells)
  R sF = R(0), sP = R(0), sD = R(0), sSD = R(0), nbad = R(0);
  R mxC = R(-INFINITY), mnF = R(INFINITY), mnP = R(INFINITY);
  // substep 2 on the interior cells
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int l = tid + it * NT;
    const int ix = l % TX, iy = l / TX;
    const int gx = x0 + ix, gy = y0 + iy;
    if (l >= TX * TY || gx >= nx || gy >= ny) continue;
    const int c = (ix + 1) + EX1 * (iy + 1);
    const int c3 = (ix + 3) + EX3 * (iy + 3);
    const bool bxl = !px && gx == 0, bxh = !px && gx == nx - 1;
    const bool byl = !py && gy == 0, byh = !py && gy == ny - 1;
    R divF = R(0), divP = R(0);
    if (p.form == FORM_W) {
      const R cw = sF3[c3], gw = sP3[c3], pw = sPhi[c], dw = sDel[c];
      R aF = R(0), aP = R(0);
#define SURF_WFACE(o, o3, skip)                                    \
      if (!(skip)) {                                               \
        aF += (pw + sPhi[o]) * (sF3[o3] - cw);                     \
        aP += (dw + sDel[o]) * (sP3[o3] - gw);                     \
      }
      SURF_WFACE(c - 1, c3 - 1, bxl)
      SURF_WFACE(c + 1, c3 + 1, bxh)
      SURF_WFACE(c - EX1, c3 - EX3, byl)
      SURF_WFACE(c + EX1, c3 + EX3, byh)
#undef SURF_WFACE
      divF = p.Db * R(0.5) * aF * p.inv_h * p.inv_h;
      divP = p.Ds * R(0.5) * aP * p.inv_h * p.inv_h;
    } else {
      // paper form: B from the centred chi gradient (chi held with halo 2)
      const int cx = ix + 1, cy = iy + 1;
      R alo = R(1), ahi = R(1);
      if constexpr (AXI) {
        const double rl = a.r0 + (double)gx * (double)p.h, rm = rl + 0.5 * (double)p.h;
        alo = (R)(rl / rm);
        ahi = (R)((rl + (double)p.h) / rm);
      }
      for (int f = 0; f < 2; ++f) {
        if (f == 0 && !bulk) continue;
        const R* x = f == 0 ? sF1 : sP1;
        const R D = f == 0 ? p.Db : p.Ds;
        R acc2 = R(0);
        for (int d = 0; d < 2; ++d) {
          const int st = d == 0 ? 1 : EX1;
          const bool blo = d == 0 ? bxl : byl, bhi = d == 0 ? bxh : byh;
          const R Bc = paper_B_lds<R>(sChi, EXC, HC, cx, cy, d, f == 0, p);
          const R wl = d == 0 ? alo : R(1), wh = d == 0 ? ahi : R(1);
          if (!blo) {
            R Bm = paper_B_lds<R>(sChi, EXC, HC, cx - (d == 0), cy - (d == 1), d, f == 0, p);
            R Bf = R(0.5) * (Bm + Bc);
            const R fl = D * (x[c] - x[c - st]) * p.inv_h + Bf * (Bf < R(0) ? x[c - st] : x[c]);
            acc2 -= AXI ? wl * fl : fl;
          }
          if (!bhi) {
            R Bp = paper_B_lds<R>(sChi, EXC, HC, cx + (d == 0), cy + (d == 1), d, f == 0, p);
            R Bf = R(0.5) * (Bc + Bp);
            const R fh = D * (x[c + st] - x[c]) * p.inv_h + Bf * (Bf < R(0) ? x[c] : x[c + st]);
            acc2 += AXI ? wh * fh : fh;
          }
        }
        if (f == 0) divF = acc2 * p.inv_h; else divP = acc2 * p.inv_h;
      }
    }
    const R Fs = sF1[c], Ps = sP1[c], ph = sPhi[c], de = sDel[c];
    R q = R(0);
    if (bulk) {
      const R cs = sF3[c3];  // c* = F* / (phi + eta)
      q = p.kin == KIN_LANGMUIR ? p.ka * cs * (p.ginf * de - Ps) - p.kd * Ps
                                : p.ka * cs * p.ginf * de - p.kd * Ps;
    }
    const R Fn = bulk ? Fs + a.dt * (divF - q) : R(0);
    const R Pn = Ps + a.dt * (divP + q);
    const R sg = eos<R>(rdiv<R>(Pn, de + p.eta_eps), p);
    const long long ci = (long long)gx + (long long)nx * gy;
    if (bulk) a.Fo[ci] = Fn;
    a.Po[ci] = Pn;
    if (a.sig) a.sig[ci] = sg;
    if constexpr (AXI) {
      const R wv = (R)(2.0 * M_PI * (a.r0 + ((double)gx + 0.5) * (double)p.h));
      sF += wv * Fn;
      sP += wv * Pn;
      sD += wv * de;
      sSD += wv * (sg * de);
    } else {
      sF += Fn;
      sP += Pn;
      sD += de;
      sSD += sg * de;
    }
    if (bulk) {
      mxC = fmax(mxC, rdiv<R>(Fn, ph + p.eta));
      mnF = fmin(mnF, Fn);
    }
    mnP = fmin(mnP, Pn);
    const bool bad = !isfinite(Pn) || !isfinite(sg) || (bulk && !isfinite(Fn));
    nbad += bad ? R(1) : R(0);
  }
  acc[P_SUM_F] = (double)sF;
  acc[P_SUM_PSI] = (double)sP;
  acc[P_SUM_DELTA] = (double)sD;
  acc[P_SUM_SIGDELTA] = (double)sSD;
  acc[P_MAX_C] = (double)mxC;
  acc[P_MIN_F] = (double)mnF;
  acc[P_MIN_PSI] = (double)mnP;
  acc[P_NBAD] = (double)nbad;
  block_partials<R, NT>(acc, a.part + (long long)t * NPART);
}

template <typename R, int KH, int NT = 512, int TX = 64, int TY = 16, bool AXI = false>
__global__ void __launch_bounds__(NT) k_step2d(Step2dArgs<R> a) {
  const int t = tile_of_block(blockIdx.x, a.tiles[0], a.per_xcd, a.diag);
  if (t >= a.ntiles) return;
  step2d_tile<R, KH, NT, TX, TY, AXI>(a, t);
}

// The moving-interface geometry alone (the step then runs the transport on
// chi_out): every tile of chi_out ends with its chi^{n+1}, quiescent tiles
// the clamp value, so that chi_out holds explicit values everywhere.  Small
// tiles (GEO_T x GEO_T) spread the sweeps of the interface band over many
// CUs.
constexpr int GEO_T = 16, GEO_THREADS = 256;
// The weighted-form moving geometry in two launches, neither with a
// device-wide atomic (those serialise across the XCDs):
//  1. k_geo_classify: one wave per tile decides from the tile's VoF and the
//     neighbour flags of the previous step whether it stays quiescent (flag
//     written; the clamp too unless chi_out's flag says the tile already
//     holds it) or is live (mark 1; its flag is left to pass 2);
//  2. k_geo_live: a fixed grid; every workgroup ranks the live marks (one
//     coalesced pass and a prefix sum) and rebuilds the live tiles of rank
//     b, b + G, ... with tile_geometry (1024 threads: 16 waves overlap each
//     sweep's LDS and barrier latency), which writes their flags.  The marks
//     live apart from the flags: workgroups that start late (the pass may
//     share the GPU with a transport) must rank the same marks as the first.
template <typename R, int KH>
__global__ void __launch_bounds__(256) k_geo_classify(Step2dArgs<R> a) {
  using T = Tile2<KH, GEO_T, GEO_T>;
  constexpr int CPL = GEO_T * GEO_T / 64;  // cells per lane
  static_assert(T::QN <= 64, "flag neighbourhood fits one wave");
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= a.ntiles) return;  // whole waves
  const int lane = threadIdx.x & 63;
  const int nx = a.g.n[0], ny = a.g.n[1];
  const int tx = t % a.tiles[0], ty = t / a.tiles[0];
  const int x0 = tx * GEO_T, y0 = ty * GEO_T;
  // the flag of the output buffer: its tile already holds the clamp when
  // the flag equals this step's quiescent sign
  const uint8_t q_had = a.q_out[t];
  // loads from cells clamped into the box, all issued before any is used;
  // only the cells inside the box vote
  bool one = true, zero = true;
  long long ci[CPL];
  bool in[CPL];
  R f[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    const int c = lane + 64 * k;
    const int gx = x0 + c % GEO_T, gy = y0 + c / GEO_T;
    in[k] = gx < nx && gy < ny;
    ci[k] = (long long)min(gx, nx - 1) + (long long)nx * min(gy, ny - 1);
    f[k] = a.vof[ci[k]];
  }
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    one = one && (!in[k] || f[k] == R(1));
    zero = zero && (!in[k] || f[k] == R(0));
  }
  int q = 255;
  if (lane < T::QN) {
    int ux = tx + lane % T::QW - T::RX, uy = ty + lane / T::QW - T::RY;
    bool ok = true;
    if (ux < 0 || ux >= a.tiles[0]) {
      if (a.g.bc[0][ux < 0 ? 0 : 1] == BC_PERIODIC) ux = (ux + a.tiles[0]) % a.tiles[0]; else ok = false;
    }
    if (uy < 0 || uy >= a.tiles[1]) {
      if (a.g.bc[1][uy < 0 ? 0 : 1] == BC_PERIODIC) uy = (uy + a.tiles[1]) % a.tiles[1]; else ok = false;
    }
    if (ok) q = a.q_in[ux + a.tiles[0] * uy];
  }
  const bool all1 = __all(one), all0 = __all(zero);
  const int want = all1 ? Q_POS : (all0 ? Q_NEG : -1);
  // the 3 x 3 neighbourhood (the flag window may be larger)
  const int dx = lane % T::QW - T::RX, dy = lane / T::QW - T::RY;
  const bool near = lane < T::QN && dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && q != 255;
  const bool quiet = __all(!near || q == want);
  const bool nb_quiet = __all(!near || q != Q_LIVE);
  if (!quiet) {
    if (lane == 0) {
      // the VoF changed under a tile whose whole neighbourhood was
      // quiescent: the interface moved farther than the clamp in one step
      if (nb_quiet) atomicOr((unsigned*)(a.state + S_FLAGS), (unsigned)STATUS_GEOM_JUMP);
      a.mark[t] = 1;  // its flag in q_out is written by the live-tile pass
    }
    return;
  }
  if ((int)q_had != want) {
    const R v = want == Q_POS ? a.p.chimax : -a.p.chimax;
#pragma unroll
    for (int k = 0; k < CPL; ++k)
      if (in[k]) a.chi_out[ci[k]] = v;
  }
  if (lane == 0) {
    a.q_out[t] = (uint8_t)want;
    a.mark[t] = 0;
  }
}

// Pass 2 ranks the tiles marked by pass 1 itself: each of its 1024 threads
// reads one 4-byte word of flags, a ballot/LDS prefix gives every marked
// tile its rank in tile order, and workgroup b takes ranks b, b + G, ...
constexpr int GEO_WG = 1024, GEO_LIVE_GRID = 512, GEO_LIVE_CAP = 32;
template <typename R, int KH>
__global__ void __launch_bounds__(GEO_WG) k_geo_live(Step2dArgs<R> a) {
  using T = Tile2<KH, GEO_T, GEO_T>;
  __shared__ R sChi[T::NC];
  __shared__ R sB[T::NC];
  __shared__ int sWave[GEO_WG / 64];
  __shared__ int sMine[GEO_LIVE_CAP];
  __shared__ int sNum;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nt = a.ntiles;
  const int G = gridDim.x, b = blockIdx.x;
  if (tid == 0) sNum = 0;
  int seen = 0;  // marked tiles in earlier chunks
  for (int base = 0; base < nt; base += 4 * GEO_WG) {
    const int t0 = base + 4 * tid;
    int cnt = 0;
    uint8_t f[4];
    if (t0 + 3 < nt) {
      // four marks in one aligned word (t0 is a multiple of 4)
      const unsigned w = *(const unsigned*)(a.mark + t0);
#pragma unroll
      for (int k = 0; k < 4; ++k) f[k] = (uint8_t)(w >> (8 * k));
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) f[k] = t0 + k < nt ? a.mark[t0 + k] : (uint8_t)0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) cnt += f[k] == 1 ? 1 : 0;
    // inclusive prefix of cnt over the wave (shuffles), then over the waves
    int inc = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int x = __shfl_up(inc, off, 64);
      if (lane >= off) inc += x;
    }
    if (lane == 63) sWave[wv] = inc;
    __syncthreads();
    int before = seen;
    for (int w = 0; w < wv; ++w) before += sWave[w];
    int rank = before + inc - cnt;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (f[k] != 1) continue;
      if (rank % G == b) {
        const int m = atomicAdd(&sNum, 1);  // LDS counter; order restored below
        if (m < GEO_LIVE_CAP) sMine[m] = t0 + k;
      }
      ++rank;
    }
    int total = 0;
    for (int w = 0; w < GEO_WG / 64; ++w) total += sWave[w];
    seen += total;
    __syncthreads();
  }
  const int mine = min(sNum, GEO_LIVE_CAP);
  if (tid == 0) {
    for (int i = 1; i < mine; ++i) {
      const int v = sMine[i];
      int j = i - 1;
      while (j >= 0 && sMine[j] > v) { sMine[j + 1] = sMine[j]; --j; }
      sMine[j + 1] = v;
    }
  }
  __syncthreads();
  for (int i = 0; i < mine; ++i) {
    tile_geometry<R, KH, GEO_WG, GEO_T, GEO_T, true>(a, sMine[i], sChi, sB, nullptr, true, false,
                                                     false);
    __syncthreads();
  }
}

// Batched form: independent static-interface instances of different sizes,
// one persistent launch walking the flattened queue of all their tiles.
// inst[i] describes instance i with its two state buffers (F/Fo, psi/Po);
// parity 1 reads the second and writes the first.  queue[q] = (instance,
// tile of that instance); the partial record of queue entry q goes to
// part[q], so each instance's records are contiguous.
template <typename R, int NT>
__global__ void __launch_bounds__(NT) k_batch2d(const Step2dArgs<R>* __restrict__ inst,
                                                const int2* __restrict__ queue, int nqueue,
                                                int parity, double* __restrict__ part) {
  for (int q = blockIdx.x; q < nqueue; q += gridDim.x) {
    const int2 e = queue[q];
    Step2dArgs<R> a = inst[e.x];
    if (parity) {
      const R* f = a.F;
      a.F = a.Fo;
      a.Fo = (R*)f;
      const R* ps = a.psi;
      a.psi = a.Po;
      a.Po = (R*)ps;
    }
    a.part = part + (long long)(q - e.y) * NPART;
    step2d_tile<R, 0, NT, 64, 16>(a, e.y);
    __syncthreads();
  }
}

// Writes the clamp value into the level-set buffer for every quiescent tile
// (consumers that read chi directly need the explicit field).
template <typename R, int TX = 64, int TY = 16>
__global__ void __launch_bounds__(BLOCK) k_materialize(Grid g, R* chi, const uint8_t* q, R chimax,
                                                       int tilesx, int ntiles) {
  int t = blockIdx.x;
  if (t >= ntiles) return;
  uint8_t f = q[t];
  if (f == Q_LIVE) return;
  R v = f == Q_POS ? chimax : -chimax;
  int x0 = (t % tilesx) * TX, y0 = (t / tilesx) * TY;
  for (int l = threadIdx.x; l < TX * TY; l += BLOCK) {
    int gx = x0 + l % TX, gy = y0 + l / TX;
    if (gx < g.n[0] && gy < g.n[1]) chi[(long long)gx + (long long)g.n[0] * gy] = v;
  }
}

__global__ void k_fill_u8(uint8_t* q, uint8_t v, int n) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) q[i] = v;
}

}  // namespace surf
