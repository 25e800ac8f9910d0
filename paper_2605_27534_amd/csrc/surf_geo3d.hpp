// surf_geo3d.hpp -- the moving-interface geometry in 3D (section 2.5):
// warm-start Jacobi sweeps restricted to the tiles near the interface.
//
// The box is cut into 16^3 tiles with one flag each (quiescent at +clamp,
// quiescent at -clamp, live).  A tile whose VoF is uniform and whose 3x3x3
// tile neighbourhood was quiescent with the same sign after the previous
// step keeps the clamp value: every cell it can reach in K <= 16 sweeps is at
// the clamp, where a Godunov sweep changes nothing.  The other tiles are
// rebuilt by K sweeps over the live tiles only.  The level set stays in one
// buffer (R); the other (S) is the sweeps' ping-pong partner.  Both hold the
// clamp on every quiescent tile, each with a flag array saying so, so that a
// sweep reads its neighbours from one buffer without looking at flags.  A
// geometry prepared while a transport still reads R sweeps between S and a
// third buffer T instead (R -> S -> T -> S ... -> T), which then becomes R:
// classify gives T the clamp on quiescent tiles too, and the last sweep
// writes T's flags.
//   k_geo3_classify  one workgroup per tile: the decision; a quiescent tile
//                    writes the clamp into S only if S's flag says S does not
//                    hold it yet, a live tile its pin data (Russo-Smereka
//                    distance of cut cells, signed infinity elsewhere); the
//                    decision goes to S's flags (live = Q_TODO);
//   k_geo3_list      one workgroup: the live tiles in tile order;
//   k_geo3_sweep     one Jacobi sweep over the listed tiles, R -> S or
//                    S -> R (K even, so the result ends in R); the last one
//                    writes R's flags.
#pragma once
#include "surf_common.hpp"
#include "surf_step2d.hpp"

namespace surf {

constexpr int G3 = 16;                    // tile edge
constexpr int G3_CELLS = G3 * G3 * G3;    // 4096
constexpr int G3_THREADS = 256;
constexpr int G3_CPT = G3_CELLS / G3_THREADS;  // cells per thread (classify)

struct Geo3Args {
  Grid g;
  int tiles[3];
  int ntiles;
  int per_xcd;  // ceil(ntiles / 8): tiles per XCD band of the classify grid
};

// map_axis written with selects only (no branches), for the uniform z
// coordinates and the per-thread x, y neighbours
__device__ __forceinline__ int map_axis_sel(int q, int n, int lo_bc, int hi_bc) {
  const int lo = lo_bc == BC_PERIODIC ? q + n : -1 - q;
  const int hi = hi_bc == BC_PERIODIC ? q - n : 2 * n - 1 - q;
  int r = q < 0 ? lo : (q >= n ? hi : q);
  r = r < 0 ? 0 : r;
  return r >= n ? n - 1 : r;
}

__device__ __forceinline__ int geo3_tile_of(const Geo3Args& t, int x, int y, int z) {
  return (x / G3) + t.tiles[0] * ((y / G3) + t.tiles[1] * (z / G3));
}

template <typename R>
__global__ void __launch_bounds__(G3_THREADS) k_geo3_classify(Geo3Args ga, Par<R> p,
                                                              const R* __restrict__ vof,
                                                              R* __restrict__ chiS,
                                                              R* __restrict__ g0,
                                                              const uint8_t* __restrict__ q_in,
                                                              uint8_t* __restrict__ q_out,
                                                              R* __restrict__ chiT,
                                                              uint8_t* __restrict__ qT,
                                                              double* __restrict__ state) {
  __shared__ uint8_t sQ[27];
  __shared__ int sVote[G3_THREADS / 64];
  // consecutive tiles (x neighbours, sharing cache lines) on one XCD
  const int b = blockIdx.x;
  const int t = (b & 7) * ga.per_xcd + (b >> 3);
  if (t >= ga.ntiles) return;
  const Grid& g = ga.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int tid = threadIdx.x;
  const int tx = t % ga.tiles[0], ty = (t / ga.tiles[0]) % ga.tiles[1],
            tz = t / (ga.tiles[0] * ga.tiles[1]);
  const int x0 = tx * G3, y0 = ty * G3, z0 = tz * G3;
  // this thread's cells: x = tid % 16, y = tid / 16, z = 0 .. 15.  The
  // loads go to mapped (always valid) cells and are all issued before any
  // is used; only the cells inside the box take part in the vote.  Columns
  // past the box edge read a valid column and store nothing.
  const int lx = tid % G3, ly = tid / G3;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool colin = gx < nx && gy < ny;
  const int cx = colin ? gx : nx - 1, cy = colin ? gy : ny - 1;
  const long long pl = (long long)nx * ny;
  const long long cxy = (long long)cx + (long long)nx * cy;
  const uint8_t qs_old = q_out[t];  // read before thread 0 rewrites it
  const uint8_t qt_old = qT ? qT[t] : (uint8_t)0;
  bool one = true, zero = true;
  R f[G3];
#pragma unroll
  for (int k = 0; k < G3; ++k)
    f[k] = vof[cxy + pl * map_axis_sel(z0 + k, nz, g.bc[2][0], g.bc[2][1])];
#pragma unroll
  for (int k = 0; k < G3; ++k) {
    const bool in = colin && z0 + k < nz;
    one = one && (!in || f[k] == R(1));
    zero = zero && (!in || f[k] == R(0));
  }
  if (tid < 27) {
    int u[3] = {tx + tid % 3 - 1, ty + (tid / 3) % 3 - 1, tz + tid / 9 - 1};
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
      if (u[d] < 0 || u[d] >= ga.tiles[d]) {
        if (g.bc[d][u[d] < 0 ? 0 : 1] == BC_PERIODIC) u[d] = (u[d] + ga.tiles[d]) % ga.tiles[d];
        else ok = false;
      }
    }
    sQ[tid] = ok ? q_in[u[0] + ga.tiles[0] * (u[1] + ga.tiles[1] * u[2])] : (uint8_t)255;
  }
  const bool w1 = __all(one), w0 = __all(zero);
  if ((tid & 63) == 0) sVote[tid >> 6] = (w1 ? 1 : 0) | (w0 ? 2 : 0);
  __syncthreads();
  int m = 3;
#pragma unroll
  for (int w = 0; w < G3_THREADS / 64; ++w) m &= sVote[w];
  const int want = (m & 1) ? Q_POS : ((m & 2) ? Q_NEG : -1);
  bool quiet = true, nb_quiet = true;
  for (int i = 0; i < 27; ++i) {
    const uint8_t q = sQ[i];
    if (q == 255) continue;
    if ((int)q != want) quiet = false;
    if (q == Q_LIVE) nb_quiet = false;
  }
  if (quiet) {  // R already holds the clamp here; S (and T) get it unless they have it
    const R v = want == Q_POS ? p.chimax : -p.chimax;
    if ((int)qs_old != want) {
#pragma unroll
      for (int k = 0; k < G3; ++k) {
        const int gz = z0 + k;
        if (colin && gz < nz) chiS[(long long)gx + (long long)nx * (gy + (long long)ny * gz)] = v;
      }
    }
    if (qT && (int)qt_old != want) {
#pragma unroll
      for (int k = 0; k < G3; ++k) {
        const int gz = z0 + k;
        if (colin && gz < nz) chiT[(long long)gx + (long long)nx * (gy + (long long)ny * gz)] = v;
      }
    }
    if (tid == 0) {
      q_out[t] = (uint8_t)want;
      if (qT) qT[t] = (uint8_t)want;
    }
    return;
  }
  if (tid == 0) {
    q_out[t] = (uint8_t)Q_TODO;
    // the VoF changed under a tile whose whole neighbourhood was quiescent
    if (nb_quiet) atomicOr((unsigned*)(state + S_FLAGS), (unsigned)STATUS_GEOM_JUMP);
  }
  if (!colin) return;
  // live: pin data of the tile's cells, in two halves of 8 planes; the
  // neighbour columns of each half are loaded before any is used
  const long long cxm = (long long)map_axis_sel(cx - 1, nx, g.bc[0][0], g.bc[0][1]) + (long long)nx * cy;
  const long long cxp = (long long)map_axis_sel(cx + 1, nx, g.bc[0][0], g.bc[0][1]) + (long long)nx * cy;
  const long long cym = (long long)cx + (long long)nx * map_axis_sel(cy - 1, ny, g.bc[1][0], g.bc[1][1]);
  const long long cyp = (long long)cx + (long long)nx * map_axis_sel(cy + 1, ny, g.bc[1][0], g.bc[1][1]);
  const R zlo = vof[cxy + pl * map_axis_sel(z0 - 1, nz, g.bc[2][0], g.bc[2][1])];
  const R zhi = vof[cxy + pl * map_axis_sel(z0 + G3, nz, g.bc[2][0], g.bc[2][1])];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    R nxm[G3 / 2], nxp[G3 / 2], nym[G3 / 2], nyp[G3 / 2];
#pragma unroll
    for (int j = 0; j < G3 / 2; ++j) {
      const long long pz = pl * map_axis_sel(z0 + half * (G3 / 2) + j, nz, g.bc[2][0], g.bc[2][1]);
      nxm[j] = vof[cxm + pz];
      nxp[j] = vof[cxp + pz];
      nym[j] = vof[cym + pz];
      nyp[j] = vof[cyp + pz];
    }
#pragma unroll
    for (int j = 0; j < G3 / 2; ++j) {
      const int k = half * (G3 / 2) + j;
      const int gz = z0 + k;
      const R x0v = (f[k] - R(0.5)) * p.h;
      const R nb[6] = {(nxm[j] - R(0.5)) * p.h, (nxp[j] - R(0.5)) * p.h,
                       (nym[j] - R(0.5)) * p.h, (nyp[j] - R(0.5)) * p.h,
                       ((k > 0 ? f[k - 1] : zlo) - R(0.5)) * p.h,
                       ((k < G3 - 1 ? f[k + 1] : zhi) - R(0.5)) * p.h};
      bool cut = false;
      R jump = R(0), grad2 = R(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const R xm = nb[2 * d], xp = nb[2 * d + 1];
        cut = cut || (x0v * xm <= R(0)) || (x0v * xp <= R(0));
        jump = fmax(jump, fmax(fabs(xm - x0v), fabs(xp - x0v)));
        const R cd = R(0.5) * (xp - xm);
        grad2 += cd * cd;
      }
      const R Delta = fmax(fmax(rsqrt_<R>(grad2), jump), R(1e-30) * p.h);
      if (colin && gz < nz)
        g0[cxy + pl * gz] = cut ? p.h * x0v / Delta : (x0v > R(0) ? R(INFINITY) : R(-INFINITY));
    }
  }
}

// live[0] = count, live[1 + r] = the r-th live tile in tile order
constexpr int G3_LIST_THREADS = 1024;
__global__ void __launch_bounds__(G3_LIST_THREADS) k_geo3_list(const uint8_t* __restrict__ q,
                                                               int ntiles, int* __restrict__ live) {
  __shared__ int sWave[G3_LIST_THREADS / 64];
  __shared__ int sBase;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) sBase = 0;
  __syncthreads();
  for (int base = 0; base < ntiles; base += G3_LIST_THREADS) {
    const int t = base + tid;
    const bool todo = t < ntiles && q[t] == Q_TODO;
    const unsigned long long mk = __ballot(todo);
    const int below = __popcll(mk & ((1ull << lane) - 1ull));
    if (lane == 0) sWave[wv] = __popcll(mk);
    __syncthreads();
    int off = sBase;
    for (int w = 0; w < wv; ++w) off += sWave[w];
    if (todo) live[1 + off + below] = t;
    __syncthreads();
    if (tid == 0) {
      int tot = 0;
      for (int w = 0; w < G3_LIST_THREADS / 64; ++w) tot += sWave[w];
      sBase += tot;
    }
    __syncthreads();
  }
  if (tid == 0) live[0] = sBase;
}

// The Godunov update of one cell from its value v, pin datum gk (finite on
// cut cells: the pinned value) and its six neighbours, clamped.
template <typename R>
__device__ __forceinline__ R geo3_update(const Par<R>& p, R dtau, R v, R gk, R xm, R xp, R ym,
                                         R yp, R zm, R zp) {
  const R sgn = gk > R(0) ? R(1) : R(-1);
  const R nb[6] = {xm, xp, ym, yp, zm, zp};
  R G2 = R(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const R a1 = sgn * (v - nb[2 * d]) * p.inv_h, b1 = sgn * (nb[2 * d + 1] - v) * p.inv_h;
    const R t1 = a1 > R(0) ? a1 * a1 : R(0), t2 = b1 < R(0) ? b1 * b1 : R(0);
    G2 += t1 > t2 ? t1 : t2;
  }
  R nv = fabs(gk) < R(INFINITY) ? gk : v - dtau * sgn * (rsqrt_<R>(G2) - R(1));
  nv = nv > p.chimax ? p.chimax : nv;
  nv = nv < -p.chimax ? -p.chimax : nv;
  return nv;
}

// One Jacobi sweep (Godunov, pinned cut cells, clamp) over the listed tiles.
// Thread (x, y, h) of a 512-thread workgroup owns G3_SZ = 8 cells of the
// tile's z-column at (x, y), half h of it: it loads those cells with one
// beyond each end, the four x and y neighbour columns over the same planes
// and the pin data, every load issued before any is used, then updates its
// cells.  Two threads per column (rather than one for all 16 cells) put
// twice the waves on the band's few hundred tiles to wait out the load
// latency.  Neighbours come from src everywhere: quiescent tiles hold the
// clamp in every buffer a sweep reads.  Persistent grid (a multiple of 8
// workgroups).  The last sweep also writes each tile's new flag.
constexpr int G3_SZ = 8;
constexpr int G3_SWEEP_THREADS = G3 * G3 * (G3 / G3_SZ), G3_SWEEP_GRID = 1024;
template <typename R>
__global__ void __launch_bounds__(G3_SWEEP_THREADS) k_geo3_sweep(Geo3Args ga, Par<R> p, R dtau,
                                                                 const R* __restrict__ src,
                                                                 R* __restrict__ dst,
                                                                 const R* __restrict__ g0,
                                                                 uint8_t* __restrict__ qr,
                                                                 const int* __restrict__ live,
                                                                 int last) {
  __shared__ int sVote[G3_SWEEP_THREADS / 64];
  const Grid& g = ga.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long pl = (long long)nx * ny;
  const int tid = threadIdx.x;
  const int lx = tid % G3, ly = (tid / G3) % G3, lz = (tid / (G3 * G3)) * G3_SZ;
  // XCD k (workgroups b with b % 8 == k) takes the k-th eighth of the list,
  // so that neighbouring tiles, which share cache lines, meet in one L2
  const int n = live[0];
  const int per = (n + 7) / 8, xcd = blockIdx.x & 7, slots = gridDim.x >> 3;
  const int lo = xcd * per, hi = min(n, lo + per);
  for (int it = lo + (blockIdx.x >> 3); it < hi; it += slots) {
    const int t = live[1 + it];
    const int x0 = (t % ga.tiles[0]) * G3, y0 = ((t / ga.tiles[0]) % ga.tiles[1]) * G3,
              z0 = (t / (ga.tiles[0] * ga.tiles[1])) * G3 + lz;  // this thread's first plane
    const int gx = x0 + lx, gy = y0 + ly;
    const bool colin = gx < nx && gy < ny;
    // columns past the box edge read a valid column and store nothing
    const int cx = colin ? gx : nx - 1, cy = colin ? gy : ny - 1;
    const long long cxy = (long long)cx + (long long)nx * cy;
    const long long cxm = (long long)map_axis_sel(cx - 1, nx, g.bc[0][0], g.bc[0][1]) + (long long)nx * cy;
    const long long cxp = (long long)map_axis_sel(cx + 1, nx, g.bc[0][0], g.bc[0][1]) + (long long)nx * cy;
    const long long cym = (long long)cx + (long long)nx * map_axis_sel(cy - 1, ny, g.bc[1][0], g.bc[1][1]);
    const long long cyp = (long long)cx + (long long)nx * map_axis_sel(cy + 1, ny, g.bc[1][0], g.bc[1][1]);
    R col[G3_SZ + 2], xm[G3_SZ], xp[G3_SZ], ym[G3_SZ], yp[G3_SZ], gv[G3_SZ];
#pragma unroll
    for (int z = -1; z <= G3_SZ; ++z) {
      const long long pz = pl * map_axis_sel(z0 + z, nz, g.bc[2][0], g.bc[2][1]);
      col[z + 1] = src[cxy + pz];
      if (z >= 0 && z < G3_SZ) {
        xm[z] = src[cxm + pz];
        xp[z] = src[cxp + pz];
        ym[z] = src[cym + pz];
        yp[z] = src[cyp + pz];
        gv[z] = g0[cxy + pz];
      }
    }
    bool allpos = true, allneg = true;
#pragma unroll
    for (int z = 0; z < G3_SZ; ++z) {
      const R nv = geo3_update<R>(p, dtau, col[z + 1], gv[z], xm[z], xp[z], ym[z], yp[z], col[z],
                                  col[z + 2]);
      if (colin && z0 + z < nz) {
        dst[cxy + pl * (z0 + z)] = nv;
        allpos = allpos && nv == p.chimax;
        allneg = allneg && nv == -p.chimax;
      }
    }
    if (last) {
      const bool wp = __all(allpos), wn = __all(allneg);
      if ((tid & 63) == 0) sVote[tid >> 6] = (wp ? 1 : 0) | (wn ? 2 : 0);
      __syncthreads();
      if (tid == 0) {
        int m = 3;
        for (int w = 0; w < G3_SWEEP_THREADS / 64; ++w) m &= sVote[w];
        qr[t] = (m & 1) ? Q_POS : ((m & 2) ? Q_NEG : Q_LIVE);
      }
      __syncthreads();
    }
  }
}


}  // namespace surf
