// surf_common.hpp -- device-side building blocks shared by the libsurf
// kernels: problem descriptors, index/ghost mapping, the phase-field maps,
// the equation of state and wave64 reductions.  gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace surf {

enum { BC_WALL = 0, BC_PERIODIC = 1, BC_OPEN = 2 };
enum { FORM_W = 0, FORM_P = 1 };
enum { KIN_LANGMUIR = 0, KIN_HENRY = 1 };
enum { EOS_LIN = 0, EOS_LANG = 1, EOS_TANH = 2 };

// per-workgroup reduction record of the step kernel
enum {
  P_SUM_F = 0, P_SUM_PSI, P_SUM_DELTA, P_SUM_SIGDELTA, P_OUTFLOW,
  P_MAX_USUM, P_MAX_C, P_MIN_F, P_MIN_PSI, P_NBAD, NPART
};

// device-resident running state (doubles) in the workspace; slot S_FLAGS
// holds a 32-bit word of status bits raised outside the finalize kernel
enum { S_TIME = 0, S_OUTCUM = 1, S_STEPS = 2, S_STATUS = 3, S_FLAGS = 4, NSTATE = 8 };

struct Grid {
  int dim;
  int n[3];
  int bc[3][2];
};

template <typename R>
struct Par {
  R h, inv_h, eps, inv_eps, Db, Ds, ka, kd, ginf, inv_ginf, sigma0, E, eta, eta_eps, chimax;
  int form, kin, eos, bulk;
};

// Cell coordinate q along axis d mapped into the box: periodic axes wrap,
// other boundaries mirror about the boundary face (zero-gradient ghost).
// The result is clamped into [0, n) so that halo cells of ragged tiles, which
// are never consumed, still address memory inside the field.
__device__ __forceinline__ int map_axis(int q, int n, int lo_bc, int hi_bc) {
  if (q < 0) {
    q = (lo_bc == BC_PERIODIC) ? q + n : -1 - q;
  } else if (q >= n) {
    q = (hi_bc == BC_PERIODIC) ? q - n : 2 * n - 1 - q;
  }
  q = q < 0 ? 0 : q;
  q = q >= n ? n - 1 : q;
  return q;
}

__device__ __forceinline__ long long cell_index(const Grid& g, int i, int j, int k) {
  return (long long)i + (long long)g.n[0] * ((long long)j + (long long)g.n[1] * k);
}

// face index along d: the d-coordinate runs 0..n_d
__device__ __forceinline__ long long face_index(const Grid& g, int d, int i, int j, int k) {
  long long mx = g.n[0] + (d == 0), my = g.n[1] + (d == 1);
  return (long long)i + mx * ((long long)j + my * k);
}

// Elementary functions.  FP32 uses the hardware approximations (exp2, log2,
// reciprocal and square root instructions, ~1 ulp), well inside the FP32
// parity budget; FP64 keeps the correctly rounded library functions.
template <typename R> __device__ __forceinline__ R rexp(R x);
template <> __device__ __forceinline__ float rexp<float>(float x) { return __expf(x); }
template <> __device__ __forceinline__ double rexp<double>(double x) { return exp(x); }

template <typename R> __device__ __forceinline__ R rlog(R x);
template <> __device__ __forceinline__ float rlog<float>(float x) { return __logf(x); }
template <> __device__ __forceinline__ double rlog<double>(double x) { return log(x); }

template <typename R> __device__ __forceinline__ R rrcp(R x);
template <> __device__ __forceinline__ float rrcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rrcp<double>(double x) { return 1.0 / x; }

template <typename R> __device__ __forceinline__ R rtanh(R x);
template <> __device__ __forceinline__ float rtanh<float>(float x) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * x));
}
template <> __device__ __forceinline__ double rtanh<double>(double x) { return tanh(x); }

template <typename R> __device__ __forceinline__ R rsqrt_(R x);
template <> __device__ __forceinline__ float rsqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double rsqrt_<double>(double x) { return sqrt(x); }

// a / b: reciprocal-multiply in FP32, division in FP64
template <typename R> __device__ __forceinline__ R rdiv(R a, R b) { return a * rrcp<R>(b); }
template <> __device__ __forceinline__ double rdiv<double>(double a, double b) { return a / b; }

// The 32-bit finalizer of MurmurHash3 (Appleby, public domain): a bijective
// mix of the bits of x.
__device__ __forceinline__ unsigned fmix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// The key of a step: a mix of the bits of the running time the step starts
// from (device state), so that every step draws other numbers and a run
// replayed from the same state draws the same ones.
__device__ __forceinline__ unsigned step_key(double t) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(t);
  return fmix32((unsigned)b ^ fmix32((unsigned)(b >> 32)));
}

// The state update a + b stored in the context precision.  FP32 rounds
// stochastically: the exact sum (two floats added in FP64) is raised by a
// random fraction of an FP32 ulp (the 16 bits of r16 on the 29 bits below
// the FP32 mantissa) and truncated, so that each of the two neighbouring
// floats comes out with the probability of its closeness and the stored
// state is unbiased.  Round-to-nearest drops every increment below half an
// ulp, and a smooth field whose per-step changes are that small stops
// evolving.  FP64 adds.
template <typename R>
__device__ __forceinline__ R upd(R a, R b, unsigned r16);
template <>
__device__ __forceinline__ float upd<float>(float a, float b, unsigned r16) {
  const double x = (double)a + (double)b;
  unsigned long long u = (unsigned long long)__double_as_longlong(x);
  u = (u + ((unsigned long long)(r16 & 0xffffu) << 13)) & ~0x1fffffffull;
  return (float)__longlong_as_double((long long)u);
}
template <>
__device__ __forceinline__ double upd<double>(double a, double b, unsigned) {
  return a + b;
}

// phi = 1/(1+e^{chi/eps}) (0 in fluid 1, 1 in the liquid), omega = 1 - phi
// evaluated without cancellation, delta = phi omega / eps.
template <typename R>
__device__ __forceinline__ void phase(R chi, const Par<R>& p, R& phi, R& om, R& del) {
  R e = rexp<R>(chi * p.inv_eps);
  phi = rrcp<R>(R(1) + e);
  om = e * phi;
  del = phi * om * p.inv_eps;
}

template <typename R>
__device__ __forceinline__ R eos(R G, const Par<R>& p) {
  R x = G * p.inv_ginf;
  if (p.eos == EOS_LIN) return p.sigma0 * (R(1) - p.E * x);
  if (p.eos == EOS_LANG) {
    // x bounded to [0, 1 - 1e-6], written as 1 - x bounded below by the
    // FP64 value of 1 - (1 - 1e-6): the same bound in FP64, and in FP32 one
    // that 1 - 1e-6 (not a float) would miss by 1.3%
    constexpr double OM_MIN = 1.0 - (1.0 - 1e-6);
    x = x < R(0) ? R(0) : x;
    const R om = R(1) - x;  // NaN stays NaN
    return p.sigma0 * (R(1) + p.E * rlog<R>(om < R(OM_MIN) ? R(OM_MIN) : om));
  }
  return p.sigma0 * (R(1) - rtanh<R>(p.E * x));
}

// minmod of two one-sided differences; the sign test avoids the underflow
// of a*b for tiny differences in FP32
template <typename R>
__device__ __forceinline__ R minmod(R a, R b) {
  R m = fabs(a) < fabs(b) ? a : b;
  bool same = (a > R(0) && b > R(0)) || (a < R(0) && b < R(0));
  return same ? m : R(0);
}

// wave64 reductions (gfx950 wavefronts are 64 lanes) with DPP row
// rotations inside each 16-lane row, then the four row results combined in
// a fixed order through readlane: no LDS permutes, deterministic.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int DPP_ROR8 = 0x128, DPP_ROR4 = 0x124, DPP_ROR2 = 0x122, DPP_ROR1 = 0x121;

enum { RED_SUM = 0, RED_MAX = 1, RED_MIN = 2 };

template <int OP>
__device__ __forceinline__ double red_op(double a, double b) {
  return OP == RED_SUM ? a + b : (OP == RED_MAX ? fmax(a, b) : fmin(a, b));
}

// every lane of the wave receives the reduction of all 64 lanes
template <int OP>
__device__ __forceinline__ double wave_reduce(double v) {
  v = red_op<OP>(v, dpp_d<DPP_ROR8>(v));
  v = red_op<OP>(v, dpp_d<DPP_ROR4>(v));
  v = red_op<OP>(v, dpp_d<DPP_ROR2>(v));
  v = red_op<OP>(v, dpp_d<DPP_ROR1>(v));
  double r0 = readlane_d(v, 0), r1 = readlane_d(v, 16);
  double r2 = readlane_d(v, 32), r3 = readlane_d(v, 48);
  return red_op<OP>(red_op<OP>(r0, r1), red_op<OP>(r2, r3));
}
__device__ __forceinline__ double wave_sum(double v) { return wave_reduce<RED_SUM>(v); }
__device__ __forceinline__ double wave_max(double v) { return wave_reduce<RED_MAX>(v); }
__device__ __forceinline__ double wave_min(double v) { return wave_reduce<RED_MIN>(v); }

}  // namespace surf
