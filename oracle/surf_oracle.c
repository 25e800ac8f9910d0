/*
 * surf_oracle.c -- plain FP64 CPU oracle of the hybrid VoF/Phase-Field
 * soluble-surfactant transport step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source, header, table or helper with the
 * HIP library; it is written from the paper's equations, one stage at a
 * time, in the paper's order, with full temporary arrays and no fusion.
 * Loops whose cells or faces are independent run over OpenMP threads; every
 * sum (the outflow budget, the divergences, the totals) keeps one serial
 * order, so the results do not depend on the thread count.
 *
 * Notation (paper -> names used here):
 *   VoF fraction of fluid 1 (bubble)        c   -> vof
 *   signed distance, > 0 inside fluid 1     chi -> chi
 *   phase field, 0 in fluid 1, 1 in liquid  phi -> phi   (omega = 1 - phi)
 *   bulk concentration per volume           F   -> F
 *   interfacial carrier Gamma*delta         f   -> psi
 *   regularised delta phi(1-phi)/eps        delta
 *   adsorption / desorption rates           r_a, r_d -> k_a, k_d
 *
 * Layout: cell fields [nz][ny][nx], x fastest.  Face fields along axis d
 * have n_d + 1 entries along d ([nz][ny][nx+1], [nz][ny+1][nx],
 * [nz+1][ny][nx]).  2D problems use nz = 1 and no z faces.
 *
 * Parameter packing (shared only in meaning with the library, not in code):
 *   ip[0] dim  ip[1..3] nx ny nz  ip[4..9] bc x-lo x-hi y-lo y-hi z-lo z-hi
 *   ip[10] flux form (0 weighted, 1 paper)  ip[11] kinetics (0 Langmuir,
 *   1 Henry)  ip[12] EoS (0 linear, 1 Langmuir, 2 tanh)  ip[13] bulk on
 *   ip[14] axisymmetric (2D only: x is the radius r, y the axis z)
 *   ip[15] slope limiter of substep 1 (0 minmod, 1 monotonized central)
 *   ip[16] BCG transverse term in substep 1 (0 off, 1 on)
 *   dp[0] h  dp[1] eps  dp[2] D_b  dp[3] D_s  dp[4] k_a  dp[5] k_d
 *   dp[6] Gamma_inf  dp[7] sigma0  dp[8] E  dp[9] eta  dp[10] chi_max/eps
 *   dp[11] advective safety factor  dp[12] diffusive safety factor
 *   dp[13] radius of the low x side (axisymmetric)
 * Boundary codes: 0 wall, 1 periodic, 2 open.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { BC_WALL = 0, BC_PERIODIC = 1, BC_OPEN = 2 };
enum { FORM_WEIGHTED = 0, FORM_PAPER = 1 };
enum { KIN_LANGMUIR = 0, KIN_HENRY = 1 };
enum { EOS_LINEAR = 0, EOS_LANGMUIR = 1, EOS_TANH = 2 };

/* totals slots */
enum {
  T_MB = 0, T_MS, T_OUT, T_OUTCUM, T_SDELTA, T_SSIGD, T_SU, T_DTNEXT,
  T_MINF, T_MINPSI, T_NBAD, T_T, T_GAVG, T_SAVG, T_MTOT, T_CMAX
};

typedef struct {
  int dim, n[3], bc[3][2];
  int form, kin, eos, bulk, axi, lim, trans;
  double h, eps, Db, Ds, ka, kd, ginf, sigma0, E, eta, chimax, cfl_a, cfl_d, r0;
  long ncell;
} Prob;

static Prob unpack(const int* ip, const double* dp) {
  Prob p;
  p.dim = ip[0];
  p.n[0] = ip[1]; p.n[1] = ip[2]; p.n[2] = ip[3];
  p.bc[0][0] = ip[4]; p.bc[0][1] = ip[5];
  p.bc[1][0] = ip[6]; p.bc[1][1] = ip[7];
  p.bc[2][0] = ip[8]; p.bc[2][1] = ip[9];
  p.form = ip[10]; p.kin = ip[11]; p.eos = ip[12]; p.bulk = ip[13]; p.axi = ip[14];
  p.lim = ip[15]; p.trans = ip[16];
  p.h = dp[0]; p.eps = dp[1]; p.Db = dp[2]; p.Ds = dp[3];
  p.ka = dp[4]; p.kd = dp[5]; p.ginf = dp[6]; p.sigma0 = dp[7]; p.E = dp[8];
  p.eta = dp[9]; p.chimax = dp[10] * dp[1]; p.cfl_a = dp[11]; p.cfl_d = dp[12];
  p.r0 = dp[13];
  p.ncell = (long)p.n[0] * p.n[1] * p.n[2];
  return p;
}

static long cell(const Prob* p, int i, int j, int k) {
  return (long)i + (long)p->n[0] * ((long)j + (long)p->n[1] * k);
}

/* Index of the cell at offset s along axis d from (i,j,k).  Outside the box
 * a periodic axis wraps; any other boundary mirrors about the boundary face
 * (ghost -1 -> 0, -2 -> 1), i.e. a zero-gradient ghost. */
static long nbr(const Prob* p, int i, int j, int k, int d, int s) {
  int c[3] = {i, j, k};
  int q = c[d] + s, n = p->n[d];
  if (q < 0 || q >= n) {
    int side = q < 0 ? 0 : 1;
    if (p->bc[d][side] == BC_PERIODIC)
      q = ((q % n) + n) % n;
    else
      q = q < 0 ? -1 - q : 2 * n - 1 - q;
  }
  c[d] = q;
  return cell(p, c[0], c[1], c[2]);
}

/* Axisymmetric geometry (Appendix B): cell (i, j) is the ring between radii
 * r_{i-1/2} = r0 + i h and r_{i+1/2} = r0 + (i+1) h, of volume
 * pi (r_{i+1/2}^2 - r_{i-1/2}^2) h = 2 pi r_i h^2 with r_i its mid radius.
 * Dividing the finite-volume balance by the volume, a flux through a radial
 * face enters with the weight r_face / r_i, an axial one with 1.  The
 * Cartesian case has every weight 1 and volume h^dim. */
static const double PI = 3.14159265358979323846;
static double r_face(const Prob* p, int i) { return p->r0 + i * p->h; }
static double r_mid(const Prob* p, int i) { return p->r0 + (i + 0.5) * p->h; }
static double cell_volume(const Prob* p, int i) {
  return p->axi ? 2.0 * PI * r_mid(p, i) * p->h * p->h : pow(p->h, p->dim);
}
/* area of face (i, j, k) along d: radial faces 2 pi r_face h, axial faces
 * 2 pi r_i h (Cartesian: h^(dim-1)) */
static double face_area(const Prob* p, int d, int i) {
  if (!p->axi) return pow(p->h, p->dim - 1);
  return 2.0 * PI * (d == 0 ? r_face(p, i) : r_mid(p, i)) * p->h;
}
/* the weights of the low and high faces of cell i along d in its balance */
static void div_weights(const Prob* p, int d, int i, double* wm, double* wp) {
  if (p->axi && d == 0) {
    *wm = r_face(p, i) / r_mid(p, i);
    *wp = r_face(p, i + 1) / r_mid(p, i);
  } else {
    *wm = 1.0;
    *wp = 1.0;
  }
}

/* number of faces along axis d and the linear index of face (i,j,k) where
 * the d-coordinate runs 0..n_d */
static long face(const Prob* p, int d, int i, int j, int k) {
  int m[3] = {p->n[0], p->n[1], p->n[2]};
  m[d] += 1;
  return (long)i + (long)m[0] * ((long)j + (long)m[1] * k);
}

/* ------------------------------------------------------------------ */
/* Geometry: VoF -> signed distance (section 2.5, Hamilton-Jacobi      */
/* redistancing with the Russo-Smereka interface-cell estimate)        */
/* ------------------------------------------------------------------ */

/* Pin data from the VoF field: the initial level set chi0 = (f - 1/2) h,
 * its sign, the set of cells whose face neighbour has the opposite (or zero)
 * sign, and for those the subcell distance estimate h chi0 / Delta. */
static void pin_data(const Prob* p, const double* vof, double* chi0,
                     signed char* sgn, unsigned char* pinned, double* D) {
  long N = p->ncell;
  #pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    chi0[c] = (vof[c] - 0.5) * p->h;
    sgn[c] = chi0[c] > 0 ? 1 : (chi0[c] < 0 ? -1 : 0);
  }
  #pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < p->n[2]; ++k)
    for (int j = 0; j < p->n[1]; ++j)
      for (int i = 0; i < p->n[0]; ++i) {
        long c = cell(p, i, j, k);
        int cut = 0;
        double jump = 0.0, grad2 = 0.0;
        for (int d = 0; d < p->dim; ++d) {
          long m = nbr(p, i, j, k, d, -1), q = nbr(p, i, j, k, d, +1);
          if (chi0[c] * chi0[m] <= 0.0) cut = 1;
          if (chi0[c] * chi0[q] <= 0.0) cut = 1;
          if (fabs(chi0[m] - chi0[c]) > jump) jump = fabs(chi0[m] - chi0[c]);
          if (fabs(chi0[q] - chi0[c]) > jump) jump = fabs(chi0[q] - chi0[c]);
          double cd = 0.5 * (chi0[q] - chi0[m]);
          grad2 += cd * cd;
        }
        double Delta = sqrt(grad2);
        if (jump > Delta) Delta = jump;
        if (1e-30 * p->h > Delta) Delta = 1e-30 * p->h;
        pinned[c] = (unsigned char)cut;
        D[c] = p->h * chi0[c] / Delta;
      }
}

/* One Jacobi sweep of d chi/d tau + sign(chi0)(|grad chi| - 1) = 0 with the
 * Godunov upwind Hamiltonian, pseudo-time step h/dim, interface cells pinned
 * to their subcell distance, and the result clamped to |chi| <= chi_max. */
static void hj_sweep(const Prob* p, const signed char* sgn,
                     const unsigned char* pinned, const double* D,
                     const double* src, double* dst) {
  double h = p->h, dtau = p->h / p->dim;
  #pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < p->n[2]; ++k)
    for (int j = 0; j < p->n[1]; ++j)
      for (int i = 0; i < p->n[0]; ++i) {
        long c = cell(p, i, j, k);
        double v;
        if (pinned[c]) {
          v = D[c];
        } else {
          double G2 = 0.0;
          for (int d = 0; d < p->dim; ++d) {
            double a = (src[c] - src[nbr(p, i, j, k, d, -1)]) / h; /* backward */
            double b = (src[nbr(p, i, j, k, d, +1)] - src[c]) / h; /* forward */
            double t1, t2;
            if (sgn[c] > 0) {
              t1 = a > 0 ? a * a : 0.0;
              t2 = b < 0 ? b * b : 0.0;
            } else {
              t1 = a < 0 ? a * a : 0.0;
              t2 = b > 0 ? b * b : 0.0;
            }
            G2 += t1 > t2 ? t1 : t2;
          }
          v = src[c] - dtau * sgn[c] * (sqrt(G2) - 1.0);
        }
        if (v > p->chimax) v = p->chimax;
        if (v < -p->chimax) v = -p->chimax;
        dst[c] = v;
      }
}

/* Build chi from vof with `iters` sweeps.  warm = 0 starts from chi0;
 * warm = 1 starts from the chi passed in (the previous step's field). */
int or_geometry(const int* ip, const double* dp, const double* vof, double* chi,
                int iters, int warm) {
  Prob p = unpack(ip, dp);
  long N = p.ncell;
  double* chi0 = malloc(N * sizeof(double));
  double* D = malloc(N * sizeof(double));
  double* tmp = malloc(N * sizeof(double));
  signed char* sgn = malloc(N);
  unsigned char* pin = malloc(N);
  if (!chi0 || !D || !tmp || !sgn || !pin) return -2;
  pin_data(&p, vof, chi0, sgn, pin, D);
  if (!warm) memcpy(chi, chi0, N * sizeof(double));
  /* Jacobi sweeps between two buffers; the last one's result ends in chi */
  double* src = chi;
  double* dst = tmp;
  for (int it = 0; it < iters; ++it) {
    hj_sweep(&p, sgn, pin, D, src, dst);
    double* t = src;
    src = dst;
    dst = t;
  }
  if (src != chi) memcpy(chi, src, N * sizeof(double));
  free(chi0); free(D); free(tmp); free(sgn); free(pin);
  return 0;
}

/* Exposes the pin data for tests (pinned flag and subcell distance). */
int or_pin_data(const int* ip, const double* dp, const double* vof,
                unsigned char* pinned, double* D) {
  Prob p = unpack(ip, dp);
  long N = p.ncell;
  double* chi0 = malloc(N * sizeof(double));
  signed char* sgn = malloc(N);
  if (!chi0 || !sgn) return -2;
  pin_data(&p, vof, chi0, sgn, pinned, D);
  free(chi0); free(sgn);
  return 0;
}

/* Phase field from the signed distance, eq. (redistance):
 * phi = (1 - tanh(chi / 2 eps)) / 2 = 1 / (1 + exp(chi/eps)); its complement
 * is evaluated on its own to avoid cancellation; delta = phi (1-phi) / eps
 * (section 2.6, the numerical estimate of |grad phi|). */
int or_cell_geometry(const int* ip, const double* dp, const double* chi,
                     double* phi, double* omega, double* delta) {
  Prob p = unpack(ip, dp);
  #pragma omp parallel for schedule(static)
  for (long c = 0; c < p.ncell; ++c) {
    double ph = 1.0 / (1.0 + exp(chi[c] / p.eps));
    double om = 1.0 / (1.0 + exp(-chi[c] / p.eps));
    if (phi) phi[c] = ph;
    if (omega) omega[c] = om;
    if (delta) delta[c] = ph * om / p.eps;
  }
  return 0;
}

/* Equation of state (section 2.3 linear and Langmuir, section 6 tanh). */
static double eos(const Prob* p, double G) {
  double x = G / p->ginf;
  if (p->eos == EOS_LINEAR) return p->sigma0 * (1.0 - p->E * x);
  if (p->eos == EOS_LANGMUIR) {
    if (x < 0.0) x = 0.0;
    if (x > 1.0 - 1e-6) x = 1.0 - 1e-6;
    return p->sigma0 * (1.0 + p->E * log(1.0 - x));
  }
  return p->sigma0 * (1.0 - tanh(p->E * x));
}

int or_eos(const int* ip, const double* dp, const double* G, long n, double* sigma) {
  Prob p = unpack(ip, dp);
  for (long c = 0; c < n; ++c) sigma[c] = eos(&p, G[c]);
  return 0;
}

/* Initial state: F = c0 phi (bulk concentration c0 in the liquid) and
 * psi = Gamma0 delta (section 2.6, f = Gamma delta). */
int or_init_state(const int* ip, const double* dp, const double* chi,
                  const double* c0, double c0_const, double gamma0,
                  double* F, double* psi) {
  Prob p = unpack(ip, dp);
  double* phi = malloc(p.ncell * sizeof(double));
  double* del = malloc(p.ncell * sizeof(double));
  if (!phi || !del) return -2;
  or_cell_geometry(ip, dp, chi, phi, NULL, del);
  #pragma omp parallel for schedule(static)
  for (long c = 0; c < p.ncell; ++c) {
    F[c] = (c0 ? c0[c] : c0_const) * phi[c];
    psi[c] = gamma0 * del[c];
  }
  free(phi); free(del);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Substep 1: explicit advection (section 3.1, BCG-type upwind face    */
/* values: the upwind cell's value carried to the half-step foot of    */
/* the characteristic with a limited slope; optionally the transverse  */
/* part of the unsplit BCG predictor)                                  */
/* ------------------------------------------------------------------ */

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

/* Monotonized central limiter (van Leer, J. Comput. Phys. 23, 1977): the
 * centred slope, bounded by twice each one-sided slope, 0 at extrema. */
static double mc_limit(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  double c = 0.5 * (a + b), m = fabs(c);
  if (2.0 * fabs(a) < m) m = 2.0 * fabs(a);
  if (2.0 * fabs(b) < m) m = 2.0 * fabs(b);
  return a > 0.0 ? m : -m;
}

static double slope(const Prob* p, double a, double b) {
  return p->lim == 1 ? mc_limit(a, b) : minmod(a, b);
}

/* Velocity of cell (c) along axis t: the mean of its two t faces (on a
 * periodic axis face n_t is face 0, as in the fluxes). */
static double cell_velocity(const Prob* p, const double* ut, int t, const int* c) {
  int a[3] = {c[0], c[1], c[2]};
  double lo = ut[face(p, t, a[0], a[1], a[2])];
  a[t] += 1;
  if (a[t] == p->n[t] && p->bc[t][0] == BC_PERIODIC) a[t] = 0;
  double hi = ut[face(p, t, a[0], a[1], a[2])];
  return 0.5 * (lo + hi);
}

/* Advective flux u * xi_face through every face along axis d.  out[0] gets
 * the amount leaving the box through open faces (dt * area * flux). */
static void advect_faces(const Prob* p, int d, const double* const* uall, const double* xi,
                         double dt, double* flux, double* out) {
  const double* u = uall[d];
  int m[3] = {p->n[0], p->n[1], p->n[2]};
  m[d] += 1;
  double h = p->h;
  #pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < m[2]; ++k)
    for (int j = 0; j < m[1]; ++j)
      for (int i = 0; i < m[0]; ++i) {
        int c[3] = {i, j, k};
        int fd = c[d], nd = p->n[d];
        long fi = face(p, d, i, j, k);
        int lo_bnd = fd == 0, hi_bnd = fd == nd;
        if ((lo_bnd || hi_bnd) && p->bc[d][hi_bnd] == BC_PERIODIC) {
          if (hi_bnd) continue; /* filled from face 0 below */
        } else if (lo_bnd || hi_bnd) {
          int side = hi_bnd;
          if (p->bc[d][side] == BC_WALL) { flux[fi] = 0.0; continue; }
          /* open: the interior cell's value, either flow direction */
          int ci[3] = {i, j, k};
          ci[d] = hi_bnd ? nd - 1 : 0;
          flux[fi] = u[fi] * xi[cell(p, ci[0], ci[1], ci[2])];
          continue;
        }
        /* interior (or periodic face 0): left cell L, right cell R */
        int cR[3] = {i, j, k};
        if (fd == nd) cR[d] = 0;
        long R = cell(p, cR[0], cR[1], cR[2]);
        long L = nbr(p, cR[0], cR[1], cR[2], d, -1);
        double uf = u[fi];
        int Uc[3] = {cR[0], cR[1], cR[2]};
        double sg;
        if (uf > 0.0) { Uc[d] = cR[d] - 1; if (Uc[d] < 0) Uc[d] += nd; sg = 1.0; }
        else sg = -1.0;
        long U = cell(p, Uc[0], Uc[1], Uc[2]);
        double xm = xi[nbr(p, Uc[0], Uc[1], Uc[2], d, -1)];
        double xp = xi[nbr(p, Uc[0], Uc[1], Uc[2], d, +1)];
        double g = slope(p, (xi[U] - xm) / h, (xp - xi[U]) / h);
        double xf = xi[U] + sg * 0.5 * (h - fabs(uf) * dt) * g;
        /* unsplit BCG: minus dt/2 times v_t d(xi)/dx_t at the upwind cell for
         * each transverse axis t, v_t the cell's mean velocity and the
         * derivative the one-sided difference on its upwind side */
        if (p->trans)
          for (int t = 0; t < p->dim; ++t) {
            if (t == d) continue;
            double vt = cell_velocity(p, uall[t], t, Uc);
            double dxt = vt > 0.0 ? xi[U] - xi[nbr(p, Uc[0], Uc[1], Uc[2], t, -1)]
                                  : xi[nbr(p, Uc[0], Uc[1], Uc[2], t, +1)] - xi[U];
            xf -= 0.5 * dt * vt * dxt / h;
          }
        (void)L;
        flux[fi] = uf * xf;
      }
  /* what leaves through open faces, summed in face order */
  for (int k = 0; k < m[2]; ++k)
    for (int j = 0; j < m[1]; ++j)
      for (int i = 0; i < m[0]; ++i) {
        int c[3] = {i, j, k};
        int hi_bnd = c[d] == p->n[d];
        if ((c[d] != 0 && !hi_bnd) || p->bc[d][hi_bnd] != BC_OPEN) continue;
        double v = flux[face(p, d, i, j, k)];
        out[0] += dt * face_area(p, d, i) * (hi_bnd ? v : -v);
      }
  /* periodic: the last face is the first face */
  if (p->bc[d][0] == BC_PERIODIC)
    for (int k = 0; k < m[2]; ++k)
      for (int j = 0; j < m[1]; ++j)
        for (int i = 0; i < m[0]; ++i) {
          int c[3] = {i, j, k};
          if (c[d] != p->n[d]) continue;
          int c0[3] = {i, j, k};
          c0[d] = 0;
          flux[face(p, d, i, j, k)] = flux[face(p, d, c0[0], c0[1], c0[2])];
        }
}

/* xi* = xi - dt/h * sum_d (w_+ flux_{+1/2} - w_- flux_{-1/2}), the weights
 * 1 except on radial faces in the axisymmetric case */
int or_advect(const int* ip, const double* dp, const double* ux, const double* uy,
              const double* uz, const double* xi, double dt, double* xs,
              double* outflow) {
  Prob p = unpack(ip, dp);
  const double* u[3] = {ux, uy, uz};
  double* fl[3] = {NULL, NULL, NULL};
  double out = 0.0;
  for (int d = 0; d < p.dim; ++d) {
    long nf = p.ncell / p.n[d] * (p.n[d] + 1);
    fl[d] = malloc(nf * sizeof(double));
    if (!fl[d]) return -2;
    advect_faces(&p, d, u, xi, dt, fl[d], &out);
  }
  #pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < p.n[2]; ++k)
    for (int j = 0; j < p.n[1]; ++j)
      for (int i = 0; i < p.n[0]; ++i) {
        long c = cell(&p, i, j, k);
        double div = 0.0;
        for (int d = 0; d < p.dim; ++d) {
          int a[3] = {i, j, k};
          long fm = face(&p, d, a[0], a[1], a[2]);
          a[d] += 1;
          long fp = face(&p, d, a[0], a[1], a[2]);
          double wm, wp;
          div_weights(&p, d, i, &wm, &wp);
          div += wp * fl[d][fp] - wm * fl[d][fm];
        }
        xs[c] = xi[c] - dt / p.h * div;
      }
  for (int d = 0; d < p.dim; ++d) free(fl[d]);
  if (outflow) *outflow = out;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Substep 2 fluxes (sections 2.6 and 3.2, Appendix A)                 */
/* ------------------------------------------------------------------ */

/* Diffusive plus anti-diffusive flux through every face along axis d for
 * one field.  Weighted form: D * wbar * (r_R - r_L)/h with r = xi / w,
 * w = phi (+eta) for the bulk and delta (+eta/eps) for the carrier -- the
 * same continuous flux as D grad xi + B xi.  Paper form: centred diffusion
 * plus B xi with B averaged to the face and xi taken upwind of the
 * transport velocity -B. */
static void substep2_faces(const Prob* p, int d, int is_bulk, const double* xs,
                           const double* phi, const double* omega,
                           const double* delta, const double* Bcell,
                           double* flux) {
  int m[3] = {p->n[0], p->n[1], p->n[2]};
  m[d] += 1;
  double h = p->h, D = is_bulk ? p->Db : p->Ds;
  (void)omega;
  #pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < m[2]; ++k)
    for (int j = 0; j < m[1]; ++j)
      for (int i = 0; i < m[0]; ++i) {
        int c[3] = {i, j, k};
        int fd = c[d], nd = p->n[d];
        long fi = face(p, d, i, j, k);
        if ((fd == 0 || fd == nd) && p->bc[d][fd == nd] != BC_PERIODIC) {
          flux[fi] = 0.0; /* walls and open faces carry no diffusive flux */
          continue;
        }
        int cR[3] = {i, j, k};
        if (fd == nd) cR[d] = 0;
        long R = cell(p, cR[0], cR[1], cR[2]);
        long L = nbr(p, cR[0], cR[1], cR[2], d, -1);
        if (p->form == FORM_WEIGHTED) {
          double wL, wR, rL, rR;
          if (is_bulk) {
            wL = phi[L]; wR = phi[R];
            rL = xs[L] / (phi[L] + p->eta); rR = xs[R] / (phi[R] + p->eta);
          } else {
            wL = delta[L]; wR = delta[R];
            rL = xs[L] / (delta[L] + p->eta / p->eps);
            rR = xs[R] / (delta[R] + p->eta / p->eps);
          }
          flux[fi] = D * 0.5 * (wL + wR) * (rR - rL) / h;
        } else {
          double Bf = 0.5 * (Bcell[L] + Bcell[R]);
          double up = Bf < 0.0 ? xs[L] : xs[R];
          flux[fi] = D * (xs[R] - xs[L]) / h + Bf * up;
        }
      }
}

/* Paper form: per-cell anti-diffusion coefficient along axis d,
 * B_F = -D_F (1-phi)/eps n,  B_f = -D_f 2(0.5-phi)/eps n, with
 * n = grad phi/|grad phi| = -grad chi/|grad chi| from centred differences. */
static void paper_B(const Prob* p, int d, int is_bulk, const double* chi,
                    const double* phi, const double* omega, double* B) {
  double D = is_bulk ? p->Db : p->Ds;
  #pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < p->n[2]; ++k)
    for (int j = 0; j < p->n[1]; ++j)
      for (int i = 0; i < p->n[0]; ++i) {
        long c = cell(p, i, j, k);
        double g[3] = {0, 0, 0}, nrm = 0.0;
        for (int e = 0; e < p->dim; ++e) {
          g[e] = (chi[nbr(p, i, j, k, e, 1)] - chi[nbr(p, i, j, k, e, -1)]) / (2.0 * p->h);
          nrm += g[e] * g[e];
        }
        nrm = sqrt(nrm);
        if (nrm < 1e-6) nrm = 1e-6;
        double n_d = -g[d] / nrm;
        double w = is_bulk ? omega[c] : (omega[c] - phi[c]);
        B[c] = -D * w / p->eps * n_d;
      }
}

/* ------------------------------------------------------------------ */
/* One full step                                                       */
/* ------------------------------------------------------------------ */

typedef struct { double s, c; } Kahan;
static void kadd(Kahan* k, double v) {
  double y = v - k->c, t = k->s + y;
  k->c = (t - k->s) - y;
  k->s = t;
}

/* Advances (F, psi) over dt: substep 1 (advection with u, skipped when
 * ux == NULL), then substep 2 (diffusion + anti-diffusion + source) taken
 * explicitly from the advected state, then the equation of state.
 * totals (16 doubles) is read for the running time and cumulative outflow
 * and rewritten.  chi is the level set of the new interface position. */
int or_step(const int* ip, const double* dp, const double* chi,
            const double* ux, const double* uy, const double* uz,
            const double* F, const double* psi, double dt,
            double* Fout, double* psiout, double* sigma, double* totals) {
  Prob p = unpack(ip, dp);
  long N = p.ncell;
  double* phi = malloc(N * sizeof(double));
  double* om = malloc(N * sizeof(double));
  double* del = malloc(N * sizeof(double));
  double* Fs = malloc(N * sizeof(double));
  double* Ps = malloc(N * sizeof(double));
  double* B = malloc(N * sizeof(double));
  double* q = malloc(N * sizeof(double));
  double* divF = calloc(N, sizeof(double));
  double* divP = calloc(N, sizeof(double));
  if (!phi || !om || !del || !Fs || !Ps || !B || !q || !divF || !divP) return -2;
  or_cell_geometry(ip, dp, chi, phi, om, del);

  /* substep 1: advection of both fields with u^n */
  double outF = 0.0, outP = 0.0;
  if (ux) {
    if (p.bulk) or_advect(ip, dp, ux, uy, uz, F, dt, Fs, &outF);
    or_advect(ip, dp, ux, uy, uz, psi, dt, Ps, &outP);
  } else {
    if (p.bulk) memcpy(Fs, F, N * sizeof(double));
    memcpy(Ps, psi, N * sizeof(double));
  }
  if (!p.bulk) memcpy(Fs, F, N * sizeof(double));

  /* substep 2 fluxes from the advected state */
  for (int d = 0; d < p.dim; ++d) {
    long nf = N / p.n[d] * (p.n[d] + 1);
    double* fl = malloc(nf * sizeof(double));
    if (!fl) return -2;
    for (int field = 0; field < 2; ++field) {
      int is_bulk = field == 0;
      if (is_bulk && !p.bulk) continue;
      if (p.form == FORM_PAPER) paper_B(&p, d, is_bulk, chi, phi, om, B);
      substep2_faces(&p, d, is_bulk, is_bulk ? Fs : Ps, phi, om, del, B, fl);
      double* div = is_bulk ? divF : divP;
      #pragma omp parallel for collapse(2) schedule(static)
      for (int k = 0; k < p.n[2]; ++k)
        for (int j = 0; j < p.n[1]; ++j)
          for (int i = 0; i < p.n[0]; ++i) {
            int a[3] = {i, j, k};
            long fm = face(&p, d, a[0], a[1], a[2]);
            a[d] += 1;
            long fp = face(&p, d, a[0], a[1], a[2]);
            double wm, wp;
            div_weights(&p, d, i, &wm, &wp);
            div[cell(&p, i, j, k)] += (wp * fl[fp] - wm * fl[fm]) / p.h;
          }
    }
    free(fl);
  }

  /* adsorption/desorption exchange, section 2.6 and Appendix C:
   * q = delta J with J = k_a c (Gamma_inf - Gamma) - k_d Gamma, c = F/phi,
   * written with psi = Gamma delta as k_a c (Gamma_inf delta - psi) - k_d psi;
   * the Henry (constant adsorption flux) law of section 4.3.1 drops the
   * saturation factor: k_a c Gamma_inf delta - k_d psi. */
  #pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    if (!p.bulk) { q[c] = 0.0; continue; }
    double cs = Fs[c] / (phi[c] + p.eta);
    if (p.kin == KIN_LANGMUIR)
      q[c] = p.ka * cs * (p.ginf * del[c] - Ps[c]) - p.kd * Ps[c];
    else
      q[c] = p.ka * cs * p.ginf * del[c] - p.kd * Ps[c];
  }

  /* update and equation of state */
  #pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    Fout[c] = p.bulk ? Fs[c] + dt * (divF[c] - q[c]) : F[c];
    psiout[c] = Ps[c] + dt * (divP[c] + q[c]);
    double G = psiout[c] / (del[c] + p.eta / p.eps);
    if (sigma) sigma[c] = eos(&p, G);
  }

  /* totals (FP64, compensated sums in cell order) */
  if (totals) {
    Kahan mb = {0, 0}, ms = {0, 0}, sd = {0, 0}, ssd = {0, 0};
    double minF = INFINITY, minP = INFINITY, cmax = -INFINITY, nbad = 0, su = 0.0;
    double* colvol = malloc(p.n[0] * sizeof(double)); /* cell volume by column */
    if (!colvol) return -2;
    for (int i = 0; i < p.n[0]; ++i) colvol[i] = cell_volume(&p, i);
    for (long c = 0; c < N; ++c) {
      double vol = colvol[c % p.n[0]];
      double sg = sigma ? sigma[c] : eos(&p, psiout[c] / (del[c] + p.eta / p.eps));
      kadd(&mb, Fout[c] * vol);
      kadd(&ms, psiout[c] * vol);
      kadd(&sd, del[c] * vol);
      kadd(&ssd, sg * del[c] * vol);
      if (Fout[c] < minF) minF = Fout[c];
      if (psiout[c] < minP) minP = psiout[c];
      double cc = Fout[c] / (phi[c] + p.eta);
      if (cc > cmax) cmax = cc;
      if (!isfinite(Fout[c]) || !isfinite(psiout[c]) || !isfinite(sg)) nbad += 1;
    }
    free(colvol);
    if (ux) {
      const double* u[3] = {ux, uy, uz};
      #pragma omp parallel for collapse(2) schedule(static) reduction(max : su)
      for (int k = 0; k < p.n[2]; ++k)
        for (int j = 0; j < p.n[1]; ++j)
          for (int i = 0; i < p.n[0]; ++i) {
            double s = 0.0;
            for (int d = 0; d < p.dim; ++d) {
              int a[3] = {i, j, k};
              double um = u[d][face(&p, d, a[0], a[1], a[2])];
              a[d] += 1;
              if (p.bc[d][1] == BC_PERIODIC && a[d] == p.n[d]) a[d] = 0; /* face n_d is face 0 */
              double up = u[d][face(&p, d, a[0], a[1], a[2])];
              /* axisymmetric: the radial mean weights each face by r_face/r_i */
              double wm, wp;
              div_weights(&p, d, i, &wm, &wp);
              s += fabs(0.5 * (wm * um + wp * up));
            }
            if (s > su) su = s;
          }
    }
    double outstep = outF + outP;
    double outcum = totals[T_OUTCUM] + outstep;
    double t = totals[T_T] + dt;
    /* stability bound of the explicit split step (substep 1: advective
     * Courant number; substep 2: sum of the diagonal coefficients) */
    double Dmax = p.bulk ? (p.Db > p.Ds ? p.Db : p.Ds) : p.Ds;
    double nd = p.dim;
    double lam = p.form == FORM_WEIGHTED
                     ? Dmax * (2.0 * nd - 1.0 + cosh(p.h / p.eps)) / (p.h * p.h)
                     : Dmax * (2.0 * nd / (p.h * p.h) + sqrt(nd) / (p.eps * p.h));
    if (p.bulk) lam += p.ka * p.ginf / p.eps + p.ka * (cmax > 0 ? cmax : 0.0) + p.kd;
    double dta = su > 0 ? p.cfl_a * p.h / su : INFINITY;
    double dtd = p.cfl_d / lam;
    totals[T_MB] = p.bulk ? mb.s : 0.0; /* the insoluble model has no bulk field */
    totals[T_MS] = ms.s;
    totals[T_OUT] = outstep;
    totals[T_OUTCUM] = outcum;
    totals[T_SDELTA] = sd.s;
    totals[T_SSIGD] = ssd.s;
    totals[T_SU] = su;
    totals[T_DTNEXT] = dta < dtd ? dta : dtd;
    totals[T_MINF] = p.bulk ? minF : 0.0;
    totals[T_MINPSI] = minP;
    totals[T_NBAD] = nbad;
    totals[T_T] = t;
    totals[T_GAVG] = ms.s / sd.s;
    totals[T_SAVG] = ssd.s / sd.s;
    totals[T_MTOT] = (p.bulk ? mb.s : 0.0) + ms.s + outcum;
    totals[T_CMAX] = p.bulk ? cmax : 0.0;
  }
  free(phi); free(om); free(del); free(Fs); free(Ps); free(B); free(q);
  free(divF); free(divP);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Marangoni face force, section 2.4: F = delta_m (I - n n) grad sigma  */
/* evaluated on the faces of the velocity grid                          */
/* ------------------------------------------------------------------ */

/* Face gradient of a cell field at the face between L and R along d:
 * compact normal difference, transverse centred differences averaged over
 * the two cells. */
static void face_grad(const Prob* p, const double* v, int d, const int* cL,
                      const int* cR, long L, long R, double* g) {
  for (int e = 0; e < p->dim; ++e) {
    if (e == d) {
      g[e] = (v[R] - v[L]) / p->h;
    } else {
      double tl = v[nbr(p, cL[0], cL[1], cL[2], e, 1)] - v[nbr(p, cL[0], cL[1], cL[2], e, -1)];
      double tr = v[nbr(p, cR[0], cR[1], cR[2], e, 1)] - v[nbr(p, cR[0], cR[1], cR[2], e, -1)];
      g[e] = (tl + tr) / (4.0 * p->h);
    }
  }
}

int or_force(const int* ip, const double* dp, const double* chi,
             const double* sigma, double* fx, double* fy, double* fz) {
  Prob p = unpack(ip, dp);
  double* out[3] = {fx, fy, fz};
  double* del = malloc(p.ncell * sizeof(double));
  if (!del) return -2;
  or_cell_geometry(ip, dp, chi, NULL, NULL, del);
  for (int d = 0; d < p.dim; ++d) {
    int m[3] = {p.n[0], p.n[1], p.n[2]};
    m[d] += 1;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < m[2]; ++k)
      for (int j = 0; j < m[1]; ++j)
        for (int i = 0; i < m[0]; ++i) {
          int c[3] = {i, j, k};
          int fd = c[d], nd = p.n[d];
          long fi = face(&p, d, i, j, k);
          if ((fd == 0 || fd == nd) && p.bc[d][fd == nd] != BC_PERIODIC) {
            out[d][fi] = 0.0;
            continue;
          }
          int cR[3] = {i, j, k};
          if (fd == nd) cR[d] = 0;
          int cL[3] = {cR[0], cR[1], cR[2]};
          cL[d] = cR[d] - 1 < 0 ? nd - 1 : cR[d] - 1;
          long R = cell(&p, cR[0], cR[1], cR[2]);
          long L = cell(&p, cL[0], cL[1], cL[2]);
          double gn[3] = {0, 0, 0}, gs[3] = {0, 0, 0};
          face_grad(&p, chi, d, cL, cR, L, R, gn);
          face_grad(&p, sigma, d, cL, cR, L, R, gs);
          double nrm = 0.0;
          for (int e = 0; e < p.dim; ++e) nrm += gn[e] * gn[e];
          nrm = sqrt(nrm);
          if (nrm < 1e-6) nrm = 1e-6;
          double ndot = 0.0;
          for (int e = 0; e < p.dim; ++e) ndot += gn[e] / nrm * gs[e];
          double dbar = 0.5 * (del[L] + del[R]);
          out[d][fi] = dbar * (gs[d] - gn[d] / nrm * ndot);
        }
  }
  free(del);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Discrete adjoint of one step (weighted flux form) and the gradient  */
/* of the interface-averaged surface tension                           */
/* ------------------------------------------------------------------ */

/* Linearisation of the advective flux through one face with the minmod
 * branch frozen at the current state: flux = wa xi[a] + wb xi[b] + wc xi[c]
 * (a behind the upwind cell b, c downwind).  Returns the number of cells
 * used (0 wall, 1 open boundary, 3 interior) and the left/right cells of the
 * face (-1 when outside the box). */
static int flux_lin(const Prob* p, int d, int i, int j, int k, const double* u,
                    const double* xi, double dt, long* cells, double* w,
                    long* L, long* R) {
  int c[3] = {i, j, k};
  int fd = c[d], nd = p->n[d];
  long fi = face(p, d, i, j, k);
  int lo = fd == 0, hi = fd == nd;
  *L = -1;
  *R = -1;
  if ((lo || hi) && p->bc[d][hi] != BC_PERIODIC) {
    if (p->bc[d][hi] == BC_WALL) return 0;
    int ci[3] = {i, j, k};
    ci[d] = hi ? nd - 1 : 0;
    long b = cell(p, ci[0], ci[1], ci[2]);
    if (hi) *L = b; else *R = b;
    cells[0] = b;
    w[0] = u[fi];
    return 1;
  }
  int cR[3] = {i, j, k};
  if (fd == nd) cR[d] = 0;
  long Rc = cell(p, cR[0], cR[1], cR[2]);
  long Lc = nbr(p, cR[0], cR[1], cR[2], d, -1);
  *L = Lc;
  *R = Rc;
  double uf = u[face(p, d, cR[0], cR[1], cR[2])];
  int Uc[3] = {cR[0], cR[1], cR[2]};
  double sg;
  if (uf > 0.0) { Uc[d] = cR[d] - 1; if (Uc[d] < 0) Uc[d] += nd; sg = 1.0; }
  else sg = -1.0;
  long b = cell(p, Uc[0], Uc[1], Uc[2]);
  long m = nbr(p, Uc[0], Uc[1], Uc[2], d, -1);
  long q = nbr(p, Uc[0], Uc[1], Uc[2], d, +1);
  /* slope g = minmod(s1, s2), s1 = (xi_b - xi_m)/h, s2 = (xi_q - xi_b)/h */
  double s1 = (xi[b] - xi[m]) / p->h, s2 = (xi[q] - xi[b]) / p->h;
  double sel1 = 0.0, sel2 = 0.0;
  if (s1 * s2 > 0.0) {
    if (fabs(s1) < fabs(s2)) sel1 = 1.0; else sel2 = 1.0;
  }
  /* xi_f = xi_b + kk (sel1 s1 + sel2 s2), kk = sg (h - |u| dt)/2 */
  double kk = sg * 0.5 * (p->h - fabs(uf) * dt) / p->h;
  cells[0] = m; w[0] = uf * (-kk * sel1);
  cells[1] = b; w[1] = uf * (1.0 + kk * sel1 - kk * sel2);
  cells[2] = q; w[2] = uf * (kk * sel2);
  return 3;
}

/* lamF, lamP (the adjoint state at t^n) from mF, mP (at t^{n+1}) for the step
 * taken from (F, psi) at t^n; adds dL/d(k_a, k_d, D_b, D_s) to dtheta.  The
 * loss term of t^n is not included (see or_loss_grad). */
int or_adjoint_step(const int* ip, const double* dp, const double* chi,
                    const double* ux, const double* uy, const double* uz,
                    const double* F, const double* psi, double dt,
                    const double* mF, const double* mP, double* lF, double* lP,
                    double* dtheta) {
  Prob p = unpack(ip, dp);
  if (p.form != FORM_WEIGHTED) return -1;
  long N = p.ncell;
  const double* u[3] = {ux, uy, uz};
  double* phi = malloc(N * sizeof(double));
  double* om = malloc(N * sizeof(double));
  double* del = malloc(N * sizeof(double));
  double* Fs = malloc(N * sizeof(double));
  double* Ps = malloc(N * sizeof(double));
  double* nF = malloc(N * sizeof(double));
  double* nP = malloc(N * sizeof(double));
  double* SF = calloc(N, sizeof(double));
  double* SP = calloc(N, sizeof(double));
  if (!phi || !om || !del || !Fs || !Ps || !nF || !nP || !SF || !SP) return -2;
  or_cell_geometry(ip, dp, chi, phi, om, del);

  /* forward substep 1 (the advected state the source and fluxes act on) */
  if (ux) {
    if (p.bulk) or_advect(ip, dp, ux, uy, uz, F, dt, Fs, NULL);
    else memcpy(Fs, F, N * sizeof(double));
    or_advect(ip, dp, ux, uy, uz, psi, dt, Ps, NULL);
  } else {
    memcpy(Fs, F, N * sizeof(double));
    memcpy(Ps, psi, N * sizeof(double));
  }

  /* transpose of substep 2: nu = mu + dt (L^T mu + dq^T (mu_psi - mu_F)) */
  for (long c = 0; c < N; ++c) {
    nF[c] = mF[c];
    nP[c] = mP[c];
  }
  for (int d = 0; d < p.dim; ++d) {
    int m[3] = {p.n[0], p.n[1], p.n[2]};
    m[d] += 1;
    for (int k = 0; k < m[2]; ++k)
      for (int j = 0; j < m[1]; ++j)
        for (int i = 0; i < m[0]; ++i) {
          int cc[3] = {i, j, k};
          int fd = cc[d], nd = p.n[d];
          if (fd == nd && p.bc[d][1] == BC_PERIODIC) continue; /* face 0 covers it */
          if ((fd == 0 || fd == nd) && p.bc[d][fd == nd] != BC_PERIODIC) continue;
          int cR[3] = {i, j, k};
          long R = cell(&p, cR[0], cR[1], cR[2]);
          long L = nbr(&p, cR[0], cR[1], cR[2], d, -1);
          double h2 = p.h * p.h;
          if (p.bulk) {
            /* forward: F+_L += dt wF (c_R - c_L), F+_R -= dt wF (c_R - c_L) */
            double wF = p.Db * 0.5 * (phi[L] + phi[R]) / h2;
            double dmu = mF[L] - mF[R];
            nF[R] += dt * wF * dmu / (phi[R] + p.eta);
            nF[L] -= dt * wF * dmu / (phi[L] + p.eta);
            double flux = 0.5 * (phi[L] + phi[R]) / h2 *
                          (Fs[R] / (phi[R] + p.eta) - Fs[L] / (phi[L] + p.eta));
            SF[L] += flux;
            SF[R] -= flux;
          }
          double wP = p.Ds * 0.5 * (del[L] + del[R]) / h2;
          double eL = del[L] + p.eta / p.eps, eR = del[R] + p.eta / p.eps;
          double dmu = mP[L] - mP[R];
          nP[R] += dt * wP * dmu / eR;
          nP[L] -= dt * wP * dmu / eL;
          double flux = 0.5 * (del[L] + del[R]) / h2 * (Ps[R] / eR - Ps[L] / eL);
          SP[L] += flux;
          SP[R] -= flux;
        }
  }
  double dka = 0.0, dkd = 0.0, dDb = 0.0, dDs = 0.0;
  for (long c = 0; c < N; ++c) {
    double diff = mP[c] - mF[c];
    if (p.bulk) {
      double cs = Fs[c] / (phi[c] + p.eta);
      double dqdF, dqdP, dqdka, dqdkd = -Ps[c];
      if (p.kin == KIN_LANGMUIR) {
        dqdF = p.ka * (p.ginf * del[c] - Ps[c]) / (phi[c] + p.eta);
        dqdP = -p.ka * cs - p.kd;
        dqdka = cs * (p.ginf * del[c] - Ps[c]);
      } else {
        dqdF = p.ka * p.ginf * del[c] / (phi[c] + p.eta);
        dqdP = -p.kd;
        dqdka = cs * p.ginf * del[c];
      }
      nF[c] += dt * dqdF * diff;
      nP[c] += dt * dqdP * diff;
      dka += dt * dqdka * diff;
      dkd += dt * dqdkd * diff;
      dDb += dt * SF[c] * mF[c];
    }
    dDs += dt * SP[c] * mP[c];
  }
  dtheta[0] += dka;
  dtheta[1] += dkd;
  dtheta[2] += dDb;
  dtheta[3] += dDs;

  /* transpose of substep 1 */
  for (long c = 0; c < N; ++c) {
    lF[c] = p.bulk ? nF[c] : mF[c];
    lP[c] = nP[c];
  }
  if (ux) {
    for (int d = 0; d < p.dim; ++d) {
      int m[3] = {p.n[0], p.n[1], p.n[2]};
      m[d] += 1;
      for (int k = 0; k < m[2]; ++k)
        for (int j = 0; j < m[1]; ++j)
          for (int i = 0; i < m[0]; ++i) {
            int cc[3] = {i, j, k};
            if (cc[d] == p.n[d] && p.bc[d][1] == BC_PERIODIC) continue;
            long cells[3], L, R;
            double w[3];
            for (int f = 0; f < 2; ++f) {
              if (f == 0 && !p.bulk) continue;
              const double* xi = f == 0 ? F : psi;
              const double* nu = f == 0 ? nF : nP;
              double* lam = f == 0 ? lF : lP;
              int nc = flux_lin(&p, d, i, j, k, u[d], xi, dt, cells, w, &L, &R);
              double g = (R >= 0 ? nu[R] : 0.0) - (L >= 0 ? nu[L] : 0.0);
              for (int s = 0; s < nc; ++s) lam[cells[s]] += dt / p.h * w[s] * g;
            }
          }
    }
  }
  free(phi); free(om); free(del); free(Fs); free(Ps); free(nF); free(nP);
  free(SF); free(SP);
  return 0;
}

/* derivative of the equation of state */
static double eos_prime(const Prob* p, double G) {
  double x = G / p->ginf;
  if (p->eos == EOS_LINEAR) return -p->sigma0 * p->E / p->ginf;
  if (p->eos == EOS_LANGMUIR) {
    if (x <= 0.0 || x >= 1.0 - 1e-6) return 0.0; /* clamped */
    return -p->sigma0 * p->E / (p->ginf * (1.0 - x));
  }
  double t = tanh(p->E * x);
  return -p->sigma0 * p->E / p->ginf * (1.0 - t * t);
}

/* gP = w d<sigma>/dpsi * sum(delta) = w sigma'(Gamma) delta / (delta + eta/eps)
 * where <sigma> = sum sigma delta / sum delta and Gamma = psi/(delta+eta/eps):
 * the loss term of a step for the weight w = dL/d<sigma> / sum(delta). */
int or_loss_grad(const int* ip, const double* dp, const double* chi, const double* psi,
                 double w, double* gP) {
  Prob p = unpack(ip, dp);
  double* del = malloc(p.ncell * sizeof(double));
  if (!del) return -2;
  or_cell_geometry(ip, dp, chi, NULL, NULL, del);
  #pragma omp parallel for schedule(static)
  for (long c = 0; c < p.ncell; ++c) {
    double e = del[c] + p.eta / p.eps;
    gP[c] = w * eos_prime(&p, psi[c] / e) * del[c] / e;
  }
  free(del);
  return 0;
}
