/*
 * surf.h -- C ABI of libsurf, the MI355X (gfx950) hybrid VoF/Phase-Field
 * soluble-surfactant transport step.
 *
 * One step advances the bulk concentration F and the interfacial carrier
 * psi = Gamma * delta (paper section 2.6) across a time step:
 *   geometry   VoF fraction -> signed distance chi by Hamilton-Jacobi
 *              redistancing (section 2.5), phi = 1/(1+exp(chi/eps)),
 *              delta = phi (1-phi)/eps (eq. (redistance), section 2.6);
 *   substep 1  explicit conservative advection (section 3.1);
 *   substep 2  confinement + diffusion + exchange source, explicit
 *              (sections 2.6, 3.1, 3.2, Appendices A and C);
 *   EoS        sigma(Gamma) (sections 2.3, 5, 6);
 * plus the Marangoni face force delta (I - n n) grad sigma (section 2.4).
 * Options of the same step: substep 2 implicit (section 3.1, Appendix C),
 * the ACDI phase field in place of the per-step level set (section 2.5),
 * axisymmetric rings (Appendix B), and the MC limiter and transverse term
 * of the unsplit BCG advection (section 3.1).  Beside the step: the
 * capillary and PLIC Marangoni forces for a flow solver (section 2.4), a
 * batched form for many small instances, and the discrete adjoint.
 *
 * Conventions
 *  - Every function returns SURF_OK (0) or a negative SURF_E* code; no
 *    exception crosses the ABI.  surf_strerror() names a code.
 *  - Ownership: the caller owns every field buffer and the workspace (device
 *    memory).  The library never allocates or frees device memory; it owns
 *    only its host-side context objects.
 *  - Streams: every call is asynchronous on the HIP stream given at init
 *    (a hipStream_t passed as void*; NULL = the null stream).  A context is
 *    bound to one stream and is not thread-safe.
 *  - Layout: cell fields are contiguous [nz][ny][nx] (x fastest), one buffer
 *    per field.  Face fields along axis d hold n_d + 1 entries along d:
 *    x faces [nz][ny][nx+1], y faces [nz][ny+1][nx], z faces [nz+1][ny][nx].
 *    2D problems use dim = 2, n[2] = 1 and no z face array.
 *  - Element type: every field buffer has the context precision (float for
 *    SURF_F32, double for SURF_F64).  Totals are always double.
 *  - Pointers must be device pointers aligned to their element size.
 *  - Numerical health is reported through a sticky status word
 *    (surf_get_status), not through return codes.
 *  - Deliberate shapes of some calls: surf_init_state takes the bulk
 *    concentration c0 and no VoF field (the level set comes first, from
 *    surf_set_geometry); surf_force takes sigma, which surf_step returns,
 *    rather than psi; surf_batch_create binds each instance's pair of state
 *    buffers once and surf_batch_step takes none (the parity says which
 *    buffer holds the state); surf_adjoint_step takes the loss weight w_n of
 *    its own time level, so that one call adds that level's loss term.
 */
#ifndef SURF_H
#define SURF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define SURF_OK 0
#define SURF_EINVAL (-1)    /* bad argument (null, size, range, alias)      */
#define SURF_ENOMEM (-2)    /* workspace too small                          */
#define SURF_EDEVICE (-3)   /* a HIP runtime error (launch or device)       */
#define SURF_ESTATE (-4)    /* call-order violation (e.g. no geometry yet)  */
#define SURF_EUNSTABLE (-5) /* reserved: reported through status bits       */

/* status bits (sticky until surf_clear_status) */
#define SURF_STATUS_NONFINITE 1u /* a non-finite F, psi or sigma was produced */
#define SURF_STATUS_NEGATIVE 2u  /* a negative F or psi was produced          */
#define SURF_STATUS_UNSTABLE 4u  /* dt exceeded the explicit stability bound  */
#define SURF_STATUS_GEOMETRY 8u  /* the VoF changed under a tile whose whole
                                  * neighbourhood was outside the band: the
                                  * interface moved farther than the clamp
                                  * distance in one step (level set stale).
                                  * A geometry prepared on a second stream
                                  * (surf_prepare_geometry) raises it when it
                                  * runs, so under pipelining it can show in
                                  * the status of the step before the one
                                  * that consumes that geometry             */
#define SURF_STATUS_SOLVE 16u    /* implicit substep 2: a linear solve ended at
                                  * cg_max_iters without meeting its test, or
                                  * broke down (matrix not positive definite) */

enum { SURF_F32 = 0, SURF_F64 = 1 };
/* substep-2 flux: weighted form D wbar grad(xi/w) (default) or the paper's
 * centred-diffusion + upwind anti-diffusion form (section 3.2) */
enum { SURF_FLUX_WEIGHTED = 0, SURF_FLUX_PAPER = 1 };
/* substep 2 in time: explicit Euler from the advected state (default), or
 * implicit Euler (section 3, Appendix C), with the interfacial and bulk
 * problems solved alternately in FP64 by Jacobi-preconditioned conjugate
 * gradients (weighted form: symmetric matrices) or BiCGSTAB (paper form:
 * the upwind anti-diffusion makes them non-symmetric) */
enum { SURF_SUBSTEP2_EXPLICIT = 0, SURF_SUBSTEP2_IMPLICIT = 1 };
/* the interface: the level set rebuilt from the VoF given to every moving
 * step (default), or the phase field phi evolved by ACDI (section 2.5, the
 * Phase-Field method) and re-initialized from a VoF field only when one is
 * given */
enum { SURF_IFACE_VOF = 0, SURF_IFACE_ACDI = 1 };
/* slope limiter of the substep-1 face values (section 3.1): minmod (default)
 * or the monotonized central limiter of van Leer (1977) */
enum { SURF_LIMITER_MINMOD = 0, SURF_LIMITER_MC = 1 };
/* exchange law: Langmuir J = k_a c (Gamma_inf - Gamma) - k_d Gamma
 * (section 2.6) or constant adsorption flux J = k_a c Gamma_inf - k_d Gamma
 * (section 4.3.1) */
enum { SURF_KIN_LANGMUIR = 0, SURF_KIN_HENRY = 1 };
/* sigma0 (1 - E x), sigma0 (1 + E ln(1 - x)), sigma0 (1 - tanh(E x)),
 * x = Gamma / Gamma_inf (sections 2.3, 5 and 6) */
enum { SURF_EOS_LINEAR = 0, SURF_EOS_LANGMUIR = 1, SURF_EOS_TANH = 2 };
/* box faces: no flux; wrap; open (advective outflow/inflow of the adjacent
 * cell value, no diffusive flux, counted in the boundary total) */
enum { SURF_BC_WALL = 0, SURF_BC_PERIODIC = 1, SURF_BC_OPEN = 2 };

/* slots of the 16-double totals record written by surf_step */
enum {
  SURF_T_MASS_BULK = 0,   /* sum F h^d after the step                      */
  SURF_T_MASS_SURF = 1,   /* sum psi h^d                                   */
  SURF_T_OUTFLOW = 2,     /* amount leaving through open faces this step   */
  SURF_T_OUTFLOW_CUM = 3, /* cumulative outflow since init_state           */
  SURF_T_SUM_DELTA = 4,   /* sum delta h^d (interface measure)             */
  SURF_T_SUM_SIGDELTA = 5,/* sum sigma delta h^d                           */
  SURF_T_MAX_USUM = 6,    /* max over cells of sum_d |cell-mean u_d|       */
  SURF_T_DT_NEXT = 7,     /* safety-factored explicit dt bound             */
  SURF_T_MIN_F = 8,       /* min F                                         */
  SURF_T_MIN_PSI = 9,     /* min psi                                       */
  SURF_T_NONFINITE = 10,  /* count of cells with a non-finite output       */
  SURF_T_TIME = 11,       /* time after the step                           */
  SURF_T_GAMMA_AVG = 12,  /* interface average sum psi / sum delta         */
  SURF_T_SIGMA_AVG = 13,  /* interface average sum sigma delta / sum delta */
  SURF_T_MASS_TOTAL = 14, /* bulk + interfacial + cumulative outflow       */
  SURF_T_C_MAX = 15       /* max F / (phi + eta)                           */
};

typedef struct surf_ctx surf_ctx;
typedef struct surf_batch surf_batch;

/* The domain (section 3.2 and Appendix A: uniform Cartesian cells; with
 * axisym, the rings of Appendix B). */
typedef struct {
  int32_t dim;       /* 2 or 3                                     */
  int32_t n[3];      /* cells per axis; n[2] = 1 in 2D              */
  int32_t bc[3][2];  /* SURF_BC_* per box face (lo, hi); periodic
                        axes must be periodic on both sides          */
  int32_t axisym;    /* 1: axisymmetric (r, z), Appendix B: 2D, x the
                        radius (the low x side at r = origin[0] >= 0,
                        not periodic), y the axis; cell (i, j) is the
                        ring of volume 2 pi r_i h^2, radial fluxes enter
                        with r_face / r_i and every total is a volume
                        or area integral over the rings.  Either flux
                        form, either substep 2, VoF or ACDI interface;
                        no adjoint; in a batch the weighted form only
                        (SURF_EINVAL otherwise).  0: Cartesian       */
  double h;          /* cell size (cubic cells)                    */
  double origin[3];  /* position of the lower box corner (axisym: the
                        radius of the low x side; else informative)  */
} surf_grid;

/* The problem's parameters (sections 2.3-2.6, Appendix C). */
typedef struct {
  int32_t precision;    /* SURF_F32 | SURF_F64                            */
  int32_t flux_form;    /* SURF_FLUX_*                                    */
  int32_t kinetics;     /* SURF_KIN_*                                     */
  int32_t eos;          /* SURF_EOS_*                                     */
  int32_t bulk_enabled; /* 0: insoluble (no bulk field, no exchange)      */
  int32_t hj_iters_init;/* redistancing sweeps for a full build (0: 2 ceil(chi_max/dtau)) */
  int32_t hj_iters_step;/* warm-start sweeps per step when the VoF moves (0: 8) */
  int32_t adjoint;      /* 1: reserve workspace for surf_adjoint_step         */
  double eps;           /* phase-field width (section 2.5)                */
  double D_b, D_s;      /* bulk and interfacial diffusivities             */
  double k_a, k_d;      /* adsorption and desorption rates                */
  double gamma_inf;     /* saturation concentration                       */
  double sigma0, eos_E; /* clean surface tension and elasticity E         */
  double eta;           /* small constant added to phi when dividing (section 2.6); 0: 1e-12 */
  double chi_max_eps;   /* distance clamp |chi| <= chi_max_eps * eps; 0: 12 */
  double cfl_adv, cfl_diff; /* safety factors of SURF_T_DT_NEXT; 0: 0.5, 0.8 */
  double dt;            /* time step used by surf_step (> 0)              */
  int32_t substep2;     /* SURF_SUBSTEP2_*                                */
  int32_t picard_iters; /* implicit: interfacial + bulk solve sweeps per step
                         * (0: 3; at most 32)                            */
  int32_t cg_max_iters; /* implicit: CG (BiCGSTAB) iterations per linear
                         * solve at most (0: 400); each is one (three)
                         * kernel launch(es), those after the test is met
                         * return at once                               */
  int32_t pad2_;
  double cg_tol;        /* implicit: ||M^-1 r|| <= cg_tol ||x|| ends a solve,
                         * M the Jacobi diagonal (0: 1e-12)               */
  int32_t interface;    /* SURF_IFACE_*                                   */
  int32_t pad3_;
  double acdi_zeta;     /* ACDI velocity scale (> 0; the paper takes 1.1
                         * times the largest speed)                      */
  double acdi_vareps;   /* ACDI: s = eps ln((phi + ve)/(1 - phi + ve))
                         * (0: 1e-6)                                      */
  int32_t limiter;      /* substep 1 slope limiter (section 3.1, BCG face
                         * values): SURF_LIMITER_MINMOD (0) or
                         * SURF_LIMITER_MC, the monotonized central limiter */
  int32_t transverse;   /* 1: the transverse term of the unsplit BCG
                         * predictor in substep 1: each face value less
                         * dt/2 times the upwind cell's mean transverse
                         * velocity times its one-sided transverse
                         * difference on the upwind side (also in the ACDI
                         * phase field's advection).  Either variant needs
                         * the weighted flux form and no adjoint, and a 2D
                         * grid (Cartesian or axisymmetric, where the face
                         * values are the Cartesian ones) unless substep 2
                         * is implicit (SURF_EINVAL otherwise)           */
} surf_params;

/* Bytes of device workspace a context needs. */
int surf_workspace_bytes(const surf_grid* grid, const surf_params* params, size_t* bytes);

/* Validates the problem, carves the caller's workspace (device memory of at
 * least surf_workspace_bytes, 256-byte aligned) and binds the stream.  No
 * device work is issued. */
int surf_init(surf_ctx** ctx, const surf_grid* grid, const surf_params* params,
              void* workspace, size_t ws_bytes, void* hip_stream);

/* VoF fraction of fluid 1 (cell field, values in [0,1]) -> signed distance
 * chi (section 2.5).  full_rebuild = 1 starts from chi0 = (f - 1/2) h and runs
 * hj_iters_init sweeps; 0 warm-starts from the cached chi with hj_iters_step
 * sweeps (SURF_ESTATE if there is no cached chi). */
int surf_set_geometry(surf_ctx* ctx, const void* vof, int full_rebuild);

/* Installs a signed-distance field directly (cell field, > 0 inside fluid 1). */
int surf_set_levelset(surf_ctx* ctx, const void* chi);

/* Copies the cached signed distance into chi_out (cell field). */
int surf_get_levelset(surf_ctx* ctx, void* chi_out);

/* ACDI interface: copies the phase field phi (cell field, 0 in fluid 1, 1 in
 * the liquid) into phi_out on the context's stream.  SURF_EINVAL for a
 * context without ACDI, SURF_ESTATE before a level set is set. */
int surf_get_phase(surf_ctx* ctx, void* phi_out);

/* Initial state F = c0 phi, psi = gamma0 delta (section 2.6, f = Gamma delta).
 * c0 is a cell field or NULL for the constant c0_const.  Resets the running
 * time, the cumulative outflow and the status word.  F_out may be NULL when
 * the bulk is disabled. */
int surf_init_state(surf_ctx* ctx, const void* c0, double c0_const, double gamma0,
                    void* F_out, void* psi_out);

/* One step from (F_in, psi_in) at t^n to (F_out, psi_out) at t^{n+1}.
 *   vof_next  VoF at t^{n+1} (after the caller's VoF advection) or NULL when
 *             the interface does not move; when given, chi is warm-started
 *             with hj_iters_step sweeps before the transport.
 *   u         face velocities u^n: u[0..dim-1] (face layouts above), or
 *             u == NULL / u[0] == NULL for no flow (substep 1 skipped).
 *   sigma_out cell field or NULL; totals_dev 16 doubles (device) or NULL.
 * Inputs and outputs must not alias (ping-pong buffers).  F_in/F_out are
 * ignored (may be NULL) when the bulk is disabled.
 * With interface = SURF_IFACE_ACDI (section 2.5) the step first advances
 * the phase field phi by one ACDI step (advection by u, then the
 * regularization flux zeta [eps grad phi - 1/4 (1 - tanh^2(s/2eps)) grad s/|grad s|],
 * s = eps ln((phi+ve)/(1-phi+ve))) and runs the transport on chi = -s(phi)
 * clamped to |chi| <= chi_max; a vof_next instead re-initializes: chi
 * warm-started from the current one with hj_iters_step sweeps, then
 * phi = 1/(1 + e^{chi/eps}).  The caller chooses the re-initialization
 * frequency by passing vof_next.  The regularization is explicit:
 * SURF_T_DT_NEXT and SURF_STATUS_UNSTABLE include its bound
 * 1/(zeta (2 dim eps/h^2 + sqrt(dim)/h)).
 * FP32 contexts (weighted flux form, explicit substep 2) store the new F and
 * psi with stochastic rounding: each value is one of the two floats
 * neighbouring the exact update, with the probability of its closeness, so
 * that increments below half an ulp are kept on average (round-to-nearest
 * drops them every step, and over thousands of steps a smooth field drifts
 * by tens of ulps).  The random numbers are a hash of the cell and of the
 * running time the step starts from (surf_set_time): a run repeated from
 * the same state and time gives the same bits.  FP64 contexts add exactly
 * as written.
 * With substep2 = SURF_SUBSTEP2_IMPLICIT (section 3, Appendix C) the step
 * advects, then takes substep 2 by implicit Euler: picard_iters sweeps of
 * the interfacial problem for Gamma and the bulk problem for c (paper form:
 * for psi and F), each solved by CG (paper form: BiCGSTAB; see cg_tol,
 * cg_max_iters); SURF_T_DT_NEXT then holds the advective
 * bound only and SURF_STATUS_UNSTABLE tests only that bound. */
int surf_step(surf_ctx* ctx, const void* vof_next, const void* const* u,
              const void* F_in, const void* psi_in, void* F_out, void* psi_out,
              void* sigma_out, double* totals_dev);

/* Pipelined moving interface (weighted flux form, 2D or 3D).  The geometry
 * of a step, chi^{n+1} from the VoF at t^{n+1} (section 2.5, as surf_step
 * does it), depends only on that VoF and chi^n, not on the transported
 * state, so it can run while the previous step's transport runs.  This call
 * enqueues it on aux_stream (a HIP stream other than the context's, at the
 * default priority) after the last transport enqueued on the context's
 * stream has consumed the level-set buffer it overwrites (2D: the other of
 * the two; 3D: the sweeps alternate between the other two of three buffers
 * and the consuming step makes the last one current; calls that write the
 * level set, and surf_interface_force in 3D, which uses the idle buffer as
 * scratch, make the geometry wait for them, while surf_force and the 2D
 * surf_interface_force, which read the current buffer, run beside it); the next
 * surf_step, which must receive the same vof_next pointer, then runs only
 * the transport, on the context's stream, after the prepared geometry.  Typical order:
 * surf_step(vof_1); then for n >= 1: surf_prepare_geometry(vof_{n+1}),
 * surf_step(vof_{n+1}).  Results equal those of plain surf_step calls.
 *   vof_next  VoF at t^{n+1}; the caller makes it ready with respect to
 *             aux_stream and keeps it unchanged until that surf_step.
 * Errors: SURF_EINVAL for a paper-form, implicit or ACDI context, more than
 * 16 sweeps per step (3D: an odd count or under 2), a 2D grid below
 * 2 (K + 2) cells per axis, null arguments or a misaligned vof_next; SURF_ESTATE without a level set or with a prepared
 * geometry still pending.  While one is pending only surf_step (with that
 * vof_next), surf_set_dt and the status calls are accepted; the level-set,
 * state, force and adjoint calls return SURF_ESTATE. */
int surf_prepare_geometry(surf_ctx* ctx, const void* vof_next, void* aux_stream);

/* Pipelined ACDI interface (section 2.5, the Phase-Field method; 2D or 3D,
 * weighted flux form, explicit substep 2).  A step's ACDI step (the advection of phi
 * by u and the regularization, then chi = -s(phi)) depends only on phi and
 * u, not on the transported state, so it can run while the previous step's
 * transport runs.  This call enqueues it on aux_stream (a HIP stream other
 * than the context's, at the default priority) after the last transport
 * enqueued on the context's stream has consumed the level-set buffer it
 * writes; the next surf_step, which must get vof_next = NULL and the same u
 * (u[0] pointer), then waits for it and runs only the transport.  Results
 * equal those of plain surf_step calls.  Steps that re-initialize from a VoF
 * field are not prepared.
 *   u  the face velocities of that step (as in surf_step; NULL for no flow),
 *      ready with respect to aux_stream and unchanged until that surf_step.
 * Errors: SURF_EINVAL for a context without ACDI, the paper flux form or
 * the implicit substep, a null aux_stream or u[1] (3D: u[2]) missing;
 * SURF_ESTATE without a level set or with a prepare still pending.  While
 * one is pending only surf_step (as above), surf_set_dt with the dt the
 * prepared step took (any other dt returns SURF_ESTATE: the phase field has
 * already advanced with it) and the status calls are accepted; the
 * level-set, phase, state, force, timing and adjoint calls return
 * SURF_ESTATE. */
int surf_prepare_phase(surf_ctx* ctx, const void* const* u, void* aux_stream);

/* Measurement aid: runs only the transport kernel of surf_step (weighted
 * form: advection, substep 2, source, equation of state and the
 * per-workgroup reduction records; no reduction to totals, no change of the
 * running time or status) `reps` times back to back on the context's stream
 * with the cached level set and the same inputs, and returns the mean time
 * of one launch between two HIP events (synchronous).  Arguments as in
 * surf_step (without vof_next); F_out, psi_out and sigma_out are
 * overwritten.  SURF_EINVAL for the paper flux form (which has no separate
 * transport kernel) or reps < 1; SURF_ESTATE without a level set or with a
 * prepared geometry pending. */
int surf_time_transport(surf_ctx* ctx, const void* const* u, const void* F_in,
                        const void* psi_in, void* F_out, void* psi_out, void* sigma_out,
                        int32_t reps, double* ms_per_launch);

/* Measurement aid for implicit substep 2: sets up the linear problem of
 * `field` (0 interface, 1 bulk) from the last implicit step's advected state
 * and iterates, and returns the mean time of `reps` back-to-back CG
 * iteration launches between two HIP events, the stop test switched off so
 * that every launch iterates.  It overwrites only solver work arrays: the
 * next surf_step is unaffected.  Waits for the stream.  SURF_EINVAL for an
 * explicit or paper-form context, field 1 without a bulk or reps < 1;
 * SURF_ESTATE before the first implicit step. */
int surf_time_solver(surf_ctx* ctx, int32_t field, int32_t reps, double* ms_per_launch);

/* Measurement aid for the ACDI interface: `reps` ACDI steps (advection and
 * regularization of phi by u, as surf_step runs them) back to back from the
 * current phase field, their results written to scratch so that the
 * context's state is unchanged; returns the mean time of one step (both
 * kernels) between two HIP events.  Waits for the stream.  SURF_EINVAL for a
 * context without ACDI or reps < 1; SURF_ESTATE without a level set. */
int surf_time_acdi(surf_ctx* ctx, const void* const* u, int32_t reps, double* ms_per_step);

/* Marangoni face force (section 2.4) from sigma (cell field) and the cached
 * chi: on each face along d, delta_face [ (grad sigma)_d - n_d (n . grad
 * sigma) ] with n = grad chi/|grad chi| from the face gradient (compact normal
 * difference, averaged transverse centred differences).  force[d] uses the
 * face layout of u.  Faces on walls and open boundaries get 0. */
int surf_force(surf_ctx* ctx, const void* sigma, void* const* force);

/* The interfacial forces of the coupling to a flow solver (section 2.4, the
 * capillary force and the Marangoni force with delta_m = A_f / V_c), 2D
 * (Cartesian or axisymmetric) or 3D Cartesian, on the faces of u.  Inputs (device, context precision, cell
 * layout): vof, the VoF fraction of fluid 1, and sigma, the surface tension
 * (e.g. surf_step's sigma_out); the context's cached level set supplies the
 * normal and the curvature fallback.  Outputs (device, caller-owned):
 * f_cap[0..1] and f_ma[0..1], the x- and y-face arrays ([ny][nx+1] and
 * [ny+1][nx]) of
 *   capillary  -sigma_f kappa_f (c_R - c_L)/h, kappa by height functions
 *              (seven-cell columns along the larger component of the Youngs
 *              normal; the level-set curvature where a column does not
 *              close) in cells with 1e-6 < c < 1 - 1e-6, on a face the mean
 *              over its interfacial cells, sigma_f the mean of both;
 *   Marangoni  delta_m,f (grad sigma - n (n . grad sigma)), delta_m the
 *              length of the PLIC line (Youngs normal, closed-form plane
 *              constant) in each interfacial cell over h, on a face the
 *              mean of both cells; grad sigma and n from the face gradients
 *              of sigma and chi as in surf_force.
 * In 3D (f_cap[0..2], f_ma[0..2], the face layouts of u): the Youngs normal
 * from the 3x3x3 stencil; kappa = (H_bb (1 + H_c^2) + H_cc (1 + H_b^2) -
 * 2 H_bc H_b H_c)/(1 + H_b^2 + H_c^2)^(3/2) from nine columns of nine cells
 * along the first axis, in the order of the normal's components, whose
 * columns all close; a cell where none closes takes the mean height
 * curvature of the interfacial cells of its 3x3x3 block, or the level-set
 * curvature moved to the interface; delta_m the area of the PLIC plane in
 * the cell over h.  The 3D call uses the context's pin-data and idle
 * level-set buffers as scratch (the next moving-geometry step rebuilds
 * what it keeps in them).
 * Either array set may be NULL (not both).  Faces on walls and open sides
 * get 0; on a periodic axis the last face repeats the first.  Enqueued on
 * the context's stream.  On axisymmetric rings (2D, x the radius) the
 * interface is a surface of revolution: kappa adds the azimuthal curvature
 * -n_r / r_i (the level-set fallback its own, moved with
 * kappa / (1 - chi kappa / 2)), and delta_m is the area the chord sweeps
 * about the axis over the ring's volume, (|chord| / h^2) r_m / r_i, r_m the
 * radius of the chord's midpoint.  SURF_EINVAL for an axis under 4 cells, in 2D (nx+1)(ny+1) >= 2^30, in 3D 2^31 or more 16^3
 * tiles, NULL inputs or a NULL array in
 * a given set; SURF_ESTATE without a level set or with a prepared geometry
 * pending. */
int surf_interface_force(surf_ctx* ctx, const void* vof, const void* sigma, void* const* f_cap,
                         void* const* f_ma);

/* Allocation-free step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): one surf_step of the weighted flux form with explicit substep
 * 2 on a given level set, with no context and no workspace.  The running
 * state and the per-workgroup records of the reduction live in a
 * file-scope device array of the library (NSTATE + 4096 x 10 doubles,
 * 320 KiB, held on every device the library runs on until the process
 * ends); the call allocates nothing, host or device.
 *   grid, params  as for surf_init (flux_form SURF_FLUX_WEIGHTED, substep2
 *                 SURF_SUBSTEP2_EXPLICIT, interface SURF_IFACE_VOF);
 *                 params->dt is ignored, dt is the step;
 *   chi           the level set of the interface at t^{n+1} (cell layout,
 *                 context precision), e.g. from surf_get_levelset;
 *   u, F_in, psi_in, F_out, psi_out, sigma_out  as for surf_step;
 *   totals_dev    16 doubles (device) or NULL: read first for the running
 *                 time (slot SURF_T_TIME) and the cumulative outflow (slot
 *                 SURF_T_OUTFLOW_CUM) of the previous step, then rewritten with
 *                 this step's totals; NULL starts from time 0 and writes
 *                 nothing;
 *   hip_stream    the stream every launch is enqueued on.
 * Results equal those of surf_step on a context holding the same level set
 * (the same kernels).  The status word is not kept: the totals carry the
 * non-finite count, the minima and the stable step.  Every call on a device
 * shares that device's array, so calls that overlap on one device race.
 * Errors: SURF_EINVAL as for surf_init and surf_step, or another flux form,
 * substep or interface; SURF_ENOMEM for a grid of more than 4096 transport
 * workgroups (2D: ceil(nx/58) ceil(ceil(ny/8)/4); 3D: ceil(nx/58)
 * ceil(ny/14) ceil(nz/16) in FP32, ceil(nz/8) in FP64); SURF_EDEVICE for a
 * HIP error. */
int surf_step_static(const surf_grid* grid, const surf_params* params, double dt,
                     const void* chi, const void* const* u, const void* F_in,
                     const void* psi_in, void* F_out, void* psi_out, void* sigma_out,
                     double* totals_dev, void* hip_stream);

/* Changes the time step used by the following steps.  SURF_EINVAL for a dt
 * that is not positive and finite; SURF_ESTATE for a different dt while an
 * ACDI step is prepared (surf_prepare_phase), which has already used the
 * current one. */
int surf_set_dt(surf_ctx* ctx, double dt);

/* Sets the running time of the context (the time a step starts from,
 * SURF_T_TIME of the previous step's totals) from one device double,
 * enqueued on the context's stream; time_dev NULL sets it to 0.  In FP32
 * the time also keys the stochastic rounding of the stored state (see
 * surf_step), so a run replayed from a stored state with that state's time
 * reproduces the original steps bit for bit (the adjoint's recomputation
 * from checkpoints does this).  SURF_ESTATE while a prepared step is
 * pending. */
int surf_set_time(surf_ctx* ctx, const double* time_dev);

/* Reads (synchronously: waits for the stream) and clears the status word. */
int surf_get_status(surf_ctx* ctx, uint32_t* bits);
int surf_clear_status(surf_ctx* ctx);

/* Implicit substep 2: the CG iterations of each linear solve of the last
 * surf_step, in the order they ran (interface, bulk, interface, bulk, ...;
 * interface only without a bulk).  Writes min(cap, *count) counts to iters
 * (host memory), *count the number of solves.  Waits for the context's
 * stream.  SURF_EINVAL for an explicit context or null arguments,
 * SURF_ESTATE before the first implicit step. */
int surf_solver_iterations(surf_ctx* ctx, int32_t* iters, int32_t cap, int32_t* count);

int surf_destroy(surf_ctx* ctx);
const char* surf_strerror(int code);

/* ---- Discrete adjoint (growth direction; weighted flux form only) ------
 * Gradients of L = (1/N) sum_{n=1..N} (<sigma>^n - target^n)^2, with
 * <sigma> = sum sigma delta / sum delta after step n, with respect to
 * (k_a, k_d, D_b, D_s) and the initial bulk field c0 (F^0 = c0 phi), by the
 * exact transpose of the discrete step: the advection with its minmod
 * branches frozen at the state, substep 2 and the exchange source.  Needs
 * params.adjoint = 1 at init, a static interface and a fixed dt. */

/* Replaces (k_a, k_d, D_b, D_s) for the following calls. */
int surf_set_kinetics(surf_ctx* ctx, double k_a, double k_d, double D_b, double D_s);

/* From the forward totals of steps 1..N (rows of `stride` doubles, device)
 * and the target history (N doubles, device): the loss weights
 * w_n = dL/d<sigma>^n / sum(delta h^d) (N doubles, device) and the loss
 * (1 double, device; may be NULL). */
int surf_loss_weights(surf_ctx* ctx, const double* totals_hist, int64_t stride,
                      const double* sigma_target, int32_t nsteps, double* w_out,
                      double* loss_out);

/* lambda^N: lamF = 0, lamPsi = w sigma'(Gamma) delta/(delta + eta/eps) at the
 * state psi^N, w = &w_out[N-1] (device). */
int surf_adjoint_seed(surf_ctx* ctx, const void* psi_N, const double* w_N, void* lamF,
                      void* lamPsi);

/* lambda^n from lambda^{n+1} for the step taken from (F_n, psi_n) with the
 * face velocities u (NULL: no flow); adds the loss term of t^n when w_n is
 * not NULL (device pointer to w_out[n-1]); adds dL/d(k_a, k_d, D_b, D_s) of
 * this step to dtheta_dev (4 doubles, device).  lamF_n/lamPsi_n must not
 * alias the inputs. */
int surf_adjoint_step(surf_ctx* ctx, const void* const* u, const void* F_n, const void* psi_n,
                      const void* lamF_np1, const void* lamPsi_np1, const double* w_n,
                      void* lamF_n, void* lamPsi_n, double* dtheta_dev);

/* The pair below lets a backward pass keep the advected state xi* of each
 * recomputed step instead of advecting again inside the adjoint step.
 *
 * surf_step_advected: surf_step on a static level set (vof_next = NULL) that
 * also writes xi* = (F*, psi*), the state after substep 1 (the advection of
 * section 2.2) and before substep 2, into F_star/psi_star (cell fields, the
 * layout of F and psi; F_star is ignored without bulk).  Outputs and totals
 * are those of surf_step.  3D contexts on the plane-marching transport only
 * (weighted flux form, no limiter or transverse terms, explicit substep 2,
 * VoF interface); SURF_EINVAL otherwise, or when an output aliases an input
 * or another output; SURF_ESTATE after surf_prepare_geometry or before a
 * level set. */
int surf_step_advected(surf_ctx* ctx, const void* const* u, const void* F_in, const void* psi_in,
                       void* F_out, void* psi_out, void* sigma_out, double* totals_dev,
                       void* F_star, void* psi_star);

/* surf_adjoint_step with xi* of the step taken from (F_n, psi_n) given, as
 * surf_step_advected wrote it for the same state, velocities and level set:
 * the adjoint of the advection reads it in place of its own recomputation.
 * Any context surf_adjoint_step accepts; F_star may be NULL without bulk.
 * lamF_n/lamPsi_n must not alias the inputs (SURF_EINVAL). */
int surf_adjoint_step_advected(surf_ctx* ctx, const void* const* u, const void* F_n,
                               const void* psi_n, const void* F_star, const void* psi_star,
                               const void* lamF_np1, const void* lamPsi_np1, const double* w_n,
                               void* lamF_n, void* lamPsi_n, double* dtheta_dev);

/* dL/dc0 = lamF^0 phi (cell field). */
int surf_adjoint_c0(surf_ctx* ctx, const void* lamF0, void* grad_c0);

/* ---- Batched form (growth direction) -----------------------------------
 * n_inst independent 2D problems (their own grid sizes, parameters and time
 * steps; one precision), static interfaces, advanced together: each step is
 * one persistent launch over the flattened queue of all their 64 x 16 tiles
 * plus one per-instance reduction; surf_batch_step records nsteps of them in
 * one HIP graph and replays it on later calls with the same step count. */

/* Bytes of device workspace for the batch. */
int surf_batch_workspace_bytes(int32_t n_inst, const surf_grid* grids, const surf_params* params,
                               size_t* bytes);

/* Validates every instance (dim 2, same precision, weighted or paper form;
 * on axisymmetric rings the weighted form) and carves the workspace.  F and psi: 2 n_inst device buffers each, the
 * state pair of instance i at [2i] and [2i+1]; sigma: n_inst buffers or NULL.
 * The state of instance i lives in buffer [2i + surf_batch_parity()]. */
int surf_batch_create(surf_batch** batch, int32_t n_inst, const surf_grid* grids,
                      const surf_params* params, void* const* F, void* const* psi,
                      void* const* sigma, void* workspace, size_t ws_bytes, void* hip_stream);

/* Full level-set build of instance i from its VoF field (section 2.5). */
int surf_batch_set_geometry(surf_batch* batch, int32_t i, const void* vof);

/* F = c0 phi, psi = gamma0 delta into buffer [2i]; resets the parity to 0
 * (initialise every instance before stepping). */
int surf_batch_init_state(surf_batch* batch, int32_t i, const void* c0, double c0_const,
                          double gamma0);

/* nsteps steps of every instance; totals_dev ([n_inst][16] doubles, device,
 * may be NULL) receives the totals of the last step. */
int surf_batch_step(surf_batch* batch, int32_t nsteps, double* totals_dev);

/* Which buffer of each pair holds the current state (0 or 1). */
int surf_batch_parity(surf_batch* batch);

/* Times the candidate launch shapes (threads per workgroup, persistent
 * workgroup count) on the bound buffers with HIP events and keeps the
 * fastest; results are unchanged by the choice.  *choice (may be NULL)
 * receives its index; times_us (may be NULL) one time per candidate. */
int surf_batch_tune(surf_batch* batch, int32_t* choice, double* times_us, int32_t max_times);

int surf_batch_destroy(surf_batch* batch);

/* Kernel timing.  While enabled, every launch of the fused transport kernel
 * and of each redistancing sweep is bracketed by HIP events recorded on the
 * context stream.  surf_profile_read waits for the recorded events, returns
 * the summed elapsed milliseconds and launch counts per kind (transport,
 * redistancing) and forgets them.  Any output pointer may be NULL. */
int surf_profile_enable(surf_ctx* ctx, int enable);
int surf_profile_read(surf_ctx* ctx, double* step_ms, int64_t* step_launches,
                      double* geom_ms, int64_t* geom_launches);

/* Library version string. */
const char* surf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SURF_H */
