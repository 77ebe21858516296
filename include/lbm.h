/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the regularised lattice
 * Boltzmann step of Brownlee, Levesley, Packwood and Gorban, "Add-ons for
 * Lattice Boltzmann Methods: Regularization, Filtering and Limiters"
 * (arXiv:1110.0270).
 *
 * One call of lbm_step advances the lattice by n time steps.  Each step is
 * the fused per-site pull-stream + collide of section 2 with
 *   - the LBGK collision (section 2, eq. CollisionIntegral),
 *   - MRT relaxation in the M1/C1 or M2/C2 basis (section 5),
 *   - ELBM with the per-site entropic root alpha (section 3),
 * and the add-on limiters of section 4: the median entropy filter, the
 * Ehrenfest step on the k sites of largest nonequilibrium entropy, and the
 * positivity rule.  lbm_backward runs the adjoint of a recorded forward
 * rollout.
 *
 * Memory layout of populations (device and caller buffers alike):
 *   structure of arrays f[i][y][x], i = 0..Q-1, y = 0..ny-1, x = 0..nx-1,
 *   x fastest, caller buffers densely packed (row pitch nx).  Velocity
 *   order ("tensor order"): D2Q9 i = 3 (b + 1) + (a + 1) for velocity
 *   (a, b) in {-1,0,1}^2, so the opposite of i is 8 - i and i = 4 is rest;
 *   D1Q3 i = a + 1 for a in {-1, 0, 1}, with ny = 1.
 *   The site index used for ties is y * nx + x.
 *   Caller populations are always unshifted f_i; the library stores the
 *   FP32, FP16 and BF16 forms internally as shifted deviations
 *   f_i - w_i rho0 (LBM_F32, LBM_F16S, LBM_BF16S).
 *
 * Ownership: the caller allocates every device buffer, including the
 * workspace (lbm_workspace_bytes); the library never allocates device
 * memory and never frees caller memory.  Buffers passed by pointer must stay
 * valid while work that uses them can still run on the stream.  The context
 * object itself is host memory owned by the library (lbm_destroy frees it).
 *
 * Streams: every call except lbm_stats, lbm_selected_count and lbm_destroy
 * only enqueues work on the stream given to lbm_init and returns.  Calls on
 * one context must not be made from two threads at once.
 *
 * Errors: every function returns an lbm_status; nothing aborts or throws
 * across the ABI.  On failure lbm_last_error() returns a message for the
 * failing call of this thread.  Invalid arguments leave the context as it
 * was.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,        /* bad configuration or argument                  */
  LBM_EWORKSPACE = -2,    /* workspace smaller than lbm_workspace_bytes     */
  LBM_EHIP = -3,          /* a HIP runtime call failed; message has details */
  LBM_EDIVERGED = -4,     /* a check found a non-finite value or rho <= 0   */
  LBM_ESTATE = -5,        /* call out of order (e.g. backward w/o forward)  */
  LBM_EUNSUPPORTED = -6,  /* valid but not implemented combination          */
  LBM_ESELECT = -7        /* Ehrenfest selection could not be resolved exactly */
} lbm_status;

/* Lattices: D1Q3 and D2Q9 (sections 2, 5, 6), and D3Q27, the tensor product
 * of D1Q3 in three dimensions (velocities (a, b, c) in {-1, 0, 1}^3, tensor
 * order i = 9 (c + 1) + 3 (b + 1) + (a + 1), weights w_a w_b w_c, product
 * equilibria), whose 27-site neighbourhood is the one of the median entropy
 * filter in 3D (section 4: the 14th of 27 values).  D3Q27 lattices are
 * periodic nx x ny x nz grids stepped with LBGK, optionally with the median
 * filter and the positivity rule; populations are (27, nz, ny, nx). */
enum { LBM_D1Q3 = 1, LBM_D2Q9 = 2, LBM_D3Q27 = 3 };
/* Boundaries: periodic in x and y; bounce-back walls on all sides; cavity =
 * bounce-back walls with the top wall moving at (u_lid, 0); couette =
 * periodic in x, resting bottom wall, moving top wall; diffusive = the
 * diffusive Maxwell wall of section 8 (First Hopf bifurcation) on the outer
 * ring of nodes, the top row moving at (u_lid, 0): after streaming, a wall
 * node sets the populations pointing into the fluid to gamma f*_i(u_wall)
 * (f* of the configured equilibrium at unit density, gamma = the sum of the
 * populations that reached the wall over the sum of those f*_i; at a corner
 * only the inward diagonal, which is bounce-back), every other population
 * whose source lies outside likewise, and does not collide; wall nodes are
 * neither Ehrenfest candidates nor median neighbours.  D2Q9, nx, ny >= 3;
 * no adjoint (checkpoint_every = 0) and no ensemble limiter. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_BOUNCEBACK = 1, LBM_BC_CAVITY = 2, LBM_BC_COUETTE = 3,
       LBM_BC_DIFFUSIVE = 4 };
enum { LBM_LBGK = 0, LBM_MRT = 1, LBM_ELBM = 2 };
enum { LBM_EQ_POLY = 0, LBM_EQ_ENTROPIC = 1 };
enum { LBM_MRT_M1 = 0, LBM_MRT_M2 = 1 };
/* Rate presets of the M1 basis (section 5 TRT; section 7 shear-wave MRT;
 * section 8 cavity study), functions of the shear rate s_nu = omega (per
 * site with an omega field):
 *   GIVEN    s_e, s_eps, s_q as configured;
 *   TRT      s_e = s_eps = s_nu, s_q = 8 (2 - s_nu) / (8 - s_nu) (the printed
 *            "8(2=s_nu)" read as 8(2 - s_nu));
 *   MRT_TRTQ s_e = 1.64, s_eps = 1.54, s_q as for TRT;
 *   MRT1     s_e = 1.64, s_eps = 1.54, s_q = 1.9;
 *   SHEAR    s_e = 1.64, s_eps = 1.54, s_q = 3 (2 - s_nu) / (3 - s_nu). */
enum { LBM_RATES_GIVEN = 0, LBM_RATES_TRT = 1, LBM_RATES_MRT_TRTQ = 2, LBM_RATES_MRT1 = 3,
       LBM_RATES_SHEAR = 4 };
/* What the Ehrenfest selection (the k sites of largest Delta S > delta)
 * does to its sites: EQUILIBRIUM sends them to f* (Ehrenfests' step); MRT
 * gives them the MRT collision of mrt_basis and its rates (with s_nu the
 * site's omega) in place of LBGK's: the MRT limiter of section 5 (LBGK
 * lattices, D2Q9 only).  The positivity rule, when on, then also acts on
 * them. */
enum { LBM_SEL_EQUILIBRIUM = 0, LBM_SEL_MRT = 1 };
/* Ensemble-dependent and smooth limiters of section 4, applied to every
 * site's pre-collision state as f* + phi (f - f*) (not with the median
 * filter; no adjoint):
 *   THRESHOLD        phi = sqrt(Delta S_t / Delta S) where Delta S >= Delta S_t,
 *                    else 1 (eq. entrHom);
 *   SMOOTH           phi = (1 + r^(k-1/2)) / (1 + r^k), r = Delta S / (alpha
 *                    E(Delta S)), E the mean over the lattice (eq. phiExamp);
 *   DOUBLE_MONOTONE  phi = (1 + (Delta S / Delta S_t)^k)^(-1/(2k)) (eq. DoublMonSpec);
 *   POINTWISE        phi = 1 / (1 + alpha Delta S^k).
 * Delta S_t = max(Delta S_0, ens_delta), with Delta S_0 the exact solution
 * over the lattice's Delta S values of eq. EntThresh:
 *   sum over sites of max(Delta S - Delta S_0, 0) = ens_delta0 * P,
 *   P = sum over sites of [1 - (omega - 1)^2] Delta S (the LBGK entropy
 *   production in quadratic approximation, section 4 "Monitoring total
 *   dissipation"); ens_delta0 <= 0 fixes Delta S_t = ens_delta.
 * Sites with Delta S = +inf (a non-positive population) take phi = 0 and are
 * left out of E and of the sums. */
enum { LBM_ENS_NONE = 0, LBM_ENS_THRESHOLD = 1, LBM_ENS_SMOOTH = 2,
       LBM_ENS_DOUBLE_MONOTONE = 3, LBM_ENS_POINTWISE = 4 };
enum { LBM_LIM_EHRENFEST = 1, LBM_LIM_POSITIVITY = 2, LBM_LIM_MEDIAN = 4 };
enum { LBM_NORM_ENTROPIC = 0, LBM_NORM_L1 = 1 };
enum { LBM_FB_POSITIVITY = 0, LBM_FB_EHRENFEST = 1 };
/* Storage forms of the lattice, and dtype codes of caller buffers
 * (caller buffers accept LBM_F64 and LBM_F32 only). */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3 };

typedef struct lbm_config {
  int lattice;            /* LBM_D1Q3 | LBM_D2Q9 | LBM_D3Q27                    */
  int nx, ny;             /* grid; ny = 1 for D1Q3                              */
  int bc;                 /* LBM_BC_*                                           */
  double u_lid;           /* moving-wall speed (cavity, couette)                */
  double rho_wall;        /* wall density in the moving-wall term (1.0)         */
  int collision;          /* LBM_LBGK | LBM_MRT | LBM_ELBM                       */
  int equilibrium;        /* LBM_EQ_POLY | LBM_EQ_ENTROPIC (ELBM: entropic)      */
  double nu;              /* viscosity; omega = 1/(3 nu + 1/2).  nu < 0: use omega */
  double omega;           /* relaxation rate when nu < 0                        */
  int mrt_basis;          /* LBM_MRT_M1 (C1 rates) | LBM_MRT_M2 (C2 rates)       */
  double s_e, s_eps, s_q; /* MRT rates of e, epsilon, q (M1 only)               */
  unsigned limiters;      /* bit set of LBM_LIM_*                               */
  long long ehr_k;        /* Ehrenfest budget: k sites per step                 */
  double ehr_delta;       /* Ehrenfest threshold: only Delta S > delta          */
  double med_delta;       /* median filter acts only where Delta S > med_delta  */
  int elbm_norm;          /* LBM_NORM_*                                         */
  int elbm_fallback;      /* no-root rule: LBM_FB_POSITIVITY | LBM_FB_EHRENFEST  */
  double elbm_eps;        /* stop when |S_f/S_f'| * ||Delta|| < eps (1e-14)     */
  int elbm_max_iter;      /* parabola iterations (32)                           */
  double elbm_dS_cut;     /* Delta S below this: plain LBGK (1e-15)             */
  double elbm_f64_below;  /* FP32 modes: sites with alpha_max below this bound
                             solve the root in FP64 (3.0)                      */
  int storage;            /* LBM_F64 | LBM_F32 | LBM_F16S | LBM_BF16S            */
  double rho0;            /* reference density of the shifted storage (1.0)     */
  int omega_field;        /* 1: a per-site relaxation field is used (lbm_set_omega) */
  int checkpoint_every;   /* K > 0: record a rollout for lbm_backward           */
  long long max_steps;    /* longest rollout lbm_backward must cover            */
  int check_interval;     /* steps between divergence checks (0: only on lbm_stats) */
  int mrt_preset;         /* LBM_RATES_* (M1 basis; GIVEN uses s_e, s_eps, s_q)   */
  int sel_action;         /* LBM_SEL_EQUILIBRIUM | LBM_SEL_MRT                   */
  int ens_limiter;        /* LBM_ENS_*                                          */
  double ens_delta0;      /* dissipation budget delta_0 of eq. EntThresh        */
  double ens_delta;       /* lower bound delta of the threshold                 */
  double ens_alpha;       /* alpha of SMOOTH and POINTWISE                      */
  double ens_k;           /* exponent k of SMOOTH, DOUBLE_MONOTONE, POINTWISE   */
  int nz;                 /* D3Q27: layers of the grid (1 otherwise)            */
  /* General nonlocal filter of section 4: after streaming, every site's
   * nonequilibrium part f - f* becomes sum_y d(y) (f - f*)(x + y) over the
   * neighbourhood shifts y (the moments, and so f*, are unchanged), before
   * the collision.  nl_coef holds d(y) in tensor order of y: D1Q3 the 3
   * shifts dx = -1, 0, 1; D2Q9 the 9 shifts, index 3 (dy + 1) + (dx + 1);
   * the remaining entries are ignored.  Periodic D1Q3 and D2Q9 lattices
   * (the shifts must map the grid into itself); not with the median filter,
   * the Ehrenfest selection, the ensemble limiters or the adjoint. */
  int nl_filter;          /* 1: the nonlocal filter is on                       */
  double nl_coef[27];     /* its coefficients d(y)                              */
} lbm_config;

typedef struct lbm_stats {
  double mass;            /* sum over sites of rho                              */
  double mom_x, mom_y;    /* sum over sites of rho u                            */
  double entropy;         /* sum over sites of -sum_i f_i ln(f_i / w_i)         */
  double min_rho;         /* smallest density                                   */
  long long steps;        /* steps taken since the last lbm_set_*               */
  long long diverged_step;/* first step at which a check failed, or -1          */
  long long n_selected;   /* Ehrenfest sites chosen in the last step            */
  long long select_fallbacks; /* steps whose selection needed a full rescan     */
  long long select_overflow;  /* steps whose boundary list overflowed          */
  long long select_candidates;/* Ehrenfest candidates examined, all steps      */
  int nonfinite;          /* 1 if the last check found NaN or Inf               */
  /* ensemble limiters, last step: Delta S_t (THRESHOLD, DOUBLE_MONOTONE;
   * +inf for the others), E(Delta S), the LBGK entropy production
   * [1 - (omega - 1)^2] sum Delta S and the limiter's own,
   * sum (1 - phi^2) Delta S (both in quadratic approximation); all 0
   * without an ensemble limiter */
  double ens_threshold;
  double ens_mean;
  double lbgk_production;
  double limiter_production;
  /* enstrophy (section 8, cavity study): the sum of the squared vorticity
   * du_y/dx - du_x/dy (central differences of u, FP64) over the sites with
   * four neighbours in the lattice (every site when periodic), divided by
   * their number; 0 for D1Q3 and D3Q27 */
  double enstrophy;
  double mom_z;           /* D3Q27: sum over sites of rho u_z (0 otherwise)     */
} lbm_stats;

typedef struct lbm_ctx lbm_ctx;

/* Fill *cfg with defaults (D2Q9 64x64 periodic LBGK, omega = 1, FP32). */
void lbm_config_default(lbm_config* cfg);

/* Bytes of device workspace lbm_init needs for cfg (0 if cfg is invalid;
 * lbm_last_error then says why).  Includes the checkpoint store when
 * cfg->checkpoint_every > 0. */
size_t lbm_workspace_bytes(const lbm_config* cfg);

/* Create a context on the current HIP device.  dev_workspace: device
 * buffer of at least lbm_workspace_bytes(cfg) bytes, 256-byte aligned,
 * owned by the caller.  stream: a hipStream_t (NULL = default stream).
 * The lattice is undefined until lbm_set_equilibrium or
 * lbm_set_populations.  Errors: LBM_EINVAL, LBM_EWORKSPACE, LBM_EHIP. */
lbm_status lbm_init(const lbm_config* cfg, void* dev_workspace, size_t ws_bytes,
                    void* stream, lbm_ctx** out);

/* Set the lattice to the equilibrium f*(rho, u) of the configured kind
 * (sections 6 and 8: 1D polynomial or entropic equilibria, and their
 * product in 2D).  rho, ux, uy: device arrays of ny*nx values of the given
 * dtype (LBM_F64 or LBM_F32); uy is ignored for D1Q3 and may be NULL.
 * Resets the step counter and the recorded rollout.  D3Q27:
 * LBM_EUNSUPPORTED (lbm_set_equilibrium3d). */
lbm_status lbm_set_equilibrium(lbm_ctx* ctx, const void* rho, const void* ux,
                               const void* uy, int dtype);

/* D3Q27: set the lattice to f*_abc = rho phi_a(ux) phi_b(uy) phi_c(uz), the
 * product of the 1D equilibria of section 6 of the configured kind.  rho,
 * ux, uy, uz: device arrays of nz*ny*nx values (index (z * ny + y) * nx + x)
 * of the given dtype.  LBM_EINVAL on other lattices.  Resets the step
 * counter. */
lbm_status lbm_set_equilibrium3d(lbm_ctx* ctx, const void* rho, const void* ux,
                                 const void* uy, const void* uz, int dtype);

/* Set the lattice to caller populations f[Q][ny][nx] (D3Q27:
 * f[27][nz][ny][nx]; device, dtype LBM_F64 or LBM_F32, unshifted).  Resets
 * the step counter and rollout. */
lbm_status lbm_set_populations(lbm_ctx* ctx, const void* f, int dtype);

/* Copy the lattice out as unshifted populations f[Q][ny][nx] (D3Q27:
 * f[27][nz][ny][nx]). */
lbm_status lbm_get_populations(lbm_ctx* ctx, void* f, int dtype);

/* Per-site relaxation rate omega(x) (device, ny*nx values, dtype LBM_F64 or
 * LBM_F32); requires cfg.omega_field = 1.  It replaces omega in LBGK and
 * ELBM (beta = omega/2) and is the shear rate s_nu of MRT (section 5). */
lbm_status lbm_set_omega(lbm_ctx* ctx, const void* omega, int dtype);

/* Advance n >= 0 time steps (section 2: free flight, then collision, with
 * the configured limiters of section 4).  Asynchronous. */
lbm_status lbm_step(lbm_ctx* ctx, long long n);

/* Density and velocity of every site, rho = sum f_i, u = sum v_i f_i / rho
 * (section 2), into device arrays of ny*nx values (uy may be NULL for
 * D1Q3).  D3Q27: LBM_EUNSUPPORTED (read the populations instead). */
lbm_status lbm_moments(lbm_ctx* ctx, void* rho, void* ux, void* uy, int dtype);

/* Adjoint of the rollout recorded since the last lbm_set_* (requires
 * cfg.checkpoint_every > 0 and at most cfg.max_steps steps).  dL_dfT: the
 * gradient of a loss with respect to the final populations f[Q][ny][nx]
 * (device, dtype, dense).  Writes dL/df0 into dL_df0 (same layout) and,
 * when dL_domega is not NULL, dL/d omega(x) into dL_domega (ny*nx): the
 * gradient with respect to a per-site relaxation rate (with a uniform
 * omega, its sum over sites is dL/d omega).  Gradients pass through the
 * limiters along the branch the forward pass took (a site the Ehrenfest
 * limiter sent to equilibrium through the Jacobian of f*; the positivity rule through
 * its coefficient and the component that set it; the median entropy filter
 * (section 4) through its homothety coefficient sqrt(med / Delta S), i.e.
 * through the site's own Delta S and that of the neighbour holding the
 * median, with equal values ranked by neighbour order and no derivative
 * through a zero median), through the ELBM root by
 * implicit differentiation of the entropy condition (section 3), and
 * through storage rounding as the identity.  The rollout is recomputed
 * from the checkpoints taken every cfg.checkpoint_every steps, with the
 * recorded Ehrenfest selections, so the recompute takes the forward pass's
 * branches bit for bit.  Work runs in the compute precision (FP64 for
 * LBM_F64 storage, FP32 otherwise).  The lattice is left in its final
 * state.  Errors: LBM_ESTATE without a recorded rollout. */
lbm_status lbm_backward(lbm_ctx* ctx, const void* dL_dfT, void* dL_df0,
                        void* dL_domega, int dtype);

/* Synchronise the stream, run a whole-lattice FP64 reduction and fill *out.
 * Returns LBM_EDIVERGED if this or an earlier check found a non-finite
 * value or rho <= 0, LBM_ESELECT if a selection overflowed. */
lbm_status lbm_stats_get(lbm_ctx* ctx, lbm_stats* out);

/* Synchronise and copy the site indices chosen by the Ehrenfest limiter in
 * the last step into the host array idx (capacity cap, ascending order).
 * *count receives the number chosen. */
lbm_status lbm_selected(lbm_ctx* ctx, long long* idx, long long cap, long long* count);

/* Synchronise and copy the cumulative limiter counters into out[0..n-1]:
 * positivity-rule activations in the collision (sites that the Ehrenfest
 * limiter then sends to equilibrium included), median-filter corrections,
 * ELBM sites with no nontrivial root, ELBM sites solved in FP64, ELBM sites
 * with a non-positive population, ELBM root iterations (summed over
 * sites). */
lbm_status lbm_counters(lbm_ctx* ctx, unsigned long long* out, int n);

/* Advance n steps exactly as lbm_step does, bracketing each step's fused
 * collide-stream kernel with HIP events on the context's stream, then
 * synchronise.  out[0] = summed duration of those kernels (ms), out[1] =
 * duration from the first kernel's start to the end of the last step's
 * work (ms).  For measurement; the events add a few microseconds per step. */
lbm_status lbm_profile_step(lbm_ctx* ctx, long long n, double out[2]);

/* lbm_backward with each step's adjoint kernel bracketed by HIP events,
 * then synchronise.  out[0] = summed duration of those kernels (ms), out[1]
 * = duration of the whole backward pass, recompute included (ms).  For
 * measurement. */
lbm_status lbm_profile_backward(lbm_ctx* ctx, const void* dL_dfT, void* dL_df0,
                                void* dL_domega, int dtype, double out[2]);

/* Size of the static device array behind lbm_step_noalloc (per device). */
#define LBM_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): one time
 * step exactly as lbm_step takes it (same kernels), from the lattice f_src
 * into the lattice f_dst, allocating nothing.  Every other buffer of the
 * step (selection state, Ehrenfest candidates and lists, histograms, limiter
 * counters, the FP64-solve list) lives in a static device array of
 * LBM_NOALLOC_SCRATCH_BYTES that each device holds until the process ends.
 *   cfg:   as for lbm_init, with checkpoint_every = 0 and omega_field = 0
 *          (check_interval is ignored).
 *   f_src, f_dst: distinct device buffers, caller-owned, in the storage form
 *          of cfg->storage, [Q][ny][nx] densely packed: LBM_F64 holds f_i;
 *          LBM_F32, LBM_F16S (_Float16) and LBM_BF16S (bfloat16) hold the
 *          shifted deviation f_i - w_i rho0 rounded to nearest even.
 *   stream: a hipStream_t (NULL = default stream); the call only enqueues.
 * Each call starts the Ehrenfest selection from its threshold (no candidate
 * floor is carried between calls), so it examines every eligible site.
 * The limiter counters are cleared at every call and not reported.
 * Errors: LBM_EINVAL (configuration, NULL or equal buffers), LBM_EWORKSPACE
 * when the configuration needs more scratch than the array holds (large
 * lattices with the Ehrenfest limiter or FP32 ELBM: use lbm_init with a
 * workspace), LBM_EHIP.  Every call on a device shares that device's
 * array: calls that overlap on one device (other streams, other threads)
 * race and must be serialised by the caller. */
lbm_status lbm_step_noalloc(const lbm_config* cfg, const void* f_src, void* f_dst, void* stream);

/* Free the context (not the caller's buffers). NULL is allowed. */
void lbm_destroy(lbm_ctx* ctx);

/* Message for the last failing call on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
