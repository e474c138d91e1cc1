/*
 * lmvd.h -- C ABI of the MI355X library for one explicit RK2 substep of the
 * pseudospectral low-Mach, variable-density method of Reuter, Oliver & Moser
 * ("A pseudospectral method for direct numerical simulation of low-Mach,
 * variable-density, turbulent flows").
 *
 * The operation (Section 4, "Time advance", Algorithm time_advanceDNS): given
 * the state S = (phi2, Omega2, z, <m>1, <m>3) at stage s, the right-hand sides
 * stored from the previous stage, and the z history, apply one substep
 * s -> s+1:
 *   1. finalize m^d (eqs. phi_poisson, md_recon, potential-matching rows of
 *      eq. bc_both);
 *   2. evaluate R_z (Section 2.1) and the BDF-like guess of dz/dt
 *      (eq. dzdt_guesses, beta^n and beta' of Appendix A);
 *   3. k_f fixed-point iterations z_t^k = L(z) z_t^{k-1} + R_z (eq. y_k,
 *      Section 3.2), L applied matrix-free (Section 4.3), then m^c
 *      (eqs. COM_fourier, CF_fourier, mc_recon, mc_mean);
 *   4. rho = f(z) (equation of state of Section 5);
 *   5. RHS of Omega2, phi2 (eqs. om, phi, with the body force -rho g delta_i2)
 *      and of <m>1, <m>3 (eq. mean_m1m3);
 *   6. explicit midpoint RK2, low-storage form:
 *      stage n:  X' = X^n + dt/2 R^n;   stage ':  X^{n+1} = X' + dt (R' - R^n/2).
 *
 * Discretisation: Fourier in x1, x3 with the Nyquist modes excluded (eq.
 * disc_f), nonlinear products on the 3/2-rule M1 x M3 grid; B-splines of
 * order p (B) and p+1 (B*, for m2) on clamped knots in x2 (Appendix C),
 * collocated at Greville points; Dirichlet rows for phi2, Omega2, Neumann
 * rows for z, <m>1, <m>3, Robin (potential-matching) rows for m2, and
 * <m2>(+L2/2) = 0 (Section 4.5).
 *
 * Array layout.  A spectral field ("S-field") is complex128 (interleaved
 * re, im doubles), shape [ny][N3-1][N1/2], index [j][n_idx][l], l fastest:
 * ny = n2 for fields in B, n2+1 for fields in B*; l = 0..N1/2-1; n_idx runs
 * over n = 0..N3/2-1 then n = -(N3/2-1)..-1.  The l = 0 column must be
 * Hermitian in n (f_{0,-n} = conj f_{0,n}) and is kept so.  The plane means
 * <m>1, <m>3 and their RHS are real double [n2].  The (0,0) entries of phi2
 * and Omega2 are ignored on input and their RHS are written as zero.
 *
 * Ownership.  Every state, output and workspace buffer is device memory owned
 * by the caller.  A plan owns only its constant tables, among them the
 * factors of A(k) for every (l, |n|) pair, which lmvd_plan_create computes
 * and checks (lmvd_factor_check).  lmvd_substep allocates nothing, does not
 * synchronise the host and only enqueues work on the given stream.
 *
 * Errors.  Every entry point returns an lmvd_status; no exceptions cross
 * the ABI.  LMVD_EINVAL: bad configuration, null or misaligned (not 16-byte)
 * pointer, or a bad argument value.  LMVD_EUNSUPPORTED: a grid size outside
 * what the kernels handle (M1/2 and M3 must be products of 2s and 3s with
 * M3 <= 1024 and M1/2 <= 768, N1/2 <= M1/2, N3-1 <= M3, order <= 9, n2 <= 4096,
 * and a band of A(k) (built on order + 1 for m2) within 8, which order 9 keeps
 * only for some breakpoint distributions).  LMVD_ENOMEM:
 * host or device allocation failed in lmvd_plan_create.  LMVD_EHIP: a HIP
 * call failed.  LMVD_ENUMERIC: a factorisation without pivoting met a
 * near-zero pivot or excessive growth at plan creation (the shared
 * projections on the host, A(k) for every (l, |n|) pair on the device).  LMVD_ENONFINITE: with check_finite set,
 * an output of lmvd_substep holds a NaN or an infinity (the outputs are
 * written all the same).
 */
#ifndef LMVD_H
#define LMVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lmvd_plan_s* lmvd_plan;

typedef enum {
  LMVD_OK = 0,
  LMVD_EINVAL = -1,
  LMVD_ENOMEM = -2,
  LMVD_EHIP = -3,
  LMVD_EUNSUPPORTED = -4,
  LMVD_ENUMERIC = -5,
  LMVD_ENONFINITE = -6
} lmvd_status;

/* Problem definition.  Symbols follow the paper. */
typedef struct {
  int32_t n1, n3;        /* Fourier modes, even; retained |l| <= n1/2-1, |n| <= n3/2-1 (eq. disc_f) */
  int32_t n2;            /* number of B coefficients (order-p B-splines); m2 uses n2+1 of order p+1 */
  int32_t order;         /* p (App. C); 3 <= p <= 9 (9: see LMVD_EUNSUPPORTED)                      */
  int32_t m1, m3;        /* physical x1, x3 grid; 3/2 rule: m = 3n/2; m1 >= n1, m3 >= n3            */
  double L1, L2, L3;     /* domain [0,L1] x [-L2/2, L2/2] x [0,L3] (Section 4)                        */
  const double* breakpoints; /* host array of n2-order+2 strictly increasing values, ends -+L2/2     */
  double dt;             /* time step (fixed per plan: the BDF-like guesses assume a uniform dt)      */
  double mu;             /* dynamic viscosity: constant part of mu(z) (see mu_z)                       */
  double rhoD;           /* rho D_z: constant part of q(z) (see rhoD_z, rhoD_form)                     */
  double g;              /* gravity along -x2 (body force -rho g delta_i2)                           */
  double rho_l, rho_h;   /* light / heavy density of the mixture EOS rho = rl rh / (rh - (rh - rl) z) */
  double beta_n, beta_p; /* free parameters of the BDF-like guesses (paper: 0, -4)                    */
  int32_t kf;            /* default number of fixed-point iterations                                  */
  int32_t plane_batch;   /* y-planes per physical-space batch (0 = all planes at once)               */
  /* Transport laws mu = g(z), D_z = h(z) (Section 2, after the stress tensor), as cubics in z:
   *   mu(z) = mu + mu_z[0] z + mu_z[1] z^2 + mu_z[2] z^3,
   *   q(z)  = rhoD + rhoD_z[0] z + rhoD_z[1] z^2 + rhoD_z[2] z^3,
   *   rho D_z = q(z) (rhoD_form 0) or f(z) q(z) (rhoD_form 1, i.e. D_z = q(z)).
   * All zero (a zero-initialised struct): constant mu and rho D, the fastest path.  A z-dependent
   * mu adds one physical-grid pass (tau_ij = mu(z) S_ij) per substep; a z-dependent rho D costs
   * nothing extra: div(rho D grad z) = rho D lap z + (rho D)'(z) |grad z|^2 is formed in the R_z
   * product.  Non-finite coefficients or another rhoD_form give LMVD_EINVAL. */
  double mu_z[3];
  double rhoD_z[3];
  int32_t rhoD_form;
  /* 1: lmvd_substep scans its outputs (z_out, phi2_out, omega2_out, the plane means, zt) for NaN
   * and infinity and returns LMVD_ENONFINITE if it finds one.  The scan synchronises the stream
   * (a diagnostic for long runs, not for timed loops); a plan with it set cannot enter a graph. */
  int32_t check_finite;
} lmvd_config;

/* Arguments of one substep.  All pointers are device pointers.  Pointers that
 * are optional may be NULL. */
typedef struct {
  int32_t stage;          /* 0 = stage n, 1 = stage ' (Section 3.2)                                    */
  int32_t kf;             /* iterations for this call; -1 = the plan's kf                               */
  int32_t guess_mode;     /* 0 = BDF-like guess from z_hist; 1 = zero guess (startup without history)  */
  /* state at stage s (inputs) */
  const void* phi2;       /* S-field (B)                                                               */
  const void* omega2;     /* S-field (B)                                                               */
  const void* z;          /* S-field (B)                                                               */
  const double* m1bar;    /* [n2]                                                                       */
  const double* m3bar;    /* [n2]                                                                       */
  /* state at stage s+1 (outputs).  phi2_out, omega2_out, m1bar_out, m3bar_out
   * may alias their inputs; z_out must not alias z (z^s is read to the end). */
  void* phi2_out;
  void* omega2_out;
  void* z_out;
  double* m1bar_out;
  double* m3bar_out;
  /* stage ' only: data stored at stage n */
  const void* rhs_phi2_prev;
  const void* rhs_omega2_prev;
  const void* zt_prev;    /* z_t^{n, k_f}                                                              */
  const double* rhs_m1_prev;
  const double* rhs_m3_prev;
  /* this stage's RHS and z_t^{s, k_f} (outputs; required at stage n, optional at stage ') */
  void* rhs_phi2;
  void* rhs_omega2;
  void* zt;
  double* rhs_m1;
  double* rhs_m3;
  /* z coefficients of the previous three stages, most recent first
   * (stage n: z^{n-1,'}, z^{n-1}, z^{n-2,'}; stage ': z^n, z^{n-1,'}, z^{n-1});
   * read only with guess_mode 0.  z_out may alias z_hist[2]. */
  const void* z_hist[3];
  /* optional diagnostics: m^d = (m1 in B, m2 in B*, m3 in B), m^c likewise */
  void* md[3];
  void* mc[3];
} lmvd_substep_args;

const char* lmvd_status_string(lmvd_status s);

/* Build the plan: host tables (knots, Greville points, collocation and
 * derivative matrices, no-pivot LU of the shared projections, FFT twiddles),
 * their upload to the current device, and the checked A(k) factors of every
 * (l, |n|) pair (computed on the device).  Host-synchronous. */
lmvd_status lmvd_plan_create(const lmvd_config* cfg, lmvd_plan* out);
lmvd_status lmvd_plan_destroy(lmvd_plan plan);

/* Element counts of an S-field in B (n2 rows) and in B* (n2+1 rows), and the
 * workspace size in bytes that lmvd_substep needs (256-byte aligned pointer). */
lmvd_status lmvd_sizes(lmvd_plan plan, size_t* sfield_elems, size_t* sfield_star_elems,
                       size_t* workspace_bytes);

/* One substep (Algorithm time_advanceDNS) on `stream` (a hipStream_t; NULL =
 * the null stream).  Asynchronous.  Not reentrant: one plan must not run on two
 * streams at once, and concurrent calls must use distinct workspaces.  It
 * allocates nothing, issues no memset and does not synchronise (unless the plan
 * sets check_finite), so a caller may capture it in a HIP graph, the first
 * call on a plan included (the A(k) factors are made at plan creation).
 * The timing hook must be off while capturing. */
lmvd_status lmvd_substep(lmvd_plan plan, const lmvd_substep_args* args, void* workspace,
                         void* stream);

/* ---- allocation-free substep ----
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): lmvd_substep with the workspace taken from a fixed array of device
 * memory that the library holds on every GPU it runs on (64 MiB, lmvd_noalloc_capacity), instead of a
 * caller buffer.  Same arguments, results and asynchrony as lmvd_substep; it calls no hipMalloc, hipFree
 * or other allocating routine.  Plans whose workspace (lmvd_sizes) exceeds the array are rejected with
 * LMVD_EUNSUPPORTED before anything is launched (64 MiB holds for example 32 x 97 x 32 or
 * 48 x 33 x 48).  Every call on a GPU uses that GPU's one array, whose contents the previous call left
 * there (a substep writes every workspace byte it reads, so nothing is carried between calls): calls that
 * overlap on one GPU (two streams, or two host threads) race and must not be made. */
lmvd_status lmvd_substep_noalloc(lmvd_plan plan, const lmvd_substep_args* args, void* stream);
lmvd_status lmvd_noalloc_capacity(size_t* bytes);

/* ---- many independent simulations in one HIP graph ----
 * For small problems, where one substep is a few dozen short launches, the
 * substeps of many independent instances (each its own plan, workspace and
 * state; any sizes the plans support) are captured into one HIP graph whose
 * instances are independent branches; one lmvd_graph_launch runs `nsub`
 * substeps of every instance.
 *
 * Instances whose substeps line up step by step share one grouped launch per
 * kernel step (one per transform size for the transforms); otherwise every
 * instance is a graph branch of its own.
 *
 * lmvd_graph_create: plans[count], workspaces[count] (one per instance,
 * distinct), args[count * nsub] with args[i * nsub + k] the k-th substep of
 * instance i (same rules as lmvd_substep; the diagnostic outputs md, mc must
 * be NULL).  The argument structs are read during the call only, but every
 * device pointer in them is baked into the graph: those buffers must stay
 * allocated, at the same addresses, while the graph exists.  A sequence of
 * args whose pointers repeat after nsub substeps (a history ring of period
 * nsub, with the stages alternating) makes repeated launches keep advancing
 * the simulations.  No plan may have its timing hook active.  Host-synchronous;
 * launches nothing else.  Errors: LMVD_EINVAL for bad arguments, LMVD_EHIP if
 * capture or instantiation fails (nothing is left allocated).
 * lmvd_graph_launch: asynchronous on `stream`; launches of one graph, and of
 * lmvd_substep on the same plans, must not overlap.
 * lmvd_graph_destroy: frees the graph (not the buffers it refers to). */
typedef struct lmvd_graph_s* lmvd_graph;
lmvd_status lmvd_graph_create(const lmvd_plan* plans, const lmvd_substep_args* args,
                              void* const* workspaces, int32_t count, int32_t nsub,
                              lmvd_graph* out);
lmvd_status lmvd_graph_launch(lmvd_graph graph, void* stream);
lmvd_status lmvd_graph_destroy(lmvd_graph graph);
/* Which form the graph took: 1 = grouped (every kernel step one launch over
 * the instances that run it; requires the instances' substeps to line up step
 * by step: same k_f, stage pattern and kernel variants), 0 = one branch per
 * instance.  Both give the results of the plain path. */
lmvd_status lmvd_graph_grouped(lmvd_graph graph, int32_t* grouped);

/* ---- tile autotuner ----
 * Chooses the tile of the register z-transform kernels of a plan with M3 < 768, as a code K = D + 8 V:
 * V in {0, 1, 2} selects the line plan (threads per z line T, radix split and stage order of the Stockham
 * FFT, whose first radix is the M3 / T points of a thread; three plans for M3 = 48, 72, 96, 144 and 192,
 * one for the other sizes, where V = 1, 2 mean the first) and D in {1, 2, 4} divides the 256 / T lines
 * per block (fewer lines per block leave fewer idle lanes when N1/2 is small).  The plans:
 *   M3 = 48:  V0 T 4 radices 12.4      V1 T 8 6.2.2.2     V2 T 2 24.2
 *   M3 = 72:  V0 T 6 12.6              V1 T 12 6.6.2      V2 T 3 24.3
 *   M3 = 96:  V0 T 8 12.4.2            V1 T 4 24.4        V2 T 8 12.2.4
 *   M3 = 144: V0 T 12 12.12            V1 T 24 6.6.2.2    V2 T 6 24.6
 *   M3 = 192: V0 T 16 12.4.4           V1 T 8 24.8        V2 T 16 12.2.2.4
 * With force = 0 it times the inverse and forward z transforms of three fields over the plan's plane
 * batch for each candidate code (a warm-up, then 5 repetitions, HIP events on the stream) on the
 * caller's workspace, whose contents it overwrites, and keeps the fastest; force = a code (1, 2, 4, 9,
 * 10, 12, 17, 18, 20) sets it without timing.  Plans without such kernels (M3 = 768, or a size without a
 * register plan) keep K = 1.  zdiv (host) receives the choice; times_ms (host, optional, 9 doubles) the
 * mean time of one repetition for K = 1, 2, 4, 9, 10, 12, 17, 18, 20 (-1 where not timed).  The choice
 * holds for every later call on the plan, graphs captured afterwards included; results do not depend
 * on it beyond rounding.  Synchronises the stream; not during graph capture or a profile
 * (LMVD_EINVAL). */
lmvd_status lmvd_autotune(lmvd_plan plan, void* workspace, void* stream, int32_t force, int32_t* zdiv,
                          double* times_ms);

/* The same tile choice made for a batch by timing the graph itself: instances run side by side in a
 * graph, where a tile that is faster alone can be slower.  Takes the arguments of lmvd_graph_create
 * (same rules) and a stream; sets K = 1 on every plan with a choice, then, one z-transform size at a
 * time, tries every other code of that size (the line plans and divisors above) for all plans of that
 * size and keeps a code that makes the graph at least 1 % faster.  Each try captures the graph,
 * launches it once, times `launches` launches (1..100) with HIP events and destroys it, so every try
 * ADVANCES EVERY INSTANCE by (1 + launches) * nsub substeps: call it where warm-up launches would go.
 * zdivs (host, optional, count entries) receives each plan's code, ms_per_launch (host, optional) the
 * best time per launch.  Graphs captured afterwards use the choice.  Synchronises the stream. */
lmvd_status lmvd_graph_autotune(const lmvd_plan* plans, const lmvd_substep_args* args, void* const* workspaces,
                                int32_t count, int32_t nsub, void* stream, int32_t launches, int32_t* zdivs,
                                double* ms_per_launch);

/* ---- operator entry points (same conventions), one per stage of the path ----
 * They expose the steps of the substep individually for verification. */

/* Inverse transform (eq. disc_f at the 3/2 grid): spectral values at the
 * Greville points (S-field of values, n2 rows) -> real physical field
 * double [n2][m3][m1], index [j][b][a] at x = a L1/m1, z = b L3/m3. */
lmvd_status lmvd_to_physical(lmvd_plan plan, const void* values, double* phys,
                             void* workspace, void* stream);
/* Forward transform: physical double [n2][m3][m1] -> values on the retained
 * modes, (1/(m1 m3)) sum u e^{-i(k1 x + k3 z)}. */
lmvd_status lmvd_to_spectral(lmvd_plan plan, const double* phys, void* values,
                             void* workspace, void* stream);
/* Projection values -> B coefficients: kind 0 = interpolation, 1 = Dirichlet
 * end rows, 2 = Neumann end rows (the end values are replaced by zero). */
lmvd_status lmvd_project(lmvd_plan plan, int32_t kind, const void* values, void* coeffs,
                         void* stream);
/* Evaluation B coefficients -> values at the Greville points: deriv 0, 1, 2.
 * With star = 1 the input is a B* S-field (n2+1 rows) and deriv must be 0. */
lmvd_status lmvd_evaluate(lmvd_plan plan, int32_t deriv, int32_t star, const void* coeffs,
                          void* values, void* stream);
/* m^d from (phi2, Omega2, <m>1, <m>3): writes m1 (B), m2 (B*), m3 (B). */
lmvd_status lmvd_md(lmvd_plan plan, const void* phi2, const void* omega2,
                    const double* m1bar, const double* m3bar, void* m1, void* m2, void* m3,
                    void* workspace, void* stream);
/* m^c from the B coefficients of rho_t: writes m1 (B), m2 (B*), m3 (B). */
lmvd_status lmvd_mc(lmvd_plan plan, const void* rhot, void* m1, void* m2, void* m3,
                    void* workspace, void* stream);

/* Steps 4 and 5 of the substep alone (Algorithm time_advanceDNS): the right-hand sides of Omega2, phi2
 * (eqs. om and phi, with the body force -rho g delta_i2) and of the plane means (eq. mean_m1m3) for a
 * given z (S-field, B) and momentum m = (m1 in B, m2 in B*, m3 in B): values at the Greville points,
 * u = m/rho, rho and C_ij = -m_i m_j/rho on the 3/2 grid, u_hat, T_ij = C_ij + tau_ij (with mu(z) when
 * the plan has it) projected, N_i, and the Dirichlet (Omega2, phi2) and Neumann (means) projections.
 * The same kernels as lmvd_substep, without the RK2 update.  Outputs: rhs_phi2, rhs_omega2 (S-fields,
 * (0,0) mode zero), rhs_m1, rhs_m3 ([n2]); all device pointers, 16-byte aligned; workspace as for
 * lmvd_substep (256-byte aligned, contents overwritten).  Asynchronous. */
lmvd_status lmvd_rhs(lmvd_plan plan, const void* z, const void* m1, const void* m2, const void* m3, void* rhs_phi2,
                     void* rhs_omega2, double* rhs_m1, double* rhs_m3, void* workspace, void* stream);

/* ---- adjoints of the linear operators (for gradients through the substep's building blocks) ----
 * Transposes in the real inner products <a, b> = sum Re(conj(a) b) over every stored entry of an
 * S-field and <f, g> = sum f g over a physical field, so that <A x, y> = <x, A^T y>.  With them the
 * operators can sit behind automatic differentiation (the binding's autograd module).
 *
 * lmvd_to_physical_adjoint: transpose of lmvd_to_physical (eq. disc_f on the 3/2 grid) on S-fields
 * with a Hermitian l = 0 column (the inputs lmvd_to_physical accepts; its output has one too): the
 * forward transform of phys times M1 M3, and times 2 for l > 0 (the real field takes c_l with its
 * conjugate partner at -l).  phys [n2][M3][M1] in, values out
 * (S-field); workspace as for lmvd_to_spectral.
 * lmvd_evaluate_adjoint: E_d^T (or F_0^T with star = 1): values at tau (n2 rows) in, coefficients out
 * (n2 rows, n2 + 1 with star); values and coeffs must not alias.
 * lmvd_project_adjoint: transpose of lmvd_project for the same kind: R A^{-T} with A = LU the kind's
 * collocation matrix (App. C) and R the end-row replacement (kinds 1, 2); coeffs in, values out,
 * not aliased.  All device pointers; asynchronous. */
lmvd_status lmvd_to_physical_adjoint(lmvd_plan plan, const double* phys, void* values, void* workspace,
                                     void* stream);
/* Transpose of lmvd_to_spectral (same contract): the inverse transform of values / (M1 M3 w_l), w_0 = 1,
 * w_l = 2.  values (S-field) in, phys out; workspace as for lmvd_to_physical. */
lmvd_status lmvd_to_spectral_adjoint(lmvd_plan plan, const void* values, double* phys, void* workspace,
                                     void* stream);
lmvd_status lmvd_evaluate_adjoint(lmvd_plan plan, int32_t deriv, int32_t star, const void* values, void* coeffs,
                                  void* stream);
lmvd_status lmvd_project_adjoint(lmvd_plan plan, int32_t kind, const void* coeffs, void* values, void* stream);

/* Transpose of lmvd_md, the map (phi2, Omega2, <m>1, <m>3) -> (m1, m2, m3) of eqs. phi_poisson,
 * bc_both and md_recon, in the same inner products (the plane means as plain real vectors): from the
 * adjoints m1, m3 (S-fields, B) and m2 (B*) it writes the adjoints phi2, omega2 (S-fields) and m1bar,
 * m3bar ([n2]).  A(k)^{-T} uses the plan's A(k) factors.  Per column the
 * adjoint of the Robin rows is zero and the (0,0) column maps to the plane means only.  workspace as
 * for lmvd_substep (one (n2+1)-row scratch field).  Device pointers, asynchronous. */
lmvd_status lmvd_md_adjoint(lmvd_plan plan, const void* m1, const void* m2, const void* m3, void* phi2,
                           void* omega2, double* m1bar, double* m3bar, void* workspace, void* stream);

/* Transpose of lmvd_mc, the map rho_t (B coefficients) -> (m1, m2, m3) of eqs. COM_fourier, CF_fourier,
 * mc_recon and mc_mean: from the adjoints m1, m3 (B) and m2 (B*) it writes the adjoint rhot (S-field,
 * B).  The (0,0) column transposes the plane-mean system (D* rows and the top condition).  workspace and
 * factors as for lmvd_md_adjoint.  Device pointers, asynchronous. */
lmvd_status lmvd_mc_adjoint(lmvd_plan plan, const void* m1, const void* m2, const void* m3, void* rhot,
                           void* workspace, void* stream);

/* ---- adjoint of the substep ----
 * Reverse mode of lmvd_substep (Algorithm time_advanceDNS) for gradients through a simulation: given
 * the substep's inputs (the same lmvd_substep_args as the forward call; its output pointers are not
 * used) and the cotangents of its outputs, it writes the gradients with respect to its inputs, in the
 * real inner products <a, b> = sum Re(conj(a) b) over the stored entries of an S-field and the plain dot
 * product of real vectors.  It recomputes the substep's intermediates from the inputs (the iterates
 * z_t^k and m^c of the fixed point, m = m^d + m^c on the grid, the grid values of z and its
 * derivatives) and transposes every step in reverse order: the RK2 update, the right-hand sides and
 * fluxes (eqs. om, phi, mean_m1m3), the final m^c (eqs. COM_fourier, CF_fourier, mc_recon, mc_mean),
 * the k_f fixed-point iterations with the matrix-free L(z) of Section 4.3, R_z, the guess (eq.
 * dzdt_guesses) and m^d (eqs. phi_poisson, md_recon), with hand-written kernels for the pointwise
 * Jacobians and the transposes of the linear operators below.
 * Gradients of S-fields are returned as their representatives with a Hermitian l = 0 column (the part
 * that pairs with the inputs the library accepts); the (0,0) entries of the phi2 and Omega2 gradients
 * are zero (those inputs are ignored).  Constant transport coefficients only (LMVD_EUNSUPPORTED for a
 * plan with mu(z) or rho D(z)).  workspace: lmvd_adjoint_sizes bytes (256-byte aligned; it contains the
 * substep workspace), overwritten.  Asynchronous on `stream`; allocates nothing. */
typedef struct {
  /* cotangents of lmvd_substep's outputs (device; required, zero arrays where an output does not
   * matter) */
  const void* phi2_out;
  const void* omega2_out;
  const void* z_out;
  const double* m1bar_out;
  const double* m3bar_out;
  const void* rhs_phi2;
  const void* rhs_omega2;
  const void* zt;
  const double* rhs_m1;
  const double* rhs_m3;
  /* cotangents of the diagnostic outputs m^d, m^c (m2 in B*; optional, NULL = zero) */
  const void* md[3];
  const void* mc[3];
  /* gradients with respect to the inputs (device, written; required) */
  void* phi2;
  void* omega2;
  void* z;
  double* m1bar;
  double* m3bar;
  /* optional (NULL = not wanted): the z history (guess_mode 0; zero with guess_mode 1) and, at stage ',
   * the stage-n data */
  void* z_hist[3];
  void* rhs_phi2_prev;
  void* rhs_omega2_prev;
  void* zt_prev;
  double* rhs_m1_prev;
  double* rhs_m3_prev;
} lmvd_substep_grads;
lmvd_status lmvd_adjoint_sizes(lmvd_plan plan, int32_t kf, size_t* workspace_bytes);
lmvd_status lmvd_substep_adjoint(lmvd_plan plan, const lmvd_substep_args* args, const lmvd_substep_grads* grads,
                                 void* workspace, void* stream);

/* Timing hook for measurements: while active, every launch of one kernel
 * class is bracketed by two HIP events recorded on the stream it is launched
 * on.  Classes (one kernel each):
 *   0 inverse z-FFT of values at tau          7 m^d solve, z values and guess
 *   1 x-pass of R_z (+ physical aux fields)   8 projection, plain store
 *   2 x-pass of L z_t                         9 projection + R_z add (+ z update)
 *   3 x-pass of rho_t                        10 values at tau of fixed fields
 *   4 x-pass of u, rho, C_ij                 11 T_ij projection + RHS emission
 *   5 forward z-FFT + truncation             12 RHS projection + RK2 + plane means
 *   6 fused m^c column kernel                13 x-pass of the transform calls
 *                                            14 z filter + wall planes of the
 *                                               non-final fixed-point iterates
 * lmvd_profile_start creates `max_launches` event pairs on the host
 * (launches beyond that are not timed); lmvd_profile_stop waits for the
 * events and returns the summed elapsed milliseconds, the number of timed
 * launches and their compulsory HBM bytes: inputs read once, outputs written
 * once, factor tables, and the stored intermediate of a two-sweep banded
 * solve; re-reads through the caches are not counted. */
lmvd_status lmvd_profile_start(lmvd_plan plan, int32_t cls, int32_t max_launches);
lmvd_status lmvd_profile_stop(lmvd_plan plan, double* total_ms, int64_t* launches, double* compulsory_bytes);

/* ---- the no-pivot factorisation of A(k) ----
 * The m^d and m^c solves use one factorisation of A(k) = E*_2 - k^2 E*_0 with the Robin rows (eqs.
 * phi_poisson, bc_both) per (l, |n|) pair, eliminated from the last row upwards without pivoting, made
 * and checked by lmvd_plan_create for every pair of the grid: with s the largest magnitude of row i of
 * A(k), the pivot of the row must reach 1e-12 s and no entry of the eliminated row may exceed
 * growth_max s (1e4 at plan creation); a NaN fails too.  A plan whose factors fail is not created
 * (LMVD_ENUMERIC).
 * lmvd_factor_check: the result of that check for a plan (growth_max = 0), or the factorisation made
 * and checked again with another growth_max > 0 (synchronous; the factors are the same, so the plan stays
 * usable; the new result replaces the old).  Outputs (host, optional): the largest growth, the smallest
 * pivot ratio, the number of rows that failed.  Returns LMVD_ENUMERIC if any row failed.
 * lmvd_factor_check_host: the same elimination and check on the host for every distinct nonzero k^2 of
 * the configuration's grid (no GPU; for validating a configuration before a plan); distinct_k receives
 * the number of k^2 checked. */
lmvd_status lmvd_factor_check(lmvd_plan plan, double growth_max, double* max_growth, double* min_pivot_ratio,
                              int64_t* bad_rows);
lmvd_status lmvd_factor_check_host(const lmvd_config* cfg, double growth_max, double* max_growth,
                                   double* min_pivot_ratio, int64_t* bad_rows, int64_t* distinct_k);

/* Host-only view of the plan's y-discretisation (for inspection; no GPU use):
 * Greville points tau [n2] and tau* [n2+1], and the dense matrices
 * E_d (d = 0,1,2; n2 x n2, row-major) of the B-splines at tau.
 * Any output pointer may be NULL. */
lmvd_status lmvd_host_tables(const lmvd_config* cfg, double* tau, double* tau_star,
                             double* E0, double* E1, double* E2);

/* Host-only values of the y basis at arbitrary points (App. C: B-splines of order p on the plan's
 * clamped knots, star = 0, or of order p + 1 for m2, star = 1): out[i * ncols + j] = B_j(y[i]),
 * ncols = n2 (n2 + 1 with star).  For quadratures in y (an objective's integral, say).  LMVD_EINVAL if
 * a point lies outside [-L2/2, L2/2]. */
lmvd_status lmvd_basis_values(const lmvd_config* cfg, int32_t npts, const double* y, int32_t star, double* out);

#ifdef __cplusplus
}
#endif
#endif /* LMVD_H */
