/*
 * gpe.h -- C ABI of libgpe, the gfx950 implementation of the hot path of the preconditioned
 * nonlinear conjugate-gradient (PCG) ground-state solver for the rotating Gross-Pitaevskii
 * energy of Antoine, Levitt and Tang (arXiv:1611.02045).
 *
 * Problem (Section 2): minimise
 *     E(phi) = int 1/2 |grad phi|^2 + V |phi|^2 + beta/2 |phi|^4 - omega conj(phi) L_z phi
 * over ||phi|| = 1, where L_z = -i (x d_y - y d_x) and beta is the paper's nonlinearity eta.
 * Discretisation (Section 3): periodic box prod_a [-L_a, L_a) with n_a points per axis,
 * h_a = 2 L_a / n_a, x_k = -L_a + k h_a; Fourier pseudo-spectral derivatives with frequencies
 * xi_p = p pi / L_a, -n_a/2 <= p < n_a/2 (the Nyquist mode is kept in odd derivatives).
 * Inner products are quadrature weighted: <f, g> = h^d sum conj(f) g, and ||phi||^2 = h^d sum |phi|^2.
 *
 * Data layout: every field is a C-ordered array with x fastest, i.e. element (k_z, k_y, k_x) at
 * offset (k_z * n_y + k_y) * n_x + k_x.  Wave functions are interleaved complex (re, im) of the
 * plan's real type; potentials are real of the same type.  All field pointers are DEVICE
 * pointers owned by the caller; the library never frees them and does not keep them after the
 * call's work has completed on the stream.  Host pointers are marked "host".
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default stream).  Calls that
 * return host scalars synchronise that stream; the others are asynchronous.  A plan owns device
 * workspace and must not be used from two streams or threads at once.
 *
 * Errors: every entry point returns a gpe_status_t; negative values are errors, and
 * gpe_last_error() returns a thread-local message describing the last error.  No C++ exception
 * crosses this boundary.
 *
 * Supported grids: dim in {1, 2, 3}; every n_a either a power of two with 8 <= n_a <= 1024 or
 * 5 * 2^k with 40 <= n_a <= 640 (the paper's M = 640 grids); other sizes give GPE_EUNSUPPORTED.
 */
#ifndef GPE_H
#define GPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem description (Sections 2-3).  n[a] and L[a] for a >= dim are ignored. */
typedef struct gpe_problem {
    int32_t dim;    /* 1, 2 or 3 */
    int32_t n[3];   /* points per axis (x, y, z) */
    double  L[3];   /* half-widths: axis a spans [-L[a], L[a]) */
    double  beta;   /* nonlinearity strength (the paper's eta) */
    double  omega;  /* rotation speed; must be 0 when dim == 1 */
} gpe_problem_t;

/* Storage and arithmetic type of the caller's fields. */
typedef enum { GPE_F64 = 0, GPE_F32 = 1 } gpe_dtype_t;

/* Preconditioners of Section 5.5: identity, P_Delta = (alpha - Delta/2)^{-1},
 * P_V = (alpha + V + beta|phi|^2)^{-1}, the symmetric P_C = P_V^{1/2} P_Delta P_V^{1/2},
 * and the non-symmetric P_C1 = P_V P_Delta, P_C2 = P_Delta P_V. */
typedef enum {
    GPE_P_NONE = 0, GPE_P_KINETIC = 1, GPE_P_POTENTIAL = 2, GPE_P_COMBINED = 3,
    GPE_P_C1 = 4, GPE_P_C2 = 5
} gpe_precond_t;

typedef enum {
    GPE_OK = 0,             /* success / converged */
    GPE_NOT_CONVERGED = 1,  /* max_iter reached; results are still written */
    GPE_EINVAL = -1,        /* invalid argument, non-SPD preconditioner, NULL pointer */
    GPE_EUNSUPPORTED = -2,  /* valid but unsupported (grid size, dimension) */
    GPE_EHIP = -3,          /* HIP runtime error */
    GPE_ENONFINITE = -4,    /* NaN or Inf met in the input or during the iteration */
    GPE_ELINESEARCH = -5    /* no step decreased the energy (FP64 phase) */
} gpe_status_t;

typedef struct gpe_plan gpe_plan_t;

/* Create a plan: validates the problem, builds twiddle tables and allocates workspace on the
 * current device.  On success *out receives the plan; on error *out is set to NULL. */
int gpe_plan_create(const gpe_problem_t* prob, int dtype, gpe_plan_t** out);
int gpe_plan_destroy(gpe_plan_t* plan);

/* Energy E(phi) of Section 2 in its discrete form (Section 3), reduced in FP64.
 * phi: device, complex, one field.  V: device, real.  E: host, receives the total.
 * parts: host, nullable; receives {kinetic <phi,T phi>, potential <phi,V phi>,
 * interaction beta/2 h^d sum|phi|^4, rotation -omega Re<phi,L_z phi>}.  Synchronises. */
int gpe_energy(gpe_plan_t* plan, const void* phi, const void* V, double* E, double* parts,
               void* stream);

/* Hphi = H_phi phi = -1/2 Delta phi + V phi + beta |phi|^2 phi - omega L_z phi (Section 2
 * mean-field Hamiltonian, Section 3 discretisation).  Device pointers; Hphi must not alias phi.
 * Asynchronous. */
int gpe_apply_H(gpe_plan_t* plan, const void* phi, const void* V, void* Hphi, void* stream);

/* Batched form: `count` wave functions stored back to back (field b at phi + b * N), all with
 * the plan's problem and the same potential V.  Asynchronous. */
int gpe_apply_H_batched(gpe_plan_t* plan, int count, const void* phi, const void* V, void* Hphi,
                        void* stream);

/* Kernel choice of every H apply (gpe_apply_H, gpe_apply_H_batched, the noalloc form, and the
 * applies inside the solvers, the backward-Euler steps and the adjoint), process-wide:
 *   GPE_APPLY_PASSES  directional passes: an x pass (with the pointwise part) into a workspace, then
 *                     a y pass (and a z pass) adding theirs: 11sN bytes in 2-D (s bytes per real, N
 *                     points), 17sN in 3-D;
 *   GPE_APPLY_PLANE   the whole-plane kernel where the xy-plane fits one workgroup's LDS (n_x, n_y
 *                     powers of two from 32 to 256, at most 16384 points for complex64 and 8192 for
 *                     complex128, within the device's LDS per workgroup; 128^2 complex64 needs
 *                     147 KiB): both directions of Section 3's discrete operator in one pass over
 *                     each plane, 5sN bytes in 2-D; in 3-D plus a z pass, 11sN.  Other grids keep
 *                     the passes;
 *   GPE_APPLY_AUTO    (default) the whole-plane kernel where it fits and the launch has enough
 *                     planes to occupy the device, else the passes.
 * Both kernels compute the same transforms and sums and agree to rounding.
 * Meant for tests and measurements: it applies to every call in the process from the next launch
 * on.  GPE_EINVAL for an unknown kind. */
typedef enum { GPE_APPLY_AUTO = 0, GPE_APPLY_PASSES = 1, GPE_APPLY_PLANE = 2 } gpe_apply_kernel_t;
int gpe_set_apply_kernel(int kind);

/* The kernel (GPE_APPLY_PASSES or GPE_APPLY_PLANE) that gpe_apply_H_batched would launch for
 * `count` fields of the plan's grid and dtype under the current setting, on the current device.
 * kind: host, receives it. */
int gpe_apply_kernel_for(gpe_plan_t* plan, int count, int* kind);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): gpe_apply_H_batched without any allocation.  The
 * intermediate between its kernels (the running sum of the directional passes, or in 3-D the
 * whole-plane kernel's xy-part; see gpe_set_apply_kernel) lives in a static device array
 * of GPE_NOALLOC_SCRATCH_BYTES per device, held until the process ends, instead of the plan's
 * growable workspace; the plan must have been created on the current device.  Same arguments,
 * layout and results as gpe_apply_H_batched (the same kernels run).  Requires
 * count * N * (16 for FP64, 8 for FP32) <= GPE_NOALLOC_SCRATCH_BYTES, else GPE_EINVAL and nothing
 * is launched.  Every call on one device shares that device's array: calls that overlap on one
 * device (concurrent streams or host threads) race and must be ordered by the caller.
 * Asynchronous. */
#define GPE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int gpe_apply_H_batched_noalloc(gpe_plan_t* plan, int count, const void* phi, const void* V, void* Hphi,
                                void* stream);

/* Pr = P r for the preconditioner `kind` of Section 5.5 at the point phi, with shift alpha.
 * alpha = NaN selects the adaptive shift lambda~(phi) = <phi,T phi> + <phi,V phi> +
 * beta h^d sum|phi|^4 (Section 5.5), computed on the device.  Returns GPE_EINVAL when
 * alpha + V + beta|phi|^2 is not positive everywhere (P would not be SPD); that check
 * synchronises the stream.  Pr must not alias r or phi. */
int gpe_precond(gpe_plan_t* plan, int kind, const void* phi, const void* V, double alpha,
                const void* r, void* Pr, void* stream);

/* Tile measurement for the plan's grid and dtype at a batch of `count` fields per launch: for each
 * axis, the directional pass (forward transform, multiplier, inverse transform) is timed for
 * every valid number of lines per workgroup and the fastest is recorded, process-wide, for every
 * later operator launch (H apply, energy, preconditioners) on that grid, dtype and batch size.
 * The solver's own passes keep their rule: they absorb one partial row per producer workgroup,
 * and the smaller workgroups an operator pass prefers made them slower.  tiles: host, 3 ints,
 * the chosen lines per workgroup per axis (0 for absent axes); us: host, 3 doubles, the time per
 * pass of the choice in microseconds; both nullable.  Uses the plan's scratch; must not run
 * concurrently with operator calls on the same grid.  Synchronises. */
int gpe_autotune(gpe_plan_t* plan, int count, int* tiles, double* us, void* stream);

/* Interpolation onto the grid with twice the points per axis and the same box: the step between
 * the nested grids M_p -> M_{p+1} of the initial-data example of Section 6.2.  Per axis, the
 * trigonometric interpolant of the Section 3 discretisation, with the Nyquist coefficient split
 * evenly between the frequencies -M/2 and +M/2 (values at the plan's grid points are kept, real
 * fields stay real).  in: device field on the plan's grid, of the plan's dtype; out: device field
 * of 2^dim N points, shape (2 n_z, 2 n_y, 2 n_x), same dtype, not aliasing in.  The norm is not
 * restored (the solver normalises its start).  GPE_EUNSUPPORTED when 2n exceeds 1024 on an axis.
 * Uses the plan's scratch (2N or 4N complex values in 2-D / 3-D).  Asynchronous. */
int gpe_prolong(gpe_plan_t* plan, const void* in, void* out, void* stream);

/* Solver options. */
typedef struct gpe_pcg_opts {
    int32_t method;        /* 0 = projected preconditioned gradient (Algorithm 1), 1 = PCG (Algorithm 2) */
    int32_t precond;       /* gpe_precond_t */
    double  tol_res_inf;   /* stop when ||H_phi phi - lambda phi||_inf <= tol (Section 5.3) */
    double  tol_energy;    /* if > 0, also stop when |E_{n+1} - E_n| <= tol_energy */
    int64_t max_iter;
    int32_t precision;     /* 0 = FP64 throughout; 1 = mixed: FP32 fields until the switch, then FP64 */
    int32_t beta_rule;     /* 0 = Polak-Ribiere max(beta_PR, 0); 1 = Fletcher-Reeves */
    double  switch_res;    /* mixed: leave FP32 once ||r||_inf <= max(tol_res_inf, switch_res), or on
                              stagnation: no progress for 100 iterations when tol_res_inf < switch_res
                              (FP32 cannot finish), else for 400 */
    double  theta_default; /* trial angle when the quadratic model has no minimum */
    int32_t max_halvings;  /* step halvings before the line search gives up */
    int32_t refresh_every; /* recompute L phi from phi every this many iterations (0 = never) */
    int32_t check_every;   /* iterations queued between convergence polls */
    int32_t record_history;/* nonzero: keep per-iteration scalars (see gpe_pcg_history) */
    int32_t use_graph;     /* nonzero: after the first chunk, replay the chunk of check_every
                            * iterations as a captured HIP graph (needs an even check_every) */
    int32_t line_search;   /* step control of Section 5.1: 0 = the trials theta_opt, theta_opt/2, ...
                            * (at most max_halvings halvings), the first that lowers E accepted;
                            * 1 = the same trials under the Armijo test
                            * E(t) - E(0) <= 1e-4 t E'(0); 2 = full line search: the global
                            * minimiser over [0, pi) of E(cos t phi + sin t phat), accepted when it
                            * lowers E; 3 = a step satisfying the strong Wolfe conditions
                            * (c1 = 1e-4, c2 = 0.1) found by bracketing from theta_opt (up to pi/2)
                            * and bisection, at most max_halvings evaluations per phase, counted
                            * as halvings.  All evaluate the exact energy polynomial of the
                            * direction pass: no extra pass over the fields */
} gpe_pcg_opts_t;

typedef struct gpe_pcg_report {
    int32_t status;        /* gpe_status_t of this solve */
    int32_t switched;      /* mixed mode: 1 if the FP64 phase was entered */
    int64_t iters;         /* total iterations (both phases) */
    int64_t iters_fp32;    /* iterations done in FP32 */
    int64_t restarts;      /* non-descent restarts (Section 5.2) */
    int64_t halvings;      /* total step halvings */
    double  E, lambda, res_inf;   /* final energy, chemical potential, ||r||_inf (fresh FP64) */
    double  dE;            /* |E_n - E_{n-1}| of the last step */
    double  dphi_inf;      /* ||phi_n - phi_{n-1}||_inf of the last step */
    double  seconds;       /* wall time of the solve (excluding plan creation) */
} gpe_pcg_report_t;

/* Fill *opts with defaults: PCG, P_C, tol 1e-8, 20000 iterations, FP64, Polak-Ribiere,
 * switch_res 1e-6, theta_default 0.1, 30 halvings, refresh every 50, poll every 16, graph replay on,
 * the decrease-test line search. */
void gpe_pcg_opts_default(gpe_pcg_opts_t* opts);

/* Ground state by PG / PCG on the unit sphere (Algorithms 1-2 with the step control of
 * Sections 5.1-5.2).  phi_inout: device, the initial guess (normalised on entry by the solver),
 * overwritten by the final iterate.  V: device.  report: host.  Synchronises.
 * Returns GPE_OK when converged, GPE_NOT_CONVERGED at max_iter, or an error. */
int gpe_pcg_solve(gpe_plan_t* plan, const void* V, void* phi_inout, const gpe_pcg_opts_t* opts,
                  gpe_pcg_report_t* report, void* stream);

/* Per-iteration record of the last solve when opts->record_history was set.  hist: host,
 * receives up to `cap` rows of 8 doubles {n, E_n, lambda_n, ||r_n||_inf, theta_n, beta_n,
 * halvings_n, restarted_n}; returns the number of rows written (>= 0) or an error. */
int gpe_pcg_history(gpe_plan_t* plan, double* hist, int cap);

/* Independent solves of `count` problems (possibly different grids, beta, omega, L); instances
 * of equal grid share each kernel launch and converged instances leave the launches.  The instances
 * of a grid are split into two parts, and the parts of all grids are solved concurrently, each
 * on its own stream (the caller's for the first, default-priority streams the call creates for
 * the others) driven by its own host thread; the created streams first wait for the work already
 * queued on the caller's stream.  Results do not depend on the split.  V[i], phi_inout[i]: device fields of instance i in its own layout and
 * in the type `dtype`.  reports: host array of `count`.  Returns the worst status.
 * Synchronises both streams before returning. */
int gpe_pcg_solve_batched(int count, const gpe_problem_t* probs, int dtype, void* const* V,
                          void* const* phi_inout, const gpe_pcg_opts_t* opts,
                          gpe_pcg_report_t* reports, void* stream);

/* Ground states on nested grids (the multigrid preparation of initial data, Section 6.2): the
 * `count` instances are solved together (as gpe_pcg_solve_batched) on the coarsest grid from
 * phi_coarse, each converged state is interpolated (gpe_prolong) onto the grid with twice the
 * points per axis and solved again, for `levels` grids in all.  coarsest[i]: the problem of
 * instance i on the coarsest grid (level l has n << l points per axis, same box, beta, omega).
 * V: levels * count device potentials, level-major (V[l * count + i] on the level-l grid).
 * phi_coarse[i]: device start on the coarsest grid (read only).  phi_fine[i]: device output on
 * the finest grid.  opts: every level; the coarse levels stop at ||r||_inf <= tol_coarse instead
 * of opts->tol_res_inf.  reports: host, levels * count, level-major.  dtype as in
 * gpe_pcg_solve_batched.  Returns the worst status of the finest level (a coarse level that does
 * not converge still hands on its state), or the first error.  Synchronises. */
int gpe_pcg_solve_nested(int count, int levels, const gpe_problem_t* coarsest, int dtype,
                         void* const* V, void* const* phi_coarse, void* const* phi_fine,
                         const gpe_pcg_opts_t* opts, double tol_coarse,
                         gpe_pcg_report_t* reports, void* stream);

/* Ground state by the backward Euler discretisation of the normalised gradient flow (the BESP
 * schemes of Section 4; BE_nu of Section 6).  Outer step n: lambda_n = <phi_n, H phi_n>; stop when
 * ||H phi_n - lambda_n phi_n||_inf <= opts->tol_res_inf or after opts->max_iter steps; otherwise
 * solve (I/dt + H_{phi_n} - s lambda_n) phit = phi_n / dt with the nonlinearity frozen at phi_n
 * (s = 1 when lambda_term, else 0) by preconditioned linear CG from phit = phi_n, to
 * ||residual|| <= inner_tol ||phi_n / dt|| (at most 10000 inner iterations), and set
 * phi_{n+1} = phit / ||phit||.  opts->precond: the inner preconditioner (GPE_P_NONE, _KINETIC,
 * _POTENTIAL or _COMBINED, with shift 1/dt); opts->check_every: inner iterations between polls;
 * the other options are ignored.  phi_inout: device, normalised on entry, overwritten.
 * inner_iters: host, nullable, the total of inner iterations (the paper's count for BE_nu).
 * report: host, nullable (iters = outer steps).  GPE_EINVAL when the inner operator is not
 * positive definite (dt too large).  Synchronises. */
int gpe_be_solve(gpe_plan_t* plan, const void* V, void* phi_inout, double dt, int lambda_term,
                 const gpe_pcg_opts_t* opts, double inner_tol, int64_t* inner_iters,
                 gpe_pcg_report_t* report, void* stream);

/* Backward of the energy (conjugate-Wirtinger convention of real-valued losses):
 * grad_phi = 2 h^d H_phi phi (device, complex), grad_V = h^d |phi|^2 (device, real, nullable),
 * *dE_dbeta = 1/2 h^d sum |phi|^4 and *dE_domega = -Re<phi, L_z phi> (host, nullable).
 * Synchronises when a host scalar is requested. */
int gpe_energy_grad(gpe_plan_t* plan, const void* phi, const void* V, void* grad_phi, void* grad_V,
                    double* dE_dbeta, double* dE_domega, void* stream);

/* Implicit adjoint at a converged ground state phi_star: solves A mu = M rhs on the tangent
 * space {f : Re<phi_star, f> = Re<i phi_star, f> = 0} with A = Pi (1/2 nabla^2 E - lambda) Pi,
 * where 1/2 nabla^2 E [f] = H f + 2 beta Re(conj(phi) f) phi (the second derivative of
 * Section 2 with its interaction term completed), by preconditioned linear CG (P_C).
 * rhs, mu: device complex fields; opts->tol_res_inf is the relative residual tolerance and
 * opts->max_iter the iteration cap.  report: host, nullable.  Synchronises. */
int gpe_adjoint_solve(gpe_plan_t* plan, const void* phi_star, const void* V, const void* rhs,
                      void* mu, const gpe_pcg_opts_t* opts, gpe_pcg_report_t* report, void* stream);

/* Parameter gradients from an adjoint state mu (the solution of gpe_adjoint_solve for a loss
 * with d l = Re<g, d phi>): d l / d theta = -Re<mu, (d_theta H) phi_star>.
 * grad_V: device, real, nullable: -h^d Re(conj(mu) phi_star) per grid point (d l / d V_k).
 * dl_dbeta: host, nullable: -Re<mu, |phi_star|^2 phi_star>.  dl_domega: host, nullable:
 * +Re<mu, L_z phi_star> (0 in 1-D).  The loss's explicit dependence on theta (for instance the
 * energy's own partial derivatives from gpe_energy_grad) is not included.  Synchronises. */
int gpe_adjoint_param_grads(gpe_plan_t* plan, const void* phi_star, const void* mu, void* grad_V,
                            double* dl_dbeta, double* dl_domega, void* stream);

/* Instrumented run for measurement (the iteration of Section 5.2, Algorithm 2): `iters` solver
 * iterations at the precision of opts->precision (0: FP64 fields, 1: FP32 fields; an FP32 plan
 * always uses FP32) from phi (device, left unchanged), every kernel launch of an iteration
 * recording a start/stop HIP event pair on `stream` around its own execution.  Host outputs,
 * `cap` entries each: avg_ms[k] = mean execution time of the k-th kernel of the iteration,
 * bytes[k] = its algorithmic HBM bytes per launch (fields read and written once), names = cap
 * rows of 32 chars.  Returns the number of kernels per iteration (>= 0) or an error.  The
 * convergence test is disabled during the run. */
int gpe_pcg_profile(gpe_plan_t* plan, const void* V, const void* phi, const gpe_pcg_opts_t* opts, int iters,
                    int cap, double* avg_ms, double* bytes, char* names, void* stream);

/* As gpe_pcg_profile for `count` instances of one grid solved together as in
 * gpe_pcg_solve_batched (same argument conventions: probs[i], V[i], phi[i] device fields of type
 * `dtype`, left unchanged); bytes[k] counts all instances.  Allocates and frees its own
 * workspace.  GPE_EINVAL if the instances do not share (dim, n). */
int gpe_pcg_profile_batched(int count, const gpe_problem_t* probs, int dtype, const void* const* V,
                            const void* const* phi, const gpe_pcg_opts_t* opts, int iters, int cap, double* avg_ms,
                            double* bytes, char* names, void* stream);

/* Message of the last error on this thread ("" if none). */
const char* gpe_last_error(void);

/* Library version string. */
const char* gpe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GPE_H */
