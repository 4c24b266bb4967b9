/*
 * tsm.h -- C ABI of the two-scale micro-batch library (libtsm.so, gfx950).
 *
 * Method (arXiv 2103.17040):
 *   - one micro problem per macro degree of freedom, posed on a shared
 *     reference cell Z = [-1,1]^2 and fed the nodal macro value u_i
 *     (Section 3.3, structure of the implementation: the micro system sits
 *     at the support point of the macro basis function);
 *   - micro integrals pulled back to Z with K = (D zeta)^{-1} and
 *     J = det D zeta (Section 3.1, equations grad_map and det_map): the
 *     stiffness weight is K K^T J per quadrature point and the boundary
 *     weight is |cof(F) nu| (change of variables, Section 3.1);
 *   - Q1 elements on the macro mesh B_H and on the reference mesh K_h
 *     (Section 3.1, spaces U_H and V_h), 2x2 Gauss per cell, 2-point Gauss
 *     per boundary edge;
 *   - macro/micro coupling through the Robin exchange kappa (p u - v) on the
 *     micro boundary and its mean as the macro source (Section 2.1, model
 *     system; the macro source carries the sign source_sign, -1 being the
 *     paper's sink);
 *   - every system solved by preconditioned conjugate gradients, the
 *     systems distributed over the processors (Section 3.5, parallelization
 *     in assembly).
 *
 * Time-dependent system stepped by implicit Euler with step dt:
 *   u_t - D Lap u = source_sign * mean_{dY_x} kappa (p u - v)  in [0,1]^2, u = 0 on the boundary
 *   v_t - d Lap_y v = 0 in Y_x,   d grad v . n = kappa (p u - v) on dY_x
 * Deformation family: zeta_x(y) = R_theta (y + a (sin(pi y1) y2, sin(pi y2) y1) / 4).
 * Each step is solved exactly: v_i = v0_i + u_i w_i with the time-invariant
 * response w_i = kappa p S_i^{-1} b_i, one micro solve per instance, one
 * macro solve.
 *
 * Conventions
 *   - Instance i is macro node i, lexicographic with x1 fastest:
 *     i = k2 (N_M+1) + k1, n_inst = (N_M+1)^2.
 *   - Micro vectors are ragged: instance i owns entries
 *     [offsets[i], offsets[i+1]) with offsets[i+1]-offsets[i] = (N_i+1)^2 and
 *     node j = j2 (N_i+1) + j1 at reference point (-1 + 2 j1/N_i, -1 + 2 j2/N_i).
 *   - "device pointer" arguments are HIP device memory owned by the caller;
 *     inputs are copied, outputs are written with stream-ordered copies on
 *     the context's stream.  "host pointer" arguments are ordinary memory.
 *   - All calls return a tsm_status; on failure tsm_last_error() gives a
 *     message (tsm_last_error(NULL): the calling thread's last tsm_create
 *     failure).  Calls on one context are not thread-safe.
 */
#ifndef TSM_H
#define TSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TSM_OK = 0,
    TSM_EINVAL = -1,   /* invalid argument or parameter */
    TSM_EGEOM = -2,    /* det D zeta <= 0 at some quadrature point */
    TSM_ENOCONV = -3,  /* some solve missed its tolerance (state still advanced) */
    TSM_EHIP = -4,     /* HIP runtime error */
    TSM_ENOMEM = -5,   /* device allocation failed or size limit exceeded */
    TSM_ESTATE = -6    /* call order violated (e.g. step before set_deformation) */
} tsm_status;

enum { TSM_FP64 = 0, TSM_FP32_REFINE = 1 };

/* flags */
#define TSM_FLAG_NO_GRAPH   (1ull << 0)  /* launch kernels directly instead of a captured hipGraph */
#define TSM_FLAG_STENCIL_STREAM (1ull << 1) /* force the streamed-stencil micro kernels */
#define TSM_FLAG_GENERIC    (1ull << 3)  /* solve every mesh size with the one-instance-per-workgroup
                                            kernels (no packed kernels for 16/32/64 cells) */
#define TSM_FLAG_GENERIC_16 (1ull << 6)  /* ... only the 16-cell meshes (likewise 32, 64): the */
#define TSM_FLAG_GENERIC_32 (1ull << 7)  /* best kernel differs per mesh size and precision    */
#define TSM_FLAG_GENERIC_64 (1ull << 8)
#define TSM_FLAG_PERSISTENT (1ull << 4)  /* all packed mesh sizes in ONE persistent launch (one
                                            workgroup per compute unit) with a work queue
                                            (largest meshes first), instead of one launch per
                                            mesh size with one workgroup per pack */
#define TSM_FLAG_MATRIX_FREE (1ull << 9) /* per-size launch plans (not TSM_FLAG_PERSISTENT): the
                                            packed refinement kernels evaluate the time-step
                                            operator matrix-free from the amplitudes at the start
                                            of every solve (Section 3.1: J and K K^T J at the
                                            quadrature points) instead of reading the operator
                                            assembled at setup.  Opt-in only: it is slower than
                                            the assembled operator, tsm_autotune never picks it
                                            by itself, and it has no extrapolated start.  Geometry
                                            from Jacobian tables always uses the assembled
                                            operator. */
#define TSM_FLAG_MACRO_PCG  (1ull << 10) /* solve the macro system (forward and adjoint) by PCG with
                                            the sine-basis solve of A_M's tensor part as
                                            preconditioner even where the sweep would do (it is
                                            used anyway where the sweep's contraction bound is
                                            0.5 or more, or where PCG needs fewer operations than
                                            the sweeps at that bound) */
#define TSM_FLAG_MULTIGRID  (1ull << 11) /* stationary contexts: the micro solves of every mesh
                                            with N = c 2^L cells per side (c <= 8, L >= 1) by CG
                                            preconditioned with one geometric multigrid V-cycle
                                            (Galerkin coarse operators of the nested meshes, two
                                            damped Jacobi sweeps before and after, dense coarsest
                                            solve).  Without it only such meshes above 64 cells
                                            per side take the V-cycle (the packed Jacobi kernels
                                            are faster at 64 and below); the other sizes keep
                                            Jacobi either way. */
#define TSM_FLAG_NO_MULTIGRID (1ull << 12) /* stationary contexts: Jacobi for every mesh */
#define TSM_FLAG_NO_EXTRAPOLATION (1ull << 13) /* time steps start every micro solve from
                                            the previous state.  By default the packed kernels
                                            with the assembled operator start it from the previous
                                            state plus the increment extrapolated quadratically
                                            from the last three steps, 3 e1 - 3 e2 + e3 (linearly,
                                            2 e1 - e2, after two; three FP32 values of history per
                                            micro DoF; an instance whose guessed residual is not
                                            smaller drops the guess; in FP32_REFINE the guess
                                            starts the first inner solve).  The FP64 residual
                                            takes the guess in exactly, so results meet rtol
                                            either way; they differ in rounding only.  The
                                            history restarts at tsm_set_state, tsm_set_flags and
                                            every change of the state other than a tsm_step.
                                            tsm_gradient's tape starts with an empty history and
                                            keeps it with every checkpoint (its recomputed
                                            segments repeat the tape bitwise); its adjoint micro
                                            solves extrapolate from their own history. */
#define TSM_FLAG_ASSEMBLED_START (1ull << 14) /* time steps form the start residual
                                            -K x0 + coef M w/dt of the packed solves on the
                                            assembled operator from the assembled planes of
                                            K = S - M/dt (one more FP64 operator read per solve).
                                            By default, for the analytic deformation family, it is
                                            formed as coef M w/dt + M x0/dt - S x0: M x0 from
                                            per-level tables (J = det(I + aG) is a sum of five
                                            products f(y1) g(y2), so with the tensor 2x2 Gauss rule
                                            M is a sum of five Kronecker products of 1D weighted
                                            masses; Sections 3.1 and 3.4), S x0 with the stencil
                                            the solve holds.  FP32_REFINE adds the low part of
                                            S x0 at its first FP64 residual update.  Results
                                            differ in rounding only.  Jacobian tables and the
                                            stationary system always read K. */
#define TSM_FLAG_TIMING     (1ull << 2)  /* tsm_step launches directly and times each phase with
                                            HIP events on the context's stream (see tsm_stats) */
#define TSM_FLAG_FIXED_POINT (1ull << 5) /* tsm_step couples macro and micro solves by the paper's
                                            alternating iteration (Section 3.3; the residual sum is
                                            the threshold of Section 3.5): macro solve with
                                            the micro data lagged, then every micro solve with the
                                            new macro values, until the residual sum (macro
                                            residual norm + mean micro residual norm) changes by
                                            less than fp_rtol times its first value.  Converges to
                                            the same step as the default exact (Schur) coupling;
                                            each iteration costs a full batch of micro solves.
                                            Launched directly (one host sync per iteration);
                                            tsm_gradient always uses the exact coupling. */

typedef struct {
    int32_t macro_cells;     /* N_M >= 2: macro Q1 cells per side on [0,1]^2 */
    double D;                /* macro diffusion, > 0 */
    double d;                /* micro diffusion, > 0 */
    double kappa;            /* Robin transfer rate, >= 0 */
    double p;                /* partition coefficient, > 0 */
    double dt;               /* time step, > 0 */
    int32_t source_sign;     /* -1 (paper's sink) or +1 */
    int32_t precision;       /* TSM_FP64 or TSM_FP32_REFINE */
    double rtol;             /* micro step solves: ||b - S x||_2 <= rtol ||b||_2 */
    double inner_rtol;       /* FP32 inner solves (refinement mode): the loosest
                                relative tolerance of one inner solve; each one
                                is solved to half of what the FP64 residual test
                                still needs, but no tighter than 2^-18 */
    double setup_rtol;       /* response solves w_i at setup */
    int32_t max_iter;        /* PCG iterations per solve (per inner solve) */
    int32_t max_refine;      /* FP64 refinement sweeps (refinement mode); a packed solve
                                still above rtol after them is solved again from its initial
                                guess by FP64 Jacobi PCG (tsm_stats.fp64_fallbacks) */
    int32_t checkpoint_every;/* adjoint checkpoint spacing in steps, >= 1 */
    uint64_t flags;          /* TSM_FLAG_* */
    double fp_rtol;          /* TSM_FLAG_FIXED_POINT: stop when the residual sum changes by
                                less than fp_rtol x its first value, > 0 */
    int32_t fp_max_iter;     /* TSM_FLAG_FIXED_POINT: iterations per step, >= 2 */
    double grad_rtol;        /* tsm_gradient: tolerance of every micro solve of the gradient
                                (its checkpointed forward, the segment recompute and the adjoint
                                solves), > 0; 0 = rtol.  The gradient of this family is small
                                against J (the cells keep their shape), so its relative error is
                                about 1e3 x the solver tolerance: 1e-11 gives ~1e-7. */
} tsm_params;

typedef struct {
    int64_t n_inst;
    int64_t n_micro_dofs;        /* sum_i (N_i+1)^2 */
    int64_t steps_taken;         /* since set_state */
    int32_t iters_min, iters_max;/* PCG iterations of the last step (inner total in refine mode) */
    double iters_mean;
    int32_t sweeps_max;          /* refinement sweeps of the last step */
    int32_t unconverged;         /* instances that missed rtol in the last step */
    int32_t macro_sweeps;        /* tensor-preconditioned macro sweeps per solve (0 under PCG) */
    double macro_contraction;    /* bound on the macro sweep contraction factor */
    double setup_ms;             /* last set_deformation */
    double step_ms;              /* last tsm_step call, between events on the stream */
    double micro_ms;             /* TSM_FLAG_TIMING: micro-solve phase, summed over the last tsm_step */
    double macro_ms;             /* TSM_FLAG_TIMING: macro solve + fluxes, summed likewise */
    int32_t timed_steps;         /* steps covered by micro_ms / macro_ms */
    int32_t micro_launches;      /* micro kernel launches per step (one per mesh-size class) */
    double grad_forward_ms;      /* last tsm_gradient: forward with checkpoints */
    double grad_backward_ms;     /* last tsm_gradient: segment recompute + adjoint + gradient */
    double sweeps_mean;          /* refinement sweeps of the last step, mean over instances
                                    (1 + the inner solves of an instance) */
    int32_t fp_iters_last;       /* TSM_FLAG_FIXED_POINT: coupling iterations of the last step */
    int32_t fp_iters_max;        /* ... and the most over the steps of the last tsm_step call */
    int32_t macro_pcg_iters;     /* macro PCG iterations per solve when PCG is used, else 0 */
    int32_t fp64_fallbacks;      /* refinement mode: packed solves that missed rtol after
                                    max_refine sweeps and were solved again in FP64 (Jacobi PCG
                                    from the step's initial guess), summed over the steps of the
                                    last tsm_step call; a solve that misses rtol there too counts
                                    in unconverged */
} tsm_stats;

typedef struct tsm_ctx tsm_ctx;

/* Fill *p with the defaults: kappa = p = 1, D = 1, d = 0.5, dt = 0.01,
 * source_sign = -1, FP64, rtol 1e-12, inner_rtol 1e-2, setup_rtol 1e-14,
 * max_iter 1000, max_refine 12, checkpoint_every 10, flags 0, fp_rtol 1e-10,
 * fp_max_iter 50, grad_rtol 0 (= rtol). */
void tsm_default_params(tsm_params* p);

/* Create a context on the current HIP device.  The parameters are those of
 * the model (Section 2.1, model problem: diffusions D and d, exchange rate
 * kappa, partition coefficient p, the sign of the macro exchange term) plus
 * the time step and the solver controls (conjugate gradients, Section 3.5).
 * p: host pointer, read during the call.  stream is a hipStream_t (NULL: the
 * context creates its own non-blocking stream).  *out receives the context,
 * which owns every device buffer it allocates (free with tsm_destroy).
 * EINVAL on a parameter out of range (message in tsm_last_error(NULL)),
 * EHIP if the device cannot be queried. */
tsm_status tsm_create(const tsm_params* p, void* stream, tsm_ctx** out);

/* Reference mesh of every instance (Section 3.1, approximation: the
 * partition K_h of the reference domain Z and its Q1 space V_h; Section
 * 3.3: one micro system per macro degree of freedom, so instance i belongs
 * to macro node i of the partition B_H): micro_cells[i] = N_i in 2..256
 * cells per side of K_h (host pointer, n_inst entries, read during the call;
 * n_inst == (N_M+1)^2, else EINVAL; a size outside 2..256: EINVAL).  Sizes
 * 16, 32 and 64 run the packed kernels; sizes above 64 run one workgroup
 * per instance in FP64 (either precision mode).
 * Allocates the ragged buffers (ENOMEM if that fails).  Invalidates any
 * deformation and state. */
tsm_status tsm_set_reference_mesh(tsm_ctx* c, const int32_t* micro_cells, int64_t n_inst);

/* Ragged layout: offsets_out[0..n_inst] (host pointer, n_inst+1 entries). */
tsm_status tsm_get_offsets(const tsm_ctx* c, int64_t* offsets_out);

/* The domain map zeta_x of every instance (Section 2.1: the micro domain
 * Y_x is the image of Z under zeta(x, .); Section 3.1, equations grad_map and
 * det_map: K = (D zeta)^{-1}, J = det D zeta, and the change of variables with
 * |cof(F) nu| on the boundary; Section 3.4, domain mappings: J and K K^T J
 * per quadrature point): the family zeta_x(y) = R_theta (y + a (sin(pi y1)
 * y2, sin(pi y2) y1) / 4) with amplitudes a_i and rotation angles theta_i
 * (device pointers, n_inst doubles each, caller-owned, read during the call;
 * theta may be NULL = 0).  EINVAL if n_inst differs from the mesh's or a
 * value is not finite, ESTATE before tsm_set_reference_mesh, EGEOM if
 * det D zeta <= 0 at some quadrature point.  Then runs setup: assembles each
 * S_i = M_i/dt + d A_i + kappa B_i, solves the responses w_i and builds the
 * macro solver.  The rotation leaves K K^T J and |cof(F) nu| unchanged, so it
 * does not enter the arithmetic. */
tsm_status tsm_set_deformation(tsm_ctx* c, const double* a, const double* theta, int64_t n_inst);

/* General maps (Section 3.1: the map zeta enters the discrete problem only
 * through its Jacobian at the quadrature points; Section 3.4, domain
 * mappings: the paper caches J and K K^T J per point).  Fcell and Fbnd (device pointers, row-major 2x2
 * Jacobians F = D zeta, entries F11 F12 F21 F22) give D zeta of every
 * instance at the reference points y = -1 + (cell + g) h, h = 2/N,
 * g in {1/2 - 1/(2 sqrt 3), 1/2 + 1/(2 sqrt 3)}:
 *   Fcell: per instance (in instance order) its N^2 cells in order
 *          c2*N + c1, each with 4 points in order g2*2 + g1 (g1 along y1):
 *          16 N_i^2 values, n_cell = sum over instances;
 *   Fbnd:  per instance its 4 sides (y2 = -1, y2 = +1, y1 = -1, y1 = +1),
 *          each with N edges in increasing coordinate and 2 points:
 *          32 N_i values, n_bnd = sum over instances.
 * J = det F, K K^T J = adj(F) adj(F)^T / J and |cof(F) nu| = |F tau| are
 * formed per point.  EINVAL on wrong sizes or NULL, EGEOM if det F <= 0 or an
 * entry is not finite at some point; otherwise the same setup as
 * tsm_set_deformation.  The tables are read during the call only.
 * tsm_gradient (derivatives with respect to amplitudes) is not available
 * for a geometry given this way (ESTATE). */
tsm_status tsm_set_jacobians(tsm_ctx* c, const double* Fcell, int64_t n_cell, const double* Fbnd, int64_t n_bnd);

/* State of the coupled system (Section 2.1, the fields u and v; Section 3.1,
 * their expansions u = sum_i u_i xi_i and v = sum_ij v_ij xi_i (eta_j pulled
 * back to Z)): u the nodal macro values (device pointer, n_u == n_inst
 * entries; macro-boundary entries are forced to 0), v the ragged micro
 * coefficients (device pointer, n_v == total micro DoFs, or NULL = 0 with n_v
 * ignored).  Copied during the call.  EINVAL on a NULL u, a wrong count or a
 * non-finite u; ESTATE before the geometry is set or on a stationary context.
 * Resets steps_taken. */
tsm_status tsm_set_state(tsm_ctx* c, const double* u, int64_t n_u, const double* v, int64_t n_v);

/* Advance n_steps >= 0 implicit-Euler steps of the coupled discrete system
 * (the discrete weak form on the reference cell, Section 3.1, in its
 * time-dependent two-field form; one micro solve per macro node, Section
 * 3.3, by preconditioned CG, Section 3.5) on the context's stream, then
 * synchronise it.  EINVAL if n_steps < 0, ESTATE before tsm_set_state,
 * ENOCONV if any solve missed its tolerance (the state is still advanced with
 * the last iterate; see tsm_get_stats), EHIP on a runtime error. */
tsm_status tsm_step(tsm_ctx* c, int32_t n_steps);

/* Outputs (caller-owned device pointers with their entry counts, written on
 * the context's stream, then synchronised; ESTATE without a state, EINVAL on
 * NULL or a wrong count):
 *   tsm_get_macro   the macro field u (Section 2.1; its nodal values,
 *                   Section 3.1), n == n_inst;
 *   tsm_get_fluxes  the mean micro Robin flux of every instance in the last
 *                   step, F_i = mean over dY_i of kappa (p u_i - v) (the
 *                   exchange integral of the macro equation, Section 2.1),
 *                   n == n_inst;
 *   tsm_get_micro   the micro field v (ragged, offsets via tsm_get_offsets),
 *                   n == total micro DoFs. */
tsm_status tsm_get_macro(const tsm_ctx* c, double* u_out, int64_t n);
tsm_status tsm_get_fluxes(const tsm_ctx* c, double* F_out, int64_t n);
tsm_status tsm_get_micro(const tsm_ctx* c, double* v_out, int64_t n);

/* Setup quantities (caller-owned device pointers, NULL to skip): response
 * functional beta_i = kappa p - (kappa/|dY_i|) b_i^T w_i and boundary length
 * |dY_i| = 1^T b_i (n_inst entries each, n_inst must match when either is
 * given), and the ragged response w (n_w == total micro DoFs when given).
 * EINVAL on a wrong count, ESTATE before the geometry is set. */
tsm_status tsm_get_setup(const tsm_ctx* c, double* beta_out, double* len_out, int64_t n_inst, double* w_out,
                         int64_t n_w);

/* y = S x for every instance with the assembled FP64 operator (the micro
 * matrix of the discrete weak form, Section 3.1); x and y are caller-owned
 * ragged device vectors of n == total micro DoFs entries.  EINVAL on NULL or
 * a wrong count, ESTATE before the geometry is set. */
tsm_status tsm_apply_operator(tsm_ctx* c, const double* x, double* y, int64_t n);

/* Gradient of J = u(T)^T M_H u(T) (the integral of u_h(T)^2) after n_steps
 * steps from the current state with respect to the amplitudes a_i of the
 * domain map (the paper has no adjoint; this is the exact derivative of the
 * discrete forward map of tsm_step): forward with checkpoints every
 * checkpoint_every steps, then the discrete adjoint backwards, segment by
 * segment.  J_out is a host pointer, dJda_out a caller-owned device pointer
 * of n == n_inst entries.  The current state is left unchanged.  EINVAL on
 * n_steps < 1, NULL or a wrong count; ESTATE before tsm_set_state or for a
 * geometry given by Jacobian tables; ENOMEM if the checkpoint buffers cannot
 * be allocated; ENOCONV if a solve missed its tolerance. */
tsm_status tsm_gradient(tsm_ctx* c, int32_t n_steps, double* J_out, double* dJda_out, int64_t n);

/* Replace the launch flags (TSM_FLAG_*) of a context; rebuilds the step
 * graph if set_deformation has run.  Results are bitwise identical under
 * every flag except TSM_FLAG_GENERIC, whose different summation order
 * changes them within the solver tolerance. */
tsm_status tsm_set_flags(tsm_ctx* c, uint64_t flags);

/* Autotuner: time the launch plans {one launch per mesh size, one persistent
 * launch for all sizes, the one-instance-per-workgroup kernels} for
 * `steps` steps each (after one warm-up step) from the current state, then,
 * from the faster packed plan, move one packed mesh size at a time to the
 * one-instance-per-workgroup kernel (TSM_FLAG_GENERIC_16/32/64) while that
 * is faster, then, if the caller asked for the matrix-free operator
 * (TSM_FLAG_MATRIX_FREE; refinement mode, packed plan, amplitude geometry),
 * time the chosen plan with the assembled operator; restore the state after
 * every trial and keep the fastest plan.  The matrix-free form is never
 * tried unless asked for.
 * ms_out[5] (host, may be NULL): ms per step of the per-size, persistent and
 * generic plans in the caller's operator form (-1 where a plan does not
 * apply), of the chosen plan, and of the chosen plan with the assembled
 * operator (-1 if not tried); *flags_out (host, may be NULL): the chosen
 * TSM_FLAG_* plan bits.  Needs set_state first. */
tsm_status tsm_autotune(tsm_ctx* c, int32_t steps, double* ms_out, uint64_t* flags_out);

/* Statistics of the last calls (host pointer *s, filled; EINVAL on NULL).
 * Bookkeeping only: iterations, sweeps and times, no passage of the method. */
tsm_status tsm_get_stats(const tsm_ctx* c, tsm_stats* s);
/* The context's last error message (owned by the context, valid until the
 * next call on it); NULL: the calling thread's last failure of a call that
 * has no context (create, mark, prolong). */
const char* tsm_last_error(const tsm_ctx* c);
/* Release the context and every device buffer it owns.  NULL-safe. */
void tsm_destroy(tsm_ctx* c);

/* ---------------------------------------------------------------------------
 * Refinement of the micro meshes from an error indicator -- an extension the
 * paper's conclusions propose (an indicator defined over all micro grids,
 * used to refine so as to reduce the error globally); the indicator, the
 * marking and the transfer below are this library's reading.
 * ------------------------------------------------------------------------- */

/* Indicator of the current micro state, gradient-jump form: eta2_out[i]
 * (device pointer, n_inst doubles) = sum over the interior edges e of
 * instance i's reference mesh of (h/12) int_e [[ d (C grad_z v_i) . nu_e ]]^2,
 * the jump of the pulled-back flux (C = K K^T J, Section 3.1) integrated with
 * the 2-point rule.  Needs set_state; ESTATE for a geometry given by Jacobian
 * tables (C is needed at points the tables do not hold) and for a
 * stationary context; EINVAL unless n == n_inst. */
tsm_status tsm_error_indicator(tsm_ctx* c, double* eta2_out, int64_t n);

/* Bulk marking over the global functional sum_i eta2[i]: the fewest
 * instances with 2 level[i] <= max_level, largest eta2 first (ties: lower
 * index first), whose indicators reach theta times the functional get
 * level_new[i] = 2 level[i]; the others keep level[i].  Host pointers, n_inst
 * entries each; *n_marked (may be NULL) receives the count.  EINVAL on
 * theta outside [0, 1], a negative or non-finite eta2 or a level outside
 * 2..256 (message in tsm_last_error(NULL)); max_level 256 lets every mesh
 * that tsm_set_reference_mesh accepts after refinement be marked. */
tsm_status tsm_mark_refine(int64_t n_inst, const double* eta2, const int32_t* level, double theta, int32_t max_level,
                           int32_t* level_new, int64_t* n_marked);

/* Nested Q1 interpolation of a ragged micro field from the meshes level_old
 * to level_new (host pointers, n_inst each; level_new[i] is level_old[i] or
 * 2 level_old[i], at most 256): v_old (ragged by level_old, n_old entries)
 * to v_new (ragged by level_new, n_new entries), device pointers.  A fine
 * node takes the coarse value at a corner, the mean of 2 on an edge
 * midpoint, of 4 at a cell centre.  Runs on `stream` (a hipStream_t, NULL:
 * the null stream) and synchronises it.  Stages the level and offset arrays
 * in device memory it allocates for the call.  EINVAL on bad levels or
 * counts (message in tsm_last_error(NULL)). */
tsm_status tsm_prolong(int64_t n_inst, const int32_t* level_old, const int32_t* level_new, const double* v_old,
                       int64_t n_old, double* v_new, int64_t n_new, void* stream);

/* tsm_prolong for callers that cannot allocate device memory (code that
 * runs under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, checks and results, with the level and
 * offset arrays staged in a static device array of the library (3 MiB per
 * GPU, held until the process ends) instead of buffers allocated per call.
 * At most 131072 instances (TSM_ENOMEM beyond, with a message in
 * tsm_last_error(NULL)).  Calls allocate nothing; every call on one GPU uses
 * that GPU's array, so calls that overlap on one GPU (from several host
 * threads) race -- serialise them. */
tsm_status tsm_prolong_noalloc(int64_t n_inst, const int32_t* level_old, const int32_t* level_new,
                               const double* v_old, int64_t n_old, double* v_new, int64_t n_new, void* stream);

/* ---------------------------------------------------------------------------
 * The paper's stationary three-field system (Section 2.1 model; the Case A/B
 * experiments of Section 4 solve it with the Table 3 parameters, the
 * convergence benchmark of Section 4.2 its manufactured form):
 *   -Lap u = f^u - int_{G^I} (k1 u - k2 v + g^v_1) dsigma_y   in [-1,1]^2,
 *            u = u_D on the Dirichlet sides, grad u . n = g^u elsewhere
 *   -Dv Lap_y v = f^v  in Y_x,   Dv grad_y v . n = k1 u - k2 v + g^v_1  on G^I
 *                                                 k3 w - k4 v + g^v_2  on G^O
 *                                                 g^v_3                on G^N
 *   -Dw Lap w = f^w - int_{G^O} (k3 w - k4 v + g^v_2) dsigma_y,
 *            Dw grad w . n = g^w on the boundary
 * The model has every g zero; by default the sources are the constants of
 * tsm_stationary_params and u_D = u_dirichlet (tsm_stationary_set_data
 * replaces them by values at the quadrature points).  G^I, G^O, G^N are
 * images of whole sides of Z (parts[]).  Same discretisation as the time-dependent system (Q1, the map
 * through its Jacobian at the quadrature points, one micro system per macro
 * node fed u_k and w_k), exchange integrals of the macro rows taken at the
 * nodes with weights L = diag(M_H 1).  Solved exactly by elimination: per
 * instance three micro PCG solves with the FP64 operator
 *   S = Dv A + k2 B^I + k4 B^O:  z^I = S^{-1} b_I,  z^O = S^{-1} b_O,
 *   z^0 = S^{-1} F^v    (b_I = B^I 1, b_O = B^O 1, F^v the load of f^v and g^v),
 * one macro PCG for (u, w) -- symmetric positive definite once the u rows
 * are scaled by k1/k2 and the w rows by k3/k4 -- and v = z^0 + k1 u z^I +
 * k3 w z^O.
 * Use: tsm_stationary_create, tsm_set_reference_mesh, tsm_set_deformation
 * or tsm_set_jacobians (assemble S, b_I, b_O, the point weights of the loads
 * and check the geometry), optionally tsm_stationary_set_data,
 * tsm_stationary_solve.  tsm_apply_operator applies this S; tsm_set_flags
 * takes the launch-plan flags; the time-stepping calls return ESTATE.
 * ------------------------------------------------------------------------- */
enum { TSM_PART_N = 0, TSM_PART_I = 1, TSM_PART_O = 2 };

typedef struct {
    int32_t macro_cells;      /* N_M in 2..256: macro Q1 cells per side on [-1,1]^2 */
    double Dv, Dw;            /* micro and macro-w diffusion, > 0 */
    double kappa1, kappa2, kappa3, kappa4;   /* exchange rates, > 0 */
    double fu, fv, fw;        /* constant bulk sources (finite; see tsm_stationary_set_data) */
    double u_dirichlet;       /* u on the Dirichlet sides (finite) */
    int32_t parts[4];         /* part of each side of Z -- bottom (y2 = -1), top (y2 = +1),
                                 left (y1 = -1), right (y1 = +1): TSM_PART_*; at least one
                                 side in G^I and one in G^O */
    int32_t dirichlet[4];     /* sides of [-1,1]^2 in the same order: nonzero = u prescribed;
                                 at least one */
    double rtol;              /* micro PCG (FP64): ||b - S x||_2 <= rtol ||b||_2 */
    double macro_rtol;        /* macro PCG: same test on the eliminated (u, w) system */
    int32_t max_iter;         /* micro PCG iterations per solve, >= 1 */
    int32_t macro_max_iter;   /* macro PCG iterations, >= 1 */
    uint64_t flags;           /* launch-plan flags (TSM_FLAG_GENERIC*, TSM_FLAG_PERSISTENT,
                                 TSM_FLAG_STENCIL_STREAM) */
} tsm_stationary_params;

typedef struct {
    int32_t micro_iters_max[3];  /* PCG iterations, most over instances, of the z^I, z^O, z^0
                                    solves of the last tsm_stationary_solve (0: not solved) */
    double micro_iters_mean[3];
    int32_t unconverged;         /* micro solves that missed rtol */
    int32_t macro_iters;         /* macro PCG iterations */
    double macro_rel_residual;   /* its final ||r||_2 / ||b||_2 */
    double solve_ms;             /* the whole solve, between events on the context's stream */
    double micro_ms;             /* the three batched micro solves */
} tsm_stationary_stats;

/* Defaults: the Table 3 parameters (Dv 1, Dw 0.1, k1..k4 = 0.5, 1, 0.25, 1,
 * f^u = f^v = f^w = 0, u_dirichlet 1), macro_cells 8, parts
 * (N, N, I, O), Dirichlet side left (x1 = -1), rtol 1e-12, macro_rtol 1e-14,
 * max_iter 20000, macro_max_iter 200000, flags 0. */
void tsm_stationary_default_params(tsm_stationary_params* p);

/* Create a stationary context on the current HIP device (stream as for
 * tsm_create).  EINVAL on bad parameters. */
tsm_status tsm_stationary_create(const tsm_stationary_params* p, void* stream, tsm_ctx** out);

/* Solve the system.  u_out, w_out: device pointers, n_inst doubles each;
 * v_out: device pointer, ragged, n_v == total micro DoFs (or NULL to skip).
 * EINVAL on a wrong count; ESTATE before the geometry is set or on a context
 * made by tsm_create; ENOCONV if a micro solve missed rtol or the macro
 * solve missed macro_rtol (outputs are still written, from the last
 * iterates). */
tsm_status tsm_stationary_solve(tsm_ctx* c, double* u_out, double* w_out, int64_t n_inst, double* v_out, int64_t n_v);

/* Data at quadrature points instead of the constants (Section 4.1, the
 * manufactured form; NULL keeps the constant of the parameters, or zero for
 * the g data).  Device pointers, copied; values must be finite.  Layouts
 * (the points of tsm_set_jacobians, one value per point):
 *   fv_cell: f^v, per instance its N_i^2 cells (c2*N+c1) x 4 points (g2*2+g1): 4 sum N_i^2 values;
 *   gv_bnd:  g^v of the part of each side, per instance its sides (bottom,
 *            top, left, right) x N_i edges x 2 points: 8 sum N_i values;
 *   fu_cell, fw_cell: f^u, f^w at the macro cells' points, same order on the
 *            N_M x N_M macro mesh of [-1,1]^2: 4 N_M^2 values each;
 *   gu_bnd, gw_bnd: grad u . n and Dw grad w . n at the macro boundary
 *            points, same order: 8 N_M values each (gu ignored on Dirichlet sides);
 *   uD: u at the (N_M+1)^2 macro nodes (read on the Dirichlet sides only).
 * Each array comes with its value count, which must equal the count above
 * (EINVAL otherwise; a NULL array's count is ignored).
 * A source at the micro points is f^v(x_k, zeta(x_k, y)) at the reference
 * point y of instance k.  Needs set_reference_mesh; a new mesh drops the data. */
tsm_status tsm_stationary_set_data(tsm_ctx* c, const double* fv_cell, int64_t n_fv, const double* gv_bnd,
                                   int64_t n_gv, const double* fu_cell, int64_t n_fu, const double* fw_cell,
                                   int64_t n_fw, const double* gu_bnd, int64_t n_gu, const double* gw_bnd,
                                   int64_t n_gw, const double* uD, int64_t n_uD);

tsm_status tsm_stationary_get_stats(const tsm_ctx* c, tsm_stationary_stats* s);

#ifdef __cplusplus
}
#endif
#endif /* TSM_H */
