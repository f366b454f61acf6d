/*
 * tdse.h -- C ABI of the MI355X (gfx950) TDSE propagation library.
 *
 * The library time-propagates dc/dt = -i [diag(E) + F(t) D] c over the
 * field-free |n,l> basis of O Broin & Nikolopoulos, "An OpenCL implementation
 * for the solution of TDSE on GPU and CPU architectures" (arXiv:1201.6062):
 *   - Sec. 3, Eqs. tdse_ode / tdse_ode_c: the projected TDSE i dC/dt = H(t) C;
 *   - Sec. 3, dipole selection rules and Fig. Matrix: H is block tridiagonal
 *     in l, diagonal blocks are the energies E_l, off-diagonal blocks are
 *     dense n x n dipole blocks coupling l and l+1;
 *   - Sec. 4, Eq. ode and the block product that follows it: the derivative
 *     is -i (E_l C_l + F (D_l C_{l+1} + D_{l-1}^T C_{l-1})) per block l;
 *   - Sec. 5: only the superdiagonal blocks D_l = D_{l,l+1} are stored, the
 *     subdiagonal block is its transpose (H is real symmetric);
 *   - Appendix B: truncated Taylor series (Eq. taylor) and explicit
 *     Runge-Kutta (Eqs. RKFinal, RKDeriv; classic RK4 tableau).
 *
 * Layout conventions (all arguments):
 *   lmax        highest partial wave; blocks l = 0..lmax, lmax >= 0.
 *   n           states per partial wave, n >= 1. nstates = (lmax+1)*n.
 *   energies    [(lmax+1)*n] doubles, block l at [l*n, (l+1)*n).
 *   dipole      [lmax][n][n] doubles, row-major; D_l[a][b] couples state a
 *               of block l (row) to state b of block l+1 (column).
 *   state c     [batch][2*nstates] doubles: complex coefficients interleaved
 *               (re, im), state j = l*n + a.
 *   field       [batch][nsteps][S] doubles, S = 3 for RK4 (the field at
 *               t_k, t_k + dt/2, t_k + dt; stages 2 and 3 share the midpoint
 *               sample), S = 1 for Taylor (H frozen over the step at the
 *               given sample, appendix B).
 *   stream      a hipStream_t passed as void*; NULL means the null stream.
 *
 * Memory: arguments named "device" must point to device memory (hipMalloc,
 * torch CUDA/HIP tensors); arguments named "host or device" may be either.
 * All device arguments must be 8-byte aligned.
 *
 * Errors: every argument is checked on the host before anything is
 * enqueued. On error nothing is enqueued, outputs are untouched, the status
 * is returned and tdse_last_error() describes the problem. HIP failures map
 * to TDSE_E_HIP.
 *
 * Asynchrony and ownership: tdse_propagate, tdse_adjoint, tdse_hmul and
 * tdse_group_propagate only enqueue work on the given stream and return;
 * caller buffers must stay valid until the stream reaches that point. The
 * library never frees caller memory. A plan or group owns its device copies
 * of the Hamiltonian, its scratch and its captured graphs. One plan may be
 * used by one stream at a time; distinct plans are independent.
 */
#ifndef TDSE_H
#define TDSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDSE_ABI_VERSION 1

typedef struct tdse_plan_s *tdse_plan;
typedef struct tdse_group_s *tdse_group;

typedef enum {
    TDSE_OK = 0,
    TDSE_E_INVAL = 1,        /* invalid argument; nothing enqueued */
    TDSE_E_NOMEM = 2,        /* device allocation failed */
    TDSE_E_HIP = 3,          /* a HIP runtime call failed */
    TDSE_E_UNSUPPORTED = 4,  /* valid request the library does not support */
    TDSE_E_UNSTABLE = 5      /* step size outside the method's stability bound */
} tdse_status;

typedef enum {
    TDSE_RK4 = 0,            /* classic 4th-order Runge-Kutta, 4 products per step */
    TDSE_TAYLOR = 1,         /* truncated Taylor series of order p, p products per step */
    TDSE_LANCZOS = 2,        /* short-iterative Lanczos, Krylov dimension m (taylor_order), m products per step */
    TDSE_RKF45 = 3           /* Runge-Kutta-Fehlberg 4(5), 6 products per step, S = 6 stage samples */
} tdse_method;

typedef enum {
    TDSE_LENGTH = 0,         /* coupling F(t) D, D real symmetric (the dipole blocks) */
    TDSE_VELOCITY = 1        /* coupling A(t) P, P = -i Q Hermitian (momentum blocks Q) */
} tdse_gauge;

/* Version of this ABI (TDSE_ABI_VERSION of the built library). */
int tdse_abi_version(void);

/* Text of the last error on the calling thread; valid until the next call on
 * this thread. Never NULL (empty string when the last call succeeded). */
const char *tdse_last_error(void);

/*
 * Create a plan for one Hamiltonian (Sec. 5: energies and superdiagonal
 * dipole blocks), and for propagating `batch` independent states (pulses)
 * at once. energies and dipole: host or device memory, copied into plan-owned,
 * re-laid-out device buffers; the call synchronises `stream`, so the caller
 * may free its inputs on return. batch >= 1; batch == 1 selects the
 * single-vector streaming kernels, batch > 1 the FP64 matrix-core kernels.
 * Errors: TDSE_E_INVAL (null out/energies, dipole null with lmax > 0,
 * lmax < 0, n < 1, batch < 1, sizes overflowing 2^40 states), TDSE_E_NOMEM,
 * TDSE_E_HIP.
 */
tdse_status tdse_create(tdse_plan *out, const double *energies, const double *dipole,
                        int32_t lmax, int32_t n, int32_t batch, void *stream);

/*
 * As tdse_create, with the gauge of the coupling (Sec. 5: the paper's runs
 * use the velocity gauge, -p.A(t)/c). TDSE_LENGTH: coupling holds the dipole
 * blocks D_l and the field samples are E(t); identical to tdse_create.
 * TDSE_VELOCITY: coupling holds the real blocks Q_l of the momentum coupling
 * P = -i Q, i.e. P_{l,l+1} = -i Q_l and P_{l+1,l} = +i Q_l^T (P Hermitian,
 * imaginary), and the field samples are the vector potential A(t); the
 * derivative is -i (E o u + A (P u)). Everything else (propagation, adjoint,
 * groups) is the same for both gauges. Errors: as tdse_create, and
 * TDSE_E_INVAL for an unknown gauge.
 */
tdse_status tdse_create_gauge(tdse_plan *out, const double *energies, const double *coupling,
                              tdse_gauge gauge, int32_t lmax, int32_t n, int32_t batch, void *stream);

/* Release a plan and everything it owns. Synchronises the device. NULL is a no-op. */
tdse_status tdse_destroy(tdse_plan plan);

/* Query the plan's shape. Any output pointer may be NULL. */
tdse_status tdse_plan_shape(tdse_plan plan, int32_t *lmax, int32_t *n, int32_t *batch);

/*
 * y = H(F) u = E o u + F (D u) for every column b of the batch with its own
 * field value F = fields[b] (Sec. 4, the block product after Eq. ode).
 * fields [batch] (device), u and y [batch][2*nstates] (device, must not
 * alias). One product per column; the building block of every step.
 */
tdse_status tdse_hmul(tdse_plan plan, const double *fields, const double *u, double *y,
                      void *stream);

/*
 * Propagate c0 over nsteps steps of size dt with RK4 (taylor_order ignored),
 * the Taylor series of order taylor_order (1 <= order <= 32), or the
 * short-iterative Lanczos propagator with Krylov dimension taylor_order
 * (1 <= m <= 64; the Krylov method named in Sec. 5.2: per step with H frozen
 * at the sample, c' = |c| V exp(-i dt T) e_1 over the Lanczos basis V of H
 * from c and its tridiagonal T; no reorthogonalisation; a vanishing beta_j
 * ends the basis early), writing c(T) to cT. field: [batch][nsteps][S]
 * device (S = 1 for Taylor and Lanczos); c0, cT: [batch][2*nstates] device;
 * cT may alias c0. nsteps == 0 copies c0 to cT.
 * ckpt: NULL, or device [batch][nsteps/ckpt_every + 1][2*nstates] receiving
 * c(k*ckpt_every*dt) for k = 0..nsteps/ckpt_every (ckpt_every >= 1).
 * The result is the discrete RK4 / Taylor map applied to the given samples.
 * Errors: TDSE_E_INVAL (null/misaligned/host pointers, dt <= 0 or not finite,
 * nsteps < 0, order out of range, ckpt_every < 1 with ckpt != NULL).
 * The Lanczos workspace ((m+2) state vectors per pulse and the recurrence
 * coefficients) is allocated on first use and kept by the plan
 * (TDSE_E_NOMEM if it cannot be).
 */
tdse_status tdse_propagate(tdse_plan plan, tdse_method method, int32_t taylor_order, double dt,
                           int64_t nsteps, const double *field, const double *c0, double *cT,
                           double *ckpt, int32_t ckpt_every, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the RK4 /
 * Taylor-p propagation of tdse_propagate on a batch-1 plan, with the same
 * arguments and the same result (the same kernels in the same order), that
 * allocates nothing. Its per-call scratch -- state vectors and product
 * partials of both launch parities and the call descriptor -- lives in one
 * fixed 16 MiB device array of the library (one per device, held until the
 * process ends) instead of the plan's own buffers, and it enqueues every
 * launch directly instead of replaying a captured graph.
 * Limits: batch-1 plans only, RK4 and Taylor only (TDSE_E_UNSUPPORTED
 * otherwise); problems whose scratch exceeds 16 MiB (96 (lmax+1) n bytes
 * plus 8 lmax ceil(n/128)^2 KiB, e.g. Lmax = 15, N = 1000) are rejected with
 * TDSE_E_UNSUPPORTED; the plan's device must be current (TDSE_E_INVAL).
 * Concurrency: every call on one device shares the array, so calls that
 * overlap on one device (on other streams or threads) race on it; calls
 * ordered on one stream are safe (each call re-initialises what it reads).
 * Other errors as tdse_propagate.
 */
tdse_status tdse_propagate_noalloc(tdse_plan plan, tdse_method method, int32_t taylor_order, double dt,
                                   int64_t nsteps, const double *field, const double *c0, double *cT,
                                   double *ckpt, int32_t ckpt_every, void *stream);

/*
 * Runge-Kutta-Fehlberg 4(5) propagation (the embedded pair of appendix B's
 * explicit Runge-Kutta family): six stages per step at t_k + c_i dt,
 * c = (0, 1/4, 3/8, 12/13, 1, 1/2), field [batch][nsteps][6] device samples
 * at those times; c advances with the fifth-order weights (the pair's
 * fifth-order solution, which the paper propagates, Sec. 5.1), and if err !=
 * NULL, err[b][k] (device [batch][nsteps]) receives |dt sum_i (b5_i - b4_i)
 * k_i|_2, the pair's embedded estimate of step k's local error (that of its
 * fourth-order member; for step-size control by the caller). tdse_propagate with TDSE_RKF45 is this call with err = NULL.
 * Batch-1 plans run it on a batched twin of themselves. Errors: as
 * tdse_propagate; TDSE_E_NOMEM if the stage workspace (5 state vectors per
 * pulse, kept by the plan) cannot be allocated.
 */
tdse_status tdse_propagate_rkf45(tdse_plan plan, double dt, int64_t nsteps, const double *field, const double *c0,
                                 double *cT, double *err, double *ckpt, int32_t ckpt_every, void *stream);

/*
 * Step-size control on the Runge-Kutta-Fehlberg error estimate (the embedded
 * pair of appendix B's explicit family): from c0 at t = 0 to t_final, one
 * step at a time. For each attempted step of size h from time t the library
 * calls field_fn(t, h, samples, ctx), which fills samples (host,
 * [batch][6]) with the field (or vector potential) at the six stage times
 * t + c_i h, c = (0, 1/4, 3/8, 12/13, 1, 1/2); runs one tdse_propagate_rkf45
 * step; and accepts it when every pulse's estimate is <= tol (or h <= dt_min).
 * The next size is max(dt_min, h min(2, max(0.2, 0.9 (tol/err)^(1/5))))
 * (2 h when err == 0); the last step is shortened to end at t_final.
 * c0, cT: [batch][2*nstates] device (may alias). steps: NULL or host
 * [max_steps], receiving the accepted step sizes; *nsteps_taken (host) their
 * count. max_steps bounds the attempted steps: TDSE_E_INVAL if t_final is not
 * reached within them (cT then holds the state at the last accepted step).
 * Synchronous: it reads every step's estimate back to the host. Batch-1 plans
 * run on their batched twin. The workspace (six samples and two states per
 * pulse) is allocated on first use and kept by the plan. Errors: TDSE_E_INVAL
 * (null plan, field_fn or nsteps_taken, non-finite or non-positive t_final,
 * dt0, dt_min or tol, device arguments as tdse_propagate), TDSE_E_NOMEM.
 */
typedef void (*tdse_field_fn)(double t, double h, double *samples, void *ctx);
tdse_status tdse_propagate_adaptive(tdse_plan plan, double t_final, double dt0, double tol, double dt_min,
                                    int64_t max_steps, tdse_field_fn field_fn, void *ctx, const double *c0,
                                    double *cT, double *steps, int64_t *nsteps_taken, void *stream);

/*
 * Stability test of a step size (appendix B's step maps on the imaginary
 * axis): one step multiplies each eigencomponent of H(F) by R(-i dt lambda),
 * R the method's stability polynomial (the Taylor polynomial of degree 4 for
 * RK4 and of degree p for Taylor-p; 1 + sum_k b^T A^(k-1) 1 z^k for the
 * Fehlberg pair's fifth-order solution). With theta = dt (max|E| + |fmax|
 * ||D||), ||D|| bounded by the largest absolute row sum of the coupling
 * (computed at plan creation), returns TDSE_OK when |R(i s)|^2 <= 1 + 1e-14
 * for every |s| <= theta, else TDSE_E_UNSTABLE (tdse_last_error gives the
 * numbers). RK4: the bound is 2 sqrt(2); Taylor orders 1, 2 (mod 4) and the
 * Fehlberg pair amplify every oscillation, so their bounds are set by the
 * 1e-14 allowance; Lanczos is unitary (always TDSE_OK). theta and bound
 * (host, either may be NULL) receive the two numbers. Host only; nothing is
 * enqueued. This is the optional pre-check of a propagation: the propagation
 * entry points do not apply it themselves (a step outside the interval is
 * still the well-defined discrete map, which short runs and tests may want).
 * Errors: TDSE_E_INVAL (null plan, unknown method, order out of range, dt
 * not finite and > 0, fmax not finite).
 */
tdse_status tdse_check_stability(tdse_plan plan, tdse_method method, int32_t taylor_order, double dt, double fmax,
                                 double *theta, double *bound);

/*
 * Discrete adjoint of tdse_propagate, for RK4 and for the Taylor series of
 * order taylor_order (appendix B steps run backwards: the co-states of the
 * RK4 stage derivatives, or of the Taylor terms Tbar_{m-1} = lambda +
 * (i dt/m) H Tbar_m). For a real loss L(c(T)) with lambdaT = dL/dRe c(T) +
 * i dL/dIm c(T) ([batch][2*nstates] device), writes grad_field[batch][nsteps][S]
 * = dL/dfield (S = 3 for RK4, 1 for Taylor; device, overwritten) and, if
 * lambda0 != NULL, lambda0 = dL/dRe c0 + i dL/dIm c0 ([batch][2*nstates]
 * device).
 * ckpt: the checkpoints written by tdse_propagate with the same field, c0,
 * dt and ckpt_every (device), or NULL: then the library recomputes them into
 * plan-owned memory first. Forward states between checkpoints are recomputed
 * segment by segment, so memory stays at one segment of stage inputs.
 * Memory: the workspace (one segment of stage inputs, ckpt_every x products
 * per step state vectors, and the internal checkpoints when ckpt is NULL) is
 * allocated on first use and kept by the plan, grown when a later call needs
 * more (TDSE_E_NOMEM if it cannot be). A batch-1 plan runs the adjoint on a
 * batched twin of itself, built on the first call: a second copy of the
 * Hamiltonian in the matrix-core layout (2 lmax Np^2 doubles, Np = n rounded
 * up to the tile height; about 31 MB at Lmax = 15, N = 500), kept by the plan
 * and shared with tdse_propagate_rkf45.
 */
tdse_status tdse_adjoint(tdse_plan plan, tdse_method method, int32_t taylor_order, double dt,
                         int64_t nsteps, const double *field, const double *c0,
                         const double *ckpt, int32_t ckpt_every, const double *lambdaT,
                         double *grad_field, double *lambda0, void *stream);

/*
 * Uneven multi-instance propagation: `count` plans (each batch == 1, any
 * lmax, n <= 1024) advanced together. Every RK4 stage of the instances still
 * running is one completion launch over all their state segments and one
 * product launch over all their dipole tiles (work lists of (instance,
 * segment) and (instance, tile), each item with its instance's own sizes,
 * buffers and field samples); chunks of 64 such rounds replay a captured HIP
 * graph. Instances are ordered by step count, so the ones still running form
 * a prefix of both lists.
 * tdse_group_create: plans[count] (host array), the group keeps references
 * (the plans must outlive the group). Every member streams its blocks at the
 * default tile count ceil(n / 128): for a plan built with another count (a
 * tuned or forced one) the group makes and owns a copy of its blocks at the
 * default count (lmax * ceil(n/128)^2 * 128 KB of device memory; created on
 * `stream`, synchronised). Errors: TDSE_E_INVAL (a plan with batch != 1,
 * plans on different devices, one plan given twice), TDSE_E_UNSUPPORTED
 * (n > 1024), TDSE_E_NOMEM (such a copy could not be allocated).
 * tdse_group_propagate: RK4 only (TDSE_E_UNSUPPORTED otherwise); nsteps[count]
 * (host), fields, c0, cT: host arrays of `count` device pointers laid out as
 * in tdse_propagate. Instance i runs its own nsteps[i] steps; instances that
 * finish early leave the later rounds. Instances without dipole blocks
 * (lmax == 0) are propagated on their own. The group keeps its work lists
 * and captured graphs between calls (reallocated when a call needs more).
 */
tdse_status tdse_group_create(tdse_group *out, int32_t count, const tdse_plan *plans,
                              void *stream);
tdse_status tdse_group_propagate(tdse_group group, tdse_method method, int32_t taylor_order,
                                 double dt, const int64_t *nsteps, const double *const *fields,
                                 const double *const *c0, double *const *cT, void *stream);
tdse_status tdse_group_destroy(tdse_group group);

/*
 * Autotuner: time the candidate tile shapes for a (lmax, n, batch) problem on
 * the current device with synthetic data and record the fastest in the JSON
 * cache at cache_path (created or updated; NULL uses $TDSE_TUNE_CACHE, else
 * no file is written). Later tdse_create calls read the cache named by
 * $TDSE_TUNE_CACHE. Synchronous; allocates and frees its own buffers.
 */
tdse_status tdse_tune(int32_t lmax, int32_t n, int32_t batch, const char *cache_path);

#ifdef __cplusplus
}
#endif

#endif /* TDSE_H */
