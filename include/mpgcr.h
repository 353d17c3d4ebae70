/*
 * mpgcr -- preconditioned non-symmetric GCR(k) solver for the elliptic depth
 * problem of a semi-implicit shallow-water model on a regular
 * longitude/latitude grid, for AMD Instinct MI355X (gfx950).
 *
 * Method: Ackmann, Dueben, Palmer, Smolarkiewicz, "Mixed-precision for linear
 * solvers in global geophysical flows" (arXiv:2103.16120), Section 2.
 *   - The problem solved is L(Phi) - R = 0 (eq. Elliptic) with the generalised
 *     Laplacian of eq. L_Operator, whose coefficient fields come from the
 *     linearised pressure gradient (eq. rhslin) and the pointwise 2x2
 *     inversion of the implicit momentum equations (eq. Qexpr).
 *   - The solver is preconditioned GCR(k) (Section 2.3) with exit test
 *     ||r_N||_2 <= eps ||r_0||_2 (eq. exitcondition) and at least one full
 *     GCR(k) cycle; the preconditioner is option 3, the semi-implicit
 *     Richardson scheme of eq. P_Operator, or one of options 0-2.
 *   - Precision forms follow Sections 4.2-4.3: double precision throughout,
 *     or low-precision storage of the operator/preconditioner with single
 *     precision Krylov vectors, a double precision solution accumulator and
 *     double precision residual recomputation.
 *
 * Grid: NX x NY cell-centred points, longitude lambda_i = i*2*pi/NX, latitude
 * phi_j = -pi/2 + (j+1/2)*pi/NY.  Every field is a contiguous row-major
 * [NY][NX] float64 array, longitude fastest, row 0 southernmost.  NX must be a
 * power of two in [8, 1024] and NY an integer in [2, 4096].
 *
 * Conventions for every entry point:
 *   - Return value: GCR_OK (0) or a positive soft status, or a negative hard
 *     error.  No exception, abort or exit crosses this interface.  After a hard
 *     error the caller's output arrays are untouched and gcr_last_error()
 *     describes the cause.
 *   - Device pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  The library never frees caller
 *     memory and never keeps caller pointers after a call returns.
 *   - A solver is used from one host thread at a time; its work is ordered on
 *     the stream given at creation (NULL = the default stream).  Calls that
 *     return results to the host synchronise that stream.
 */
#ifndef MPGCR_H
#define MPGCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gcr_solver gcr_solver; /* opaque; owned by the library */

/* status codes */
enum {
  GCR_OK = 0,            /* converged: ||r|| <= rtol ||r_0|| after >= min_iters      */
  GCR_NOT_CONVERGED = 1, /* max_iters reached; x holds the last iterate               */
  GCR_STAGNATED = 2,     /* breakdown or no decrease over a whole cycle; x = last     */
  GCR_FALLBACK_USED = 3, /* converged, but the learned preconditioner was replaced
                            by the semi-implicit one during the solve               */
  GCR_EINVAL = -1,       /* invalid argument                                          */
  GCR_ENOMEM = -2,       /* device or host allocation failed                          */
  GCR_EHIP = -3,         /* HIP runtime error (includes: no usable GPU)               */
  GCR_ESTATE = -4        /* call out of order (e.g. solve before set_operator)        */
};

/* precision forms (paper Sections 4.1-4.3) */
enum {
  GCR_FP64 = 0,          /* everything in float64                                     */
  GCR_MIXED = 1,         /* operator and preconditioner coefficients stored as
                            float16 (float32 in the polar rows), float32 arithmetic;
                            float32 Krylov vectors and inner products; solver
                            increments accumulated in float32 and added to the
                            float64 solution at exit                                 */
  GCR_MIXED_FP64DOT = 2, /* as GCR_MIXED, plus float64 inner products, a float64
                            solution accumulator, and the residual recomputed in
                            float64 from the solution at every restart
                            (residual replacement)                                 */
  GCR_MIXED_HALF_PC = 3, /* as GCR_MIXED_FP64DOT, but the operator applied inside
                            the Krylov iteration keeps float32 coefficients: half
                            precision only in the preconditioner, the step the
                            paper finds most robust to reduced precision          */
  GCR_SINGLE = 4,        /* the paper's single-precision solver cycle (Section 4.2,
                            option two): operator and preconditioner in float32
                            (coefficients formed from the float32 depth),
                            float32 Krylov vectors, inner products and
                            preconditioner intermediates, float32 solution
                            increments added to the float64 solution at exit;
                            float64 initial and final residual                    */
  GCR_SINGLE_POLAR64 = 5 /* as GCR_SINGLE, but the rows within polar_rows of either
                            pole compute the operator and the preconditioner in
                            float64 from float64 coefficients (Section 4.2,
                            option three); vectors stay float32                   */
};

/* preconditioners (paper Section 2.3, options 0-3; 4 is a learned network) */
enum {
  GCR_PC_NONE = 0,           /* P = I                                                 */
  GCR_PC_DIAG = 1,           /* P = diagonal of L                                     */
  GCR_PC_RICHARDSON = 2,     /* explicit Richardson on L, diagonally preconditioned   */
  GCR_PC_SEMI_IMPLICIT = 3,  /* semi-implicit Richardson, eq. P_Operator (default)    */
  GCR_PC_LEARNED = 4         /* option 3 plus a 3x3 convolution network correction
                                (not from the paper); needs gcr_set_learned           */
};

/* flags */
#define GCR_F_RECORD_HISTORY 0x1u  /* keep ||r_nu||/||r_0|| per iteration in reports  */
#define GCR_F_ONE_STREAM 0x2u      /* solve the whole batch on the solver's stream; by
                                      default a large batch is split into two groups
                                      of members, one solved on that stream, one on a
                                      stream of the library forked from and joined
                                      back to it                                   */
#define GCR_F_LINF_EXIT 0x4u       /* exit test in the maximum norm, max|r| <= rtol
                                      max|r_0| (paper Section 4.1 discussion: the
                                      alternative exit condition); the iteration,
                                      its stagnation test and the reported relative
                                      residuals stay Euclidean                     */
#define GCR_F_FAULT_NAN_PC 0x8u    /* tests of the exit logic: the preconditioner
                                      output computed after iteration k (the first
                                      one of the second GCR(k) cycle) is replaced
                                      by NaN in every member; the breakdown is
                                      reported as GCR_STAGNATED with x the iterate
                                      after k+1 updates (the last finite one)      */
#define GCR_F_FAULT_ZERO_DIR 0x10u /* as GCR_F_FAULT_NAN_PC with an all-zero
                                      preconditioner output, i.e. a zero search
                                      direction (<L p, L p> = 0)                   */
#define GCR_F_SPLIT_R0 0x20u       /* GCR_SINGLE / GCR_SINGLE_POLAR64 only: the
                                      initial residual is the split single-
                                      precision evaluation of Section 4.2.1 (eq.
                                      L_Operator_SP) on x_0 = Phi_hat + Phi_tilde,
                                      Phi_hat the member's base stored by
                                      gcr_set_split_base (the caller renews it at
                                      the cadence it chooses; the paper keeps it
                                      for many time steps), Phi_tilde =
                                      fl32(x_0 - Phi_hat); every member needs a
                                      base (GCR_ESTATE otherwise)                 */
#define GCR_F_GRAPH 0x40u          /* replay the kernels of every GCR iteration and
                                      cycle end from HIP graphs, captured once per
                                      window position and ring slot on first use
                                      (the host still reads the done flags once per
                                      cycle); results are bitwise those without.
                                      Not used with the learned preconditioner or
                                      with per-kernel timing.  With a NULL stream
                                      the solver orders its work on a blocking
                                      stream of its own (the null stream cannot
                                      be captured; its work stays ordered with
                                      that stream's)                              */

typedef struct {
  int32_t batch;          /* number of independent solves, 1..4096                    */
  const int32_t* nx;      /* host array [batch]: longitudes per member                */
  const int32_t* ny;      /* host array [batch]: latitudes per member                 */
  int32_t k;              /* GCR(k) window, 1..8 (paper: 3)                           */
  int32_t precision;      /* GCR_FP64 / GCR_MIXED / GCR_MIXED_FP64DOT / _HALF_PC      */
  int32_t precond;        /* GCR_PC_*                                                 */
  int32_t richardson_iters; /* Richardson iterations in options 2-3, 1..16 (paper: 2) */
  int32_t polar_rows;     /* rows per pole kept in float32 in the mixed forms;
                             -1 = max(1, log2(NY/32)), i.e. 1/2/3 at NY = 64/128/256  */
  int32_t min_iters;      /* no exit before this many iterations; -1 = k+1            */
  int32_t max_iters;      /* 1..100000                                                */
  double rtol;            /* exit when ||r||_2 <= rtol * ||r_0||_2; >= 0              */
  void* stream;           /* hipStream_t all work is ordered on; NULL = default        */
  uint32_t flags;         /* GCR_F_* (other bits: GCR_EINVAL)                         */
} gcr_params;

typedef struct {
  double dt;              /* time step, s (> 0)                                       */
  double g;               /* gravity, m s^-2 (> 0)                                    */
  double omega;           /* rotation rate, s^-1 (f = 2 omega sin(lat)); 0 allowed    */
  double radius;          /* sphere radius, m (> 0)                                   */
  double absorber;        /* polar absorber strength alpha_max, s^-1 (>= 0): alpha
                             rises linearly from 0 at 3*pi/64 from a pole to
                             alpha_max at the pole (paper Section 3.2)               */
  const double* depth;    /* Phi*, explicit depth predictor [NY][NX], m, > 0          */
  const double* orography;/* H0 [NY][NX], m, or NULL for a flat surface               */
  int32_t b_terms;        /* 1 = the paper's operator; 0 drops the B^I terms (tests)  */
  int32_t mem_is_device;  /* 1 if depth/orography are device pointers, 0 if host      */
} gcr_operator;

typedef struct {
  int32_t status;             /* GCR_OK / NOT_CONVERGED / STAGNATED / FALLBACK_USED  */
  int32_t iterations;         /* number of step-2 updates                            */
  int32_t restarts;           /* residual recomputations (FP64DOT / HALF_PC forms)   */
  int32_t fallback_used;      /* 1 if the learned preconditioner was abandoned       */
  double r0_norm;             /* ||L(x_0) - R||_2                                    */
  double rel_res_recursive;   /* ||r_N|| / ||r_0|| of the iterated residual         */
  double rel_res_true;        /* ||L(x_N) - R||_2 / ||r_0||, recomputed in float64   */
  double* history;            /* host buffer supplied by the caller, or NULL         */
  int32_t history_cap;        /* entries available in history                        */
  int32_t history_len;        /* entries written: ||r_nu||/||r_0||, nu = 0..N        */
} gcr_report;

/* Fill *p with defaults for one member of size nx x ny: k = 3, GCR_FP64,
 * GCR_PC_SEMI_IMPLICIT, 2 Richardson iterations, polar_rows = -1,
 * min_iters = -1, max_iters = 200, rtol = 1e-8, default stream, no flags.
 * The nx/ny pointers are left NULL; the caller must set them.  Returns
 * GCR_EINVAL if p is NULL. */
int gcr_default_params(gcr_params* p);

/* Create a solver for params->batch independent members.  Validates the
 * parameters, selects the device that is current, and allocates all device
 * workspace for the declared sizes (the solve path allocates nothing).
 * On success *out receives the solver; on failure *out is set to NULL.
 * Errors: GCR_EINVAL (bad sizes or options), GCR_ENOMEM, GCR_EHIP (no GPU).
 * gcr_last_error(NULL) describes a creation failure. */
int gcr_create(const gcr_params* params, gcr_solver** out);

/* Build the coefficient fields of member `member` (0-based) from the
 * physical inputs (paper eqs. rhslin, Qexpr, L_Operator; Section 2.2).  All
 * precision forms of the coefficients are built on the device, on the
 * solver's stream.  Host inputs are copied before the call returns; device
 * inputs are read in place by the assembly kernel, so they must stay valid
 * until that kernel has run (see gcr_set_operators).
 * Errors: GCR_EINVAL, GCR_EHIP. */
int gcr_set_operator(gcr_solver* s, int32_t member, const gcr_operator* op);

/* Batched form of gcr_set_operator: members[t] (distinct, 0-based) gets
 * operator ops[t], t = 0..count-1, all assembled by one kernel launch.  Device
 * inputs (mem_is_device = 1) are read in place and must stay valid until the
 * work on the solver's stream has run (any later call that synchronises the
 * stream, e.g. gcr_solve, guarantees that); host inputs are copied before the
 * call returns.  Errors: GCR_EINVAL, GCR_EHIP. */
int gcr_set_operators(gcr_solver* s, int32_t count, const int32_t* members, const gcr_operator* ops);

/* Solve L(x_m) = rhs_m for every member m (paper Section 2.3).
 * rhs, x: host arrays [batch] of device pointers to float64 [NY][NX] fields;
 * x[m] holds the initial guess on entry and the solution on return.  Both
 * are used in place: rhs is read by every residual recomputation, x is read
 * by the first kernel and written by the last one, so no x[m] may overlap an
 * rhs field or another member's x.  reports: host array
 * [batch], or NULL.  Returns the worst soft status over the members (or a
 * hard error, with every x untouched).  Synchronises the solver's stream.
 * Errors: GCR_EINVAL (NULL pointers), GCR_ESTATE (a member without operator),
 * GCR_EHIP. */
int gcr_solve(gcr_solver* s, const double* const* rhs, double* const* x, gcr_report* reports);

/* y = L(x) for member `member` in float64 (eq. L_Operator), device pointers
 * [NY][NX]; y must not overlap x.  Asynchronous on the solver's stream. */
int gcr_apply_operator(gcr_solver* s, int32_t member, const double* x, double* y);

/* Split single-precision residual (paper Section 4.2.1, eq. L_Operator_SP).
 * The depth is carried as a float32 base Phi_hat plus a float32 correction
 * Phi_tilde.  gcr_set_split_base stores Phi_hat = fl32(phi0) of member
 * `member` (device float64 [NY][NX]) and the float32 differences of Phi_hat
 * that the operator's gradient terms use (taken in float64, rounded once);
 * the paper renews the base only every so many time steps.  The first call
 * allocates the solver's split buffers (6 float32 values per pooled point;
 * GCR_ENOMEM on failure).  Needs the member's operator (GCR_ESTATE).
 * gcr_residual_split computes r = L_SP(Phi_hat + Phi_tilde) - R: the gradient
 * terms take the stored differences of Phi_hat plus those of phi_tilde, the B
 * and C terms take Phi_hat + phi_tilde, all in float32, with the face
 * coefficients formed in float64 and rounded to float32; the rows within
 * polar_rows (gcr_params) of either pole use
 * the float64 operator on Phi_hat + phi_tilde.  phi_tilde: device float32,
 * rhs and r: device float64, all [NY][NX]; r holds float32 values outside the
 * polar bands and must not overlap an input.  GCR_ESTATE without a split
 * base.  Asynchronous on the solver's stream; uses the solver's pooled
 * scratch fields (not during a solve). */
int gcr_set_split_base(gcr_solver* s, int32_t member, const double* phi0);
int gcr_residual_split(gcr_solver* s, int32_t member, const float* phi_tilde, const double* rhs, double* r);

/* e = P^{-1}(r) for member `member` with the solver's preconditioner and
 * Richardson count, in float64 (eq. P_Operator for option 3), device
 * pointers [NY][NX]; e must not overlap r.  Asynchronous on the stream. */
int gcr_apply_precond(gcr_solver* s, int32_t member, const double* r, double* e);

/* The operator and the preconditioner of member `member` in the solver's own
 * precision form, with the kernels its solve runs (Sections 4.2-4.3: the
 * storage and arithmetic precision of each quantity as listed for the forms
 * above).  Device pointers [NY][NX] float64; the output must not overlap the
 * input.
 *   gcr_apply_operator_form: y = L(x) as the Krylov iteration applies it to a
 *     direction: x is rounded to the form's vector type (float32 in every
 *     form but GCR_FP64), L is evaluated with the form's operator
 *     coefficients (float16 storage with float32 polar rows in GCR_MIXED and
 *     GCR_MIXED_FP64DOT; float32 formed from the float32 depth in
 *     GCR_MIXED_HALF_PC and GCR_SINGLE; float64 polar rows in
 *     GCR_SINGLE_POLAR64), rounded to the vector type, and returned in
 *     physical units.
 *   gcr_apply_precond_form: e = P^{-1}(r) as the solve applies it to a
 *     residual: r is rounded to the vector type (in the mixed forms' scaled
 *     units s r, s = dt / (2 a^2)), the preconditioner runs with the form's
 *     coefficients and intermediate storage (float16 with one scale per row in
 *     GCR_MIXED, GCR_MIXED_FP64DOT and GCR_MIXED_HALF_PC; float32 in
 *     GCR_SINGLE; float64 polar rows in GCR_SINGLE_POLAR64), and e is returned
 *     as held (physical units).  With GCR_PC_LEARNED the network correction
 *     is applied too.
 * In GCR_FP64 they equal gcr_apply_operator and gcr_apply_precond.  Both use
 * the solver's Krylov buffers and are asynchronous on the solver's stream.
 * Errors: GCR_EINVAL, GCR_ESTATE (no operator; learned without parameters),
 * GCR_EHIP. */
int gcr_apply_operator_form(gcr_solver* s, int32_t member, const double* x, double* y);
int gcr_apply_precond_form(gcr_solver* s, int32_t member, const double* r, double* e);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): e =
 * P^{-1}(r) for one member with operator `op`, the semi-implicit Richardson
 * preconditioner (option 3) with `richardson_iters` iterations in float64 --
 * the result of gcr_apply_precond on a GCR_FP64 solver whose member has this
 * operator and Richardson count.  No solver is needed and nothing is
 * allocated: every buffer besides r and e is a static device array of the
 * library (about 13 MiB per GPU it runs on, held until the process ends),
 * and the call only launches kernels on `stream` (hipStream_t, NULL = the
 * default stream; asynchronous).
 *   nx: power of two in [8, 1024]; ny in [2, 4096]; nx * ny <=
 *     GCR_STATIC_MAX_POINTS (larger sizes: GCR_EINVAL);
 *   op: depth (and orography, or NULL) must be device pointers
 *     (mem_is_device = 1), [NY][NX] float64, valid until the work on the
 *     stream has run; r, e: device float64 [NY][NX], not overlapping.
 * Calls on one GPU share the static array, and the last call's contents stay
 * in it: calls that overlap on one GPU (unordered streams or threads) race.
 * Errors: GCR_EINVAL, GCR_EHIP; gcr_last_error(NULL) describes the last
 * failure on the calling thread. */
#define GCR_STATIC_MAX_POINTS 131072
int gcr_apply_precond_static(int32_t nx, int32_t ny, const gcr_operator* op, int32_t richardson_iters,
                             const double* r, double* e, void* stream);

/* Release every resource of the solver.  NULL is accepted (no-op). */
int gcr_destroy(gcr_solver* s);

/* Text of a status or error code (static storage). */
const char* gcr_status_string(int code);

/* Description of the last hard error on `s` (or of the last failed
 * gcr_create when s is NULL); static or solver-owned storage, valid until the
 * next call on the same solver. */
const char* gcr_last_error(const gcr_solver* s);

/* Kernel kinds for per-kernel timing. */
enum {
  GCR_K_ASSEMBLE = 0,   /* coefficient assembly (gcr_set_operator)                  */
  GCR_K_RESIDUAL = 1,   /* float64 residual L(x) - R                                 */
  GCR_K_SWEEP1 = 2,     /* step-2 update fused with the first row solve              */
  GCR_K_SWEEP2 = 3,     /* later Richardson iterations (P^M + row solve)             */
  GCR_K_APPLY_L = 4,    /* L(e) with fused inner products                            */
  GCR_K_ORTH = 5,       /* step-4 direction update with fused inner products         */
  GCR_K_CONTROL = 6,    /* per-member scalar updates                                 */
  GCR_K_COPY = 7,       /* gather/scatter of caller fields                           */
  GCR_K_LEARNED = 8,    /* learned correction: features, five convolutions, update   */
  GCR_K_SOLUTION = 9,   /* step-2 solution updates, applied once per GCR cycle       */
  GCR_K_SI_STEP = 10,   /* gcr_si_step's explicit part and momentum recovery         */
  GCR_K_COUNT = 11
};

/* Enable (1) or disable (0) timing of every kernel the solver launches with
 * HIP events recorded on its stream around each launch, and reset the
 * accumulated times.  Timing adds two event records per launch. */
int gcr_set_kernel_timing(gcr_solver* s, int32_t enable);

/* Launch count and summed duration (milliseconds) of kernel kind `kind`
 * (GCR_K_*) since timing was last enabled.  Synchronises the stream. */
int gcr_kernel_time(gcr_solver* s, int32_t kind, int64_t* launches, double* total_ms);

/* Name of a kernel kind (static storage). */
const char* gcr_kernel_name(int32_t kind);

/* Library version string, e.g. "mpgcr 0.1.0 gfx950". */
const char* gcr_version(void);

/* ------------------------------------------------------------------------
 * Learned preconditioner (GCR_PC_LEARNED; not from the paper).
 *
 * After the semi-implicit Richardson output e_2 = P^{-1}(r) (option 3 with
 * the solver's Richardson count) a convolution network N adds a correction
 * that passes through the preconditioner's row operator T = I - eta (P^Z -
 * P^H) (eq. P_Operator):
 *     e = e_2 + T^{-1}( s * sigma * N(r / sigma, e_2 / (s * sigma), cos(lat)) ),
 * with s = dt / (2 a^2) and sigma = ||r||_2 / sqrt(NX*NY) in physical units
 * (L is of size 1/s, so both inputs are of order one), so the result is
 * independent of the scale of r.  GCR minimises the residual over whatever
 * directions it is given, so a preconditioner that changes between
 * iterations is allowed.  N: 3x3 convolutions 3 -> 32 -> 32 -> 32 -> 32 -> 1,
 * ReLU between layers, periodic in longitude, the row beyond a pole is the
 * polar row shifted by NX/2 (the operator's closure).  Weights and
 * activations bf16, float32 accumulation.
 * ------------------------------------------------------------------------ */
#define GCR_LEARNED_CHANNELS 3

typedef struct cnn_net cnn_net; /* opaque; owned by the library */

/* Parameters of a network with c_in input channels, float32, in the order
 * w_1 [32][c_in][3][3], b_1 [32], w_2..w_4 [32][32][3][3], b_2..b_4 [32],
 * w_5 [1][32][3][3], b_5 [1]; w[co][ci][dy+1][dx+1] multiplies the input at
 * (lat + dy, lon + dx). */
int64_t cnn_param_count(int c_in);

/* Create a network for batches of up to max_batch images of ny x nx pixels
 * (nx a power of two in [64, 1024], 2 <= ny <= 4096) with c_in (1..32)
 * input channels.  Parameters start at zero (N = 0).  All device memory is
 * allocated here; work is ordered on `stream` (hipStream_t, NULL = default).
 * Errors: GCR_EINVAL, GCR_ENOMEM, GCR_EHIP (no GPU); *out = NULL then. */
int cnn_create(int32_t nx, int32_t ny, int32_t max_batch, int32_t c_in, void* stream, cnn_net** out);

/* Copy `count` (= cnn_param_count(c_in)) float32 parameters from / to host
 * memory; setting them also resets the Adam moments.  Synchronous.
 * Errors: GCR_EINVAL (NULL or wrong count), GCR_EHIP. */
int cnn_set_params(cnn_net* n, const float* host, int64_t count);
int cnn_get_params(cnn_net* n, float* host, int64_t count);

/* out[b][y][x] = N(in[b][.][y][x]); in: device float32 [batch][c_in][ny][nx],
 * out: device float32 [batch][ny][nx].  Asynchronous on the network's stream.
 * Errors: GCR_EINVAL (batch outside 1..max_batch, NULL), GCR_EHIP. */
int cnn_forward(cnn_net* n, int32_t batch, const float* in, float* out);

/* Gradient of sum(dy * N(in)) with respect to every parameter, written to
 * host memory in the parameter order (cnn_param_count floats); in and dy are
 * device float32 [batch][c_in][ny][nx] and [batch][ny][nx].  Synchronous.
 * Errors: as cnn_forward. */
int cnn_gradients(cnn_net* n, int32_t batch, const float* in, const float* dy, float* grads_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * mean squared error mean((N(in) - target)^2) over the batch; in and target
 * as in cnn_gradients.  *loss (may be NULL) receives the loss before the
 * step, which makes the call synchronous.  Errors: as cnn_forward, and
 * GCR_EINVAL for lr not finite and positive. */
int cnn_train_step(cnn_net* n, int32_t batch, const float* in, const float* target, float lr, double* loss);

/* Release the network.  NULL is accepted. */
int cnn_destroy(cnn_net* n);

/* Description of the last error on n (or of the last failed cnn_create when
 * n is NULL). */
const char* cnn_last_error(const cnn_net* n);

/* Give solver s (created with precond = GCR_PC_LEARNED, every member of one
 * size) the network parameters `params` (cnn_param_count(3) floats, host).
 * The solver keeps its own copy and inference buffers.  fallback_ratio in
 * (0, 1]: a member whose residual shrinks by less than this factor over a GCR
 * cycle drops the learned correction for the rest of the solve (reported as
 * fallback_used / GCR_FALLBACK_USED); a cycle without any decrease also
 * triggers it instead of GCR_STAGNATED.  Synchronous.
 * Errors: GCR_EINVAL (wrong precond, uneven sizes, count, ratio), GCR_ENOMEM,
 * GCR_EHIP. */
int gcr_set_learned(gcr_solver* s, const float* params, int64_t count, double fallback_ratio);

/* Reference residual history for the learned preconditioner's fallback:
 * rel_res[i] (i = 1..n, host array of n+1 values, entry 0 ignored) is the
 * relative residual ||r_i|| / ||r_0|| the plain semi-implicit preconditioner
 * reaches after iteration i on this workload (e.g. the geometric mean over
 * the members of a plain solve's histories).  A member whose residual after
 * iteration i <= n is above rel_res[i] has fallen behind the method without
 * the network and drops the network from its next preconditioner application
 * on (reported as fallback_used / GCR_FALLBACK_USED).  n = 0 removes the
 * reference (only the per-cycle fallback_ratio test of gcr_set_learned stays).
 * n <= max_iters.  Synchronous.  Errors: GCR_EINVAL (no learned
 * preconditioner, n out of range, NULL with n > 0, values not finite and
 * positive), GCR_ENOMEM, GCR_EHIP. */
int gcr_set_learned_reference(gcr_solver* s, const double* rel_res, int32_t n);

/* Training data for member `member`: with r = L(x) - rhs (float64),
 * e_lo = P^{-1}(r) with the solver's Richardson count and, if hi_iters > 0,
 * e_hi = P^{-1}(r) with hi_iters Richardson iterations, write
 *   feat [3][NY][NX] = (r / sigma, e_lo / (s sigma), cos(lat))   (float32)
 *   target [NY][NX]  = T(e_hi - e_lo) / (s sigma)                (float32)
 * (target only if hi_iters > 0 and target != NULL).  x, rhs: device float64
 * [NY][NX]; feat, target: device float32.  *sigma (may be NULL) receives
 * sigma; a zero residual gives sigma = 0 and zero features.  Synchronous.
 * Errors: GCR_EINVAL, GCR_ESTATE (no operator), GCR_EHIP. */
int gcr_learned_features(gcr_solver* s, int32_t member, const double* x, const double* rhs, int32_t hi_iters,
                         float* feat, float* target, double* sigma);

/* ---- the semi-implicit time step around the solve (paper Sections 2.1-2.2) */

/* One member's state for gcr_si_step.  All fields are device float64
 * [NY][NX] arrays of the member's size.  Variables: fluid thickness Phi (m),
 * momenta Q_x, Q_y (Phi times the zonal / meridional velocity, m^2 s^-1). */
typedef struct {
  const double* phi;      /* Phi^n                                                   */
  const double* qx;       /* Q_x^n                                                   */
  const double* qy;       /* Q_y^n                                                   */
  const double* phi_old;  /* Phi^{n-1} (first step: Phi^n)                           */
  const double* qx_old;   /* Q_x^{n-1}                                               */
  const double* qy_old;   /* Q_y^{n-1}                                               */
  const double* orography;/* H0, or NULL for a flat surface                          */
  const double* qbar_x;   /* relaxation target of the polar absorber, or NULL (zero) */
  const double* qbar_y;
  double* phi_new;        /* Phi^{n+1} (written; must not alias any input field)     */
  double* qx_new;         /* Q_x^{n+1}                                               */
  double* qy_new;         /* Q_y^{n+1}                                               */
  double dt, g, omega, radius, absorber;   /* as in gcr_operator                     */
} gcr_si_member;

/* One time step n -> n+1 of the shallow-water equations in the paper's
 * semi-implicit form (eqs. SWE1-SWE3, RSWE2-RSWE3, MPDATA, rhslin, Qexpr,
 * Elliptic, vadv) for every member of the solver's batch:
 *   forcings R^n; Q~ = Q^n + dt/2 R^n; the advective velocity at n + 1/2
 *   extrapolated from n and n-1 as face Courant numbers; MPDATA (donor cell
 *   plus one corrective pass, |psi| in the ratios, no limiter) of Phi^n, Q~_x,
 *   Q~_y giving Phi* and Qhat; the implicit Coriolis / relaxation / pressure
 *   terms inverted pointwise (eq. Qexpr); the elliptic problem
 *   L(Phi^{n+1}) = D(F^n) + D(Fhathat) - C Phi^n assembled from Phi* and H0
 *   (replacing each member's operator) and solved by gcr_solve from Phi^n;
 *   then Q^{n+1} from eq. Qexpr.
 * members: host array [batch].  reports: host array [batch] or NULL (the
 * solve's reports).  The step's work fields (18 per member, ~ 8 * 18 * NX *
 * (NY+1) bytes) are allocated by the first call and kept.  Returns the
 * solve's worst soft status, or a hard error.  Synchronous.  Errors:
 * GCR_EINVAL (NULL fields, a new field equal to another new field or to an
 * input field (fields must not overlap at all), dt / g / radius
 * not > 0, absorber < 0, and every error of gcr_set_operators / gcr_solve,
 * e.g. a non-positive Phi*), GCR_ENOMEM, GCR_EHIP. */
int gcr_si_step(gcr_solver* s, const gcr_si_member* members, gcr_report* reports);

#ifdef __cplusplus
}
#endif

#endif /* MPGCR_H */
