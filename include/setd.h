/*
 * setd.h - C ABI of the split-ETD3 library (libsetd.so) for AMD Instinct
 * MI355X (gfx950).
 *
 * The library advances stiff semilinear systems
 *
 *     u'(t) = K u(t) + g(u(t)),   K = A_d (+) ... (+) A_1   (Kronecker sum),
 *
 * with the third-order directionally split exponential Runge-Kutta method
 * exprk3ds_real of Cassini, "Efficient third order tensor-oriented
 * directional splitting for exponential integrators" (problem statement:
 * Section 1, eqs. ODE and kronsum; method: eq. exprk3 with the splittings of
 * Sections 2.1 and 2.3; pseudocode: Algorithms 1 and 2 of the appendix).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Tensors.  An order-d tensor V of size n_1 x ... x n_d is a flat array of
 *   N = n_1 ... n_d elements with index i_1 fastest ("vec stacks by columns",
 *   Section 2): element (i_1, ..., i_d) sits at
 *   i_1 + n_1 (i_2 + n_2 (i_3 + ...)).
 * Matrices.  Square n x n matrices are column-major: entry (i, j) at i + n j.
 * Memory.  Every data pointer is DEVICE memory of the current HIP device unless
 *   the argument says "host".  The caller owns all buffers passed in; the
 *   library never frees them and never keeps them past the call (a context
 *   copies what it needs).
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the legacy
 *   default stream).  Calls are asynchronous on that stream unless stated.
 * Errors.  Every function returns SETD_OK (0) or a negative SETD_E* code.
 *   Arguments are validated before anything is launched; on a validation
 *   error nothing is written.  setd_last_error() gives a message for the
 *   calling thread's last failure.  Nothing throws or aborts across the ABI.
 */
#ifndef SETD_H
#define SETD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define SETD_OK            0
#define SETD_EINVAL       -1   /* bad size, null pointer, aliasing, bad enum   */
#define SETD_ENOMEM       -2   /* device allocation failed                     */
#define SETD_EHIP         -3   /* a HIP runtime call or kernel launch failed   */
#define SETD_ENONFINITE   -4   /* a non-finite value where one is not allowed  */
#define SETD_EUNSUPPORTED -5   /* valid request outside what is implemented    */

/* ---- arithmetic of the mu-mode products ---- */
#define SETD_PREC_F64     0    /* FP64 operands, FP64 accumulate                */
#define SETD_PREC_F32     1    /* FP32 operands and intermediates, FP32 accum.  */
#define SETD_PREC_BF16X3  2    /* three-term bf16 split x = h + m + l (each the
                                  bf16 rounding of what is left); the six
                                  products h*h, h*m, m*h, h*l, l*h, m*m on MFMA
                                  with FP32 accumulate; FP32 intermediates     */
#define SETD_PREC_BF16X2  3    /* two-term split x = h + l; h*h, h*l, l*h (three
                                  products): faster, about 16 significant bits */
#define SETD_PREC_I8X4    4    /* error-free int8 slicing (Ozaki scheme): every
                                  phi row and tensor fibre rounded to a 30-bit
                                  integer relative to its largest entry, four
                                  int8 digits each; the thirteen digit products
                                  of order >= 2 summed exactly in int32 on the
                                  int8 matrix cores, combined in FP64 (about
                                  2^-29 of |x|max |p|max per product term);
                                  FP64 inputs, outputs and sums; intermediates
                                  kept as digits where the next product can
                                  take them so (bit-identical to slicing the
                                  FP64 intermediate; the environment variable
                                  SETD_I8_EMIT=0 turns this off, for tests)  */

/* ---- reaction terms g (eq. twocompdisc: two components u, v) ---- */
#define SETD_G_NONE         0  /* g = 0; nparams = 0                            */
#define SETD_G_SCHNAKENBERG 1  /* params (gamma, a, b):
                                  g1 = gamma (a - u + u^2 v), g2 = gamma (b - u^2 v)
                                  (Section 3.1 model)                            */
#define SETD_G_FHN          2  /* params (eps, a1, a0[, rho]), rho = 1 if absent:
                                  g1 = rho (u - u^3 - v), g2 = rho eps (u - a1 v - a0)
                                  (Section 3.2 model)                            */

/* ---- stages of eq. exprk3 (argument scale c_s of the phi bank) ---- */
#define SETD_STAGE_2  2        /* c = 1/3 */
#define SETD_STAGE_3  3        /* c = 2/3 */
#define SETD_STAGE_F  4        /* c = 1   */

/*
 * phi-functions of a small dense matrix (Section 1 definition
 * phi_l(X) = sum_k X^k/(k+l)!; computed as in Section 2.4: rational Pade
 * approximation with modified scaling and squaring, here entirely in FP64 on
 * the GPU).
 *
 *   A     n x n column-major FP64 (device).
 *   n     1 <= n <= 4096.
 *   tau   scalar; the argument is X = tau * A.  Must be finite.
 *   ell   0 <= ell <= 4.
 *   out   (ell + 1) consecutive n x n column-major blocks (device):
 *         phi_0(tau A), phi_1(tau A), ..., phi_ell(tau A).  Must not alias A.
 *
 * Synchronises `stream` once (the scaling exponent is chosen on the host from
 * the norm computed on the device).  Returns SETD_ENONFINITE if A holds a
 * non-finite value.
 */
int setd_phi_matrices(const double* A, int64_t n, double tau, int ell, double* out, void* stream);

/*
 * Tucker operator (Section 2, eq. krontomu):
 *
 *     W <- alpha * (V x_1 M_1 x_2 M_2 ... x_d M_d) + beta * W
 *
 *   V, W   N-element tensors (device), FP64, must not overlap.
 *   d      1 <= d <= 8.
 *   dims   host array of d sizes, 1 <= n_mu <= 4096, at most 2^36 elements
 *          in all.
 *   M      host array of d device pointers; M[mu] is the n_mu x n_mu
 *          column-major FP64 matrix applied along mode mu+1.  NULL means the
 *          identity (that mode is skipped).
 *   prec   SETD_PREC_F64, SETD_PREC_F32, SETD_PREC_BF16X3, SETD_PREC_BF16X2 or
 *          SETD_PREC_I8X4 (arithmetic of the mode products; V and W stay FP64).
 *   ws     device workspace of at least setd_tucker_workspace_bytes(d, dims,
 *          prec) bytes, or NULL to let the library use its own (grown on
 *          demand, kept until setd_release_workspace or process exit).
 *
 * beta = 0 ignores the old contents of W (NaN included).  An argument error or
 * a failed workspace allocation returns before W is touched.
 * setd_tucker_workspace_bytes returns 0 for arguments setd_tucker_apply would
 * reject.
 */
int setd_tucker_apply(const double* V, double* W, int d, const int64_t* dims,
                      const double* const* M, double alpha, double beta, int prec,
                      void* ws, size_t ws_bytes, void* stream);
size_t setd_tucker_workspace_bytes(int d, const int64_t* dims, int prec);
int setd_release_workspace(void);

/*
 * setd_tucker_apply without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, kernels and results as
 * setd_tucker_apply, but the Tucker intermediates and packed matrices live in
 * a scratch array of SETD_NOALLOC_SCRATCH_BYTES (64 MiB) that the library
 * holds on each GPU until the process ends; a tensor whose
 * setd_tucker_workspace_bytes exceeds it (e.g. beyond 128^3 in FP64, whose
 * need is 34 MB) is rejected with SETD_EINVAL before anything runs.  The
 * call allocates nothing and does not synchronise `stream`.
 * Every call on one GPU uses that GPU's single array: calls that overlap in
 * time on one GPU (different streams or threads) race and must be serialised
 * by the caller.  Nothing in the array needs to be cleared between calls.
 */
#define SETD_NOALLOC_SCRATCH_BYTES (64ll << 20)
int setd_tucker_apply_noalloc(const double* V, double* W, int d, const int64_t* dims,
                              const double* const* M, double alpha, double beta, int prec,
                              void* stream);

/*
 * Integration context: one grid, one set of matrices A_mu^(c) per component,
 * one step size tau and one arithmetic.  Creating it builds the phi bank
 * P_{i,s}^(l){mu} = phi_{l_i}(c_s tau alpha_{i,mu}^(l) A_mu) of Algorithm 1
 * (d = 2, Table 1 real coefficients, 2 terms) or Algorithm 2 (d >= 3,
 * Table 3, 3 terms), with the '+' coefficient set of Section 2.4, and every
 * work buffer of the time step.
 *
 *   d       2 <= d <= 3.
 *   dims    host array of d sizes, 2 <= n_mu <= 4096.
 *   ncomp   number of components, 1 or 2 (the reactions need 2).
 *   A       host array of ncomp*d device pointers: A[c*d + mu] is A_{mu+1}^(c),
 *           n_mu x n_mu column-major FP64.  Copied; the caller may free them.
 *   tau     step size > 0.
 *   prec    arithmetic of the mu-mode products (SETD_PREC_*); u and the
 *           stage accumulators are FP64 in every case.
 *
 * Synchronises `stream`.  Device memory held: about (23 N + bank) * 8 bytes
 * per component in FP64.
 */
typedef struct setd_ctx setd_ctx;
int setd_ctx_create(setd_ctx** ctx, int d, const int64_t* dims, int ncomp,
                    const double* const* A, double tau, int prec, void* stream);
int setd_ctx_destroy(setd_ctx* ctx);

/*
 * Split approximation of a phi-function action (eqs. split2d / splitnd3):
 *
 *     W <- beta * W + scale * S_l(c_s tau) V,
 *     S_l(c tau) V = sum_i eta_i^(l) T(V, {P_{i,s}^(l){mu}})
 *
 *   comp    component whose matrices are used, 0 <= comp < ncomp.
 *   ell     1 or 2 (stage SETD_STAGE_2 has ell = 1 only, as in the algorithms).
 *   stage   SETD_STAGE_2, SETD_STAGE_3 or SETD_STAGE_F.
 *   V, W    N-element FP64 tensors (device); must not overlap.
 */
int setd_split_phi_apply(setd_ctx* ctx, int comp, int ell, int stage, const double* V,
                         double* W, double scale, double beta, void* stream);

/*
 * Time stepping: nsteps steps of eq. exprk3 with the split phi actions
 * (the time loop of Algorithms 1 and 2), in place.
 *
 *   u        ncomp * N FP64 (device), component-major: u then v.
 *   nsteps   >= 0.
 *   tau      step size; if it differs from the context's, the phi bank is
 *            rebuilt first (synchronising).
 *   g_kind   SETD_G_*; params (host) and nparams as documented there.
 *
 * The diffusion coefficients live in the matrices A.  The K action uses a
 * fused 3-point stencil when every A_mu^(c) is tridiagonal and dense mu-mode
 * products otherwise.
 */
int setd_etd_step(setd_ctx* ctx, double* u, int nsteps, double tau, int g_kind,
                  const double* params, int nparams, void* stream);

/*
 * Second-order split integrator etd2rkds (the paper's comparison method,
 * Section 1): eq. ETD2RK
 *     u2 = u + tau phi_1(tau K) f(u),  u_new = u2 + tau phi_2(tau K)(g(u2) - g(u)),
 * with phi_l(tau K) v replaced by the second-order splitting eq. secondord,
 * l!^(d-1) T(V, {phi_l(tau A_mu)}): one Tucker operator per phi action.
 * Same context, arguments and in-place semantics as setd_etd_step.
 */
int setd_etd2_step(setd_ctx* ctx, double* u, int nsteps, double tau, int g_kind,
                   const double* params, int nparams, void* stream);

/*
 * exprk3ds_cplx: the same step with the two-term complex splitting (Table 1
 * complex column for d = 2, Table 2 for d > 2; Algorithm 1's complex
 * variant), each split action taken as the real part of its two complex
 * Tucker operators (the exact phi action is real; the imaginary part is
 * O(tau^3)).  Same context, arguments and in-place semantics as
 * setd_etd_step.  FP64 contexts only.  The first call (and a call with a new
 * tau) builds the complex phi matrices, through the real 2n x 2n
 * representation of the complex matrices, and synchronises; device memory
 * grows by 12 (d = 2) or 24 (d = 3) N doubles per component.
 */
int setd_etd_cplx_step(setd_ctx* ctx, double* u, int nsteps, double tau, int g_kind,
                       const double* params, int nparams, void* stream);

/*
 * Adjoint of one split-ETD3 step (vector-Jacobian product), for gradients of
 * a loss of the final state.  With U' = step(U; params, sigma) the step of
 * setd_etd_step (eq. exprk3 with the split phi actions) and
 * ubar = dL/dU' on entry, on return
 *     ubar = dL/dU = (dU'/dU)^T ubar_in,
 *     grad[k]            += (dU'/dparams_k)^T ubar_in     (k < nparams),
 *     grad[nparams + c]  += (dU'/dsigma_c)^T ubar_in      (bit c of sigma_mask),
 * where sigma_c scales every A_mu^(c) (derivative at sigma_c = 1; for
 * A^(c) = d_c D this is d_c dL/dd_c).  The transposed split actions are
 * Tucker operators with the transposed phi matrices (Section 2, eq.
 * krontomu); the phi derivative uses z phi_l'(z) = phi_{l-1}(z) - l phi_l(z).
 *
 *   u           state U at the start of the step (ncomp*N, device, read only).
 *   ubar        ncomp*N (device), in place; must not overlap u.
 *   g_kind, params, nparams   as for setd_etd_step (the same values).
 *   sigma_mask  components whose diffusion-size gradient is wanted (0..3);
 *               each costs 2d extra Tucker groups.
 *   grad        device accumulators (nparams + ncomp doubles), added to,
 *               never cleared; reduced in a fixed order (deterministic).
 * FP64 contexts only (SETD_EUNSUPPORTED otherwise).  The first call builds
 * the transposed and derivative phi matrices (synchronising); device memory
 * grows by about 11 ncomp N doubles.  Checkpointing is the caller's: keep
 * U at the start of each step (or recompute it) and call this backwards.
 */
int setd_etd_adjoint_step(setd_ctx* ctx, const double* u, double* ubar, int g_kind,
                          const double* params, int nparams, int sigma_mask, double* grad,
                          void* stream);

/*
 * One split-ETD3 step that also keeps the step's stage quantities, for a
 * later setd_etd_adjoint_step_recorded (a checkpointed backward pass steps
 * forward from a checkpoint anyway; recording there spares the adjoint step
 * its own forward recomputation of the stages).
 *
 *   u     as for setd_etd_step (one step, in place).
 *   rec   6 * ncomp * N doubles (device), written: G = g(U), F = K U + G,
 *         U2, D2 = g(U2) - G, U3, D3 = g(U3) - G (eq. exprk3 with the split
 *         phi actions), each ncomp * N, component-major.  Must not overlap u.
 * FP64 contexts only.  Plain launches (no graph replay).
 */
int setd_etd_step_record(setd_ctx* ctx, double* u, double tau, int g_kind, const double* params,
                         int nparams, double* rec, void* stream);

/*
 * setd_etd_adjoint_step with the stage quantities of the step taken from
 * `rec`, as setd_etd_step_record wrote them for the same u, tau and
 * parameters (read only; must not overlap ubar).  Same results as
 * setd_etd_adjoint_step, without its forward recomputation.
 */
int setd_etd_adjoint_step_recorded(setd_ctx* ctx, const double* u, const double* rec, double* ubar,
                                   int g_kind, const double* params, int nparams, int sigma_mask,
                                   double* grad, void* stream);

/*
 * Batched integration: nbatch independent instances of one kind of problem
 * (same d, ncomp and tau; each with its own grid, matrices A_mu^(c) and
 * reaction parameters) advanced together by split-ETD3 steps (the same step
 * as setd_etd_step, applied to every instance; the paper's method is per
 * instance, the batching is how the small instances fill the GPU).
 * Every stage of a step is one launch over all instances: the mu-mode
 * products of a Tucker group run from a work list of (instance, output,
 * tile) entries walked by a persistent grid, the pointwise kernels over the
 * points of all instances.  The step is captured in a hipGraph and replayed.
 * Tile shapes and grid sizes are chosen by timing candidates on the batch's
 * own work lists (setd_batch_tune; run automatically before the first step
 * unless setd_batch_set_tiles chose them or SETD_BATCH_TUNE=0).
 *
 * setd_batch_create
 *   nbatch  1 <= nbatch <= 65536 instances.
 *   d       2 or 3 (every instance).
 *   dims    host array of nbatch*d sizes: dims[b*d + mu] = n_{mu+1} of
 *           instance b, 2 <= n <= 1024 (grids may be non-square and differ
 *           between instances).
 *   ncomp   1 or 2.
 *   A       host array of nbatch*ncomp*d device pointers: A[(b*ncomp + c)*d +
 *           mu] is A_{mu+1}^(c) of instance b (column-major FP64).  Copied.
 *   tau     step size shared by all instances, > 0.
 *   prec    SETD_PREC_F64 only (others: SETD_EUNSUPPORTED).
 *   Builds the phi bank of every instance (one phi build per distinct
 *   matrix, scalars and packing; identical matrices are shared) and the work
 *   buffers.  Synchronises `stream`.
 *
 * Layout of the batch state u (device, FP64, owned by the caller): instance
 * b occupies elements off[b] .. off[b+1]-1 with component c of its grid
 * (Fortran-ordered as everywhere in this header) at off[b] + c*cs[b], where
 * cs[b] = N_b rounded up to a multiple of 8 (the gap, if any, is ignored).
 * setd_batch_layout writes off (host, nbatch+1 entries; off[nbatch] = total
 * length of u) and, if cs != NULL, cs (host, nbatch entries).
 *
 * setd_batch_step: nsteps steps of every instance, in place on u.
 *   g_kind  SETD_G_* for every instance.
 *   params  host array of nbatch*nparams values, instance b's at
 *           params[b*nparams] (as for setd_etd_step); NULL if nparams = 0.
 * The work lists refer to u itself: a call with another u rebuilds them
 * (synchronising); calls that overlap on the same u race.
 *
 * setd_batch_tune times every candidate tile shape (2 or 4 tiles of 16 on
 * each side) and grid cap on the phi_1 group of the step, separately for
 * mode 1 and for modes >= 2, and keeps the fastest.  Synchronises `stream`.
 * setd_batch_set_tiles fixes them instead: cfg (host) = {tm, tn, cap} for
 * mode 1 followed by {tm, tn, cap} for modes >= 2 (cap = largest number of
 * workgroups of a launch, 0 = one per tile).
 * setd_batch_info (host, SETD_BATCH_INFO entries): the six tile values as
 * for setd_batch_set_tiles, whether they were tuned or set, launches per
 * step (0 before the first step), the length of u, and the number of
 * distinct packed matrix sets.
 */
typedef struct setd_batch setd_batch;
#define SETD_BATCH_INFO 10
int setd_batch_create(setd_batch** batch, int nbatch, int d, const int64_t* dims, int ncomp,
                      const double* const* A, double tau, int prec, void* stream);
int setd_batch_destroy(setd_batch* batch);
int setd_batch_layout(const setd_batch* batch, int64_t* off, int64_t* cs);
int setd_batch_step(setd_batch* batch, double* u, int nsteps, int g_kind, const double* params,
                    int nparams, void* stream);
int setd_batch_tune(setd_batch* batch, void* stream);
int setd_batch_set_tiles(setd_batch* batch, const int* cfg);
int setd_batch_info(const setd_batch* batch, int64_t* info);

/*
 * Norms for error reporting (deterministic fixed-order reductions):
 *   out[0] = ||x||_2, out[1] = ||x||_inf, and when y != NULL
 *   out[2] = ||x - y||_2, out[3] = ||x - y||_inf   (out is host, 4 doubles).
 * Synchronises `stream`.
 */
int setd_field_norms(const double* x, const double* y, int64_t n, double* out, void* stream);

/*
 * Kernel timing for measurement.  While enabled, every kernel launch of the
 * library is bracketed by a pair of hipEvents recorded on the launch stream,
 * and the launch's algorithmic work is noted: 2 N n flops per mu-mode product
 * term (N tensor entries, n the contracted size; Section 2 cost count) and
 * the bytes a single pass must move (inputs read once, outputs written once).
 * Kernel classes:
 *   0 mode-1 products, FP64          1 modes >= 2 products, FP64
 *   2 mode-1 products, FP32/BF16x3   3 modes >= 2 products, FP32/BF16x3
 *   4 pointwise (G/F, stage differences)
 *   5 modes >= 2 products, FP64, matrix panel in LDS (single-term jobs with
 *     192 <= n <= 256)
 * setd_profile_read synchronises the recorded events and writes, per class
 * c, out[4c..4c+3] = {launches, total milliseconds, total flops, total bytes}
 * (out is host memory of SETD_PROF_CLASSES*4 doubles); reset != 0 clears the
 * record.  Enabling costs one event pair per launch.
 */
#define SETD_PROF_CLASSES 6
int setd_profile_enable(int on);
int setd_profile_read(double* out, int reset);

/* Message for the calling thread's last error ("" if none). */
const char* setd_last_error(void);
/* Waits for `stream` and reports an asynchronous HIP error as SETD_EHIP. */
int setd_sync(void* stream);
/* Library version string. */
const char* setd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SETD_H */
