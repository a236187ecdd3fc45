/*
 * arrow.h -- C ABI of libarrow, an MI355X (gfx950) FP64 eigensolver for real
 * symmetric arrowhead matrices and the two problems the method extends to.
 *
 * Method: Jakovcevic Stor, Slapnicar, Barlow, "Accurate eigenvalue
 * decomposition of arrowhead matrices and applications".  Each eigenpair is
 * computed independently by shifting to the nearest pole, inverting the
 * shifted matrix, evaluating its one sensitive element b in double-double and
 * bisecting for the extreme eigenvalue of the inverse (Algorithms 1-5).
 *
 * Conventions shared by every call:
 *   - All array arguments are DEVICE pointers (HIP device memory of the
 *     handle's device), owned by the caller.  The library never frees them.
 *   - Calls are asynchronous on the handle's stream (arrow_set_stream; the
 *     default is the null stream).  Outputs are valid once that stream has
 *     completed the call.  One handle must not be used by two threads at once;
 *     calls on one handle reuse its workspace and are ordered by its stream.
 *   - Eigenvalues (singular values) are returned in descending order.
 *   - Matrices are column-major with leading dimension ld >= n; column k is
 *     the vector of the k-th largest eigenvalue; rows follow the caller's
 *     original (unsorted) order of d.
 *   - Return value: ARROW_OK (0), a negative value -i when argument i
 *     (1-based, counting the handle as argument 1) is invalid, or a positive
 *     ARROW_ERR_* for a host-side failure.  Conditions that depend on the
 *     data (reducible input, remedies used) never fail the call; they are
 *     reported per eigenvalue in info[] (ARROW_INFO_* bits) on the device.
 */
#ifndef ARROW_H
#define ARROW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct arrow_handle_s* arrow_handle_t;

/* status codes */
#define ARROW_OK 0
#define ARROW_ERR_HIP 1      /* a HIP runtime call failed (launch, allocation) */
#define ARROW_ERR_NOMEM 2    /* device workspace could not be allocated */
#define ARROW_ERR_STATE 3    /* null or destroyed handle */

/* info bits, one uint32 per eigenvalue */
#define ARROW_INFO_DD_B 1u        /* b evaluated in double-double (Sec. 4, Theorem 6) */
#define ARROW_INFO_REMEDY_A 2u    /* shifted to the other neighbouring pole (Remark 2(a)) */
#define ARROW_INFO_REMEDY_B 4u    /* DPR1 inverse at a shift near lambda (Remark 2(b)) */
#define ARROW_INFO_NEAR_ZERO 8u   /* eigenvalue closest to 0 taken from A^{-1} (Remark 1), with
                                     f(0) summed exactly where double-double cannot resolve it */
#define ARROW_INFO_REDUCIBLE 16u  /* dpr1_eig / arrow_svd / arrow_eig_herm: some z_j = 0 or d_i = d_j
                                     (Sec. 1): not solved, outputs NaN (arrow_eig deflates instead) */
#define ARROW_INFO_NONFINITE 32u  /* non-finite input: not solved, outputs NaN */
#define ARROW_INFO_KB_LARGE 64u   /* K_b (eq. K2) beyond what double-double resolves */
#define ARROW_INFO_KNU_LARGE 128u /* reserved */
#define ARROW_INFO_BAD_INPUT 256u /* arrow_svd: some d_j = 0: not solved, outputs NaN */
#define ARROW_INFO_POLE_SHIFT 512u /* dpr1_eig: smallest eigenvalue measured from the pole d_n */
#define ARROW_INFO_DEFLATED 1024u  /* arrow_eig: eigenpair deflated from a reducible matrix (Sec. 1) */
#define ARROW_INFO_F0_UNRESOLVED 2048u /* Remark 1: the Pick function at 0 is 0 as far as an exact sum of
                                          its terms' FP64 quotient digits reaches (down to 2^-1074);
                                          lambda carries that absolute uncertainty */

/* largest order n that arrow_eig, arrow_eig_herm, dpr1_eig and arrow_svd accept (2^25; they
 * return -2 above it): one solve launches up to 64 lanes per eigenvalue, n * 64 <= 2^31 */
#define ARROW_N_MAX 33554432

/* options for arrow_set_option */
#define ARROW_OPT_TAU_NU 1     /* K_nu above which a Remark 2 remedy is applied (default 100) */
#define ARROW_OPT_TAU_ZERO 2   /* (|d_i|+|mu|)/|lambda| above which Remark 1 applies (default 10) */
#define ARROW_OPT_FP64_B 3     /* 1: b in FP64 only (Algorithm 2), a negative control (default 0) */
#define ARROW_OPT_REMEDIES 4   /* 0: no K_nu / near-zero remedies (default 1) */
#define ARROW_OPT_LANES 5      /* lanes per eigenvalue: 0 = automatic, else 1,2,4,...,64 */
#define ARROW_OPT_TIMING 6     /* 1: record HIP events around each stage of later calls */
#define ARROW_OPT_ROOT 7       /* root finder for the extreme eigenvalue of the inverse:
                                  0 = bisection (Algorithm 3), 1 = safeguarded rational
                                  (secular) iteration on the same function (default) */
#define ARROW_OPT_TAU_B 8      /* K_b (eq. K2) at or below which b is taken from an FP64 pass
                                  alone, as Algorithm 5 allows; the double-double pass (Theorem 6)
                                  runs only above it.  0 = always double-double (default).  With a
                                  bound of a few, eigenvalues carry about K_b times the FP64 sums'
                                  rounding instead of double-double's: a few ulps to ~1e-14 */
#define ARROW_OPT_CHECK_LANES 9 /* batched plans: lanes per eigenvalue in the check stage (K_nu test,
                                  norms): 4 (default), 8, 16, 32 or 64, or 0 for those of the first
                                  pass; the Remark 2 remedies and the DPR1 re-measure that the test
                                  calls for are re-run on whole wavefronts */

/* Create a handle on HIP device `device`.  *h receives the handle. */
int arrow_create(arrow_handle_t* h, int device);

/* Destroy a handle after synchronising its stream; frees its workspace. */
int arrow_destroy(arrow_handle_t h);

/* Set the HIP stream (a hipStream_t passed as void*) all later calls use. */
int arrow_set_stream(arrow_handle_t h, void* hip_stream);

/* Set one ARROW_OPT_* option.  Returns -2 for an unknown option, -3 for a bad value. */
int arrow_set_option(arrow_handle_t h, int option, double value);

/* Device workspace (bytes) one problem of order n needs; 0 for an order outside
 * 1..ARROW_N_MAX.  The handle grows its own workspace on demand (allocation
 * synchronises its stream). */
size_t arrow_workspace_size(int64_t n);

/*
 * Eigen-decomposition of the real symmetric arrowhead matrix
 *     A = [ diag(d)  z ; z^T  alpha ]            (Sec. 1, eqs. (A), (z))
 * of order n >= 1.  d, z: n-1 entries each, any order and signs (the
 * symmetric permutation to decreasing d and the sign normalisation of Sec. 1
 * are done inside; n == 1 allows null d, z).
 *   lambda: n eigenvalues, descending.
 *   V:      n x n eigenvectors (ldv >= n), or null for eigenvalues only.
 *           v_k = x/||x||, x = [(D - lambda_k I)^{-1} z; -1] (eq. Aeigenvec),
 *           so V[n-1, k] < 0.
 *   shift, mu: optional (null allowed); lambda_k = shift_k + mu_k exactly in
 *           real arithmetic, where shift_k is the pole the eigenvalue was
 *           computed from (Remark 3); this pair carries ~32 digits.
 *   info:   optional, n uint32 ARROW_INFO_* bits.
 * Reducible input (Sec. 1: some z_j = 0, or d_i = d_j) is deflated on the
 * device: a pole d_j with z_j = 0 is an eigenvalue with the unit vector e_j;
 * r > 1 equal poles with nonzero z are merged by rotations into one pole
 * with shaft (sum z^2)^(1/2), and the r - 1 directions the rotations remove
 * are eigenvectors for that pole: for the run's t-th nonzero member
 * (sorted order, ties in caller order), entries z_i z_t / (R_{t-1} R_t) on
 * the run's earlier rows and -R_{t-1}/R_t on its own row, R_t^2 = sum of
 * z_i^2 up to t.  These eigenpairs carry ARROW_INFO_DEFLATED, shift = the
 * pole, mu = 0.  The irreducible rest is solved as above, its vectors given
 * by eq. (Aeigenvec) on every row (0 where z_j = 0).  Columns are the merge
 * of both sets in descending order; on equal values the solved one first.
 */
int arrow_eig(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha,
              double* lambda, double* V, int64_t ldv, double* shift, double* mu, uint32_t* info);

/*
 * arrow_eig without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as arrow_eig, for
 * 1 <= n <= ARROW_NOALLOC_N_MAX (above it: -2).  Instead of the handle's
 * workspace it uses a scratch array in static device memory, 16 + 26
 * ARROW_NOALLOC_N_MAX doubles (6.5 MiB), which every device the library runs
 * on holds until the process ends; its address is looked up in arrow_create
 * (ARROW_ERR_HIP if that failed).  It calls no hipMalloc, hipFree or other
 * allocating routine.  The scratch is shared by every arrow_eig_noalloc call on
 * that device, through any handle: calls whose executions overlap on one
 * device (different streams, or different host threads) race and give wrong
 * results; calls ordered on one stream are safe.  Each call's kernels set up
 * every scratch word they read (the last call's contents stay behind).
 */
#define ARROW_NOALLOC_N_MAX 32768
int arrow_eig_noalloc(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha,
                      double* lambda, double* V, int64_t ldv, double* shift, double* mu, uint32_t* info);

/*
 * Eigen-decomposition of the Hermitian arrowhead C = [ diag(d)  z ; z^*  alpha ]
 * (Sec. 6.1) of order n >= 1: d real (n-1), z complex (n-1 (re, im) pairs of
 * doubles, any order; 8-byte aligned), alpha real.  Solved as the real
 * arrowhead Phi^* C Phi = [D |z|; |z|^T alpha], Phi = diag(z_j/|z_j|, 1), with
 * |z_j|^2 formed in double-double; u = Phi v.
 *   lambda: n eigenvalues, descending.
 *   U:      n x n complex eigenvectors as (re, im) pairs, column-major with
 *           leading dimension ldu >= n counted in complex entries, 16-byte
 *           aligned (a complex128 array), or null.  u_k = x/||x||,
 *           x = [(D - lambda_k I)^{-1} z; -1], so U[n-1, k] is real and < 0.
 *   shift, mu, info: as for arrow_eig.  Reducible input (some z_j = 0 or
 *           d_i = d_j) is reported (ARROW_INFO_REDUCIBLE, outputs NaN), not deflated.
 */
int arrow_eig_herm(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha,
                   double* lambda, double* U, int64_t ldu, double* shift, double* mu, uint32_t* info);

/*
 * Eigen-decomposition of the real symmetric DPR1 matrix M = diag(d) + rho u u^T
 * (Sec. 6.3) of order n >= 1, rho != 0.  d, u: n entries, any order; d distinct,
 * u_j != 0 (else info reports REDUCIBLE).  rho < 0 is solved as the negation of
 * (-D) + |rho| u u^T (the reduction of Sec. 6.3 needs rho > 0; the closing
 * remark of Sec. 6 names D - u u^T as the case it does not cover).
 *   lambda: n eigenvalues, descending.
 *   Q:      n x n eigenvectors (ldq >= n) or null; q_k = x/||x||,
 *           x = (D - lambda_k I)^{-1} u, for either sign of rho.
 *   info:   optional.
 */
int dpr1_eig(arrow_handle_t h, int64_t n, const double* d, const double* u, double rho,
             double* lambda, double* Q, int64_t ldq, uint32_t* info);

/*
 * Singular value decomposition B = U Sigma V^T of the upper-triangular
 * arrowhead B = [ diag(d)  z ; 0  alpha ] of order n >= 1 (Sec. 6.2).
 * d: n-1 nonzero entries with distinct |d_j|; z: n-1 nonzero entries.
 *   sigma: n singular values, descending.
 *   U, V:  n x n (ldu, ldv >= n) or null.  v_k is the eigenvector of the
 *          arrowhead B^T B with V[n-1, k] < 0; u_k = B v_k / sigma_k.
 *   info:  optional.
 */
int arrow_svd(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha,
              double* sigma, double* U, int64_t ldu, double* V, int64_t ldv, uint32_t* info);

/*
 * Eigen-decomposition of the symmetric tridiagonal T = tridiag(b, a, b) of
 * order 1 <= n <= 46340 by divide and conquer, each merge a DPR1 eigenproblem
 * solved by the accurate method (Sec. 1 names the arrowhead/DPR1 problem as
 * the merge step of divide-and-conquer solvers).  T is torn at every
 * off-diagonal (T = diag(T1', T2') + b_k v v^T, the tearing of Cuppen's
 * method) down to 1x1 blocks; a level's merges
 * diag(L1, L2) + b_k u u^T, u = [last row of Q1; first row of Q2], run as one
 * batched DPR1 plan (either sign of b_k; b_k = 0 merges two sorted lists), and
 * Q = diag(Q1, Q2) Qh as FP64 GEMMs (rocBLAS).
 *   a: n diagonal entries, b: n-1 off-diagonal entries (device).
 *   lambda: n eigenvalues, descending.  Q: n x n (ldq >= n), column k the
 *   eigenvector of lambda_k (sign as produced by the merges).
 *   info: optional, n words: the top merge's ARROW_INFO_* bits (a merge that
 *   is reducible, e.g. exactly equal eigenvalues of two halves, is reported
 *   there and its outputs are NaN).
 * Synchronous: it reads b to the host to plan the tree, keeps its device
 * buffers (about 4 n^2 doubles) in the handle, grown on demand, and waits for
 * the handle's stream before returning.
 */
int tridiag_eig(arrow_handle_t h, int64_t n, const double* a, const double* b, double* lambda, double* Q,
                int64_t ldq, uint32_t* info);

/* ------------------------------------------------------------------------
 * Batched solves: many independent problems of uneven order in one plan.
 *
 * Each problem is described by offsets (counted in elements) into three
 * caller-owned device pools.  Vector outputs of a problem are column-major
 * with leading dimension n.  Problems are independent: each one's results are
 * the same whether it is solved alone or inside any batch (same order n gives
 * the same schedule).
 */
#define ARROW_KIND_ARROW 0   /* arrowhead: d, z (n-1 each), scalar = alpha */
#define ARROW_KIND_DPR1 1    /* diag(d) + rho u u^T: d, u (n each), scalar = rho != 0 */
#define ARROW_KIND_SVD 2     /* triangular arrowhead SVD: d, z (n-1 each), scalar = alpha */
#define ARROW_KIND_HERM 3    /* Hermitian arrowhead: d (n-1), z (n-1 complex = 2(n-1) doubles as
                                (re, im) pairs), scalar = alpha; vectors complex (2n^2 doubles,
                                vec_off must leave them 16-byte aligned) */

typedef struct {
  int32_t kind;       /* ARROW_KIND_* */
  int32_t n;          /* matrix order, 1 <= n <= 46340 */
  int64_t d_off;      /* in_pool offset of d */
  int64_t z_off;      /* in_pool offset of z (DPR1: u) */
  double scalar;      /* alpha, or rho for DPR1 */
  int64_t lam_off;    /* out_pool offset of the n eigenvalues (SVD: singular values) */
  int64_t vec_off;    /* out_pool offset of the n x n vectors (V, Q, or SVD right vectors), -1: none */
  int64_t left_off;   /* SVD: out_pool offset of the n x n left vectors U, -1: none */
  int64_t info_off;   /* info_pool offset of n uint32 ARROW_INFO_* words, -1: none */
} arrow_desc_t;

typedef struct arrow_batch_s* arrow_batch_t;

#define ARROW_BATCH_GRAPH 1   /* capture the plan's launches in a HIP graph on its first run */
#define ARROW_BATCH_TIMING 2  /* (without ARROW_BATCH_GRAPH) every run stamps HIP events at the start and end
                                 of each of its five kernels, by the kernels' own dispatches */

/* Device bytes a plan for these problems needs (descriptor tables + per-problem workspace). */
size_t arrow_batch_workspace_size(int64_t count, const arrow_desc_t* descs);

/*
 * Build a plan for `count` problems described by the HOST array `descs`.
 * in_pool, out_pool, info_pool: device pools the offsets refer to (info_pool
 * may be null when no problem asks for info).  workspace: device memory of at
 * least arrow_batch_workspace_size bytes owned by the caller, or null to let
 * the plan allocate (and free) its own.  The plan records the handle's options
 * (ARROW_OPT_*) and lanes table as they are at creation: later
 * arrow_set_option calls change neither its eager nor its graph runs.  Each
 * arrow_batch_run launches on the handle's stream as set at that call; the
 * descriptor tables are copied to the device on the handle's stream.
 * Invalid descriptors fail with -3.
 */
int arrow_batch_create(arrow_handle_t h, int64_t count, const arrow_desc_t* descs, const double* in_pool,
                       double* out_pool, uint32_t* info_pool, void* workspace, size_t workspace_bytes, int flags,
                       arrow_batch_t* plan);

/* Launch the plan on the handle's stream (asynchronous).  Can be run again. */
int arrow_batch_run(arrow_batch_t plan);

/* Synchronise the handle's stream and free the plan (and its own workspace). */
int arrow_batch_destroy(arrow_batch_t plan);

/*
 * Diagnostics of a plan.
 *
 * arrow_batch_timing: ms[0..4] receive the durations (milliseconds) of the five
 *   kernels of the plan's latest run -- prologue (sort, weights, corner), root
 *   stage (shift, b, root of the inverse, for every eigenvalue), check stage
 *   (K_nu, norms, the repair list), repairs, vectors -- from the events their
 *   dispatches stamped (ARROW_BATCH_TIMING).  Waits for that run.
 *   ARROW_ERR_STATE when the plan has no timed run.
 * arrow_batch_counters: out[0..5] receive, summed over all problems p, m_p times
 *   the bisection (or rational) steps, double-double O(n) passes and plain O(n)
 *   passes of the root stage (out[0..2]) and of the check stage and repairs
 *   (out[3..5]) over the eigenvalues of p, m_p being the number of poles a pass
 *   of p visits; out[6] = sum of the orders.  So out[c] counts pole terms.
 *   Reads the counters of the plan's latest run (synchronises the stream;
 *   allocates and frees a small device buffer).
 */
int arrow_batch_timing(arrow_batch_t plan, double* ms);
int arrow_batch_counters(arrow_batch_t plan, double* out);

/* The same problems solved one after another with the single-problem entry
 * points (one launch sequence per problem, on the handle's stream, sharing the
 * handle's workspace): the reference the batched plan is measured against. */
int arrow_solve_sequential(arrow_handle_t h, int64_t count, const arrow_desc_t* descs, const double* in_pool,
                           double* out_pool, uint32_t* info_pool);

/* create + run + destroy; returns after the solve has finished. */
int arrow_solve_batched(arrow_handle_t h, int64_t count, const arrow_desc_t* descs, const double* in_pool,
                        double* out_pool, uint32_t* info_pool);

/*
 * Schedule: how many lanes of a 64-lane wavefront cooperate on one eigenvalue
 * (64: a wavefront per eigenvalue; fewer: 64/lanes eigenvalues share one
 * wavefront and its loads of the pole data) for problems of order
 * n <= n_max[e] (first matching entry; n_max strictly increasing, >= 1; at
 * most 16 entries).  Results differ between lane counts only in rounding.
 *
 *   scope ARROW_SCHEDULE_SINGLE: arrow_eig / dpr1_eig / arrow_svd calls;
 *     lanes 1, 2, 4, ..., 64.  n beyond the table and entries = 0 use the
 *     built-in rule (about 8 pole terms per lane, at most 64 lanes).  The
 *     option ARROW_OPT_LANES, when nonzero, overrides the table.
 *   scope ARROW_SCHEDULE_BATCH: plans created afterwards; lanes 4, ..., 64;
 *     n beyond the table uses 64; entries = 0 restores the built-in table
 *     {24: 4, 48: 8, 96: 16, 192: 32, larger: 64}.
 *
 * The package's autotuner measures these tables on the device and the Python
 * binding loads its result into every handle it creates.
 * Returns 0, or -1 bad handle, -2 bad scope, -3 bad entries, -4 bad n_max,
 * -5 bad lanes (the handle is unchanged on error).
 */
#define ARROW_SCHEDULE_SINGLE 0
#define ARROW_SCHEDULE_BATCH 1
int arrow_set_lanes_table(arrow_handle_t h, int scope, int32_t entries, const int32_t* n_max, const int32_t* lanes);

/*
 * Diagnostics of the most recent single-problem call on this handle.
 *
 * arrow_last_timing: ms[0..4] receive the elapsed times (milliseconds, from
 *   HIP events on the handle's stream) of the stages front (sortedness check;
 *   for input already in decreasing order also the copy and the shaft weights
 *   and corner), sort (input not in that order: rank sort, copy, weights and
 *   corner), root (shift, b, root of the inverse), check (K_nu, repairs, norm)
 *   and vectors.  The events are stamped by the kernels' own dispatches (no
 *   marker packets between launches): root and vectors are their kernels'
 *   durations, front and sort run from one kernel's start to the next one's,
 *   check from the end of the root kernel to the start of the vector kernel,
 *   so the five sum to the whole call.  Needs ARROW_OPT_TIMING set before that
 *   call; waits for it to finish.  Returns ARROW_ERR_STATE when no timed call
 *   exists.
 * arrow_timing_of: the same for the most recent timed call (age 0) or the one
 *   before it (age 1): the handle keeps the stage events of two timed calls, so
 *   a caller can read a call's stages after queuing the next one without
 *   draining the stream.  -3 for another age; ARROW_ERR_STATE when fewer than
 *   age + 1 timed calls were made.
 * arrow_last_counters: out[0..6] receive, summed over all eigenvalues, the
 *   bisection steps, double-double O(n) passes and plain O(n) passes executed
 *   by the root stage (out[0..2]) and by the check stage (out[3..5]), and the
 *   matrix order n (out[6]; a pass visits the n-1 poles, n for DPR1 norms).
 *   Synchronises the stream and copies 24 n bytes to the host.
 */
/*
 * arrow_conditions: the condition numbers of the most recent single-problem
 * call on this handle (arrow_eig, arrow_eig_noalloc, arrow_eig_herm, dpr1_eig,
 * arrow_svd), per output column: kb[k] = K_b (Sec. 3, eq. (K2)) of the element
 * b at the shift the first pass chose for the k-th eigenvalue, knu[k] = K_nu
 * (eq. (K0)), the test that decides the Remark 2 remedies.  kb, knu: device
 * arrays of n doubles, either may be null; NaN where a value was not
 * evaluated (n = 1, remedies off, deflated or unsolved eigenpairs).  Copied on
 * the handle's stream (asynchronous); call it before the handle's next solve,
 * which reuses the workspace they are kept in.  ARROW_ERR_STATE: no call yet.
 */
int arrow_conditions(arrow_handle_t h, double* kb, double* knu);

int arrow_last_timing(arrow_handle_t h, double* ms);
int arrow_timing_of(arrow_handle_t h, int age, double* ms);
int arrow_last_counters(arrow_handle_t h, int64_t* out);

/*
 * Calibration kernels (not part of the solve): the rates the device sustains
 * for the resources the solver is bound by, measured by the caller around
 * these asynchronous launches on `stream` (a hipStream_t passed as void*).
 *
 * arrow_probe_fma:  blocks x 256 threads, each running 8 independent chains of
 *   `iters` dependent FP64 FMAs (16 * iters FP64 flops per thread); writes one
 *   double per thread to out[0 .. blocks*256) (device memory, caller-owned).
 *   Returns -1 out null, -2 blocks outside [1, 2^24], -3 iters < 1.
 * arrow_probe_fill: streams `bytes` (a positive multiple of 16) of copies of
 *   `value` to dst (16-byte aligned device memory) with 16-byte non-temporal
 *   stores.  Returns -1 bad dst, -2 bad bytes.
 * arrow_probe_copy: copies `bytes` (a positive multiple of 16) from src to dst
 *   (16-byte aligned, not overlapping) with 16-byte loads and stores: a plain
 *   copy of known size, to scale hardware traffic counters.  Returns -1 bad
 *   dst, -2 bad src, -3 bad bytes.
 * arrow_probe_rcp: the solver's three reciprocals of x[0 .. n) (device memory,
 *   finite, nonzero, in the normal range): out[i] the hardware estimate alone,
 *   out[n + i] after one Newton step, out[2n + i] after two (out: 3n doubles,
 *   device memory, caller-owned).  Their accuracy is what the solver's choice
 *   of reciprocal per pass relies on.  Returns -1 x null, -2 out null, -3 n < 1.
 * All return ARROW_ERR_HIP if the launch fails.
 */
int arrow_probe_fma(double* out, int64_t blocks, int iters, void* stream);
int arrow_probe_fill(double* dst, int64_t bytes, double value, void* stream);
int arrow_probe_copy(double* dst, const double* src, int64_t bytes, void* stream);
int arrow_probe_rcp(const double* x, double* out, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ARROW_H */
