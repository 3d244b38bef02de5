/*
 * fracctl -- rank-truncated preconditioned CG for the fractional control
 * equation on MI355X (gfx950).
 *
 * Problem (paper Section 3.1, control equation after eliminating state and
 * adjoint, finite differences so the mass matrix is the identity):
 *
 *     (beta A^-alpha + (gamma/beta) A^alpha) u = y,
 *     A = A_1 (x) I (x) I + I (x) A_2 (x) I + I (x) I (x) A_3        (Section 3.2)
 *
 * where A_l is the 1D finite-difference Sturm-Liouville matrix of
 * -d/dx a_l(x) d/dx with homogeneous Dirichlet conditions on n interior nodes,
 * h = 1/(n+1):  A_l = (1/h^2) tridiag(-a_{i-1/2}, a_{i-1/2}+a_{i+1/2}, -a_{i+1/2}).
 * The fractional powers are spectral (Section 2).  The solve runs in the
 * eigenbasis of the three A_l (Section 3.3, eqn. DiagKron3D): operator and
 * preconditioner are separable (low Kronecker rank) diagonal scalings there,
 * and the iteration is Algorithm 1 (Appendix 2) with a rank truncation after
 * every update (canonical-to-Tucker by reduced HOSVD, Appendix 1).
 *
 * Tensor layout at the boundary: a canonical tensor
 *     T = sum_s w[s] * U1[:,s] o U2[:,s] o U3[:,s]
 * is passed as three column-major n x rank FP64 factor matrices (leading
 * dimension n) and an FP64 weight vector.  Factor entries are the values at
 * the grid nodes x_i = i/(n+1), i = 1..n.  Outputs have unit-norm columns and
 * carry norms and signs in the weights.
 *
 * Memory: every pointer documented as DEVICE is a device (HBM) pointer owned
 * by the caller; HOST pointers are ordinary host memory.  The plan owns all
 * of its device state and workspace; fc_solve performs no device allocation.
 * Streams: `hip_stream` is a hipStream_t (NULL = the default stream); all
 * device work of a call is enqueued on it.  fc_setup_ex is the exception: a
 * NULL stream there means a private non-blocking stream that the setup
 * creates, and with any stream the plan is complete when it returns.  A plan
 * must not be used by two threads at once; distinct plans may run
 * concurrently on distinct streams, and plans may be built concurrently on
 * several threads.
 *
 * Errors: every entry point returns an fc_status; no exception crosses the
 * boundary.  fc_last_error() returns a thread-local text describing the last
 * failure.
 */
#ifndef FRACCTL_H
#define FRACCTL_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fc_plan_s* fc_plan;

typedef enum {
    FC_OK = 0,
    FC_ERR_INVALID_ARG = 1,   /* argument out of range; nothing was touched      */
    FC_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed (setup only)   */
    FC_ERR_NOT_CONVERGED = 3, /* max_iter reached; best iterate still written     */
    FC_ERR_RANK_OVERFLOW = 4, /* result rank exceeds cap_u (*rank_u = required)   */
    FC_ERR_NUMERIC = 5,       /* NaN/Inf met, or a setup accuracy gate failed     */
    FC_ERR_HIP = 6,           /* a HIP runtime call failed                        */
    FC_ERR_INTERNAL = 7       /* internal capacity exceeded (Tucker rank > max)   */
} fc_status;

/* FC_FP64: every operation in FP64.  FC_MIXED_FP32: outer FP64 iterative
 * refinement of the true residual around an inner PCG whose bulk
 * contractions (the Hadamard truncation's projections and core
 * contractions) run on the FP32 matrix cores with FP32 accumulation; Grams,
 * eigensolves, the short sums' projections, PCG scalars and the refinement
 * residual stay FP64.  Stop rule of the mixed path: the refinement sweeps
 * end when an error estimate, the preconditioned residual ratio
 * ||D~_p (.) R|| / ||D~_p (.) B|| (formed to two digits), is <= tol; if it
 * stops falling by half from one sweep to the next, the solve ends and counts
 * as converged when the estimate is <= 3 tol (else FC_ERR_NOT_CONVERGED).
 * The FP64 Euclidean residual ||R|| / ||Y|| of the last sweep is reported in
 * fc_info.rel_residual. */
typedef enum { FC_FP64 = 0, FC_MIXED_FP32 = 1 } fc_precision;

/* Preconditioner (Section 3.5).
 * FC_PRECOND_EIGEN (case (B)): D~_p ~ 1/f(lambda1 + lambda2 + lambda3) in the
 *   eigenbasis of the variable-coefficient matrices, no transforms.
 * FC_PRECOND_LAPLACE (case (A)): P = (beta B^-alpha + (gamma/beta) B^alpha)^-1
 *   (eqn Precond_var) for the constant-coefficient anisotropic Laplacian
 *   B = sum_l b0_l Delta_l (eqn PrecClassA), diagonal in the sine (DST-I)
 *   basis (eqn DiagLaplace) with entries 1/f(b0_1 mu_i + b0_2 mu_j + b0_3 mu_k),
 *   mu_k = (4/h^2) sin^2(k pi h/2).  Each application maps the iterate's
 *   factors from the eigenbasis of A_l to the sine basis with the dense
 *   orthogonal W_l = S V_l (S the orthonormal DST-I matrix, formed at setup),
 *   applies the separable symbol there and maps back with W_l^T.  b0_l = 1 in
 *   every mode is the classical Laplacian of the paper's 3D tests (Section 4). */
typedef enum { FC_PRECOND_EIGEN = 0, FC_PRECOND_LAPLACE = 1 } fc_precond_kind;

/* Setup parameters.  Zero-valued optional fields select the defaults. */
typedef struct {
    int n;                  /* interior nodes per mode, 2 <= n <= 4096                        */
    const double* a[3];     /* HOST: n+1 samples a_l((i+1/2)/(n+1)), i = 0..n, finite, > 0      */
    double alpha;           /* 0 <= alpha <= 1                                                 */
    double beta, gamma;     /* > 0                                                             */
    double eps;             /* truncation threshold, 0 < eps < 1 (paper: 1e-6)                 */
    double tol;             /* stop when ||R|| <= tol ||Y||; 0 -> eps                          */
    double op_accuracy;     /* entrywise relative accuracy of the operator; 0 -> eps           */
    int max_iter;           /* 0 -> 100                                                        */
    int max_rank;           /* Tucker rank capacity per mode; 0 -> 96, at most 128 (the small
                               eigenproblems of the truncations are at most 128 x 128)         */
    int precond_rank;       /* Kronecker rank of the preconditioner (the paper's tests use 6,
                               Section 4), at most 16; 0 -> automatic: the first of 6, 8, ...,
                               16 whose fit of 1/f reaches a relative error of 1e-3 (else the
                               best)                                                          */
    fc_precision precision; /* FC_FP64 or FC_MIXED_FP32                                        */
    fc_precond_kind precond; /* FC_PRECOND_EIGEN (0, default) or FC_PRECOND_LAPLACE             */
    double precond_b0[3];   /* case (A) constants b0_l; <= 0 -> (max a_l + min a_l)/2 over the
                               samples (eqn modcoeff); finite                                  */
    int dims;               /* 3 (or 0) or 2: the d = 2 problem on (0,1)^2 (a[2] ignored), solved
                               with fc_solve2d.  The plan then carries a third mode A_3 - sigma I
                               (A_3 the Laplacian, sigma its smallest eigenvalue, so the third
                               eigenvalues start at exactly 0) and every tensor is u (x) v_1 with
                               v_1 the first eigenvector: the Tucker truncation of such a tensor
                               is the reduced SVD truncation of the matrix u (Section 3.6).    */
} fc_setup_params;

/* Per-solve report (HOST struct). */
typedef struct {
    int iterations;         /* PCG iterations taken (Algorithm 1 loop count, all sweeps)       */
    int refinements;        /* outer refinement sweeps (FC_MIXED_FP32), else 0                 */
    int rank_u;             /* canonical rank of the result                                    */
    int tucker_rank[3];     /* Tucker rank of the final iterate                                */
    int max_tucker_rank;    /* largest Tucker rank met during the iteration                    */
    int op_rank;            /* Kronecker rank of the operator                                  */
    int precond_rank;       /* Kronecker rank of the preconditioner                            */
    double rel_residual;    /* ||R|| / ||Y|| of the recursively updated residual at exit       */
    double op_max_rel_err;  /* max over the spectrum of |D~/D - 1| (setup gate value)          */
    double precond_max_rel_err; /* max over the preconditioner's spectrum (of A, case (B); of B,
                                   case (A)) of |D~_p f - 1|                                   */
    int state_rank;         /* Kronecker rank of the state map beta A^-alpha                   */
    double state_max_rel_err; /* max over the spectrum of its relative error (setup gate)      */
    double subspace_miss;   /* largest, over the Hadamard truncations of the solve, ratio of the
                               energy their mode subspaces miss (twice an estimate from 8 rank-1
                               Gaussian probes; charged to the truncation's budget) to that
                               truncation's error budget: below 1 the error bound holds       */
} fc_info;

/* Plan with gamma = 1, FP64 and defaults; see fc_setup_ex.  a1..a3 are HOST. */
fc_status fc_setup(int n, const double* a1, const double* a2, const double* a3,
                   double alpha, double beta, double eps, fc_plan* out);

/* Build a plan (paper Sections 3.2-3.5), on the device: the three 1D FD
 * matrices (host, O(n)), their eigenpairs (divide and conquer on the
 * device), the separable operator D~ ~ f(lambda1+lambda2+lambda3),
 * f(s) = beta s^-alpha + (gamma/beta) s^alpha, the state map and the
 * preconditioner (case (B): D~_p ~ 1/f in the same eigenbasis; case (A):
 * 1/f on the spectrum of the anisotropic Laplacian in the sine basis, see
 * fc_precond_kind), all as exponential sums with positive weights (Section
 * 3.4: nonnegative least squares on a geometric node grid for the operator
 * and the state map, free nodes for the preconditioner), fitted by one
 * workgroup per candidate grid or rank on the device; then the factors
 * exp(-t lambda) on the device, the solve workspace and the autotuner's
 * launch choices.  The device work runs on hip_stream, or on a private
 * non-blocking stream when it is NULL (so that setups on several threads do
 * not serialise on the default stream); the stream is synchronised before
 * the call returns.  Fails with FC_ERR_NUMERIC if the operator misses
 * op_accuracy anywhere on [s_min, s_max] or a separable factor is not
 * positive. */
fc_status fc_setup_ex(const fc_setup_params* p, void* hip_stream, fc_plan* out);

/* Solve F(A) u = y for one design function given in canonical format.
 *   rank_y            number of terms of y, 1 <= rank_y <= 256
 *   w_y               DEVICE, rank_y weights, or NULL for all ones
 *   Y1, Y2, Y3        DEVICE, n x rank_y column-major factors of y
 *   cap_u             capacity (columns) of the output buffers
 *   rank_u            HOST out: rank of u (on FC_ERR_RANK_OVERFLOW: the required rank)
 *   w_u               DEVICE out: cap_u weights
 *   U1, U2, U3        DEVICE out: n x cap_u column-major unit-norm factors
 *   info              HOST out, may be NULL
 * Synchronises the stream before returning (ranks are read on the host).
 * Algorithm 1 of the paper with X0 = 0, trunc = reduced-HOSVD
 * canonical-to-Tucker after every update, and the Tucker-to-canonical
 * transform of the final iterate (Appendix 1). */
fc_status fc_solve(fc_plan plan, int rank_y, const double* w_y,
                   const double* Y1, const double* Y2, const double* Y3,
                   int cap_u, int* rank_u, double* w_u, double* U1, double* U2, double* U3,
                   fc_info* info, void* hip_stream);

/* The d = 2 problem (Section 2 with d = 2, the 2D tests of Section 4): plan
 * built with dims = 2.  y = sum_s w_y[s] Y1[:, s] Y2[:, s]^T, u returned as
 * sum_k w_u[k] U1[:, k] U2[:, k]^T; arguments, ranks, synchronisation and
 * errors as fc_solve (rank_u <= max_rank).  FC_ERR_INVALID_ARG if the plan
 * is three-dimensional (and fc_solve, fc_solve_state reject d = 2 plans). */
fc_status fc_solve2d(fc_plan plan, int rank_y, const double* w_y, const double* Y1,
                     const double* Y2, int cap_u, int* rank_u, double* w_u, double* U1,
                     double* U2, fc_info* info, void* hip_stream);

/* fc_solve, then the state y = beta A^-alpha u (eqn `State`, Section 3.1) and
 * the cost functional J = 1/2 ||y - y_Omega||^2 + gamma/2 ||u||^2 (Section 3.1
 * with the finite-difference mass matrix M = I, Euclidean norms).  The state
 * is the Hadamard product of the Tucker solution with the separable state
 * map (an exponential sum for beta s^-alpha, gated like the operator),
 * truncated to relative accuracy eps, then converted to canonical format and
 * transformed to the grid like u.  J is evaluated from exact Tucker inner
 * products of y, u and the design in eigen-coordinates.
 *   cap_s, rank_s, w_s, S1..S3   as cap_u, rank_u, w_u, U1..U3, for y
 *   J                            HOST out, may be NULL
 * Other arguments, synchronisation and errors as fc_solve; FC_ERR_RANK_OVERFLOW
 * when either output exceeds its capacity. */
fc_status fc_solve_state(fc_plan plan, int rank_y, const double* w_y, const double* Y1,
                         const double* Y2, const double* Y3, int cap_u, int* rank_u, double* w_u,
                         double* U1, double* U2, double* U3, int cap_s, int* rank_s, double* w_s,
                         double* S1, double* S2, double* S3, double* J, fc_info* info,
                         void* hip_stream);

/* Solve a batch of independent problems, one plan per problem (plans may
 * differ in n and alpha).  Arrays are HOST arrays of length `count`; the
 * per-problem pointers follow fc_solve.  status[i] receives each problem's
 * own status; the return value is FC_OK if every problem succeeded, else the
 * first failing status.  Problems run concurrently: worker threads (16, or
 * the environment variable FC_BATCH_STREAMS, at most 64) each solve on a
 * stream of their own after the given stream's pending work; the call
 * returns when all are done.  The workers and their streams are created by
 * the first batched call on a device and kept for the process; batched calls
 * made at the same time on one device run one after the other.  The HIP
 * runtime maps streams onto GPU_MAX_HW_QUEUES hardware queues
 * (4 unless set before the runtime starts), which bounds the concurrency.
 * Plans built with dims = 2 are solved as by fc_solve2d: their Y3[i] and
 * U3[i] are not used (the arrays must still have `count` entries; those
 * entries may be NULL). */
fc_status fc_solve_batched(int count, const fc_plan* plans, const int* rank_y,
                           const double* const* w_y, const double* const* Y1,
                           const double* const* Y2, const double* const* Y3,
                           const int* cap_u, int* rank_u, double* const* w_u,
                           double* const* U1, double* const* U2, double* const* U3,
                           fc_status* status, fc_info* info, void* hip_stream);

/* Release every resource of a plan (NULL is allowed). */
void fc_destroy(fc_plan plan);

/* Plan introspection (HOST outputs).  lam: 3*n ascending eigenvalues, mode
 * after mode (d = 2: the third mode's shifted ones, starting at 0); V (may be
 * NULL): 3 n x n column-major eigenvector matrices. */
fc_status fc_plan_spectrum(fc_plan plan, double* lam, double* V);

/* Separable factors of the operator (which = 0), the preconditioner
 * (which = 1) or the state map (which = 2) in eigen-coordinates: *rank terms, w (HOST, capacity cap) and
 * F (HOST, 3 consecutive n x cap column-major matrices, may be NULL).  For
 * FC_PRECOND_LAPLACE the preconditioner's rows are indexed by the sine mode k
 * (ascending mu_k), not by the eigenpairs of A_l. */
fc_status fc_plan_separable(fc_plan plan, int which, int cap, int* rank, double* w, double* F);

/* Launch choices the autotuner picked for the plan at setup (per device, n
 * and operator rank; kept in a disk cache, environment FC_TUNE_CACHE, else
 * $HOME/.cache/fracctl/tune_v2.txt; FC_TUNE=0 keeps the defaults).  HOST
 * outputs: choices[0..5] = wavefronts per workgroup of the Gram kernel for
 * batched and for single products (8 or 16), of the fused Kronecker
 * application (8 or 16), K chunk of the streaming transform kernel (128 or
 * 256), Gram-Schmidt panel width (8 or 16), 1 if tuned; us (may be NULL):
 * the measured times of the ten candidates (us; two per choice, in that
 * order, the panel widths per orthonormalisation of three n x 96 blocks). */
fc_status fc_plan_tuning(fc_plan plan, int* choices, double* us);

/* ---- building blocks of the path, exposed for testing (DEVICE buffers) ---- */

/* Mode transform (Section 3.3): out = V_l^T X (transpose = 1, into
 * eigen-coordinates) or out = V_l X (transpose = 0, back to the grid), X and
 * out n x m column-major.  On the plan's eigenbasis of mode l. */
fc_status fc_mode_transform(fc_plan plan, int mode, int transpose, int m,
                            const double* X, double* out, void* hip_stream);

/* Canonical scalar product (Appendix 1): <A, B> = sum_k sum_m wa_k wb_m
 * prod_l <A_l[:,k], B_l[:,m]>, A_l n x ra, B_l n x rb (DEVICE), result to
 * HOST *out.  wa/wb may be NULL (ones). */
fc_status fc_cp_inner(fc_plan plan, int ra, const double* wa, const double* A1, const double* A2,
                      const double* A3, int rb, const double* wb, const double* B1,
                      const double* B2, const double* B3, double* out, void* hip_stream);

/* fc_cp_inner for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no plan, no allocation, no host synchronisation.
 *   n                 rows of every factor (n >= 1)
 *   ra, wa, A1..A3    as fc_cp_inner (DEVICE)
 *   rb, wb, B1..B3    as fc_cp_inner (DEVICE)
 *   out               DEVICE out: one double, <A, B>
 * The three cross Grams A_l^T B_l live in a file-scope device array of the
 * library (3 x 65536 doubles, 1.5 MiB per GPU, held until the process ends),
 * so ra * rb <= 65536; larger ranks return FC_ERR_INVALID_ARG and enqueue
 * nothing.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (different streams, or threads without ordering) race and give
 * wrong results.  The result is enqueued on hip_stream and is ready when the
 * stream reaches it.  The cross Grams run on the same kernels as
 * fc_cp_inner's, so the result is bit-identical to fc_cp_inner's. */
fc_status fc_cp_inner_noalloc(int n, int ra, const double* wa, const double* A1,
                              const double* A2, const double* A3, int rb, const double* wb,
                              const double* B1, const double* B2, const double* B3,
                              double* out, void* hip_stream);

/* Rank truncation of a canonical tensor (Appendix 1, C2T by reduced HOSVD
 * followed by the Tucker-to-canonical transform) to relative accuracy eps:
 * the result T' satisfies ||T - T'|| <= eps ||T|| (Euclidean norm).
 * Input as in fc_solve (DEVICE, rank m), output as in fc_solve. */
fc_status fc_cp_truncate(fc_plan plan, int m, const double* w, const double* X1,
                         const double* X2, const double* X3, double eps, int cap,
                         int* rank_out, double* w_out, double* O1, double* O2, double* O3,
                         void* hip_stream);

/* Apply the operator (which = 0), preconditioner (which = 1) or state map
 * (which = 2) to a canonical
 * tensor given in eigen-coordinates, with truncation to relative accuracy eps
 * (Section 3.3, eqn. Gen3DtimesX, evaluated in eigen-coordinates; for
 * FC_PRECOND_LAPLACE eqn Lap3DtimesX with the sine-basis maps W_l, W_l^T
 * around the separable symbol, result in eigen-coordinates).  DEVICE buffers
 * as in fc_cp_truncate.  Accuracy floor (this call, fc_cp_truncate and every
 * truncation of the solve): subspaces and ranks come from unfolding Grams,
 * which square the singular values, so relative accuracies below about 1e-8
 * are not resolved (eps = 1e-8 gives errors up to ~5e-8; eps >= 1e-7 is
 * met). */
fc_status fc_apply_separable(fc_plan plan, int which, int m, const double* w, const double* X1,
                             const double* X2, const double* X3, double eps, int cap,
                             int* rank_out, double* w_out, double* O1, double* O2, double* O3,
                             void* hip_stream);

/* ---- host-only helpers (no device needed), exposed for testing ---- */

/* Eigenpairs of the 1D FD matrix built from n+1 midpoint samples (HOST):
 * lam ascending (n), V column-major n x n (may be NULL). */
fc_status fc_host_fd_eigen(int n, const double* a_mid, double* lam, double* V);

/* Exponential sum sum_k c_k exp(-t_k s) fitted to target(s) with relative
 * accuracy on [s_min, s_max].  kind 0: target = s^-nu (nu = p1);
 * kind 1: target = 1/(p1 s^-p2 + p3 s^p2)  (preconditioner symbol 1/f);
 * kind 2: target = p1 s^(-p2-1) + p3 s^(p2-1)  (f(s)/s).
 * terms = K requested; on return t, c hold K values (HOST) and *max_rel_err
 * the maximum relative error on a dense logarithmic grid. */
fc_status fc_host_expsum(int kind, double p1, double p2, double p3, double s_min, double s_max,
                         int terms, double* t, double* c, double* max_rel_err);

/* Host-only construction of the setup phase (no device needed): the
 * eigenpairs (implicit QL) and the separable operator (which = 0),
 * preconditioner (which = 1) or state map (which = 2) by the fits that
 * fc_setup_ex runs on the device (the same algorithms, node grids, candidate
 * ranks and selection rules; results agree to rounding, which may move a
 * node of a nonnegative fit in or out of its active set), returned like
 * fc_plan_separable; *max_rel_err (may be NULL) receives the gate value
 * max over [s_min, s_max] of |D~/f - 1| (operator) or |D~_p f - 1|. */
fc_status fc_host_separable(const fc_setup_params* p, int which, int cap, int* rank, double* w,
                            double* F, double* max_rel_err);

/* Timing of the FP64 matrix-core GEMM kernel (the dominant kernel of the
 * path) for roofline reporting.  fc_profile_gemm(1) clears the counters and
 * brackets every subsequent GEMM launch of the library with a pair of HIP
 * events on its stream (inside fc_solve_batched: the launches of its first
 * worker stream only, a sample); fc_profile_gemm(0) stops recording.  The
 * event pool grows as needed and is kept, so a profiled warm-up run sizes it
 * for a later profiled run.
 * fc_profile_gemm_read waits for the recorded events and returns the launch
 * count, the summed kernel time (ms), and the algorithmic work of those
 * launches: 2 M N K flops and 8 (M K + K N + M N) bytes per GEMM.
 * Process-wide; not thread-safe; meant for benchmarks. */
fc_status fc_profile_gemm(int enable);
fc_status fc_profile_gemm_read(long* launches, double* total_ms, double* flops, double* bytes);

/* The same for one kernel family timed while fc_profile_gemm is on (HIP
 * events around each launch; algorithmic work as stated):
 *   kind 0  the short-reduction LDS-tiled GEMMs (2 M N K flops; operands
 *           read and the result written once, operands shared by a batch
 *           counted once)
 *   kind 1  the Gram-Schmidt panel kernel (16 n b bytes: its n x b panel
 *           read and written once; 4 n b^2 flops per two passes)
 *   kind 2  the symmetric eigensolver (16 k^2 bytes and (4/3 + 2) k^3 flops
 *           per matrix)
 *   kind 3  the mode transforms V^T Y, V Z (and case (A)'s sine-basis maps):
 *           8 (n^2 + 2 n m) bytes and 2 n^2 m flops per mode
 *   kind 4  the long-reduction Gram engine (Gram-type products, the scaled
 *           Grams Z^T diag(d) X of the Hadamard truncation, the core
 *           contractions over long reductions), counted as kind 0
 *   kind 5  the fused Kronecker application sum_q diag(D[:,q]) Z T^q:
 *           2 n p r Q flops; Z, D, T read and the n x p result written once
 * fc_profile_gemm_read returns kinds 0, 3, 4 and 5 together. */
fc_status fc_profile_kernel_read(int kind, long* launches, double* total_ms, double* flops,
                                 double* bytes);

/* Self-test of the matrix-core operand layouts: one 16x16x4 product of fixed
 * matrices on the FP64 matrix core (out[0..255], row-major) and on the FP32
 * matrix core (out[256..511]); 512 values written to HOST out.  Returns 0 on
 * success. */
int fc_selftest_mfma(double* host_out);

/* Self-test of the device symmetric eigensolver used by the truncations:
 * A_host is a k x k column-major symmetric matrix (k <= 128); eigenvalues
 * (descending) and eigenvectors (columns) are returned to host memory.
 * Returns 0 on success. */
int fc_selftest_eig(int k, const double* A_host, double* evals_host, double* V_host);

const char* fc_status_string(fc_status s);
const char* fc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FRACCTL_H */
