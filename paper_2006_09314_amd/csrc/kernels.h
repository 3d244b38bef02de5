// Device kernels of the fracctl library (gfx950).  All arithmetic is FP64.
#pragma once
#include <hip/hip_runtime.h>

namespace fc {

// C[b] = alpha * op(A[b]) * diag(d[b]) * op(B[b]) + beta * C[b]
// op(A) is M x K, op(B) is K x N, C is M x N; all column-major.
// Strides are in elements; a zero stride shares the operand across the batch.
// d (length K, may be null) scales the inner dimension.
// Two-level batch: entry b uses operand offsets (b / inner) * stride + (b % inner) * strideIn.
struct GemmArgs {
    int M = 0, N = 0, K = 0, batch = 1, inner = 1;
    double alpha = 1.0, beta = 0.0;
    const double* A = nullptr; long lda = 0, strideA = 0, strideAin = 0;
    const double* B = nullptr; long ldb = 0, strideB = 0, strideBin = 0;
    double* C = nullptr; long ldc = 0, strideC = 0, strideCin = 0;
    const double* d = nullptr; long strideD = 0;
    // split-K workspace: when few output tiles face a long reduction, K is
    // split over extra workgroups whose partial products land here and are
    // summed in a fixed order by a second kernel (deterministic).
    double* part = nullptr; long part_cap = 0;
    // FP32 matrix cores (operands rounded to FP32, FP32 accumulation, FP64
    // in and out) instead of FP64
    bool lowp = false;
};

hipError_t gemm(bool transA, bool transB, const GemmArgs& g, hipStream_t s);
// C = alpha op(A) diag(d) op(B) + beta C over a long reduction
// (op(A) op(B) = A^T B, A B^T or A B; batched over g.batch with strides, d
// advancing by strideD per batch entry; inner == 1, FP64): the Gram-type
// products of the truncations and the diagonally scaled Grams Z^T diag(d) X
// of the Hadamard truncation, one workgroup per 32 x 32 output tile.
// staged: the workgroup stages K chunks of both operands in LDS with
// coalesced loads (the next chunk fetched while the current one is used);
// direct: each wavefront loads its K slice straight into the matrix-core
// layout, with no barrier in the K loop.
// group (1, 2 or 4): batches of scaled Grams A^T diag(d_q) B with A and B
// shared by the batch (strideA = strideB = 0) run with that many terms per
// workgroup, their operand chunks staged once for the group (16 wavefronts
// take two terms at most); other products ignore it.
hipError_t gram(bool transA, bool transB, const GemmArgs& g, hipStream_t s, int waves = 16,
                bool staged = false, int group = 1);
// Up to kMaxGramJobs Gram-type products (each as in gram, batched or not) in
// one launch.
constexpr int kMaxGramJobs = 3;
struct GramJobs {
    int count = 0;
    GemmArgs g[kMaxGramJobs];
};
hipError_t gram_multi(bool transA, bool transB, const GramJobs& jobs, hipStream_t s,
                      int waves = 16, bool staged = false, int group = 1);
// Streaming products C = alpha op(A) op(B) + beta C over a long reduction
// with op(A) op(B) = A^T B (layout 0), A B^T (1) or A B (2), up to three
// jobs (of any sizes) in one launch on the FP64 matrix cores: the mode
// transforms (A an n x n eigenvector matrix, streamed once) and Gram-type
// products with few output tiles.  K is split into chunks of kc (128 or 256)
// values, one workgroup per chunk and 32-row block; with more than one
// chunk the partial tiles go to `part` (jobs x chunks x max M N doubles,
// part_cap available: stream_fits says whether they fit) and a second
// kernel adds them in chunk order.
struct StreamJob {
    int M = 0, N = 0, K = 0;
    double alpha = 1.0, beta = 0.0;
    const double* A = nullptr; long lda = 0;
    const double* B = nullptr; long ldb = 0;
    double* C = nullptr; long ldc = 0;
};
struct StreamJobs {
    int count = 0;
    StreamJob job[3];
};
hipError_t stream_multi(int layout, const StreamJobs& jobs, int kc, double* part, long part_cap,
                        hipStream_t s);
bool stream_fits(const StreamJobs& jobs, int kc, long part_cap);
// Up to three independent plain FP64 products C = alpha op(A) op(B) + beta C
// (strided or two-level batches, no scaling vector, whole K per block) in
// one launch on the matrix cores: 32 x 32 tiles, one wavefront each.
hipError_t gemm_multi(bool transA, bool transB, const GramJobs& jobs, hipStream_t s);

// out = sum_q diag(D[:, q]) Z T^q for up to three jobs in one launch (one
// per mode): Z n x r (ld ldz), D n x Q (ld n), T^q the r x p block at
// T + q r p (ld r), out n x p (ld ldo).  The row-wise Kronecker product
// Z (.) D is formed in registers (never stored); FP64 matrix cores.
struct KronJob {
    int r = 0, p = 0;
    const double* Z = nullptr; long ldz = 0;
    const double* D = nullptr;
    const double* T = nullptr;
    double* out = nullptr; long ldo = 0;
};
struct KronJobs {
    int count = 0;
    KronJob job[3];
};
hipError_t kron_apply_multi(int n, int Q, const KronJobs& jobs, hipStream_t s,
                            int waves = 16);

// Symmetric eigen-decomposition of a batch of k x k matrices (k <= 128),
// cyclic Jacobi with the matrix in LDS.  A (column-major, leading dimension
// lda, batch stride strideA) is read only.  Eigenvalues go to evals[b*k + i]
// in descending order, eigenvectors to V[b*strideV + i*ldv + j] (column i).
// scratch: batch * (k+1)^2 doubles of device memory.
hipError_t sym_eig(int k, int batch, const double* A, long lda, long strideA, double* evals,
                   double* V, long ldv, long strideV, double* scratch, hipStream_t s);

// Up to four independent eigenproblems of different sizes in one launch
// (Householder tridiagonalisation + bisection + inverse iteration).  Each job
// needs 6 k^2 doubles of device scratch.
struct EigJob {
    const double* A = nullptr; long lda = 0; int k = 0;
    double* evals = nullptr; double* V = nullptr; long ldv = 0; double* scratch = nullptr;
    // Eigenvectors wanted: all when budget < 0; else the first
    // min(max(numrank, 1), max(rr + margin, 1)), rr the smallest count whose
    // tail sum of positive eigenvalues is <= budget and numrank the count
    // above 1e-17 of the largest (the rank rule of the truncations, applied
    // to the same eigenvalues in the same order).  The other columns of V are
    // left as they are.
    double budget = -1.0; int margin = 0;
};
struct EigJobs {
    EigJob job[4];
    int count = 0;
    int kpmax = 0;
};
hipError_t sym_eig_multi(const EigJobs& jobs, hipStream_t s);

// Tucker-to-canonical term selection on the device: N candidate terms
// with energies sig2[e] (e = nu r1 + j); ordered by (energy, e) ascending,
// the smallest are dropped while the cumulative dropped energy is <= budget2.
// keep[t] (t < K) receives the kept term indices in descending order, *count
// (device int) K.  N <= kT2cMaxTerms; scratch: 12 * N_pad bytes (N_pad the
// next power of two) of device memory, used when N_pad > 8192.
constexpr int kT2cMaxTerms = 1 << 16;
hipError_t t2c_select(int N, const double* sig2, double budget2, void* scratch, int* keep,
                      int* count, hipStream_t s);
// The canonical factors of the K kept terms (see t2c_select): c0 r0 x K,
// c1 r1 x K, c2 r2 x K (column-major, ld r0, r1, r2) and the weights w (K),
// from the core (r0 x r1 x r2, r0 <= 128) and the slice-Gram eigenpairs
// (values ev[nu r1 + j], vectors as columns of the r1 x r1 blocks at
// V + nu r1 r1).
hipError_t t2c_coef(int r0, int r1, int r2, int K, const double* core, const double* V,
                    const double* ev, const int* keep, double* c0, double* c1, double* c2,
                    double* w, hipStream_t s);

// Probe sums of the projection check of the Hadamard truncation, for two
// problems y = 0, 1 and S probes t:
//   out[2 t + y] = sum_q sum_k U2_t[k, q] sum_j M_t[j + r1 k + r1 r2 q] U1_t[j, q]
// with M_t at M + t mstride, U1_t (r1 x Q) at U1 + t r1 Q, U2_t (r2 x Q) at
// U2 + t r2 Q, r1 <= 128.
struct ProbeSum {
    int r1 = 0, r2 = 0, Q = 0;
    const double* M = nullptr; long mstride = 0;
    const double* U1 = nullptr;
    const double* U2 = nullptr;
};
struct ProbeSums {
    ProbeSum p[2];
    double* out = nullptr;
};
hipError_t probe_sums(const ProbeSums& a, int S, hipStream_t s);

// E[i + n*(j + r*c)] = Z[i + ldz*j] * X[i + ldx*c]   (row-wise Kronecker product)
hipError_t rowkron(int n, int r, int p, const double* Z, long ldz, const double* X, long ldx,
                   double* E, hipStream_t s);
// out[i + ldo*c] = sum_j Z[i + ldz*j] * F[i + n*(j + r*c)]   (row-wise contraction)
hipError_t rowcontract(int n, int r, int p, const double* Z, long ldz, const double* F,
                       double* out, long ldo, hipStream_t s);

// Up to three row-wise Kronecker products (out = E of rowkron, X the right
// factor) or row-wise contractions (X = F, out the n x p result, ld ldo) in
// one launch.
struct RowJob {
    int r = 0, p = 0;
    const double* Z = nullptr; long ldz = 0;
    const double* X = nullptr; long ldx = 0;
    double* out = nullptr; long ldo = 0;
};
struct RowJobs {
    int count = 0;
    RowJob job[3];
};
hipError_t rowkron_multi(int n, const RowJobs& jobs, hipStream_t s);
hipError_t rowcontract_multi(int n, const RowJobs& jobs, hipStream_t s);

// dst = permutation of a dense r0 x r1 x r2 column-major core that brings
// mode `mode` first: mode 0 -> identity copy, mode 1 -> (r1, r0, r2),
// mode 2 -> (r2, r0, r1).  Batched with strides.
hipError_t permute_core(int r0, int r1, int r2, int mode, int batch, const double* src,
                        long sstride, double* dst, long dstride, hipStream_t s);
// the mode-1 and mode-2 permutations of one core (into dst1, dst2) in one launch
hipError_t permute_core12(int r0, int r1, int r2, const double* src, double* dst1, double* dst2,
                          hipStream_t s);

// y[i] = a * x[i] (+ y[i] if accumulate)
hipError_t axpby(long n, double a, const double* x, double b, double* y, hipStream_t s);
// out[0] = x . y for a long vector in one launch: 256-thread partial sums in
// up to 256 blocks (part: 256 doubles of scratch), summed in block order by
// the last block to finish.  count: one unsigned that is zero before the call
// and is zero again after it (calls sharing it must not overlap).
hipError_t dot_long(long n, const double* x, const double* y, double* part, unsigned* count,
                    double* out, hipStream_t s);
// X[:, c] *= scale[c] (or /= if divide) for an n x m column-major matrix
hipError_t scale_cols(int n, int m, double* X, long ldx, const double* scale, int divide,
                      hipStream_t s);
// fill up to three vectors with deterministic pseudo-random normal-like
// sequences (counter hash of the seed and the index) in one launch
struct FillJob {
    long n = 0;
    unsigned seed = 0;
    double* x = nullptr;
};
struct FillJobs {
    int count = 0;
    FillJob job[3];
};
hipError_t fill_random_multi(const FillJobs& jobs, hipStream_t s);
// out[:, j] = v for j < m (out n x m, leading dimension ld).
hipError_t fill_columns(int n, int m, const double* v, double* out, long ld, hipStream_t s);
// w[k] *= <U[:, k], v> for k < K (U n x K, leading dimension ld).
hipError_t scale_by_dot(int n, int K, const double* U, long ld, const double* v, double* w,
                        hipStream_t s);
// Scale the columns of the three n x K factors (ld) to unit length and
// multiply w[t] by the product of the three column norms.
hipError_t normalize_factors(int n, int K, double* U0, double* U1, double* U2, long ld, double* w,
                             hipStream_t s);
// copy a column-major m x n block
hipError_t copy2d(int rows, int cols, const double* src, long lds, double* dst, long ldd,
                  hipStream_t s);
// Up to kMaxCopyJobs column-major block copies in one launch.
constexpr int kMaxCopyJobs = 12;
struct CopyJob {
    const double* src = nullptr; long lds = 0;
    double* dst = nullptr; long ldd = 0;
    int rows = 0, cols = 0;
};
struct CopyJobs {
    int count = 0;
    CopyJob job[kMaxCopyJobs];
};
hipError_t copy_multi(const CopyJobs& jobs, hipStream_t s);
// Block-symmetric k x k matrices (ld k) split into nb diagonal blocks at
// off[0] = 0 < off[1] < ... < off[nb] = k, with the blocks on and above the
// diagonal filled: the blocks below are set to the transposes of their
// mirror images.  Up to three matrices in one launch.
constexpr int kMaxSymBlocks = 4;
struct SymJob {
    double* M = nullptr;
    int k = 0, nb = 0;
    int off[kMaxSymBlocks + 1] = {};
};
struct SymJobs {
    int count = 0;
    SymJob job[3];
};
hipError_t sym_blocks(const SymJobs& jobs, hipStream_t s);
// nonfinite check: flag[0] = 1 if any of n values is NaN/Inf
hipError_t check_finite(long n, const double* x, int* flag, hipStream_t s);

// out[0] = sum_{k<ra, m<rb} wa[k] wb[m] G0[k,m] G1[k,m] G2[k,m]  (ld ra, wa/wb may be null)
hipError_t cp_inner_reduce(int ra, int rb, const double* G0, const double* G1, const double* G2,
                           const double* wa, const double* wb, double* out, hipStream_t s);

// Panel step of a blocked Gram-Schmidt: orthonormalise the n x b panel Y
// (ld n, b <= 32) in place with `passes`-pass MGS; a column whose norm after
// projection is <= drop * norm0[j] (norm0 null: drop * 1) is set to zero and
// flagged 0 in keep[j].  Up to kMaxPanelJobs panels (of different matrices)
// per launch, one workgroup each.
constexpr int kMaxPanelJobs = 3;
struct PanelJob {
    double* Y = nullptr;
    const double* norm0 = nullptr;
    double drop = 0.0;
    int* keep = nullptr;
    int b = 0;
};
struct PanelJobs {
    int count = 0;
    PanelJob job[kMaxPanelJobs];
};
hipError_t panel_mgs(int n, const PanelJobs& jobs, int passes, hipStream_t s);
// Block projection update P -= Y C of up to kMaxPanelJobs panels per launch:
// P n x b (ld n, b <= 16), Y n x j0 (ld n, 1 <= j0 <= 256), C j0 x b (ld j0).
struct UpdateJob {
    const double* Y = nullptr;
    const double* C = nullptr;
    double* P = nullptr;
    int j0 = 0, b = 0;
};
struct UpdateJobs {
    int count = 0;
    UpdateJob job[kMaxPanelJobs];
};
hipError_t panel_update(int n, const UpdateJobs& jobs, hipStream_t s);
// Move the kept columns (j < done, or keep[j] != 0) of each n x m matrix Y
// (m <= 512) to the front, in order, in place, and write their number to
// *count (device int); up to kMaxPanelJobs matrices per launch.
struct CompactJob {
    double* Y = nullptr;
    int m = 0, done = 0;
    const int* keep = nullptr;
    int* count = nullptr;
};
struct CompactJobs {
    int count = 0;
    CompactJob job[kMaxPanelJobs];
};
hipError_t compact_cols(int n, const CompactJobs& jobs, hipStream_t s);
// Column 2-norms of up to kMaxPanelJobs n x m matrices (ld n) in one launch.
struct NormJob {
    const double* X = nullptr;
    int m = 0;
    double* out = nullptr;
};
struct NormJobs {
    int count = 0;
    NormJob job[kMaxPanelJobs];
};
hipError_t col_norms(int n, const NormJobs& jobs, hipStream_t s);

// dst (cols x rows) = src^T, src rows x cols (ld lds), dst ld ldd
hipError_t transpose(int rows, int cols, const double* src, long lds, double* dst, long ldd,
                     hipStream_t s);

hipError_t mfma_probe(double* out, hipStream_t s);

}  // namespace fc
