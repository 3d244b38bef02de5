// fracctl: rank-truncated PCG for (beta A^-alpha + (gamma/beta) A^alpha) u = y on MI355X.
//
// Everything after the entry transform runs in the eigen-coordinates of the
// three 1D Sturm-Liouville matrices (paper Section 3.3): there the operator
// and the preconditioner are Hadamard products with separable (low Kronecker
// rank) positive tensors, and Algorithm 1 (Appendix 2) runs on Tucker iterates
// (orthonormal bases Z_l, n x r_l, dense core r0 x r1 x r2).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>
#include <type_traits>
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>
#include <sys/stat.h>

#include "../../include/fracctl.h"
#include "host_math.h"
#include "fit.h"
#include "kernels.h"

namespace {

// largest small-space dimension (union bases, projected cores, Jacobi size)
constexpr int KM = 128;

thread_local std::string g_last_error;

fc_status fail(fc_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            throw FcError(FC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
    } while (0)

struct FcError {
    fc_status status;
    std::string msg;
    FcError(fc_status s, std::string m) : status(s), msg(std::move(m)) {}
};

// A Tucker tensor in device memory: T = core x_1 Z0 x_2 Z1 x_3 Z2.
struct Tucker {
    int r[3] = {0, 0, 0};
    double* Z[3] = {nullptr, nullptr, nullptr};  // n x rcap each, ld n
    double* core = nullptr;                     // capacity ccap
    bool empty() const { return r[0] == 0 || r[1] == 0 || r[2] == 0; }
    long csize() const { return (long)r[0] * r[1] * r[2]; }
};

struct Arena {
    std::vector<void*> blocks;
    double* alloc(size_t count) {
        void* p = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(double));
        if (e != hipSuccess) throw FcError(FC_ERR_OUT_OF_MEMORY, "hipMalloc failed");
        blocks.push_back(p);
        return (double*)p;
    }
    int* alloc_int(size_t count) {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(int));
        if (e != hipSuccess) throw FcError(FC_ERR_OUT_OF_MEMORY, "hipMalloc failed");
        blocks.push_back(p);
        return (int*)p;
    }
    void release(void* q) {
        for (size_t i = 0; i < blocks.size(); ++i)
            if (blocks[i] == q) {
                (void)hipFree(q);
                blocks.erase(blocks.begin() + (long)i);
                return;
            }
    }
    ~Arena() {
        for (void* p : blocks) (void)hipFree(p);
    }
};

}  // namespace

// A separable positive tensor in eigen-coordinates: sum_q (x)_l D_l[:, q]
// with the positive weights folded into the factors (cube root per mode).
struct Separable {
    int Q = 0;
    double* D[3] = {nullptr, nullptr, nullptr};   // n x Q
    double* D2[3] = {nullptr, nullptr, nullptr};  // elementwise squares
    std::vector<double> w;                        // host copy of the weights (pre-folding)
    std::vector<double> F[3];                     // host-built plans: unweighted factors n x Q
    double* Fd[3] = {nullptr, nullptr, nullptr};  // device-built plans: the same on the device
};

enum {
    SITE_Z = 0, SITE_S, SITE_X, SITE_R, SITE_P, SITE_MISC, SITE_OS, SITE_OR, SITE_OU, SITE_ST, SITE_ZE,
    NSITES
};

// Launch choices picked by the autotuner for a plan's size (see autotune):
// wavefronts per workgroup of the Gram kernel for batched (scaled) and for
// unbatched products, of the fused Kronecker application, the K chunk of the
// streaming transform kernel, the Gram-Schmidt panel width; and the measured
// time (us) of every candidate.
struct Tuning {
    int gram_batched = 16, gram_single = 16, kron = 16, stream_kc = 128, panel_b = 16;
    double us[10] = {};
    bool tuned = false;
};

struct WarmBasis {
    double* W[3] = {nullptr, nullptr, nullptr};
    int pk[3] = {0, 0, 0};
    bool valid = false;
};

struct fc_plan_s {
    int n = 0;
    double alpha = 0, beta = 1, gamma = 1, eps = 1e-6, tol = 1e-6, op_acc = 0;
    int max_iter = 100, rcap = 64, pcap = 96, precond_rank = 6;
    std::vector<double> lam[3];   // host eigenvalues
    std::vector<double> Vh[3];    // host eigenvectors
    double* V[3] = {nullptr, nullptr, nullptr};
    // V_l^T stored as well (n x n each), so that both transform directions
    // read their matrix along columns (coalesced): HBM is plentiful, the
    // transforms are bandwidth-bound
    double* Vt[3] = {nullptr, nullptr, nullptr};
    Separable op, pc, st;   // operator ~ f, preconditioner ~ 1/f, state map ~ beta s^-alpha
    double op_err = 0, pc_err = 0, st_err = 0;
    // preconditioner case (A): 1/f on the spectrum of the anisotropic
    // Laplacian in the sine basis, and the maps W_l = S V_l into that basis
    int pc_kind = FC_PRECOND_EIGEN;
    // d = 2: the third mode is a Laplacian shifted by its smallest eigenvalue,
    // and designs and results carry its first eigenvector (Y3d, U3d: n x 256)
    int dims = 3;
    double *Y3d = nullptr, *U3d = nullptr;
    double b0[3] = {1.0, 1.0, 1.0};
    std::vector<double> mu[3];    // host: b0_l (4/h^2) sin^2(k pi h/2), ascending
    Separable pcA;
    double pcA_err = 0;
    double* Wsin[3] = {nullptr, nullptr, nullptr};
    double* WsinT[3] = {nullptr, nullptr, nullptr};   // W_l^T
    Arena arena;
    // workspace
    Tucker slot[14];
    fc_precision precision = FC_FP64;
    double *E = nullptr, *Gd[3] = {}, *Mq = nullptr, *c1 = nullptr, *c2 = nullptr;
    double *Xs = nullptr, *HX = nullptr, *Ys = nullptr, *Ts = nullptr;
    double *Bp = nullptr, *Ev = nullptr, *Evec = nullptr, *W[3] = {}, *As[3] = {};
    double *T1 = nullptr, *T2 = nullptr, *C = nullptr, *Cp = nullptr, *Cg = nullptr;
    double *Cev = nullptr, *Cvec = nullptr, *Cn1 = nullptr, *Cn2 = nullptr;
    double *Phi[3] = {}, *Map = nullptr, *scal = nullptr, *tmpn = nullptr, *tmpn2 = nullptr;
    double *cw = nullptr, *cf[3] = {}, *Yh[3] = {};
    int* icount = nullptr;
    int* t2c_keep = nullptr;   // kept T2C term indices (rcap^2)
    void* t2c_ws = nullptr;    // T2C sort scratch beyond the LDS capacity
    double* jac = nullptr;
    WarmBasis warm[NSITES];
    Tuning tune;
    double *qrN = nullptr, *qrC = nullptr;
    double *Xs3[3] = {}, *HX3[3] = {}, *Bp3 = nullptr, *Ev3 = nullptr, *Evec3 = nullptr;
    int* qrKeep = nullptr;
    double* splitws = nullptr;
    long splitws_cap = 0;
    double *SG[3] = {}, *SM[3] = {};
    long qchunk = 1;
    long cbig = 0;     // doubles in c1 (= T1) and in c2 (= T2)
    long cap_canon = 0;
    int* dflag = nullptr;
    unsigned* dotcnt = nullptr;   // zero between calls of the device dot
    long ys_cap = 0;              // doubles in Ys and in Ts
    long e_cap = 0;               // doubles in E
    hipStream_t stream = nullptr;   // the setup's stream (set during fc_setup_ex only)
    // statistics of the last solve
    int max_seen_rank = 0;
    double worst_missed = 0;   // largest missed-energy charge / budget of a Hadamard truncation
    double site_ms[16] = {};   // wall time per truncation site (with FC_TRACE)
    int site_calls[16] = {};
    std::mutex use_mu;   // one solve at a time per plan
    // pinned host landing area for the small device-to-host reads of a solve
    // (ranks, spectra, scalars): a direct copy, no pageable staging.  (The
    // kernels writing these results straight into coherent pinned host
    // memory, with a stream synchronisation as the only wait, saved under 1%;
    // one batched run in about fifty then stopped on a zero inner product,
    // so the copies stay.)
    static constexpr size_t kPinnedBytes = 64 * 1024;
    void* pinned = nullptr;
    ~fc_plan_s() {
        if (pinned) (void)hipHostFree(pinned);
    }
};

namespace {

using fc::GemmArgs;

// Convergence trace on stderr (ranks and residuals per iteration and per
// refinement sweep), switched on by the environment variable FC_TRACE.
const bool g_trace = std::getenv("FC_TRACE") != nullptr;
#define FC_TRACE_PRINT(...)                         \
    do {                                            \
        if (g_trace) {                              \
            std::fprintf(stderr, "[fc] " __VA_ARGS__); \
            std::fflush(stderr);                    \
        }                                           \
    } while (0)

// Optional timing of every matrix-core GEMM launch with HIP events on the
// launching stream (for roofline reporting); off unless enabled.
struct GemmShape {
    bool ta, tb;
    int M, N, K, batch, inner;
    bool lowp;
    int kind;   // profile kind of the launch (see KernelProfile)
    double flops, bytes;
};
struct GemmProfile {
    bool on = false;
    std::vector<hipEvent_t> ev;   // pairs
    std::vector<GemmShape> shapes;
    size_t used = 0;
    double flops = 0, bytes = 0;
    long launches = 0;
};
GemmProfile g_prof;
std::mutex g_prof_mu;
thread_local bool t_no_profile = false;   // set in batch workers

// Profile kinds: the products are split into the short-reduction LDS-tiled
// GEMMs (0), the mode transforms V^T Y, V Z (3), the long-reduction Gram
// engine (4: Gram-type products, scaled Grams, core contractions) and the
// fused Kronecker application (5), all timed through the GEMM profile; the
// Gram-Schmidt panel kernel (1) and the eigensolver (2) have event pairs of
// their own, enabled together with the GEMM timing.
constexpr int kProfKinds = 6;
thread_local int t_tag = -1;   // kind override for the launches of a scope
struct KindTag {
    int saved;
    explicit KindTag(int k) : saved(t_tag) { t_tag = k; }
    ~KindTag() { t_tag = saved; }
};
struct KernelProfile {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    double flops = 0, bytes = 0;
    long launches = 0;
};
KernelProfile k_prof[kProfKinds];

// Event pair around one product-type launch, with its shape and work
// (profile on, not a batch worker).
template <class F>
void record_product(hipStream_t s, const GemmShape& shape, F&& launch) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof.used + 2 > g_prof.ev.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            g_prof.ev.push_back(e);
        }
    }
    HIPCHK(hipEventRecord(g_prof.ev[g_prof.used], s));
    HIPCHK(launch());
    HIPCHK(hipEventRecord(g_prof.ev[g_prof.used + 1], s));
    g_prof.used += 2;
    g_prof.shapes.push_back(shape);
    g_prof.flops += shape.flops;
    g_prof.bytes += shape.bytes;
    g_prof.launches += 1;
}

// algorithmic work of a batch of symmetric eigenproblems: Householder
// tridiagonalisation 4/3 k^3 and back-transformation 2 k^2 k flops per
// matrix; the matrix read and the vectors written once
double eig_flops(const fc::EigJobs& j) {
    double f = 0;
    for (int i = 0; i < j.count; ++i) f += (4.0 / 3.0 + 2.0) * std::pow((double)j.job[i].k, 3);
    return f;
}
double eig_bytes(const fc::EigJobs& j) {
    double b = 0;
    for (int i = 0; i < j.count; ++i) b += 16.0 * (double)j.job[i].k * j.job[i].k;
    return b;
}

template <class F>
hipError_t timed_launch(int kind, hipStream_t s, double flops, double bytes, F&& launch) {
    if (!g_prof.on || t_no_profile) return launch();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    KernelProfile& kp = k_prof[kind];
    if (kp.used + 2 > kp.ev.size())
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            hipError_t er = hipEventCreate(&e);
            if (er != hipSuccess) return er;
            kp.ev.push_back(e);
        }
    hipError_t e = hipEventRecord(kp.ev[kp.used], s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(kp.ev[kp.used + 1], s);
    kp.used += 2;
    kp.flops += flops;
    kp.bytes += bytes;
    kp.launches += 1;
    return e;
}

struct Ctx {
    fc_plan_s* p;
    hipStream_t s;
    int n;
    bool lowp = false;   // bulk contractions on the FP32 matrix cores
    bool clamp = false;  // search directions: cap HOSVD ranks at max_rank instead of failing
};

// Algorithmic work of one product: 2 M N K flops per batch entry; each
// operand read once (once in all when shared by the batch, stride 0), the
// result written once.
double prod_flops(const GemmArgs& g) { return 2.0 * g.M * g.N * (double)g.K * g.batch; }
double prod_bytes(const GemmArgs& g) {
    const double nb = g.batch;
    const bool two = g.inner > 1;
    const double a = (double)g.M * g.K * ((g.strideA || (two && g.strideAin)) ? nb : 1.0);
    const double b = (double)g.K * g.N * ((g.strideB || (two && g.strideBin)) ? nb : 1.0);
    const double dd = g.d ? (double)g.K * (g.strideD ? nb : 1.0) : 0.0;
    return 8.0 * (a + b + dd + (double)g.M * g.N * nb);
}

// Gram-type products go to the split-over-waves kernel: every FP64 product
// over a reduction of at least 256 (the mode transforms V^T Y and V Z, the
// diagonally scaled Grams Z^T diag(d) X of the Hadamard truncation, the
// long contractions of the core), and the unbatched A^T B with a small
// result (M, N <= 128).  Not A^T B^T, not two-level batches.
bool gram_type(bool ta, bool tb, const GemmArgs& g) {
    if (g.lowp || g.inner != 1 || g.K <= 0 || (ta && tb)) return false;
    if (g.K >= 256) return true;
    return !g.d && g.batch == 1 && g.M <= 128 && g.N <= 128 && ta;
}

// A mode transform: C = A B with A the n x n matrix of a mode (M = K = n),
// FP64, unbatched, alpha = 1, beta = 0.
bool is_transform(const Ctx& c, bool ta, bool tb, const GemmArgs& g) {
    return !ta && !tb && !g.d && !g.lowp && g.inner == 1 && g.batch == 1 && g.M == c.n &&
           g.K == c.n && g.alpha == 1.0 && g.beta == 0.0 && g.N > 0;
}

// wavefronts per workgroup of the Gram kernel for a product: the tuned
// choice for batched (the scaled Grams) and for single products
int gram_waves(const Ctx& c, const GemmArgs& g) {
    return g.batch > 1 ? c.p->tune.gram_batched : c.p->tune.gram_single;
}

// staged or direct Gram tile for a product (see fc::gram): staged for
// A^T B, whose operands are contiguous along the reduction (measured per
// shape on the n = 1024 workload: 0.7-0.9 of the direct tile's time), direct
// for A B^T (1.4-2.1x faster than staged there); FC_GRAM_MODE = staged |
// direct forces one (a diagnostic)
const int g_gram_mode = [] {
    const char* m = std::getenv("FC_GRAM_MODE");
    if (!m) return -1;
    return std::strcmp(m, "staged") == 0 ? 1 : std::strcmp(m, "direct") == 0 ? 0 : -1;
}();
bool gram_staged(bool ta) {
    if (g_gram_mode >= 0) return g_gram_mode == 1;
    return ta;
}

// terms per workgroup of the batched scaled Grams (fc::gram's group): four
// (two at sixteen wavefronts).  A workgroup then stages its A and B chunks
// once for the group; a batch holds a fraction of the compute units, which
// the concurrent solves of a batched call use (64 solves at n = 1024, six
// timed steps: one term 151-154, two 164-165, four 166-167 solves/s; one
// solve alone unchanged).  FC_GRAM_GROUP = 1 | 2 | 4 overrides it (a
// diagnostic); the results do not depend on it.
const int g_gram_group = [] {
    const char* m = std::getenv("FC_GRAM_GROUP");
    const int v = m ? std::atoi(m) : 4;
    return (v == 1 || v == 2 || v == 4) ? v : 4;
}();
// FC_KRON_WAVES = 8 | 16 overrides the tuned wavefronts of the fused
// Kronecker application (a diagnostic)
const int g_kron_waves = [] {
    const char* m = std::getenv("FC_KRON_WAVES");
    const int v = m ? std::atoi(m) : 0;
    return (v == 8 || v == 16) ? v : 0;
}();
int kron_waves(const Ctx& c) { return g_kron_waves ? g_kron_waves : c.p->tune.kron; }
int gram_group(const GemmArgs& g) { return g.batch > 1 ? g_gram_group : 1; }

// The mode transforms run on the streaming kernel (K split over workgroups,
// partials added by a second kernel).  The small Gram-type products stay on
// the Gram kernel: one launch each, where the split would need two (the
// batched path is bound by the launch rate).
int stream_layout(bool ta, bool tb) { return ta ? 0 : (tb ? 1 : 2); }

// Up to three products in one launch of the streaming kernel (split-K
// partials in the plan's GEMM workspace).
hipError_t run_stream(const Ctx& c, bool ta, bool tb, const GemmArgs* g, int count) {
    fc::StreamJobs sj;
    for (int t = 0; t < count; ++t) {
        fc::StreamJob& J = sj.job[sj.count++];
        J.M = g[t].M; J.N = g[t].N; J.K = g[t].K;
        J.alpha = g[t].alpha; J.beta = g[t].beta;
        J.A = g[t].A; J.lda = g[t].lda;
        J.B = g[t].B; J.ldb = g[t].ldb;
        J.C = g[t].C; J.ldc = g[t].ldc;
    }
    fc_plan_s* p = c.p;
    const int kc = fc::stream_fits(sj, p->tune.stream_kc, p->splitws_cap) ? p->tune.stream_kc : 256;
    if (!fc::stream_fits(sj, kc, p->splitws_cap)) {
        // partials beyond the workspace: the Gram kernel, one product at a time
        for (int t = 0; t < count; ++t) {
            const hipError_t e = fc::gram(ta, tb, g[t], c.s, gram_waves(c, g[t]), gram_staged(ta),
                                          gram_group(g[t]));
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    return fc::stream_multi(stream_layout(ta, tb), sj, kc, p->splitws, p->splitws_cap, c.s);
}

// Route one product: Gram-type ones to the split-over-waves kernel, the
// rest (short reductions, two-level batches, FP32 cores) to the LDS-tiled
// matrix-core GEMM.  Every product of a solve runs on the library's own
// kernels.
hipError_t run_gemm(const Ctx& c, bool ta, bool tb, const GemmArgs& g) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (t_tag == 3 && is_transform(c, ta, tb, g)) return run_stream(c, ta, tb, &g, 1);
    if (gram_type(ta, tb, g))
        return fc::gram(ta, tb, g, c.s, gram_waves(c, g), gram_staged(ta), gram_group(g));
    return fc::gemm(ta, tb, g, c.s);
}

// One product given as GemmArgs (split-K workspace from the plan), timed
// with HIP events when the GEMM profile is on.
void gemm_args(const Ctx& c, bool ta, bool tb, GemmArgs g) {
    g.part = c.p->splitws; g.part_cap = c.p->splitws_cap;
    const int M = g.M, N = g.N, K = g.K, batch = g.batch;
    if (g_prof.on && !t_no_profile && M > 0 && N > 0 && K > 0 && batch > 0) {
        const int kind = t_tag >= 0 ? t_tag : (gram_type(ta, tb, g) ? 4 : 0);
        record_product(c.s, {ta, tb, M, N, K, batch, g.inner, g.lowp, kind, prod_flops(g),
                             prod_bytes(g)},
                       [&] { return run_gemm(c, ta, tb, g); });
        return;
    }
    HIPCHK(run_gemm(c, ta, tb, g));
}

void gemm(const Ctx& c, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
          long lda, const double* B, long ldb, double beta, double* C, long ldc, int batch = 1,
          long sA = 0, long sB = 0, long sC = 0, int inner = 1, long sAi = 0, long sBi = 0,
          long sCi = 0, const double* d = nullptr, long sD = 0, bool bulk = false) {
    GemmArgs g;
    g.lowp = c.lowp && bulk;
    g.M = M; g.N = N; g.K = K; g.batch = batch; g.inner = inner;
    g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.strideA = sA; g.strideAin = sAi;
    g.B = B; g.ldb = ldb; g.strideB = sB; g.strideBin = sBi;
    g.C = C; g.ldc = ldc; g.strideC = sC; g.strideCin = sCi;
    g.d = d; g.strideD = sD;
    gemm_args(c, ta, tb, g);
}

// bulk contraction: runs on the FP32 matrix cores when the context asks for it
void gemmb(const Ctx& c, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
           long lda, const double* B, long ldb, double beta, double* C, long ldc, int batch = 1,
           long sA = 0, long sB = 0, long sC = 0, int inner = 1, long sAi = 0, long sBi = 0,
           long sCi = 0) {
    gemm(c, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, batch, sA, sB, sC, inner, sAi,
         sBi, sCi, nullptr, 0, true);
}

// Up to three independent FP64 products of the same form (op(A) op(B) with
// the given transposes) issued together: those that are Gram-type (the same
// rule as run_gemm: M, N <= 128 and A^T B, or a reduction of at least 256)
// share one launch of the Gram kernel, two or more others with a short
// reduction (K <= 256, or any with long_k) share one launch of the grouped
// matrix-core GEMM, the rest go through gemm one by one.  Products may be
// strided or two-level batches (a batch is never Gram-type here).  Timed
// like gemm when the GEMM profile is on.
void launch_group(const Ctx& c, bool ta, bool tb, const fc::GramJobs& jobs, bool gram) {
    if (jobs.count == 0) return;
    bool transform = gram && t_tag == 3 && !ta && !tb;
    for (int t = 0; t < jobs.count && transform; ++t) transform = is_transform(c, ta, tb, jobs.g[t]);
    auto run = [&] {
        if (transform) return run_stream(c, ta, tb, jobs.g, jobs.count);
        return gram ? fc::gram_multi(ta, tb, jobs, c.s, gram_waves(c, jobs.g[0]), gram_staged(ta),
                                     gram_group(jobs.g[0]))
                    : fc::gemm_multi(ta, tb, jobs, c.s);
    };
    if (g_prof.on && !t_no_profile) {
        // one shape entry per launch: the first product's shape, with the
        // number of products as its batch; the work of all of them
        const fc::GemmArgs& g0 = jobs.g[0];
        GemmShape sh{ta, tb, g0.M, g0.N, g0.K, jobs.count, 1, false,
                     t_tag >= 0 ? t_tag : (gram ? 4 : 0), 0.0, 0.0};
        for (int t = 0; t < jobs.count; ++t) {
            sh.flops += prod_flops(jobs.g[t]);
            sh.bytes += prod_bytes(jobs.g[t]);
        }
        record_product(c.s, sh, run);
        return;
    }
    HIPCHK(run());
}

void gemm_group(const Ctx& c, bool ta, bool tb, const fc::GemmArgs* prods, int count,
                bool long_k = false) {
    fc::GramJobs grams, others;
    auto one = [&](const fc::GemmArgs& g) { gemm_args(c, ta, tb, g); };
    for (int t = 0; t < count; ++t) {
        const fc::GemmArgs& g = prods[t];
        if (g.M <= 0 || g.N <= 0) continue;
        if (gram_type(ta, tb, g))
            grams.g[grams.count++] = g;
        else if (g.K > 0 && !g.d && !g.lowp && (g.K <= 256 || long_k))
            others.g[others.count++] = g;
        else
            one(g);
    }
    launch_group(c, ta, tb, grams, true);
    if (others.count == 1)
        one(others.g[0]);
    else
        launch_group(c, ta, tb, others, false);
}

// out_l = sum_q diag(D_l[:, q]) Z_l T_l^q for the jobs (fused row-wise
// Kronecker product and contraction), timed with the GEMM family when the
// GEMM profile is on: 2 n p r Q flops, Z, D, T read and out written once.
void kron_apply(const Ctx& c, int Q, const fc::KronJobs& kj) {
    if (kj.count == 0) return;
    const int n = c.n;
    if (g_prof.on && !t_no_profile) {
        const fc::KronJob& J0 = kj.job[0];
        GemmShape sh{false, false, n, J0.p, J0.r * Q, kj.count, 1, false, 5, 0.0, 0.0};
        for (int t = 0; t < kj.count; ++t) {
            const fc::KronJob& J = kj.job[t];
            sh.flops += 2.0 * n * J.p * (double)J.r * Q;
            sh.bytes += 8.0 * ((double)n * J.r + (double)n * Q + (double)J.r * J.p * Q +
                               (double)n * J.p);
        }
        record_product(c.s, sh,
                       [&] { return fc::kron_apply_multi(n, Q, kj, c.s, kron_waves(c)); });
        return;
    }
    HIPCHK(fc::kron_apply_multi(n, Q, kj, c.s, kron_waves(c)));
}

fc::GemmArgs prod(int M, int N, int K, const double* A, long lda, const double* B, long ldb,
                  double* C, long ldc) {
    fc::GemmArgs g;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
    return g;
}

void sync(const Ctx& c) { HIPCHK(hipStreamSynchronize(c.s)); }

// With FC_TRACE: wall time of one truncation, stream drained at both ends.
struct SiteClock {
    const Ctx& c;
    int site;
    std::chrono::steady_clock::time_point t0;
    SiteClock(const Ctx& c_, int site_) : c(c_), site(site_) {
        if (g_trace) {
            (void)hipStreamSynchronize(c.s);
            t0 = std::chrono::steady_clock::now();
        }
    }
    ~SiteClock() {
        if (!g_trace) return;
        (void)hipStreamSynchronize(c.s);
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        c.p->site_ms[site] += ms;
        c.p->site_calls[site] += 1;
    }
};

template <class T>
void d2h(const Ctx& c, T* dst, const T* src, size_t count) {
    const size_t bytes = count * sizeof(T);
    void* pin = c.p->pinned;
    if (pin && bytes <= fc_plan_s::kPinnedBytes) {
        HIPCHK(hipMemcpyAsync(pin, src, bytes, hipMemcpyDeviceToHost, c.s));
        sync(c);
        std::memcpy(dst, pin, bytes);
        return;
    }
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.s));
    sync(c);
}
template <class T>
void h2d(const Ctx& c, T* dst, const T* src, size_t count) {
    HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, c.s));
}

// ---- core mode products ---------------------------------------------------
// out = core x_mode M, core r0 x r1 x r2, M is m x r_mode (ld ldm); out has
// r_mode replaced by m.
// With transM the stored matrix is r_mode x m and op(M) = M^T.
void mode_product(const Ctx& c, const double* core, const int r[3], int mode, const double* M,
                  long ldm, int m, double* out, double alpha = 1.0, double beta = 0.0,
                  bool transM = false, bool bulk = false) {
    if (mode == 0) {
        gemm(c, transM, false, m, r[1] * r[2], r[0], alpha, M, ldm, core, r[0], beta, out, m, 1, 0,
             0, 0, 1, 0, 0, 0, nullptr, 0, bulk);
    } else if (mode == 1) {
        // for each k: (r0 x r1) * op(M)^T (r1 x m)
        gemm(c, false, !transM, r[0], m, r[1], alpha, core, r[0], M, ldm, beta, out, r[0], r[2],
             (long)r[0] * r[1], 0, (long)r[0] * m, 1, 0, 0, 0, nullptr, 0, bulk);
    } else {
        gemm(c, false, !transM, r[0] * r[1], m, r[2], alpha, core, (long)r[0] * r[1], M, ldm,
             beta, out, (long)r[0] * r[1], 1, 0, 0, 0, 1, 0, 0, 0, nullptr, 0, bulk);
    }
}

// permuted dims for "mode first"
void perm_dims(const int r[3], int mode, int out[3]) {
    if (mode == 0) { out[0] = r[0]; out[1] = r[1]; out[2] = r[2]; }
    else if (mode == 1) { out[0] = r[1]; out[1] = r[0]; out[2] = r[2]; }
    else { out[0] = r[2]; out[1] = r[0]; out[2] = r[1]; }
}

double host_dot(const Ctx& c, long n, const double* x, const double* y) {
    fc_plan_s* p = c.p;
    HIPCHK(fc::dot_long(n, x, y, p->scal + 256, p->dotcnt, p->scal, c.s));
    double v = 0;
    d2h(c, &v, p->scal, 1);
    return v;
}

// ---- rank-revealing orthonormalisation of n x m columns (in place) --------
// Blocked classical Gram-Schmidt with reorthogonalisation (BCGS2): panels of
// 16 columns are projected against all earlier columns by two GEMM passes and
// then orthonormalised by a two-pass MGS panel kernel.  Columns whose norm
// after projection drops below `drop` times their input norm are removed.
// Returns the number of kept columns (compacted to the front).
// `done` leading columns are already orthonormal and are kept as they are.
// Rank-revealing orthonormalisation of up to three n x m_l blocks (one per
// mode, in place; block l only when use[l]): BCGS2 with panels of b columns.
// Per panel: block projection against the earlier columns, panel MGS (two
// passes, drop test), a second block projection and panel pass.  The second
// round removes what normalising a nearly dependent column magnified of its
// rounding components along the earlier columns; a column with less than
// half its length left after it was rounding noise and is dropped.  The
// first done_l columns are already orthonormal.  The modes run in lockstep:
// each panel step of the three modes is one launch (a workgroup per mode),
// the compaction of the kept columns one launch, and the three counts one
// read; m[l] receives the count.
void orthonormalize3(const Ctx& c, int m[3], double* const Y[3], double drop, const int done_in[3],
                     const bool use[3]) {
    fc_plan_s* p = c.p;
    const int n = c.n;
    int done[3];
    bool on[3];
    fc::NormJobs nj;
    for (int l = 0; l < 3; ++l) {
        on[l] = use[l] && m[l] > 0;
        done[l] = on[l] ? std::max(0, std::min(done_in[l], m[l])) : 0;
        if (on[l]) {
            fc::NormJob& J = nj.job[nj.count++];
            J.X = Y[l]; J.m = m[l]; J.out = p->qrN + l * 512L;
        }
    }
    HIPCHK(fc::col_norms(n, nj, c.s));
    // panel width: the panel lives in LDS (<= 144 KiB)
    const int b = std::max(1, std::min(p->tune.panel_b, (int)((144L * 1024 / 8) / n)));
    // block projection P -= Y (Y^T P) of the modes' current panels: the
    // coefficients per mode (Gram-type product), the updates in one launch
    auto project = [&](const fc::PanelJobs& pj, const int* j0s, const int* modes) {
        fc::UpdateJobs uj;
        fc::GemmArgs coef[3];
        int nc = 0;
        for (int t = 0; t < pj.count; ++t) {
            const int l = modes[t];
            if (j0s[l] == 0) continue;
            double* Cl = p->qrC + (long)l * 256 * 16;
            coef[nc++] = prod(j0s[l], pj.job[t].b, n, Y[l], n, pj.job[t].Y, n, Cl, j0s[l]);
            fc::UpdateJob& U = uj.job[uj.count++];
            U.Y = Y[l]; U.C = Cl; U.P = pj.job[t].Y; U.j0 = j0s[l]; U.b = pj.job[t].b;
        }
        gemm_group(c, true, false, coef, nc);   // C_l = Y_l^T P_l
        HIPCHK(fc::panel_update(n, uj, c.s));
    };
    for (int pi = 0;; ++pi) {
        fc::PanelJobs first, second;
        int j0s[3] = {0, 0, 0}, modes[3] = {0, 0, 0};
        double flops1 = 0, bytes1 = 0, flops2 = 0, bytes2 = 0;
        for (int l = 0; l < 3; ++l) {
            if (!on[l]) continue;
            const int j0 = done[l] + pi * b;
            if (j0 >= m[l]) continue;
            const int bw = std::min(b, m[l] - j0);
            double* P = Y[l] + (long)j0 * n;
            j0s[l] = j0;
            modes[first.count] = l;
            fc::PanelJob& J = first.job[first.count++];
            J.Y = P; J.norm0 = p->qrN + l * 512L + j0; J.drop = drop;
            J.keep = p->qrKeep + l * 512L + j0; J.b = bw;
            // algorithmic work: the panel read and written once, two MGS passes
            flops1 += 4.0 * n * bw * bw;
            bytes1 += 16.0 * n * bw;
        }
        if (first.count == 0) break;
        project(first, j0s, modes);
        HIPCHK(timed_launch(1, c.s, flops1, bytes1,
                            [&] { return fc::panel_mgs(n, first, 2, c.s); }));
        int modes2[3] = {0, 0, 0};
        for (int t = 0; t < first.count; ++t) {
            const int l = modes[t];
            if (j0s[l] == 0) continue;
            const fc::PanelJob& J1 = first.job[t];
            modes2[second.count] = l;
            fc::PanelJob& J = second.job[second.count++];
            J = J1;
            J.norm0 = nullptr; J.drop = 0.5;
            flops2 += 2.0 * n * J1.b * J1.b;
            bytes2 += 16.0 * n * J1.b;
        }
        if (second.count > 0) project(second, j0s, modes2);
        if (second.count > 0)
            HIPCHK(timed_launch(1, c.s, flops2, bytes2,
                                [&] { return fc::panel_mgs(n, second, 1, c.s); }));
    }
    fc::CompactJobs cj;
    int slot[3] = {-1, -1, -1};
    for (int l = 0; l < 3; ++l) {
        if (!on[l]) continue;
        fc::CompactJob& J = cj.job[cj.count];
        J.Y = Y[l]; J.m = m[l]; J.done = done[l]; J.keep = p->qrKeep + l * 512L;
        J.count = p->icount + 4 + cj.count;
        slot[l] = cj.count++;
    }
    if (cj.count == 0) {
        for (int l = 0; l < 3; ++l) if (use[l]) m[l] = 0;
        return;
    }
    HIPCHK(fc::compact_cols(n, cj, c.s));
    int cnt[3] = {0, 0, 0};
    d2h(c, cnt, p->icount + 4, cj.count);
    for (int l = 0; l < 3; ++l)
        if (use[l]) m[l] = on[l] ? cnt[slot[l]] : 0;
}

// Diagnostic (environment variable FC_CHECK): largest deviation of M^T M
// from the identity for an m x k matrix, printed when above 1e-10.
const bool g_check = std::getenv("FC_CHECK") != nullptr;
// FC_UNGROUPED: the truncations issue their per-mode products, row-wise
// products and term passes mode by mode instead of in grouped launches (the
// paths taken when the grouped slices do not fit the plan's buffers), so
// those paths can be checked on any problem
const bool g_ungrouped = std::getenv("FC_UNGROUPED") != nullptr;
void check_cols(const Ctx& c, const double* M, long ld, int m, int k, const char* what, int tag) {
    if (!g_check || k <= 0) return;
    fc_plan_s* p = c.p;
    double* G = p->Bp3 + 2L * KM * KM;   // scratch for k <= 128
    gemm(c, true, false, k, k, m, 1.0, M, ld, M, ld, 0.0, G, k);
    std::vector<double> g((size_t)k * k);
    d2h(c, g.data(), G, g.size());
    double worst = 0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            worst = std::max(worst, std::fabs(g[i + (size_t)j * k] - (i == j ? 1.0 : 0.0)));
    if (worst > 1e-10)
        std::fprintf(stderr, "[fc] check %s[%d]: max |M^T M - I| = %.3e (%d x %d)\n", what, tag,
                     worst, m, k);
}

// ---- HOSVD truncation of a dense core in given bases ----------------------
// Input: core C (k0 x k1 x k2) expressed in orthonormal bases B_l (n x k_l).
// Output: Tucker `out` with ranks chosen so that the dropped energy is at
// most thr2 (the exact HOSVD bound sum_l tail_l <= thr2, split evenly).
void hosvd_core(const Ctx& c, const double* C, const int k[3], double* const B[3], double thr2,
                Tucker& out, const char* what) {
    fc_plan_s* p = c.p;
    const int n = c.n;
    const long csz = (long)k[0] * k[1] * k[2];
    if (csz == 0) { out.r[0] = out.r[1] = out.r[2] = 0; return; }
    for (int l = 0; l < 3; ++l)
        if (k[l] > KM) throw FcError(FC_ERR_INTERNAL, std::string(what) + ": subspace > 128");
    // unfolding Grams (modes 1 and 2 from permuted copies, one launch)
    {
        fc::GemmArgs grams[3];
        double* perm[3] = {nullptr, p->Cp, p->Cn1};
        HIPCHK(fc::permute_core12(k[0], k[1], k[2], C, perm[1], perm[2], c.s));
        for (int l = 0; l < 3; ++l) {
            int pd[3];
            perm_dims(k, l, pd);
            const double* src = (l == 0) ? C : perm[l];
            grams[l] = prod(pd[0], pd[0], pd[1] * pd[2], src, pd[0], src, pd[0],
                            p->Cg + (long)l * KM * KM, pd[0]);
        }
        gemm_group(c, false, true, grams, 3);
    }
    // per-mode share of the budget: the HOSVD bound sum_l tail_l <= thr2.  With
    // d = 2 the core is a matrix (third rank 1, no tail) and cutting both
    // modes at tails <= thr2 is the reduced SVD truncation, whose error is
    // exactly the smaller of the two tails.
    const double per_mode = p->dims == 2 ? thr2 : thr2 / 3.0;
    {
        fc::EigJobs jobs;
        jobs.count = 3;
        for (int l = 0; l < 3; ++l) {
            fc::EigJob& J = jobs.job[l];
            J.A = p->Cg + (long)l * KM * KM; J.lda = k[l]; J.k = k[l];
            J.evals = p->Cev + l * KM; J.V = p->Cvec + (long)l * KM * KM; J.ldv = k[l];
            J.scratch = p->jac + (long)l * 6 * KM * KM;
            J.budget = per_mode;   // vectors for the kept rank only
            J.margin = 0;
        }
        HIPCHK(timed_launch(2, c.s, eig_flops(jobs), eig_bytes(jobs),
                            [&] { return fc::sym_eig_multi(jobs, c.s); }));
    }
    std::vector<double> ev(3 * KM);
    d2h(c, ev.data(), p->Cev, 3 * KM);
    double tot = 0;
    for (int i = 0; i < k[0]; ++i) tot += std::max(ev[i], 0.0);
    int r[3];
    for (int l = 0; l < 3; ++l) {
        // smallest r with tail(r) <= the mode's share
        double tail = 0;
        int rr = k[l];
        for (int i = k[l] - 1; i >= 0; --i) {
            tail += std::max(ev[l * KM + i], 0.0);
            if (tail <= per_mode) rr = i; else break;
        }
        int numrank = 0;
        const double tmax = std::max(ev[l * KM], 0.0);
        while (numrank < k[l] && ev[l * KM + numrank] > 1e-17 * tmax) ++numrank;
        r[l] = std::min(rr, numrank);
    }
    if (r[0] == 0 || r[1] == 0 || r[2] == 0 || tot <= thr2) {
        out.r[0] = out.r[1] = out.r[2] = 0;
        return;
    }
    for (int l = 0; l < 3; ++l)
        if (r[l] > p->rcap) {
            // a search direction (Z, P) only steers the iteration: its best
            // rank-max_rank approximation keeps every recursion consistent
            // (S is the operator applied to the P actually used)
            if (!c.clamp)
                throw FcError(FC_ERR_INTERNAL, std::string(what) + ": Tucker rank " +
                                                   std::to_string(r[l]) + " exceeds max_rank");
            FC_TRACE_PRINT("%s: mode %d rank %d capped at %d\n", what, l, r[l], p->rcap);
            r[l] = p->rcap;
        }
    // core projection: C x_l U_l^T
    int cur[3] = {k[0], k[1], k[2]};
    const double* src = C;
    double* bufs[2] = {p->Cn1, p->Cn2};
    for (int l = 0; l < 3; ++l) {
        double* dst = (l == 2) ? out.core : bufs[l & 1];
        // C x_l U_l[:, :r_l]^T
        mode_product(c, src, cur, l, p->Cvec + (long)l * KM * KM, k[l], r[l], dst, 1.0, 0.0, true,
                     true);
        cur[l] = r[l];
        src = dst;
    }
    // bases: Z_l = B_l U_l[:, :r_l], the modes together
    fc::GemmArgs bases[3];
    for (int l = 0; l < 3; ++l) {
        bases[l] = prod(n, r[l], k[l], B[l], n, p->Cvec + (long)l * KM * KM, k[l], out.Z[l], n);
        out.r[l] = r[l];
    }
    gemm_group(c, false, false, bases, 3);
    p->max_seen_rank = std::max({p->max_seen_rank, r[0], r[1], r[2]});
}

// H_l X_l for the selected modes: through `apply.all` when the operator
// offers it (its products then go out grouped over the modes), else mode by
// mode.
template <class A, class = void>
struct has_all : std::false_type {};
template <class A>
struct has_all<A, std::void_t<decltype(&A::all)>> : std::true_type {};
template <class Apply>
void apply_modes(Apply& apply, const bool sel[3], double* const* X, const int q[3],
                 double* const* HX) {
    if constexpr (has_all<Apply>::value) {
        apply.all(sel, X, q, HX);
    } else {
        for (int l = 0; l < 3; ++l)
            if (sel[l]) apply(l, X[l], q[l], HX[l]);
    }
}

// Dominant subspaces of the three mode Grams H_l (given by `apply`, which
// writes H_l X to its output), the three modes in lockstep:
//  * start: the basis found at the same place of the previous iteration (a
//    warm start, within one solve) padded with 2 * margin random columns, or
//    kcap random columns; orthonormalised;
//  * one power step followed by a rank-revealing orthonormalisation;
//  * Rayleigh-Ritz: eigenpairs of X_l^T H_l X_l in one batched launch, then
//    W_l = X_l V_l[:, :pk_l] with pk_l = (smallest rank whose Ritz tail is
//    <= tail_budget) + margin, capped by the numerical rank.
//  * If a mode's Ritz tail leaves less than `margin` spare columns, its
//    subspace is enlarged (Ritz vectors plus random columns) and the power
//    step and Rayleigh-Ritz are repeated for that mode.
// Returns false if some H_l is zero.
// span[l] (optional, n x kcap[l]): columns spanning the whole range of H_l;
// then the start is exactly that span and no power step is needed;
// span_ortho[l] of its leading columns are already orthonormal.
template <class Apply>
bool find_subspaces(const Ctx& c, int site, const int kcap[3], Apply& apply, double tail_budget,
                    int margin, int pk[3], const double* const* span = nullptr,
                    const int* span_ortho = nullptr, const int* cold = nullptr) {
    fc_plan_s* p = c.p;
    const int n = c.n;
    WarmBasis& wb = p->warm[site];
    int kk[3], have[3], first_cols[3] = {0, 0, 0};
    bool exact[3], active[3], dropped[3] = {false, false, false};
    fc::CopyJobs starts;   // the start bases of the three modes, copied in one launch
    for (int l = 0; l < 3; ++l) {
        exact[l] = span && span[l];
        active[l] = true;
        const double* from = nullptr;
        if (exact[l]) {
            kk[l] = have[l] = kcap[l];
            first_cols[l] = span_ortho ? span_ortho[l] : 0;
            from = span[l];
        } else if (wb.valid) {
            have[l] = std::min(wb.pk[l], kcap[l]);
            // the earlier basis plus padding, and at least the cold-start size
            // (the input's rank may have grown since)
            kk[l] = std::min(kcap[l], std::max(have[l] + 2 * margin, cold ? cold[l] : 0));
            from = wb.W[l];
        } else {
            have[l] = 0;
            kk[l] = cold ? std::max(1, std::min(kcap[l], cold[l])) : kcap[l];
        }
        if (from && have[l] > 0) {
            fc::CopyJob& J = starts.job[starts.count++];
            J.src = from; J.lds = n; J.dst = p->Xs3[l]; J.ldd = n; J.rows = n; J.cols = have[l];
        }
    }
    HIPCHK(fc::copy_multi(starts, c.s));
    std::vector<double> th(3 * KM);
    for (int round = 0;; ++round) {
        // start bases of the active modes, orthonormalised together
        int start_done[3] = {0, 0, 0};
        fc::FillJobs fills;   // the random padding of the three modes, one launch
        for (int l = 0; l < 3; ++l) {
            if (!active[l]) continue;
            if (kk[l] > have[l]) {
                fc::FillJob& F = fills.job[fills.count++];
                F.n = n * (long)(kk[l] - have[l]);
                F.seed = 1234u + 7u * l + 101u * site + 7919u * round;
                F.x = p->Xs3[l] + (long)have[l] * n;
            }
            start_done[l] = exact[l] ? first_cols[l] : have[l];
        }
        HIPCHK(fc::fill_random_multi(fills, c.s));
        orthonormalize3(c, kk, p->Xs3, 1e-13, start_done, active);
        bool power[3] = {false, false, false};
        int before[3] = {0, 0, 0};
        for (int l = 0; l < 3; ++l) {
            if (!active[l]) continue;
            if (kk[l] == 0) return false;
            check_cols(c, p->Xs3[l], n, n, kk[l], "start basis", l);
            if (exact[l]) continue;
            // one power step moves the start into the range of H_l
            power[l] = true;
            before[l] = kk[l];
        }
        apply_modes(apply, power, p->Xs3, kk, p->HX3);
        const int none[3] = {0, 0, 0};
        orthonormalize3(c, kk, p->HX3, 1e-13, none, power);
        for (int l = 0; l < 3; ++l) {
            if (!power[l]) continue;
            dropped[l] = kk[l] < before[l];
            if (kk[l] == 0) return false;
            std::swap(p->Xs3[l], p->HX3[l]);
            check_cols(c, p->Xs3[l], n, n, kk[l], "power-step basis", l);
        }
        fc::EigJobs jobs;
        jobs.count = 0;
        fc::GemmArgs rr_mats[3];
        int nrr = 0;
        apply_modes(apply, active, p->Xs3, kk, p->HX3);
        for (int l = 0; l < 3; ++l) {
            if (!active[l]) continue;
            rr_mats[nrr++] = prod(kk[l], kk[l], n, p->Xs3[l], n, p->HX3[l], n,
                                  p->Bp3 + (long)l * KM * KM, kk[l]);
        }
        gemm_group(c, true, false, rr_mats, nrr);   // Rayleigh-Ritz matrices X^T H X
        for (int l = 0; l < 3; ++l) {
            if (!active[l]) continue;
            double* Bl = p->Bp3 + (long)l * KM * KM;
            fc::EigJob& J = jobs.job[jobs.count++];
            J.A = Bl; J.lda = kk[l]; J.k = kk[l];
            J.evals = p->Ev3 + l * KM; J.V = p->Evec3 + (long)l * KM * KM; J.ldv = kk[l];
            J.scratch = p->jac + (long)l * 6 * KM * KM;
            J.budget = tail_budget;   // vectors for the rank rule below only
            J.margin = margin;
        }
        HIPCHK(timed_launch(2, c.s, eig_flops(jobs), eig_bytes(jobs),
                            [&] { return fc::sym_eig_multi(jobs, c.s); }));
        d2h(c, th.data(), p->Ev3, 3 * KM);
        bool again = false;
        fc::CopyJobs keep;   // the modes finished this round, saved for a warm start
        fc::GemmArgs fin[3];   // their subspaces W_l = X_l V_l, formed together
        int nfin = 0;
        for (int l = 0; l < 3; ++l) {
            if (!active[l]) continue;
            double tail = 0;
            int rr = kk[l];
            for (int i = kk[l] - 1; i >= 0; --i) {
                tail += std::max(th[l * KM + i], 0.0);
                if (tail <= tail_budget) rr = i; else break;
            }
            int numrank = 0;
            const double tmax = std::max(th[l * KM], 0.0);
            while (numrank < kk[l] && th[l * KM + numrank] > 1e-17 * tmax) ++numrank;
            const double* Vl = p->Evec3 + (long)l * KM * KM;
            FC_TRACE_PRINT("subspace site %d round %d mode %d kk %d/%d rr %d numrank %d\n", site,
                           round, l, kk[l], kcap[l], rr, numrank);
            // Too few spare columns: restart from all Ritz vectors, enlarged.  Not
            // when the power step dropped columns: then the subspace already holds
            // the numerical range of H_l.
            if (!dropped[l] && !exact[l] && rr + margin > kk[l] && kk[l] < kcap[l] &&
                numrank == kk[l] && round < 3) {
                gemm(c, false, false, n, kk[l], kk[l], 1.0, p->Xs3[l], n, Vl, kk[l], 0.0, p->W[l], n);
                HIPCHK(fc::copy2d(n, kk[l], p->W[l], n, p->Xs3[l], n, c.s));
                have[l] = kk[l];
                kk[l] = std::min(kcap[l], std::max(kk[l], rr) + 2 * margin);
                again = true;
                continue;
            }
            const int use = std::min(std::max(numrank, 1), std::max(rr + margin, 1));
            check_cols(c, Vl, kk[l], kk[l], use, "Ritz vectors", l);
            fin[nfin++] = prod(n, use, kk[l], p->Xs3[l], n, Vl, kk[l], p->W[l], n);
            pk[l] = use;
            fc::CopyJob& J = keep.job[keep.count++];
            J.src = p->W[l]; J.lds = n; J.dst = wb.W[l]; J.ldd = n; J.rows = n; J.cols = use;
            wb.pk[l] = use;
            active[l] = false;
        }
        gemm_group(c, false, false, fin, nfin);
        for (int t = 0; t < nfin; ++t)
            check_cols(c, fin[t].C, n, n, fin[t].N, "subspace W", t);
        HIPCHK(fc::copy_multi(keep, c.s));
        if (!again) break;
    }
    wb.valid = true;
    return true;
}

// H_l X = B_l (M_l (B_l^T X)) for the sum truncation (B_l in Phi[l], M_l in
// SM[l]); all() runs the three stages for the selected modes with one
// grouped launch per stage (per-mode slices of Ys and Ts).
struct SumGramApply {
    const Ctx& c;
    const int* k;
    void operator()(int l, const double* X, int q, double* HXo) const {
        fc_plan_s* p = c.p;
        const int n = c.n;
        gemm(c, true, false, k[l], q, n, 1.0, p->Phi[l], n, X, n, 0.0, p->Ys, k[l]);
        gemm(c, false, false, k[l], q, k[l], 1.0, p->SM[l], k[l], p->Ys, k[l], 0.0, p->Ts, k[l]);
        gemm(c, false, false, n, q, k[l], 1.0, p->Phi[l], n, p->Ts, k[l], 0.0, HXo, n);
    }
    void all(const bool sel[3], double* const* X, const int q[3], double* const* HX) const {
        fc_plan_s* p = c.p;
        const int n = c.n;
        long need = 0;
        for (int l = 0; l < 3; ++l)
            if (sel[l]) need += (long)k[l] * q[l];
        if (g_ungrouped || need > p->ys_cap) {
            for (int l = 0; l < 3; ++l)
                if (sel[l]) (*this)(l, X[l], q[l], HX[l]);
            return;
        }
        fc::GemmArgs s1[3], s2[3], s3[3];
        int cnt = 0;
        long off = 0;
        for (int l = 0; l < 3; ++l) {
            if (!sel[l]) continue;
            double* Ysl = p->Ys + off;
            double* Tsl = p->Ts + off;
            off += (long)k[l] * q[l];
            s1[cnt] = prod(k[l], q[l], n, p->Phi[l], n, X[l], n, Ysl, k[l]);
            s2[cnt] = prod(k[l], q[l], k[l], p->SM[l], k[l], Ysl, k[l], Tsl, k[l]);
            s3[cnt] = prod(n, q[l], k[l], p->Phi[l], n, Tsl, k[l], HX[l], n);
            ++cnt;
        }
        gemm_group(c, true, false, s1, cnt);
        gemm_group(c, false, false, s2, cnt);
        gemm_group(c, false, false, s3, cnt);
    }
};

// ---- exact truncation of a short sum of Tucker tensors ---------------------
// T = sum_t c_t T_t (t < 4).  With the concatenated bases B_l = [Z_l^0 ...]
// (not orthonormal) and the block-diagonal core, the mode-l unfolding Gram
// is H_l = B_l M_l B_l^T, M_l[t,t'] = c_t c_t' core_t,(l) (G_b^{tt'} (x) G_a^{tt'})
// core_t',(l)^T with the cross Grams G^{tt'} = Z^t^T Z^t'.  Its dominant
// subspace comes from subspace iteration in R^n; T is projected onto it
// exactly, and the HOSVD of the projected core finishes the truncation.
// ||T||^2 = trace(M_l G_l) is exact, so the energy the subspace misses is
// known and charged to the tolerance.
void sum_trunc(const Ctx& c, const std::vector<std::pair<double, const Tucker*>>& terms_in,
               double tol_rel, double floor_abs, Tucker& out, const char* what, int site) {
    SiteClock clock(c, site);
    fc_plan_s* p = c.p;
    const int n = c.n;
    std::vector<std::pair<double, const Tucker*>> terms;
    for (auto& t : terms_in)
        if (t.first != 0.0 && !t.second->empty()) terms.push_back(t);
    if (terms.empty()) { out.r[0] = out.r[1] = out.r[2] = 0; return; }
    const int m = (int)terms.size();
    int k[3], off[4][3];
    for (int l = 0; l < 3; ++l) {
        int tot = 0;
        for (int t = 0; t < m; ++t) { off[t][l] = tot; tot += terms[t].second->r[l]; }
        k[l] = tot;
        if (tot > 256) throw FcError(FC_ERR_INTERNAL, std::string(what) + ": too many columns");
    }
    {
        // concatenated bases, every mode and term in one launch
        fc::CopyJobs cj;
        for (int l = 0; l < 3; ++l)
            for (int t = 0; t < m; ++t) {
                fc::CopyJob& J = cj.job[cj.count++];
                J.src = terms[t].second->Z[l]; J.lds = n;
                J.dst = p->Phi[l] + (long)off[t][l] * n; J.ldd = n;
                J.rows = n; J.cols = terms[t].second->r[l];
            }
        HIPCHK(fc::copy_multi(cj, c.s));
    }
    {
        // full Grams of the concatenated bases (k_l x k_l), the modes together
        fc::GemmArgs grams[3];
        for (int l = 0; l < 3; ++l)
            grams[l] = prod(k[l], k[l], n, p->Phi[l], n, p->Phi[l], n, p->SG[l], k[l]);
        gemm_group(c, true, false, grams, 3);
    }
    // block unfolding Grams M_l (k_l x k_l), symmetric: the blocks M[t,u],
    // u >= t, are computed and the ones below the diagonal are their
    // transposes.  With two terms each term's core is permuted once per mode
    // (into Cn2 and Cp); with more, per use.
    const bool hoist = m <= 2;
    for (int l = 0; l < 3; ++l) {
        const int a = (l == 0) ? 1 : 0, b = (l == 2) ? 1 : 2;
        const double* pcore[4] = {nullptr, nullptr, nullptr, nullptr};
        for (int t = 0; t < m; ++t) {
            const Tucker& Tt = *terms[t].second;
            pcore[t] = Tt.core;
            if (l != 0 && hoist) {
                double* dst = (t == 0) ? p->Cn2 : p->Cp;
                HIPCHK(fc::permute_core(Tt.r[0], Tt.r[1], Tt.r[2], l, 1, Tt.core, 0, dst, 0, c.s));
                pcore[t] = dst;
            }
        }
        if (hoist) {
            // the pairs t <= u of this mode in three grouped stages, on
            // per-pair slices of c1 and c2 when they fit
            long n1 = 0, n2c = 0;
            for (int t = 0; t < m; ++t)
                for (int u = t; u < m; ++u) {
                    int pt[3], pu[3];
                    perm_dims(terms[t].second->r, l, pt);
                    perm_dims(terms[u].second->r, l, pu);
                    n1 += (long)pu[0] * pu[1] * pt[2];
                    n2c += (long)pu[0] * pt[1] * pt[2];
                }
            if (!g_ungrouped && n1 <= p->cbig && n2c <= p->cbig) {
                fc::GemmArgs s1[3], s2[3], s3[3];
                int np = 0;
                long o1 = 0, o2 = 0;
                for (int t = 0; t < m; ++t)
                    for (int u = t; u < m; ++u) {
                        int pt[3], pu[3];
                        perm_dims(terms[t].second->r, l, pt);
                        perm_dims(terms[u].second->r, l, pu);
                        double* c1 = p->c1 + o1;
                        double* c2 = p->c2 + o2;
                        o1 += (long)pu[0] * pu[1] * pt[2];
                        o2 += (long)pu[0] * pt[1] * pt[2];
                        // c1 = core_u x_3 G_b^{tu}
                        s1[np] = prod(pu[0] * pu[1], pt[2], pu[2], pcore[u], (long)pu[0] * pu[1],
                                      p->SG[b] + off[t][b] + (long)off[u][b] * k[b], k[b], c1,
                                      (long)pu[0] * pu[1]);
                        // c2 = c1 x_2 G_a^{tu}, a batch over the third index
                        fc::GemmArgs g2 = prod(pu[0], pt[1], pu[1], c1, pu[0],
                                               p->SG[a] + off[t][a] + (long)off[u][a] * k[a], k[a],
                                               c2, pu[0]);
                        g2.batch = pt[2];
                        g2.strideA = (long)pu[0] * pu[1];
                        g2.strideB = 0;
                        g2.strideC = (long)pu[0] * pt[1];
                        s2[np] = g2;
                        // M[t,u] = c_t c_u core_t,(1) c2_(1)^T
                        fc::GemmArgs g3 = prod(pt[0], pu[0], pt[1] * pt[2], pcore[t], pt[0], c2,
                                               pu[0], p->SM[l] + off[t][l] + (long)off[u][l] * k[l],
                                               k[l]);
                        g3.alpha = terms[t].first * terms[u].first;
                        s3[np] = g3;
                        ++np;
                    }
                gemm_group(c, false, true, s1, np);
                gemm_group(c, false, true, s2, np);
                gemm_group(c, false, true, s3, np);
                continue;
            }
        }
        for (int t = 0; t < m; ++t) {
            const Tucker& Tt = *terms[t].second;
            int pt[3];
            perm_dims(Tt.r, l, pt);
            const double* coret = pcore[t];
            if (l != 0 && !hoist) {
                HIPCHK(fc::permute_core(Tt.r[0], Tt.r[1], Tt.r[2], l, 1, Tt.core, 0, p->Cn2, 0, c.s));
                coret = p->Cn2;
            }
            for (int u = t; u < m; ++u) {
                const Tucker& Tu = *terms[u].second;
                int pu[3];
                perm_dims(Tu.r, l, pu);
                const double* coreu = pcore[u];
                if (l != 0 && !hoist) {
                    HIPCHK(fc::permute_core(Tu.r[0], Tu.r[1], Tu.r[2], l, 1, Tu.core, 0, p->Cp, 0, c.s));
                    coreu = p->Cp;
                }
                // c1 = core_u x_3 G_b^{tu}   (G_b^{tu}: r_t,b x r_u,b block of SG[b])
                const int cur1[3] = {pu[0], pu[1], pu[2]};
                mode_product(c, coreu, cur1, 2, p->SG[b] + off[t][b] + (long)off[u][b] * k[b], k[b],
                             pt[2], p->c1);
                const int cur2[3] = {pu[0], pu[1], pt[2]};
                mode_product(c, p->c1, cur2, 1, p->SG[a] + off[t][a] + (long)off[u][a] * k[a], k[a],
                             pt[1], p->c2);
                // M[t,u] = c_t c_u core_t,(1) c2_(1)^T : (pt0 x pt1 pt2)(pt1 pt2 x pu0)
                gemm(c, false, true, pt[0], pu[0], pt[1] * pt[2], terms[t].first * terms[u].first,
                     coret, pt[0], p->c2, pu[0], 0.0, p->SM[l] + off[t][l] + (long)off[u][l] * k[l],
                     k[l]);
            }
        }
    }
    if (m > 1) {
        fc::SymJobs sj;
        for (int l = 0; l < 3; ++l) {
            fc::SymJob& J = sj.job[sj.count++];
            J.M = p->SM[l];
            J.k = k[l];
            J.nb = m;
            for (int t = 0; t < m; ++t) J.off[t] = off[t][l];
            J.off[m] = k[l];
        }
        HIPCHK(fc::sym_blocks(sj, c.s));
    }
    const double n2 = host_dot(c, (long)k[0] * k[0], p->SM[0], p->SG[0]);
    if (!std::isfinite(n2)) throw FcError(FC_ERR_NUMERIC, std::string(what) + ": non-finite");
    const double thr2 = std::max(tol_rel * tol_rel * n2, floor_abs * floor_abs);
    if (n2 <= thr2) { out.r[0] = out.r[1] = out.r[2] = 0; return; }
    // dominant subspaces of H_l = B M B^T
    int pk[3], kcap[3];
    SumGramApply apply{c, k};
    const double* span[3] = {nullptr, nullptr, nullptr};
    for (int l = 0; l < 3; ++l) {
        kcap[l] = std::min({p->pcap, n, k[l]});
        if (k[l] <= p->pcap && k[l] <= n) span[l] = p->Phi[l];   // range(H_l) within span(B_l)
    }
    int span_ortho[3];
    for (int l = 0; l < 3; ++l) span_ortho[l] = terms[0].second->r[l];
    if (!find_subspaces(c, site, kcap, apply, thr2 / 6.0, 8, pk, span, span_ortho)) {
        out.r[0] = out.r[1] = out.r[2] = 0;
        return;
    }
    // exact projection C = sum_t c_t core_t x_l (W_l^T Z_l^t), in FP64 on
    // every path: ||C||^2 decides the energy the subspace misses, which is
    // charged to the tolerance
    for (int l = 0; l < 3; ++l)
        gemm(c, true, false, pk[l], k[l], n, 1.0, p->W[l], n, p->Phi[l], n, 0.0,
             p->Map + (long)l * KM * 256, pk[l]);
    const long Csz = (long)pk[0] * pk[1] * pk[2];
    for (int t = 0; t < m; ++t) {
        const Tucker& T = *terms[t].second;
        int cur[3] = {T.r[0], T.r[1], T.r[2]};
        const double* src = T.core;
        double* bufs[2] = {p->Cn1, p->Cn2};
        for (int l = 0; l < 3; ++l) {
            const bool last = (l == 2);
            double* dst = last ? p->C : bufs[l & 1];
            mode_product(c, src, cur, l, p->Map + (long)l * KM * 256 + (long)off[t][l] * pk[l], pk[l],
                         pk[l], dst, last ? terms[t].first : 1.0, (last && t > 0) ? 1.0 : 0.0, false,
                         false);
            cur[l] = pk[l];
            src = dst;
        }
    }
    const double c2 = host_dot(c, Csz, p->C, p->C);
    const double missed = std::max(n2 - c2, 0.0);
    const double thr_core = std::max(thr2 - missed, 0.0);
    double* B[3] = {p->W[0], p->W[1], p->W[2]};
    hosvd_core(c, p->C, pk, B, thr_core, out, what);
}

// The Q diagonally scaled Grams C^q = A^T diag(D[:, q]) B (A n x M, B n x N,
// D n x Q, all ld n) as one batched product: C^q is M x N with ld M at
// C + q M N.  This is the row-wise Kronecker product of A and B contracted
// with D (E^T D with E[i, (j, c)] = A[i, j] B[i, c]) without forming E.
fc::GemmArgs scaled_gram(int M, int N, int n, int Q, const double* A, const double* B,
                         const double* D, double* C) {
    fc::GemmArgs g;
    g.M = M; g.N = N; g.K = n; g.batch = Q;
    g.A = A; g.lda = n; g.B = B; g.ldb = n; g.C = C; g.ldc = M; g.strideC = (long)M * N;
    g.d = D; g.strideD = n;
    return g;
}

// ---- truncation of a Hadamard product with a separable positive tensor ----
// T = D~ (.) P = sum_q P x_l diag(D_l[:,q]).  Subspace per mode from the
// block reduced HOSVD (sum over q of the unfolding Grams of the terms),
// exact projection of T onto it, then HOSVD of the projected core.
// Hh_l X = sum_q D^q Z M^q Z^T D^q X for the Hadamard truncation: the scaled
// Grams Y^q = Z^T D^q X (stack r q x Q, one batched launch), T^q = M^q Y^q,
// and sum_q D^q Z T^q in one fused launch (the row-wise Kronecker products
// Z (.) X and Z (.) D are never stored).  all() runs each stage for the
// selected modes in one launch, on per-mode slices of Ys and Ts when they
// fit (else mode by mode).
struct HadGramApply {
    const Ctx& c;
    const Separable& op;
    const Tucker& P;
    double* const* Mq;
    void operator()(int l, const double* X, int q, double* HXo) const {
        fc_plan_s* p = c.p;
        const int n = c.n, Q = op.Q;
        const int* r = P.r;
        {
            const fc::GemmArgs g1 = scaled_gram(r[l], q, n, Q, P.Z[l], X, op.D[l], p->Ys);
            gemm_group(c, true, false, &g1, 1);
        }
        gemm(c, false, false, r[l], q, r[l], 1.0, Mq[l], r[l], p->Ys, r[l], 0.0, p->Ts, r[l], Q,
             (long)r[l] * r[l], (long)r[l] * q, (long)r[l] * q);
        fc::KronJobs kj;
        fc::KronJob& J = kj.job[kj.count++];
        J.r = r[l]; J.p = q; J.Z = P.Z[l]; J.ldz = n; J.D = op.D[l]; J.T = p->Ts; J.out = HXo;
        J.ldo = n;
        kron_apply(c, Q, kj);
    }
    void all(const bool sel[3], double* const* X, const int q[3], double* const* HX) const {
        fc_plan_s* p = c.p;
        const int n = c.n, Q = op.Q;
        const int* r = P.r;
        long ny = 0;
        for (int l = 0; l < 3; ++l)
            if (sel[l]) ny += (long)r[l] * q[l] * Q;
        if (g_ungrouped || ny > p->ys_cap) {
            for (int l = 0; l < 3; ++l)
                if (sel[l]) (*this)(l, X[l], q[l], HX[l]);
            return;
        }
        fc::KronJobs kj;
        fc::GemmArgs s1[3], s2[3];
        int cnt = 0;
        long oy = 0;
        for (int l = 0; l < 3; ++l) {
            if (!sel[l]) continue;
            const long rq = (long)r[l] * q[l];
            double* Ysl = p->Ys + oy;
            double* Tsl = p->Ts + oy;
            oy += rq * Q;
            s1[cnt] = scaled_gram(r[l], q[l], n, Q, P.Z[l], X[l], op.D[l], Ysl);
            fc::GemmArgs g2 = prod(r[l], q[l], r[l], Mq[l], r[l], Ysl, r[l], Tsl, r[l]);
            g2.batch = Q;
            g2.strideA = (long)r[l] * r[l];
            g2.strideB = rq;
            g2.strideC = rq;
            s2[cnt] = g2;
            fc::KronJob& J = kj.job[kj.count++];
            J.r = r[l]; J.p = q[l]; J.Z = P.Z[l]; J.ldz = n; J.D = op.D[l]; J.T = Tsl;
            J.out = HX[l]; J.ldo = n;
            ++cnt;
        }
        gemm_group(c, true, false, s1, cnt);
        gemm_group(c, false, false, s2, cnt);
        kron_apply(c, Q, kj);
    }
};

void had_trunc(const Ctx& c, const Separable& op, const Tucker& P, double tol_rel,
               double floor_abs, Tucker& out, const char* what, int site) {
    SiteClock clock(c, site);
    fc_plan_s* p = c.p;
    const int n = c.n;
    const int Q = op.Q;
    if (P.empty()) { out.r[0] = out.r[1] = out.r[2] = 0; return; }
    const int* r = P.r;
    // 1. diagonal Grams Gd_l^q = Z_l^T diag(D_l[:,q]^2) Z_l  -> stack r_l^2 x Q,
    //    the Q terms of the three modes as batched scaled Grams in one launch
    {
        fc::GemmArgs gd[3];
        for (int l = 0; l < 3; ++l)
            gd[l] = scaled_gram(r[l], r[l], n, Q, P.Z[l], P.Z[l], op.D2[l], p->Gd[l]);
        if (g_ungrouped)
            for (int l = 0; l < 3; ++l) gemm_group(c, true, false, gd + l, 1);
        else
            gemm_group(c, true, false, gd, 3);
    }
    // 2. per-term unfolding Grams M_l^q = core_(l) (G_b^q (x) G_a^q) core_(l)^T
    double* Mq[3];
    for (int l = 0; l < 3; ++l) Mq[l] = p->Mq + (long)l * Q * p->rcap * p->rcap;
    const long csz3 = (long)r[0] * r[1] * r[2];
    const bool grouped = !g_ungrouped && 3L * Q * csz3 <= p->cbig;
    if (grouped) {
        // all terms of the three modes at once, each mode on its own slices
        // of c1 and c2 (the permuted cores of modes 1 and 2 in Cp and Cn2)
        HIPCHK(fc::permute_core12(r[0], r[1], r[2], P.core, p->Cp, p->Cn2, c.s));
        const double* cores[3] = {P.core, p->Cp, p->Cn2};
        fc::GemmArgs s1[3], s2[3], s3[3];
        for (int l = 0; l < 3; ++l) {
            int pd[3];
            perm_dims(r, l, pd);
            const int a = (l == 0) ? 1 : 0, b = (l == 2) ? 1 : 2;
            double* c1 = p->c1 + (long)l * Q * csz3;
            double* c2 = p->c2 + (long)l * Q * csz3;
            // c1^q = core x_3 G_b^q
            fc::GemmArgs g1 = prod(pd[0] * pd[1], pd[2], pd[2], cores[l], (long)pd[0] * pd[1],
                                   p->Gd[b], pd[2], c1, (long)pd[0] * pd[1]);
            g1.batch = Q;
            g1.strideA = 0;
            g1.strideB = (long)r[b] * r[b];
            g1.strideC = csz3;
            s1[l] = g1;
            // c2^q = c1^q x_2 G_a^q: batch over (q, k)
            fc::GemmArgs g2 = prod(pd[0], pd[1], pd[1], c1, pd[0], p->Gd[a], pd[1], c2, pd[0]);
            g2.batch = Q * pd[2];
            g2.inner = pd[2];
            g2.strideA = csz3;
            g2.strideB = (long)r[a] * r[a];
            g2.strideC = csz3;
            g2.strideAin = (long)pd[0] * pd[1];
            g2.strideBin = 0;
            g2.strideCin = (long)pd[0] * pd[1];
            s2[l] = g2;
            // M^q = core_(1) c2^q_(1)^T
            fc::GemmArgs g3 = prod(pd[0], pd[0], pd[1] * pd[2], cores[l], pd[0], c2, pd[0], Mq[l],
                                   pd[0]);
            g3.batch = Q;
            g3.strideA = 0;
            g3.strideB = csz3;
            g3.strideC = (long)pd[0] * pd[0];
            s3[l] = g3;
        }
        gemm_group(c, false, true, s1, 3);
        gemm_group(c, false, true, s2, 3);
        gemm_group(c, false, true, s3, 3);
    }
    for (int l = 0; l < 3 && !grouped; ++l) {
        int pd[3];
        perm_dims(r, l, pd);
        const int a = (l == 0) ? 1 : 0, b = (l == 2) ? 1 : 2;   // other modes in order
        const double* core = P.core;
        if (l != 0) {
            HIPCHK(fc::permute_core(r[0], r[1], r[2], l, 1, P.core, 0, p->Cp, 0, c.s));
            core = p->Cp;
        }
        const long csz = (long)r[0] * r[1] * r[2];
        // as many terms per pass as c1 and c2 hold at the actual core size
        const long qstep = std::max<long>(1, std::min<long>(Q, p->cbig / std::max<long>(1, csz)));
        for (long q0 = 0; q0 < Q; q0 += qstep) {
            const int qc = (int)std::min<long>(qstep, Q - q0);
            // c1^q = core x_3 G_b^q : (pd0 pd1 x pd2) * G^T
            gemm(c, false, true, pd[0] * pd[1], pd[2], pd[2], 1.0, core, (long)pd[0] * pd[1],
                 p->Gd[b] + q0 * (long)r[b] * r[b], pd[2], 0.0, p->c1, (long)pd[0] * pd[1], qc, 0,
                 (long)r[b] * r[b], csz);
            // c2^q = c1^q x_2 G_a^q : batch over (q, k)
            gemm(c, false, true, pd[0], pd[1], pd[1], 1.0, p->c1, pd[0],
                 p->Gd[a] + q0 * (long)r[a] * r[a], pd[1], 0.0, p->c2, pd[0], qc * pd[2], csz,
                 (long)r[a] * r[a], csz, pd[2], (long)pd[0] * pd[1], 0, (long)pd[0] * pd[1]);
            // M^q = core_(1) c2^q_(1)^T
            gemm(c, false, true, pd[0], pd[0], pd[1] * pd[2], 1.0, core, pd[0], p->c2, pd[0], 0.0,
                 Mq[l] + q0 * (long)pd[0] * pd[0], pd[0], qc, 0, csz, (long)pd[0] * pd[0]);
        }
    }
    // trace = sum_q ||T_q||^2 = sum_q <M_0^q, Gd_0^q>
    const double trH = host_dot(c, (long)Q * r[0] * r[0], Mq[0], p->Gd[0]);
    if (!std::isfinite(trH)) throw FcError(FC_ERR_NUMERIC, std::string(what) + ": non-finite");
    if (trH <= 0) { out.r[0] = out.r[1] = out.r[2] = 0; return; }
    const double tau2_est = std::max(tol_rel * tol_rel * trH, floor_abs * floor_abs);
    // 3. dominant subspaces of Hh_l = sum_q D^q Z M^q Z^T D^q
    int pk[3], kcap[3];
    HadGramApply apply{c, op, P, Mq};
    // a cold start (no basis from an earlier call at this site) begins with
    // twice the input rank plus the margin; the search enlarges it when the
    // Ritz tail needs more
    int cold[3];
    for (int l = 0; l < 3; ++l) {
        kcap[l] = std::min({p->pcap, n, Q * r[l]});
        cold[l] = 2 * r[l] + 32;
    }
    if (!find_subspaces(c, site, kcap, apply, tau2_est / 3.0, 16, pk, nullptr, nullptr, cold)) {
        out.r[0] = out.r[1] = out.r[2] = 0;
        return;
    }
    // 4. projection A_l^q = W_l^T D^q Z_l -> stack (pk*r x Q): in FP64 the
    //    scaled Grams of the three modes in one launch; on the FP32 matrix
    //    cores (mixed inner solve) the row-wise Kronecker products contracted
    //    with D
    if (!c.lowp) {
        fc::GemmArgs pa[3];
        for (int l = 0; l < 3; ++l)
            pa[l] = scaled_gram(pk[l], r[l], n, Q, p->W[l], P.Z[l], op.D[l], p->As[l]);
        if (g_ungrouped)
            for (int l = 0; l < 3; ++l) gemm_group(c, true, false, pa + l, 1);
        else
            gemm_group(c, true, false, pa, 3);
    } else if (!g_ungrouped &&
               (long)n * (pk[0] * r[0] + pk[1] * r[1] + pk[2] * r[2]) <= p->e_cap) {
        fc::RowJobs kr;
        double* El[3];
        long oe = 0;
        for (int l = 0; l < 3; ++l) {
            El[l] = p->E + oe;
            oe += (long)n * pk[l] * r[l];
            fc::RowJob& J = kr.job[kr.count++];
            J.r = pk[l]; J.p = r[l]; J.Z = p->W[l]; J.ldz = n; J.X = P.Z[l]; J.ldx = n;
            J.out = El[l];
        }
        HIPCHK(fc::rowkron_multi(n, kr, c.s));
        for (int l = 0; l < 3; ++l)
            gemmb(c, true, false, pk[l] * r[l], Q, n, 1.0, El[l], n, op.D[l], n, 0.0, p->As[l],
                  (long)pk[l] * r[l]);
    } else {
        for (int l = 0; l < 3; ++l) {
            HIPCHK(fc::rowkron(n, pk[l], r[l], p->W[l], n, P.Z[l], n, p->E, c.s));
            gemmb(c, true, false, pk[l] * r[l], Q, n, 1.0, p->E, n, op.D[l], n, 0.0, p->As[l],
                  (long)pk[l] * r[l]);
        }
    }
    // 5. C = sum_q core x_1 A_0^q x_2 A_1^q x_3 A_2^q
    const long csz = (long)r[0] * r[1] * r[2];
    const long t1sz = (long)pk[0] * r[1] * r[2];
    const long t2sz = (long)pk[0] * pk[1] * r[2];
    const long qstep =
        std::max<long>(1, std::min<long>(Q, p->cbig / std::max<long>(1, std::max(t1sz, t2sz))));
    for (long q0 = 0; q0 < Q; q0 += qstep) {
        const int qc = (int)std::min<long>(qstep, Q - q0);
        // T1^q = A_0^q core_(1): (pk0 x r0)(r0 x r1 r2)
        gemmb(c, false, false, pk[0], r[1] * r[2], r[0], 1.0, p->As[0] + q0 * pk[0] * (long)r[0],
              pk[0], P.core, r[0], 0.0, p->T1, pk[0], qc, (long)pk[0] * r[0], 0, t1sz);
        // T2^q = T1^q x_2 A_1^q: batch (q, k)
        gemmb(c, false, true, pk[0], pk[1], r[1], 1.0, p->T1, pk[0],
              p->As[1] + q0 * pk[1] * (long)r[1], pk[1], 0.0, p->T2, pk[0], qc * r[2], t1sz,
              (long)pk[1] * r[1], t2sz, r[2], (long)pk[0] * r[1], 0, (long)pk[0] * pk[1]);
        // C += [T2^q]_q [A_2^q]_q^T  ((pk0 pk1) x (qc r2)) ((qc r2) x pk2)
        gemmb(c, false, true, pk[0] * pk[1], pk[2], qc * r[2], 1.0, p->T2, (long)pk[0] * pk[1],
              p->As[2] + q0 * pk[2] * (long)r[2], pk[2], q0 == 0 ? 0.0 : 1.0, p->C,
              (long)pk[0] * pk[1]);
    }
    const long Csz = (long)pk[0] * pk[1] * pk[2];
    HIPCHK(fc::dot_long(Csz, p->C, p->C, p->scal + 256, p->dotcnt, p->scal, c.s));
    // 6. a-posteriori check of the subspaces: the energy of T outside them,
    //    ||T - PT||^2, estimated with S rank-1 Gaussian probes
    //    g_t = g_0,t (x) g_1,t (x) g_2,t (E <X, g_t>^2 = ||X||^2), read back with
    //    ||PT||^2 = ||C||^2 and charged to the core's budget
    const long per_probe = (long)r[1] * r[2] * Q;
    int S = (int)std::min<long>(8, p->cbig / std::max<long>(1, per_probe));
    if ((long)S * Q * (r[0] + r[1] + r[2]) > p->ys_cap) S = 0;
    if (S >= 2) {
        fc::FillJobs fills;
        for (int l = 0; l < 3; ++l) {
            fc::FillJob& F = fills.job[fills.count++];
            F.n = (long)n * S;
            F.seed = 4099u + 7u * l + 101u * site;
            F.x = p->Xs3[l];
        }
        HIPCHK(fc::fill_random_multi(fills, c.s));
        fc::GemmArgs ug[3], vg[3];
        double* Ul[3];
        long ou = 0;
        for (int l = 0; l < 3; ++l) {
            Ul[l] = p->Ys + ou;
            ou += (long)r[l] * Q * S;
            // U_l,t = Z_l^T diag(g_l,t) D_l, the S probes as a batch
            ug[l] = scaled_gram(r[l], Q, n, S, P.Z[l], op.D[l], p->Xs3[l], Ul[l]);
            vg[l] = prod(pk[l], S, n, p->W[l], n, p->Xs3[l], n, p->Map + (long)l * KM * 256, pk[l]);
        }
        gemm_group(c, true, false, ug, 3);
        gemm_group(c, true, false, vg, 3);
        // Mb_t = core_(1)^T U_0,t  (r1 r2 x Q per probe)
        gemm(c, true, false, r[1] * r[2], Q, r[0], 1.0, P.core, r[0], Ul[0], r[0], 0.0, p->T1,
             (long)r[1] * r[2], S, 0, (long)r[0] * Q, per_probe);
        // Yv_t = C_(1)^T v_0,t  (pk1 pk2 x 1 per probe)
        const long ppk = (long)pk[1] * pk[2];
        gemm(c, true, false, (int)ppk, S, pk[0], 1.0, p->C, pk[0], p->Map, pk[0], 0.0, p->T2, ppk);
        fc::ProbeSums ps;
        ps.p[0].r1 = r[1]; ps.p[0].r2 = r[2]; ps.p[0].Q = Q;
        ps.p[0].M = p->T1; ps.p[0].mstride = per_probe;
        ps.p[0].U1 = Ul[1]; ps.p[0].U2 = Ul[2];
        ps.p[1].r1 = pk[1]; ps.p[1].r2 = pk[2]; ps.p[1].Q = 1;
        ps.p[1].M = p->T2; ps.p[1].mstride = ppk;
        ps.p[1].U1 = p->Map + (long)KM * 256; ps.p[1].U2 = p->Map + 2L * KM * 256;
        ps.out = p->scal + 1;
        HIPCHK(fc::probe_sums(ps, S, c.s));
    }
    double vals[1 + 2 * 8];
    d2h(c, vals, p->scal, 1 + 2 * (S >= 2 ? S : 0));
    const double n2 = vals[0];
    if (!std::isfinite(n2)) throw FcError(FC_ERR_NUMERIC, std::string(what) + ": non-finite");
    double missed = 0.0;
    for (int t = 0; S >= 2 && t < S; ++t) {
        const double dlt = vals[1 + 2 * t] - vals[2 + 2 * t];
        missed += dlt * dlt / S;
    }
    const double thr2 = std::max(tol_rel * tol_rel * n2, floor_abs * floor_abs);
    if (n2 <= thr2) { out.r[0] = out.r[1] = out.r[2] = 0; return; }
    // the estimate's spread over S probes: charge twice the estimate
    const double charge = 2.0 * missed;
    p->worst_missed = std::max(p->worst_missed, charge / thr2);
    FC_TRACE_PRINT("%s: missed-energy estimate %.3e of budget %.3e (%d probes)\n", what, missed,
                   thr2, S);
    double* B[3] = {p->W[0], p->W[1], p->W[2]};
    hosvd_core(c, p->C, pk, B, std::max(thr2 - charge, 0.0), out, what);
    (void)csz;
}

const Separable& active_pc(const fc_plan_s* p) {
    return p->pc_kind == FC_PRECOND_LAPLACE ? p->pcA : p->pc;
}

double active_pc_err(const fc_plan_s* p) {
    return p->pc_kind == FC_PRECOND_LAPLACE ? p->pcA_err : p->pc_err;
}

// Z = trunc(precond(R)) for an iterate in eigen-coordinates.  Case (B): the
// Hadamard product with D~_p in the same coordinates.  Case (A) (eqn
// Lap3DtimesX): the factors go to the sine basis (W_l Z_l, still
// orthonormal), the Hadamard product with the Laplacian's symbol is truncated
// there, and the result's factors come back with W_l^T.
void apply_precond(const Ctx& c, const Tucker& R, double tol_rel, Tucker& Z, const char* what,
                   int site) {
    fc_plan_s* p = c.p;
    if (p->pc_kind != FC_PRECOND_LAPLACE) {
        had_trunc(c, p->pc, R, tol_rel, 0.0, Z, what, site);
        return;
    }
    if (R.empty()) { Z.r[0] = Z.r[1] = Z.r[2] = 0; return; }
    const int n = c.n;
    Tucker& tmp = p->slot[13];
    Tucker Rs;
    {
        KindTag tag(3);
        fc::GemmArgs to_sine[3];
        for (int l = 0; l < 3; ++l) {
            Rs.r[l] = R.r[l];
            Rs.Z[l] = tmp.Z[l];
            to_sine[l] = prod(n, R.r[l], n, p->Wsin[l], n, R.Z[l], n, Rs.Z[l], n);
        }
        gemm_group(c, false, false, to_sine, 3);
    }
    Rs.core = R.core;
    had_trunc(c, p->pcA, Rs, tol_rel, 0.0, Z, what, site);
    if (Z.empty()) return;
    {
        KindTag tag(3);
        fc::GemmArgs back[3];
        for (int l = 0; l < 3; ++l)
            back[l] = prod(n, Z.r[l], n, p->WsinT[l], n, Z.Z[l], n, tmp.Z[l], n);
        gemm_group(c, false, false, back, 3);
    }
    for (int l = 0; l < 3; ++l) std::swap(Z.Z[l], tmp.Z[l]);
}

// ---- canonical -> Tucker (exact unfolding spectra) ------------------------
// Factors X_l (n x m, ld n) and weights w (m, device, may be null).
void canon_to_tucker(const Ctx& c, int m, const double* w, const double* const X[3],
                     double tol_rel, Tucker& out, const char* what) {
    fc_plan_s* p = c.p;
    const int n = c.n;
    int k[3];
    for (int l = 0; l < 3; ++l) {
        HIPCHK(fc::copy2d(n, m, X[l], n, p->Phi[l], n, c.s));
    }
    int cnt[3] = {m, m, m};
    {
        const int none[3] = {0, 0, 0};
        const bool all[3] = {true, true, true};
        orthonormalize3(c, cnt, p->Phi, 1e-13, none, all);
    }
    for (int l = 0; l < 3; ++l) {
        k[l] = cnt[l];
        if (k[l] > KM) throw FcError(FC_ERR_INTERNAL, std::string(what) + ": input basis > 128");
        if (k[l] == 0) { out.r[0] = out.r[1] = out.r[2] = 0; return; }
    }
    // coefficients M_l = Phi_l^T X_l  (k_l x m); scale M_2 columns by w
    double* Ml[3];
    {
        fc::GemmArgs coefs[3];
        for (int l = 0; l < 3; ++l) {
            Ml[l] = p->cf[l];
            coefs[l] = prod(k[l], m, n, p->Phi[l], n, X[l], n, Ml[l], k[l]);
        }
        gemm_group(c, true, false, coefs, 3);
    }
    if (w) HIPCHK(fc::scale_cols(k[2], m, Ml[2], k[2], w, 0, c.s));
    // Khatri-Rao: KR[(i,j), s] = M0[i,s] M1[j,s]  -> use rowkron on transposes: build
    // M0^T (m x k0) and M1^T (m x k1), then rowkron gives E[s, i + k0 j]
    double* M0t = p->Ys;
    double* M1t = p->Ts;
    HIPCHK(fc::transpose(k[0], m, Ml[0], k[0], M0t, m, c.s));
    HIPCHK(fc::transpose(k[1], m, Ml[1], k[1], M1t, m, c.s));
    HIPCHK(fc::rowkron(m, k[0], k[1], M0t, m, M1t, m, p->E, c.s));
    // core_(3)^T = KR^T-ish: C[(i,j), kk] = sum_s E[s, (i,j)] M2[kk, s]
    gemm(c, true, true, k[0] * k[1], k[2], m, 1.0, p->E, m, Ml[2], k[2], 0.0, p->C,
         (long)k[0] * k[1]);
    const long csz = (long)k[0] * k[1] * k[2];
    const double n2 = host_dot(c, csz, p->C, p->C);
    if (!std::isfinite(n2)) throw FcError(FC_ERR_NUMERIC, std::string(what) + ": non-finite input");
    const double thr2 = tol_rel * tol_rel * n2;
    if (n2 <= 0) { out.r[0] = out.r[1] = out.r[2] = 0; return; }
    double* B[3] = {p->Phi[0], p->Phi[1], p->Phi[2]};
    hosvd_core(c, p->C, k, B, thr2, out, what);
}

double tucker_inner(const Ctx& c, const Tucker& A, const Tucker& B) {
    fc_plan_s* p = c.p;
    const int n = c.n;
    if (A.empty() || B.empty()) return 0.0;
    for (int l = 0; l < 3; ++l)
        gemm(c, true, false, A.r[l], B.r[l], n, 1.0, A.Z[l], n, B.Z[l], n, 0.0,
             p->Map + (long)l * KM * KM, A.r[l]);
    int cur[3] = {B.r[0], B.r[1], B.r[2]};
    const double* src = B.core;
    double* bufs[3] = {p->Cn1, p->Cn2, p->Cn1};
    for (int l = 0; l < 3; ++l) {
        double* dst = (l == 2) ? p->Cp : bufs[l];
        mode_product(c, src, cur, l, p->Map + (long)l * KM * KM, A.r[l], A.r[l], dst);
        cur[l] = A.r[l];
        src = dst;
    }
    return host_dot(c, A.csize(), A.core, p->Cp);
}

double tucker_norm2(const Ctx& c, const Tucker& A) {
    if (A.empty()) return 0.0;
    return host_dot(c, A.csize(), A.core, A.core);
}

void check_orth(const Ctx& c, const Tucker& T, const char* what) {
    if (!g_check || T.empty()) return;
    for (int l = 0; l < 3; ++l) check_cols(c, T.Z[l], c.n, c.n, T.r[l], what, l);
}

void tucker_copy(const Ctx& c, const Tucker& src, Tucker& dst, double scale = 1.0) {
    for (int l = 0; l < 3; ++l) {
        HIPCHK(fc::copy2d(c.n, src.r[l], src.Z[l], c.n, dst.Z[l], c.n, c.s));
        dst.r[l] = src.r[l];
    }
    HIPCHK(fc::axpby(src.csize(), scale, src.core, 0.0, dst.core, c.s));
}

// ---- Tucker -> canonical (T2C) and output in grid coordinates -------------
// The core of a HOSVD-truncated tensor is all-orthogonal; each mode-3 slice
// core[:,:,nu] is split by its SVD (eigenpairs of the slice Gram), and
// (slice, singular value) terms are dropped smallest first while the dropped
// energy stays within budget2 (Appendix 1).  Selection and coefficient
// assembly run on the device; the host reads the kept count only.
// Returns the rank; writes nothing if the rank exceeds cap.
int tucker_to_canon_out(const Ctx& c, const Tucker& X, double budget2, bool to_grid, int cap,
                        double* w_u, double* const U[3]) {
    fc_plan_s* p = c.p;
    const int n = c.n;
    if (X.empty()) return 0;
    const int r0 = X.r[0], r1 = X.r[1], r2 = X.r[2];
    // slice Grams S_nu = core[:,:,nu]^T core[:,:,nu]  (r1 x r1), batch r2
    gemm(c, true, false, r1, r1, r0, 1.0, X.core, r0, X.core, r0, 0.0, p->Bp, r1, r2,
         (long)r0 * r1, (long)r0 * r1, (long)r1 * r1);
    HIPCHK(fc::sym_eig(r1, r2, p->Bp, r1, (long)r1 * r1, p->Ev, p->Evec, r1, (long)r1 * r1, p->jac, c.s));
    HIPCHK(fc::t2c_select(r1 * r2, p->Ev, budget2, p->t2c_ws, p->t2c_keep, p->icount + 8, c.s));
    int K = 0;
    d2h(c, &K, p->icount + 8, 1);
    if (K > cap || K == 0) return K;
    HIPCHK(fc::t2c_coef(r0, r1, r2, K, X.core, p->Evec, p->Ev, p->t2c_keep, p->cf[0], p->cf[1],
                        p->cf[2], w_u, c.s));
    const int rr[3] = {r0, r1, r2};
    const double* Zl[3] = {X.Z[0], X.Z[1], X.Z[2]};
    if (to_grid) {
        // exit transform V_l Z_l of the three bases in one launch
        KindTag tag(3);
        double* G[3] = {p->tmpn, p->tmpn2, p->Xs3[0]};
        fc::GemmArgs tr[3];
        for (int l = 0; l < 3; ++l) {
            tr[l] = prod(n, rr[l], n, p->V[l], n, X.Z[l], n, G[l], n);
            Zl[l] = G[l];
        }
        gemm_group(c, false, false, tr, 3);
    }
    fc::GemmArgs outs[3];
    for (int l = 0; l < 3; ++l) outs[l] = prod(n, K, rr[l], Zl[l], n, p->cf[l], rr[l], U[l], n);
    gemm_group(c, false, false, outs, 3);
    // exact unit columns (the bases are orthonormal only to rounding)
    HIPCHK(fc::normalize_factors(n, K, U[0], U[1], U[2], n, w_u, c.s));
    sync(c);
    return K;
}

void reset_warm(fc_plan_s* p) {
    for (int st = 0; st < NSITES; ++st) p->warm[st].valid = false;
}

void alloc_workspace(fc_plan_s* p) {
    const int n = p->n;
    const long rc = p->rcap, pc = p->pcap;
    const int Q = std::max({p->op.Q, p->pc.Q, p->st.Q, p->pcA.Q});
    Arena& A = p->arena;
    for (int s = 0; s < 14; ++s) {
        for (int l = 0; l < 3; ++l) p->slot[s].Z[l] = A.alloc((size_t)n * rc);
        p->slot[s].core = A.alloc((size_t)rc * rc * rc);
    }
    const long ecols = std::max(rc * rc, pc * rc);
    p->e_cap = std::max<long>((long)n * ecols, 256L * KM * KM);
    p->E = A.alloc((size_t)p->e_cap);
    for (int l = 0; l < 3; ++l) p->Gd[l] = A.alloc((size_t)Q * rc * rc);
    p->Mq = A.alloc((size_t)3 * Q * rc * rc);
    p->qchunk = std::max<long>(1, std::min<long>(Q, (8L << 20) / std::max<long>(1, rc * rc * rc)));
    // c1/c2 and T1/T2 need qchunk cores of up to pc*pc*rc
    const long big = p->qchunk * std::max(rc * rc * rc, pc * pc * rc);
    p->cbig = big;
    p->c1 = A.alloc(big);
    p->c2 = A.alloc(big);
    p->T1 = p->c1;
    p->T2 = p->c2;
    p->Xs = A.alloc((size_t)n * pc);
    p->HX = A.alloc((size_t)n * pc);
    p->ys_cap = std::max<long>(rc * pc * Q, 256L * KM);
    p->Ys = A.alloc((size_t)p->ys_cap);
    p->Ts = A.alloc((size_t)p->ys_cap);
    p->Bp = A.alloc((size_t)std::max<long>(pc * pc, rc * rc * rc));
    p->Ev = A.alloc((size_t)std::max<long>(pc, rc * rc));
    p->Evec = A.alloc((size_t)std::max<long>(pc * pc, rc * rc * rc));
    for (int l = 0; l < 3; ++l) {
        p->W[l] = A.alloc((size_t)n * pc);
        p->As[l] = A.alloc((size_t)pc * rc * Q);
        p->Phi[l] = A.alloc((size_t)n * 256);
        p->cf[l] = A.alloc((size_t)std::max<long>(KM * 256, rc * rc * rc));
        p->Yh[l] = A.alloc((size_t)n * 256);
    }
    const size_t kcube = (size_t)KM * KM * KM;
    p->C = A.alloc(kcube);
    p->Cp = A.alloc(kcube);
    p->Cn1 = A.alloc(kcube);
    p->Cn2 = A.alloc(kcube);
    p->Cg = A.alloc((size_t)3 * KM * KM);
    p->Cev = A.alloc((size_t)3 * KM);
    p->Cvec = A.alloc((size_t)3 * KM * KM);
    p->Map = A.alloc((size_t)3 * KM * 256);
    for (int l = 0; l < 3; ++l) {
        p->SG[l] = A.alloc((size_t)256 * 256);
        p->SM[l] = A.alloc((size_t)256 * 256);
    }
    p->jac = A.alloc((size_t)std::max<long>(3L * 6 * KM * KM, (long)rc * (rc + 1) * (rc + 1)));
    p->scal = A.alloc(512);
    p->tmpn = A.alloc((size_t)n * std::max<long>(rc, 256));
    p->tmpn2 = A.alloc((size_t)n * std::max<long>(rc, 256));
    p->icount = A.alloc_int(16);
    p->t2c_keep = A.alloc_int((size_t)rc * rc);
    {
        long np2 = 1;
        while (np2 < rc * rc) np2 <<= 1;
        p->t2c_ws = A.alloc((size_t)(12 * np2 + 7) / 8);
    }
    p->qrN = A.alloc(3 * 512);
    p->qrC = A.alloc(3 * 256 * 16);
    p->qrKeep = A.alloc_int(3 * 512);
    for (int l = 0; l < 3; ++l) {
        p->Xs3[l] = A.alloc((size_t)n * pc);
        p->HX3[l] = A.alloc((size_t)n * pc);
    }
    p->Bp3 = A.alloc((size_t)3 * KM * KM);
    for (int st = 0; st < NSITES; ++st)
        for (int l = 0; l < 3; ++l) p->warm[st].W[l] = A.alloc((size_t)n * pc);
    p->Ev3 = A.alloc((size_t)3 * KM);
    p->Evec3 = A.alloc((size_t)3 * KM * KM);
    p->splitws_cap = 8L << 20;
    p->splitws = A.alloc((size_t)p->splitws_cap);
    p->dflag = A.alloc_int(4);
    p->dotcnt = (unsigned*)A.alloc_int(1);
    const unsigned zero = 0;
    if (hipMemcpy(p->dotcnt, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
        throw FcError(FC_ERR_HIP, "hipMemcpy failed");
}


double f_control(double s, double alpha, double beta, double gamma) {
    return beta * std::pow(s, -alpha) + (gamma / beta) * std::pow(s, alpha);
}

// Operator D~ ~ f(s), f(s) = s g(s), g(s) = beta s^(-alpha-1) + (gamma/beta) s^(alpha-1):
// g is completely monotone, so g ~ sum_k c_k exp(-t_k s) with c_k > 0 and
// s exp(-t s) = (l1 + l2 + l3) exp(-t l1) exp(-t l2) exp(-t l3) gives three
// separable terms per exponential.  alpha = 0 and alpha = 1 carry exact
// constant / linear parts.
void build_operator(fc_plan_s* p, double smin, double smax) {
    const int n = p->n;
    const double a = p->alpha, b = p->beta, gm = p->gamma;
    Separable& S = p->op;
    auto add_term = [&](double w, const double* t_or_null, double t, int lambda_mode) {
        S.w.push_back(w);
        for (int l = 0; l < 3; ++l) {
            for (int i = 0; i < n; ++i) {
                const double lam = p->lam[l][i];
                double v = t_or_null ? std::exp(-t * lam) : 1.0;
                if (l == lambda_mode) v *= lam;
                S.F[l].push_back(v);
            }
        }
        S.Q++;
    };
    if (a == 0.0) {
        add_term(b + gm / b, nullptr, 0.0, -1);
        p->op_err = 0.0;
        return;
    }
    // alpha = 1: g = gamma/beta + beta s^-2 carries an exact constant.
    const double cexact = (a == 1.0) ? gm / b : 0.0;
    auto g = [&](double s) { return b * std::pow(s, -a - 1.0) + (gm / b) * std::pow(s, a - 1.0); };
    auto h = [&](double s) { return g(s) - cexact; };
    std::vector<double> t, cc;
    double cfit = 0.0, err = 1e300;
    // node range: the fastest useful exponential decays over ~ln(1/acc)/s_min,
    // the slowest is replaced by the constant term below ~acc/s_max
    const double t_hi = (std::log(1.0 / p->op_acc) + 10.0) / smin;
    const double t_lo = std::pow(p->op_acc, 0.7) / smax;
    for (double hstep : {0.7, 0.6, 0.5, 0.42, 0.35}) {
        if (!fc::fit_expsum_nnls(h, g, smin, smax, t_lo, t_hi, hstep, a < 1.0, t, cc, cfit, err))
            continue;
        if (err <= p->op_acc) break;
    }
    if (!(err <= p->op_acc))
        throw FcError(FC_ERR_NUMERIC, "operator exponential sum misses the accuracy gate (err " +
                                          std::to_string(err) + ")");
    const double c0 = cexact + cfit;
    if (c0 > 0.0)
        for (int m = 0; m < 3; ++m) add_term(c0, nullptr, 0.0, m);
    for (int k = 0; k < (int)t.size(); ++k)
        for (int m = 0; m < 3; ++m) add_term(cc[k], &t[0], t[k], m);
    // gate on the spectrum: |D~(s)/f(s) - 1| over a dense grid of [smin, smax]
    double emax = 0;
    const int G = 20000;
    for (int i = 0; i <= G; ++i) {
        const double s = std::exp(std::log(smin) + (std::log(smax) - std::log(smin)) * i / G);
        double v = c0 * s;
        for (size_t k = 0; k < t.size(); ++k) v += s * cc[k] * std::exp(-t[k] * s);
        emax = std::max(emax, std::fabs(v / f_control(s, a, b, gm) - 1.0));
    }
    p->op_err = emax;
    if (!(emax <= p->op_acc))
        throw FcError(FC_ERR_NUMERIC, "operator gate failed: max rel err " + std::to_string(emax));
}

// Preconditioner: 1/f with precond_rank positive exponentials on [smin, smax],
// separable over the per-mode spectra lam[l] (case (B): the eigenvalues of
// A_l; case (A): those of b0_l Delta_l).
void build_preconditioner(fc_plan_s* p, double smin, double smax, const std::vector<double>* lam,
                          Separable& S, double& err_out) {
    const int n = p->n;
    const double a = p->alpha, b = p->beta, gm = p->gamma;
    auto add = [&](double w, double t) {
        S.w.push_back(w);
        for (int l = 0; l < 3; ++l)
            for (int i = 0; i < n; ++i) S.F[l].push_back(std::exp(-t * lam[l][i]));
        S.Q++;
    };
    if (a == 0.0) {
        add(1.0 / (b + gm / b), 0.0);
        err_out = 0.0;
        return;
    }
    auto pf = [&](double s) { return 1.0 / f_control(s, a, b, gm); };
    // largest usable rank <= Kmax: positive weights and a relative error < 0.9
    auto fit = [&](int Kmax, std::vector<double>& t, std::vector<double>& cc, double& err) {
        for (int K = Kmax; K >= 1; --K) {
            if (!fc::fit_expsum(pf, pf, smin, smax, K, t, cc, err)) continue;
            bool pos = true;
            for (double x : cc) pos = pos && x > 0;
            if (pos && err < 0.9) return K;
        }
        return 0;
    };
    std::vector<double> t, cc;
    double err = 0;
    int K = 0;
    if (p->precond_rank > 0) {
        K = fit(p->precond_rank, t, cc, err);
    } else {
        // automatic rank: the relative error of a fixed number of exponentials
        // grows with the width of the spectrum, and every point of it costs
        // PCG iterations, while a few more terms cost little in the Hadamard
        // truncation; take the first of 6, 8, ..., 16 that reaches 1e-3
        double best = 1e300;
        for (int K0 = 6; K0 <= 16; K0 += 2) {
            std::vector<double> t2, c2;
            double e2 = 0;
            const int k2 = fit(K0, t2, c2, e2);
            if (k2 > 0 && e2 < best) { best = e2; K = k2; t = t2; cc = c2; err = e2; }
            if (best <= 1e-3) break;
        }
    }
    if (K == 0) throw FcError(FC_ERR_NUMERIC, "preconditioner fit failed");
    for (int k = 0; k < K; ++k) add(cc[k], t[k]);
    err_out = err;
}

// Spectrum of the case (A) preconditioner: mu_l[k] = b0_l (4/h^2) sin^2(k pi h/2)
// (eqn DiagLaplace, Section 3.4), b0_l the mid-range of the samples unless
// given (eqn modcoeff).
void laplace_spectrum(fc_plan_s* p, const fc_setup_params* prm) {
    const int n = p->n;
    const double h = 1.0 / (n + 1);
    for (int l = 0; l < 3; ++l) {
        double lo = prm->a[l][0], hi = prm->a[l][0];
        for (int i = 1; i <= n; ++i) { lo = std::min(lo, prm->a[l][i]); hi = std::max(hi, prm->a[l][i]); }
        p->b0[l] = prm->precond_b0[l] > 0 ? prm->precond_b0[l] : 0.5 * (lo + hi);
        p->mu[l].resize(n);
        for (int k = 1; k <= n; ++k) {
            const double sn = std::sin(k * M_PI * h / 2.0);
            p->mu[l][k - 1] = p->b0[l] * 4.0 / (h * h) * sn * sn;
        }
    }
}

// State map y = beta A^-alpha u (eqn `State`): beta s^-alpha is completely
// monotone, so it is an exponential sum with positive weights on the same
// geometric node grid as the operator (one separable term per node; the
// constant beta when alpha = 0), gated like the operator.
void build_state_map(fc_plan_s* p, double smin, double smax) {
    const int n = p->n;
    const double a = p->alpha, b = p->beta;
    Separable& S = p->st;
    auto add = [&](double w, double t) {
        S.w.push_back(w);
        for (int l = 0; l < 3; ++l)
            for (int i = 0; i < n; ++i) S.F[l].push_back(t > 0 ? std::exp(-t * p->lam[l][i]) : 1.0);
        S.Q++;
    };
    if (a == 0.0) {
        add(b, 0.0);
        p->st_err = 0.0;
        return;
    }
    auto h = [&](double s) { return b * std::pow(s, -a); };
    const double t_hi = (std::log(1.0 / p->op_acc) + 10.0) / smin;
    const double t_lo = std::pow(p->op_acc, 0.7) / smax;
    std::vector<double> t, cc;
    double c0 = 0.0, err = 1e300;
    for (double hstep : {0.7, 0.6, 0.5, 0.42, 0.35}) {
        if (!fc::fit_expsum_nnls(h, h, smin, smax, t_lo, t_hi, hstep, false, t, cc, c0, err))
            continue;
        if (err <= p->op_acc) break;
    }
    if (!(err <= p->op_acc))
        throw FcError(FC_ERR_NUMERIC, "state-map exponential sum misses the accuracy gate (err " +
                                          std::to_string(err) + ")");
    for (size_t k = 0; k < t.size(); ++k) add(cc[k], t[k]);
    p->st_err = err;
}

// The separable factors from the spectra (Sections 3.4, 3.5, 3.1): the
// exponential-sum fits are independent host problems, run on threads of
// their own.
// The spectra the fits run on: with d = 2 the third mode's eigenvalues are
// shifted by the smallest one; case (A) adds the Laplacian's spectrum.
void prepare_spectra(fc_plan_s* p, const fc_setup_params* prm) {
    if (p->dims == 2) {
        // A_3 - lambda_3,1 I: its first eigenvector spans a null space, so a
        // design y (x) v_1 has the solution u (x) v_1 with u the d = 2 control
        const double sig = p->lam[2][0];
        for (double& x : p->lam[2]) x -= sig;
        p->lam[2][0] = 0.0;
    }
    if (p->pc_kind == FC_PRECOND_LAPLACE) {
        laplace_spectrum(p, prm);
        if (p->dims == 2) {
            const double sig = p->mu[2][0];
            for (double& x : p->mu[2]) x -= sig;
            p->mu[2][0] = 0.0;
        }
    }
}

void build_separables(fc_plan_s* p, const fc_setup_params* prm) {
    prepare_spectra(p, prm);
    double smin = 0, smax = 0;
    for (int l = 0; l < 3; ++l) { smin += p->lam[l].front(); smax += p->lam[l].back(); }
    auto now = [] { return std::chrono::steady_clock::now(); };
    const auto t0 = now();
    std::exception_ptr err[4];
    auto run = [&](int i, auto fn) {
        try { fn(); } catch (...) { err[i] = std::current_exception(); }
    };
    std::vector<std::thread> th;
    th.emplace_back([&] { run(0, [&] { build_operator(p, smin, smax); }); });
    th.emplace_back([&] { run(1, [&] { build_state_map(p, smin, smax); }); });
    if (p->pc_kind == FC_PRECOND_LAPLACE)
        th.emplace_back([&] {
            run(2, [&] {
                double mmin = 0, mmax = 0;
                for (int l = 0; l < 3; ++l) { mmin += p->mu[l].front(); mmax += p->mu[l].back(); }
                build_preconditioner(p, mmin, mmax, p->mu, p->pcA, p->pcA_err);
            });
        });
    run(3, [&] { build_preconditioner(p, smin, smax, p->lam, p->pc, p->pc_err); });
    for (auto& t : th) t.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
    FC_TRACE_PRINT("setup fits: %.1f ms (operator Q %d)\n",
                   std::chrono::duration<double, std::milli>(now() - t0).count(), p->op.Q);
}

// ---- the separable factors on the device ----------------------------------
// The same fits as build_separables (operator and state map: nonnegative
// sums on the node grids of hstep 0.7 ... 0.35, the first grid meeting the
// accuracy taken; preconditioner: the largest usable rank, automatic rank
// the first of 6, 8, ..., 16 reaching 1e-3), every candidate an independent
// workgroup of one launch (fit.hip); the host reads the results, applies the
// same selection rules, and the factors exp(-t lam) are formed on the device.
struct TermList {
    std::vector<double> w, t;   // weight, node (< 0: no exponential)
    std::vector<int> lm;        // mode whose factor carries the eigenvalue (-1: none)
    void add(double wq, double tq, int m) { w.push_back(wq); t.push_back(tq); lm.push_back(m); }
};

// Stream-ordered temporaries of the setup: plans set up on concurrent host
// threads must not wait for each other's kernels, which hipFree would do.
// Freed on the plan's stream when the holder goes out of scope (also when
// the setup throws).
struct SetupTmp {
    hipStream_t s;
    std::vector<void*> held;
    explicit SetupTmp(hipStream_t st) : s(st) {}
    template <typename T>
    T* get(size_t count) {
        void* q = nullptr;
        if (hipMallocAsync(&q, std::max<size_t>(count, 1) * sizeof(T), s) != hipSuccess)
            throw FcError(FC_ERR_OUT_OF_MEMORY, "hipMallocAsync failed");
        held.push_back(q);
        return (T*)q;
    }
    ~SetupTmp() {
        for (void* q : held) (void)hipFreeAsync(q, s);
    }
};

void device_factors(fc_plan_s* p, const TermList& tl, const std::vector<double>* spec,
                    Separable& S) {
    const int n = p->n, Q = (int)tl.w.size();
    S.Q = Q;
    S.w = tl.w;
    std::vector<double> lamh((size_t)3 * n), tw((size_t)2 * Q);
    std::vector<int> lm(tl.lm);
    for (int l = 0; l < 3; ++l) std::copy(spec[l].begin(), spec[l].end(), lamh.begin() + (long)l * n);
    for (int q = 0; q < Q; ++q) { tw[q] = tl.w[q]; tw[Q + q] = tl.t[q]; }
    SetupTmp tmp(p->stream);
    double* lamd = tmp.get<double>(lamh.size());
    double* twd = tmp.get<double>(tw.size());
    int* lmd = tmp.get<int>(lm.size());
    HIPCHK(hipMemcpyAsync(lamd, lamh.data(), sizeof(double) * lamh.size(), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipMemcpyAsync(twd, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipMemcpyAsync(lmd, lm.data(), sizeof(int) * lm.size(), hipMemcpyHostToDevice, p->stream));
    for (int l = 0; l < 3; ++l) {
        S.Fd[l] = p->arena.alloc((size_t)n * Q);
        S.D[l] = p->arena.alloc((size_t)n * Q);
        S.D2[l] = p->arena.alloc((size_t)n * Q);
    }
    HIPCHK(fc::expsum_factors(n, Q, lamd, twd, twd + Q, lmd, S.Fd, S.D, S.D2, p->stream));
    // the host vectors are read by the copies above before they go out of scope
    HIPCHK(hipStreamSynchronize(p->stream));
}

// A set of fit jobs run in one launch pair; results copied back per job.
struct FitBatch {
    fc::FitJobs jobs;
    std::vector<std::vector<double>> out;
    int add(const fc::FitJob& j) {
        if (jobs.count >= fc::kMaxFitJobs) throw FcError(FC_ERR_INTERNAL, "too many fit jobs");
        jobs.job[jobs.count] = j;
        return jobs.count++;
    }
    void run(fc_plan_s* p) {
        out.assign(jobs.count, {});
        if (jobs.count == 0) return;
        std::vector<long> woff(jobs.count), ooff(jobs.count + 1);
        long wtot = 0;
        ooff[0] = 0;
        for (int k = 0; k < jobs.count; ++k) {
            woff[k] = wtot;
            wtot += fc::fit_work_doubles(jobs.job[k]);
            ooff[k + 1] = ooff[k] + fc::fit_out_doubles(jobs.job[k]);
        }
        SetupTmp tmp(p->stream);
        double* work = tmp.get<double>((size_t)wtot);
        double* outd = tmp.get<double>((size_t)ooff[jobs.count]);
        for (int k = 0; k < jobs.count; ++k) {
            jobs.job[k].work = work + woff[k];
            jobs.job[k].out = outd + ooff[k];
        }
        std::vector<double> h((size_t)ooff[jobs.count]);
        HIPCHK(fc::fit_run(jobs, p->stream));
        HIPCHK(hipMemcpyAsync(h.data(), outd, sizeof(double) * h.size(), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        for (int k = 0; k < jobs.count; ++k)
            out[k].assign(h.begin() + ooff[k], h.begin() + ooff[k + 1]);
    }
};

void device_separables(fc_plan_s* p, const fc_setup_params* prm) {
    prepare_spectra(p, prm);
    const auto t0 = std::chrono::steady_clock::now();
    const double a = p->alpha, b = p->beta, gm = p->gamma;
    double smin = 0, smax = 0, mmin = 0, mmax = 0;
    for (int l = 0; l < 3; ++l) { smin += p->lam[l].front(); smax += p->lam[l].back(); }
    const bool lap = p->pc_kind == FC_PRECOND_LAPLACE;
    if (lap)
        for (int l = 0; l < 3; ++l) { mmin += p->mu[l].front(); mmax += p->mu[l].back(); }
    if (!(smin > 0) || !(smax >= smin) || (lap && (!(mmin > 0) || !(mmax >= mmin))))
        throw FcError(FC_ERR_NUMERIC, "spectrum not positive");
    const double hsteps[5] = {0.7, 0.6, 0.5, 0.42, 0.35};
    const double t_hi = (std::log(1.0 / p->op_acc) + 10.0) / smin;
    const double t_lo = std::pow(p->op_acc, 0.7) / smax;
    const double cexact = (a == 1.0) ? gm / b : 0.0;
    auto nonneg_job = [&](int target, double hs) {
        fc::FitJob J;
        J.target = target; J.alpha = a; J.beta = b; J.gamma = gm;
        J.cexact = target == fc::FIT_OPERATOR ? cexact : 0.0;
        J.smin = smin; J.smax = smax; J.log_tlo = std::log(t_lo); J.hstep = hs;
        int cnt = 0;
        for (double x = std::log(t_lo); x <= std::log(t_hi) + 1e-12; x += hs) ++cnt;
        J.nodes = cnt;
        J.with_constant = (target == fc::FIT_OPERATOR && a < 1.0) ? 1 : 0;
        if (cnt < 1 || cnt + J.with_constant > fc::kFitMaxNodes)
            throw FcError(FC_ERR_NUMERIC, "exponential-sum node grid out of range");
        return J;
    };
    auto free_job = [&](double lo, double hi, int kmax) {
        fc::FitJob J;
        J.target = fc::FIT_PRECOND; J.alpha = a; J.beta = b; J.gamma = gm;
        J.smin = lo; J.smax = hi; J.kmax = kmax;
        return J;
    };
    // a nonnegative fit passes when it ran and its error meets the accuracy
    auto passes = [&](const fc::FitJob& J, const std::vector<double>& o) {
        const int N = J.nodes + J.with_constant;
        return o[N + 2] == 1.0 && o[N] <= p->op_acc;
    };
    TermList op, st, pc, pcA;
    int jobs_run = 0;
    if (a == 0.0) {
        op.add(b + gm / b, -1.0, -1);
        p->op_err = 0.0;
        st.add(b, -1.0, -1);
        p->st_err = 0.0;
        pc.add(1.0 / (b + gm / b), 0.0, -1);
        p->pc_err = 0.0;
        if (lap) { pcA.add(1.0 / (b + gm / b), 0.0, -1); p->pcA_err = 0.0; }
    } else {
        // stage 1: the three coarser node grids of both nonnegative fits and
        // every preconditioner candidate; stage 2: the finer grids of a fit
        // none of whose coarser grids met the accuracy (the selection takes
        // the first grid that does, so the finer ones only matter then)
        std::vector<int> kmaxes;
        if (p->precond_rank > 0) kmaxes.push_back(p->precond_rank);
        else
            for (int K0 = 6; K0 <= 16; K0 += 2) kmaxes.push_back(K0);
        FitBatch s1;
        int opi[5], sti[5];
        std::vector<int> pci, pai;
        for (int h = 0; h < 3; ++h) {
            opi[h] = s1.add(nonneg_job(fc::FIT_OPERATOR, hsteps[h]));
            sti[h] = s1.add(nonneg_job(fc::FIT_STATE, hsteps[h]));
        }
        for (int K0 : kmaxes) pci.push_back(s1.add(free_job(smin, smax, K0)));
        if (lap)
            for (int K0 : kmaxes) pai.push_back(s1.add(free_job(mmin, mmax, K0)));
        s1.run(p);
        jobs_run += s1.jobs.count;
        // chosen results: (job, outputs) per target
        fc::FitJob opJ, stJ;
        std::vector<double> opO, stO;
        double op_last = 1e300, st_last = 1e300;
        auto first_pass = [&](FitBatch& B, const int* idx, int from, int to, fc::FitJob& J,
                              std::vector<double>& O, double& last) {
            for (int h = from; h < to; ++h) {
                const fc::FitJob& Jh = B.jobs.job[idx[h]];
                const std::vector<double>& o = B.out[idx[h]];
                const int N = Jh.nodes + Jh.with_constant;
                if (o[N + 2] == 1.0) last = o[N];
                if (passes(Jh, o)) { J = Jh; O = o; return true; }
            }
            return false;
        };
        bool opok = first_pass(s1, opi, 0, 3, opJ, opO, op_last);
        bool stok = first_pass(s1, sti, 0, 3, stJ, stO, st_last);
        if (!opok || !stok) {
            FitBatch s2;
            for (int h = 3; h < 5; ++h) {
                if (!opok) opi[h] = s2.add(nonneg_job(fc::FIT_OPERATOR, hsteps[h]));
                if (!stok) sti[h] = s2.add(nonneg_job(fc::FIT_STATE, hsteps[h]));
            }
            s2.run(p);
            jobs_run += s2.jobs.count;
            if (!opok) opok = first_pass(s2, opi, 3, 5, opJ, opO, op_last);
            if (!stok) stok = first_pass(s2, sti, 3, 5, stJ, stO, st_last);
        }
        if (!opok)
            throw FcError(FC_ERR_NUMERIC, "operator exponential sum misses the accuracy gate (err " +
                                              std::to_string(op_last) + ")");
        if (!stok)
            throw FcError(FC_ERR_NUMERIC, "state-map exponential sum misses the accuracy gate (err " +
                                              std::to_string(st_last) + ")");
        {
            const int N0 = opJ.nodes, N = N0 + opJ.with_constant;
            const double* o = opO.data();
            const double c0 = cexact + (opJ.with_constant ? o[N0] : 0.0);
            if (c0 > 0.0)
                for (int m = 0; m < 3; ++m) op.add(c0, -1.0, m);
            for (int j = 0; j < N0; ++j)
                if (o[j] > 0)
                    for (int m = 0; m < 3; ++m) op.add(o[j], o[N + 3 + j], m);
            p->op_err = o[N + 1];
            if (!(p->op_err <= p->op_acc))
                throw FcError(FC_ERR_NUMERIC, "operator gate failed: max rel err " + std::to_string(p->op_err));
        }
        {
            const int N = stJ.nodes;
            const double* o = stO.data();
            for (int j = 0; j < N; ++j)
                if (o[j] > 0) st.add(o[j], o[N + 3 + j], -1);
            p->st_err = o[N];
        }
        // preconditioner: fixed rank, or the automatic rule over the candidates
        auto pick_free = [&](const std::vector<int>& idx, TermList& tl, double& err_out) {
            int kbest = -1;
            double best = 1e300;
            for (size_t c = 0; c < idx.size(); ++c) {
                const std::vector<double>& o = s1.out[idx[c]];
                const int K = (int)o[2 * fc::kFitMaxK + 1];
                const double e = o[2 * fc::kFitMaxK];
                if (K > 0 && e < best) { best = e; kbest = idx[c]; }
                if (best <= 1e-3) break;
            }
            if (kbest < 0) throw FcError(FC_ERR_NUMERIC, "preconditioner fit failed");
            const std::vector<double>& o = s1.out[kbest];
            const int K = (int)o[2 * fc::kFitMaxK + 1];
            for (int k = 0; k < K; ++k) tl.add(o[K + k], o[k], -1);
            err_out = best;
        };
        pick_free(pci, pc, p->pc_err);
        if (lap) pick_free(pai, pcA, p->pcA_err);
    }
    const auto t1 = std::chrono::steady_clock::now();
    device_factors(p, op, p->lam, p->op);
    device_factors(p, st, p->lam, p->st);
    device_factors(p, pc, p->lam, p->pc);
    if (lap) device_factors(p, pcA, p->mu, p->pcA);
    FC_TRACE_PRINT("setup fits on the device: %.1f ms (%d jobs), factors %.1f ms (operator Q %d)\n",
                   std::chrono::duration<double, std::milli>(t1 - t0).count(), jobs_run,
                   std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count(),
                   p->op.Q);
}

// Host construction (no device): implicit-QL eigenpairs, then the fits.
void host_spectra_and_separables(fc_plan_s* p, const fc_setup_params* prm) {
    const int n = p->n;
    std::vector<std::thread> th;
    bool ok[3] = {false, false, false};
    for (int l = 0; l < 3; ++l) {
        p->lam[l].resize(n);
        p->Vh[l].resize((size_t)n * n);
        th.emplace_back([&, l] { ok[l] = fc::fd_eigen(n, prm->a[l], p->lam[l].data(), p->Vh[l].data()); });
    }
    for (auto& t : th) t.join();
    for (int l = 0; l < 3; ++l)
        if (!ok[l] || !(p->lam[l][0] > 0))
            throw FcError(FC_ERR_NUMERIC, "tridiagonal eigensolver failed");
    build_separables(p, prm);
}

// Eigenpairs of the three 1D matrices (Section 3.3) on the device: divide
// and conquer on the symmetric tridiagonal matrices (rocSOLVER stedc, on a
// handle of its own that manages its workspace), eigenvalues ascending,
// eigenvectors straight into the plan's V_l.  The eigenvalues come back to
// the host for the fits.
void device_spectra(fc_plan_s* p, const fc_setup_params* prm) {
    const int n = p->n;
    std::vector<double> dh((size_t)3 * n), eh((size_t)3 * n, 0.0);
    for (int l = 0; l < 3; ++l) fc::fd_tridiag(n, prm->a[l], &dh[(size_t)l * n], &eh[(size_t)l * n]);
    SetupTmp tmp(p->stream);
    double* D = tmp.get<double>((size_t)3 * n);
    double* E = tmp.get<double>((size_t)3 * n);
    int* info = tmp.get<int>(3);
    HIPCHK(hipMemcpyAsync(D, dh.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipMemcpyAsync(E, eh.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, p->stream));
    // a library handle from a process-wide pool: creating and destroying one
    // per plan frees its device workspace, which waits for the whole device
    // (plans set up on concurrent threads would wait for each other)
    struct HandleLease {
        rocblas_handle h = nullptr;
        HandleLease() {
            {
                std::lock_guard<std::mutex> lk(pool_mutex());
                if (!pool().empty()) { h = pool().back(); pool().pop_back(); }
            }
            if (!h && rocblas_create_handle(&h) != rocblas_status_success)
                throw FcError(FC_ERR_HIP, "rocblas_create_handle failed");
        }
        ~HandleLease() {
            std::lock_guard<std::mutex> lk(pool_mutex());
            pool().push_back(h);
        }
        static std::vector<rocblas_handle>& pool() { static std::vector<rocblas_handle> v; return v; }
        static std::mutex& pool_mutex() { static std::mutex m; return m; }
    } lease;
    rocblas_handle h = lease.h;
    if (rocblas_set_stream(h, p->stream) != rocblas_status_success)
        throw FcError(FC_ERR_HIP, "rocblas_set_stream failed");
    for (int l = 0; l < 3; ++l) {
        p->V[l] = p->arena.alloc((size_t)n * n);
        if (rocsolver_dstedc(h, rocblas_evect_tridiagonal, n, D + (size_t)l * n, E + (size_t)l * n,
                             p->V[l], n, info + l) != rocblas_status_success)
            throw FcError(FC_ERR_HIP, "rocsolver_dstedc failed");
    }
    int ih[3];
    HIPCHK(hipMemcpyAsync(dh.data(), D, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipMemcpyAsync(ih, info, sizeof(int) * 3, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    for (int l = 0; l < 3; ++l) {
        p->Vt[l] = p->arena.alloc((size_t)n * n);
        HIPCHK(fc::transpose(n, n, p->V[l], n, p->Vt[l], n, p->stream));
    }
    HIPCHK(hipStreamSynchronize(p->stream));
    for (int l = 0; l < 3; ++l) {
        p->lam[l].assign(dh.begin() + (long)l * n, dh.begin() + (long)(l + 1) * n);
        if (ih[l] != 0 || !(p->lam[l][0] > 0))
            throw FcError(FC_ERR_NUMERIC, "tridiagonal eigensolver failed (mode " +
                                              std::to_string(l) + ", info " + std::to_string(ih[l]) + ")");
    }
}

// W_l = S V_l: eigen-coordinates of A_l -> sine coordinates.  S[i,k] =
// sqrt(2/(n+1)) sin(pi i k/(n+1)) with the integer i k reduced modulo
// 2(n+1) before the sine; the product runs on the device.
void build_sine_maps(fc_plan_s* p) {
    const int n = p->n;
    std::vector<double> S((size_t)n * n);
    const double sc = std::sqrt(2.0 / (n + 1));
    for (int k = 1; k <= n; ++k)
        for (int i = 1; i <= n; ++i) {
            const long m = ((long)i * k) % (2L * (n + 1));
            S[(size_t)(k - 1) * n + (i - 1)] = sc * std::sin(M_PI * (double)m / (n + 1));
        }
    SetupTmp tmp(p->stream);
    double* Sd = tmp.get<double>((size_t)n * n);
    HIPCHK(hipMemcpyAsync(Sd, S.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, p->stream));
    Ctx c{p, p->stream, n};
    for (int l = 0; l < 3; ++l) {
        p->Wsin[l] = p->arena.alloc((size_t)n * n);
        gemm(c, false, false, n, n, n, 1.0, Sd, n, p->V[l], n, 0.0, p->Wsin[l], n);
        p->WsinT[l] = p->arena.alloc((size_t)n * n);
        HIPCHK(fc::transpose(n, n, p->Wsin[l], n, p->WsinT[l], n, p->stream));
    }
    HIPCHK(hipStreamSynchronize(p->stream));
}

// ---- autotuner ------------------------------------------------------------
// Picks, per device, grid size n and operator rank Q, the launch choices of
// Tuning by timing every candidate on the plan's own buffers and operator:
//   wavefronts per workgroup of the Gram kernel (8 or 16) on the scaled Grams
//   Z^T diag(D_q) X (48 x 96, Q terms) and on three 32 x 16 products over n;
//   wavefronts of the fused Kronecker application (8 or 16, r = 48, p = 96);
//   the K chunk of the streaming transform kernel (128 or 256, three modes,
//   m = 16); the Gram-Schmidt panel width (8 or 16, three n x 96 blocks).
// Results are kept for the process and in a text cache on disk (environment
// FC_TUNE_CACHE, else $HOME/.cache/fracctl/tune_v2.txt; one line per key),
// so plans of the same size take the same choices and give the same bits.
// FC_TUNE=0 keeps the defaults.
std::mutex g_tune_mu;
std::vector<std::pair<std::string, Tuning>> g_tune_table;

std::string tune_cache_path() {
    if (const char* e = std::getenv("FC_TUNE_CACHE")) return e;
    const char* home = std::getenv("HOME");
    if (!home || !*home) return std::string();
    return std::string(home) + "/.cache/fracctl/tune_v2.txt";
}

bool tune_lookup_disk(const std::string& key, Tuning& t) {
    const std::string path = tune_cache_path();
    if (path.empty()) return false;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        const char* bar = std::strchr(line, '|');
        if (!bar || std::string(line, (size_t)(bar - line)) != key) continue;
        Tuning x;
        int got = std::sscanf(bar + 1, "%d %d %d %d %d | %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf",
                              &x.gram_batched, &x.gram_single, &x.kron, &x.stream_kc, &x.panel_b,
                              &x.us[0], &x.us[1], &x.us[2], &x.us[3], &x.us[4], &x.us[5], &x.us[6],
                              &x.us[7], &x.us[8], &x.us[9]);
        const bool ok = got == 15 && (x.gram_batched == 8 || x.gram_batched == 16) &&
                        (x.gram_single == 8 || x.gram_single == 16) && (x.kron == 8 || x.kron == 16) &&
                        (x.stream_kc == 128 || x.stream_kc == 256) &&
                        (x.panel_b == 8 || x.panel_b == 16);
        if (ok) {   // the last valid line for the key wins
            x.tuned = true;
            t = x;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_store_disk(const std::string& key, const Tuning& t) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0)
        for (size_t i = 1; i <= slash; ++i)   // mkdir -p of the parent directory
            if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s|%d %d %d %d %d | %.2f %.2f %.2f %.2f %.2f %.2f %.2f %.2f %.2f %.2f\n",
                 key.c_str(), t.gram_batched, t.gram_single, t.kron, t.stream_kc, t.panel_b, t.us[0],
                 t.us[1], t.us[2], t.us[3], t.us[4], t.us[5], t.us[6], t.us[7], t.us[8], t.us[9]);
    std::fclose(f);
}

// mean time (us) of `reps` launches after one warm-up, HIP events on s
template <class F>
double time_launches(hipStream_t s, int reps, F&& launch) {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(launch());
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) HIPCHK(launch());
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return 1e3 * ms / reps;
}

void autotune(fc_plan_s* p) {
    const char* off = std::getenv("FC_TUNE");
    if (off && std::strcmp(off, "0") == 0) return;
    const int n = p->n, Q = p->op.Q;
    hipDeviceProp_t prop;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    const std::string key = std::string(prop.gcnArchName) + " n=" + std::to_string(n) +
                            " Q=" + std::to_string(Q);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& e : g_tune_table)
        if (e.first == key) { p->tune = e.second; return; }
    Tuning t;
    if (tune_lookup_disk(key, t)) {
        g_tune_table.emplace_back(key, t);
        p->tune = t;
        return;
    }
    const hipStream_t s = p->stream;
    Ctx c{p, s, n};
    // random inputs in the subspace buffers
    fc::FillJobs fills;
    for (int l = 0; l < 3; ++l) {
        fc::FillJob& F = fills.job[fills.count++];
        F.n = (long)n * p->pcap;
        F.seed = 97u + 13u * l;
        F.x = p->Xs3[l];
    }
    HIPCHK(fc::fill_random_multi(fills, s));
    const int reps = 5;
    // 1. scaled Grams Z^T diag(D_q) X, 48 x 96 over Q terms
    {
        const int r = std::min(48, n), q = std::min(96, n);
        const fc::GemmArgs g = scaled_gram(r, q, n, Q, p->Xs3[0], p->Xs3[1], p->op.D[0], p->Ys);
        for (int w = 0; w < 2; ++w)
            t.us[w] = time_launches(s, reps, [&] { return fc::gram(true, false, g, s, w ? 16 : 8, gram_staged(true)); });
        t.gram_batched = t.us[0] < t.us[1] ? 8 : 16;
    }
    // 2. three 32 x 16 Gram-type products over n (the panel coefficients)
    {
        fc::GramJobs jobs;
        for (int l = 0; l < 3; ++l) {
            fc::GemmArgs& g = jobs.g[jobs.count++];
            g.M = std::min(32, n); g.N = std::min(16, n); g.K = n;
            g.A = p->Xs3[l]; g.lda = n; g.B = p->Xs3[(l + 1) % 3]; g.ldb = n;
            g.C = p->HX3[l]; g.ldc = g.M;
        }
        for (int w = 0; w < 2; ++w)
            t.us[2 + w] = time_launches(s, reps, [&] {
                return fc::gram_multi(true, false, jobs, s, w ? 16 : 8, gram_staged(true));
            });
        t.gram_single = t.us[2] < t.us[3] ? 8 : 16;
    }
    // 3. fused Kronecker application, r = 48, p = 96, Q terms
    {
        fc::KronJobs kj;
        fc::KronJob& J = kj.job[kj.count++];
        J.r = std::min(48, n); J.p = std::min(96, n); J.Z = p->Xs3[0]; J.ldz = n; J.D = p->op.D[0];
        J.T = p->Ts; J.out = p->HX3[0]; J.ldo = n;
        HIPCHK(fc::fill_random_multi(fc::FillJobs{1, {fc::FillJob{(long)J.r * J.p * Q, 5u, p->Ts}}}, s));
        for (int w = 0; w < 2; ++w)
            t.us[4 + w] = time_launches(s, reps, [&] {
                return fc::kron_apply_multi(n, Q, kj, s, w ? 16 : 8);
            });
        t.kron = t.us[4] < t.us[5] ? 8 : 16;
    }
    // 4. streaming transforms of the three modes, m = 16
    {
        fc::StreamJobs sj;
        for (int l = 0; l < 3; ++l) {
            fc::StreamJob& J = sj.job[sj.count++];
            J.M = n; J.N = std::min(16, n); J.K = n;
            J.A = p->V[l]; J.lda = n; J.B = p->Xs3[l]; J.ldb = n; J.C = p->HX3[l]; J.ldc = n;
        }
        const int kcs[2] = {128, 256};
        for (int w = 0; w < 2; ++w)
            t.us[6 + w] = fc::stream_fits(sj, kcs[w], p->splitws_cap)
                              ? time_launches(s, reps, [&] {
                                    return fc::stream_multi(2, sj, kcs[w], p->splitws,
                                                            p->splitws_cap, s);
                                })
                              : 1e30;
        t.stream_kc = t.us[6] <= t.us[7] ? 128 : 256;
    }
    // 5. Gram-Schmidt panel width: three n x 96 blocks orthonormalised
    if ((long)n * 16 * 8 <= 144L * 1024 && n >= 96) {
        const int pw[2] = {8, 16};
        for (int w = 0; w < 2; ++w) {
            p->tune.panel_b = pw[w];
            double best = 1e30;
            for (int r = 0; r < 2; ++r) {
                HIPCHK(fc::fill_random_multi(fills, s));
                HIPCHK(hipStreamSynchronize(s));
                const auto t0 = std::chrono::steady_clock::now();
                int m[3] = {96, 96, 96};
                const int none[3] = {0, 0, 0};
                const bool all[3] = {true, true, true};
                orthonormalize3(c, m, p->Xs3, 1e-13, none, all);
                HIPCHK(hipStreamSynchronize(s));
                best = std::min(best, std::chrono::duration<double, std::micro>(
                                          std::chrono::steady_clock::now() - t0).count());
            }
            t.us[8 + w] = best;
        }
        t.panel_b = t.us[8] < t.us[9] ? 8 : 16;
    } else {
        t.us[8] = t.us[9] = 0.0;
    }
    // the times as the disk cache keeps them (two decimals), so that a plan
    // reading the cache reports the same values
    for (double& u : t.us) u = std::round(u * 100.0) / 100.0;
    t.tuned = true;
    p->tune = t;
    g_tune_table.emplace_back(key, t);
    tune_store_disk(key, t);
    FC_TRACE_PRINT("autotune %s: gram %d/%d (%.1f %.1f | %.1f %.1f us) kron %d (%.1f %.1f) kc %d "
                   "(%.1f %.1f) panel %d (%.0f %.0f)\n",
                   key.c_str(), t.gram_batched, t.gram_single, t.us[0], t.us[1], t.us[2], t.us[3],
                   t.kron, t.us[4], t.us[5], t.stream_kc, t.us[6], t.us[7], t.panel_b, t.us[8],
                   t.us[9]);
}

void setup_plan(fc_plan_s* p, const fc_setup_params* prm) {
    const auto t0 = std::chrono::steady_clock::now();
    device_spectra(p, prm);
    const auto t1 = std::chrono::steady_clock::now();
    FC_TRACE_PRINT("setup eigenpairs on the device: %.1f ms\n",
                   std::chrono::duration<double, std::milli>(t1 - t0).count());
    device_separables(p, prm);
    alloc_workspace(p);
    if (p->pc_kind == FC_PRECOND_LAPLACE) build_sine_maps(p);
    HIPCHK(hipHostMalloc(&p->pinned, fc_plan_s::kPinnedBytes, hipHostMallocDefault));
    autotune(p);
    if (p->dims == 2) {
        p->Y3d = p->arena.alloc((size_t)p->n * 256);
        p->U3d = p->arena.alloc((size_t)p->n * 256);
    }
    HIPCHK(hipStreamSynchronize(p->stream));
}

// The rank-truncated PCG (Algorithm 1) on Tucker iterates in eigen-coordinates.
struct SolveOut {
    int iterations = 0;
    double rel_res = 0;
    bool converged = false;
};

// floor_abs: absolute accuracy to which S and R are resolved (the plain solve
// uses eps/10 of ||B||; a refinement correction needs no more than the outer
// solve's absolute level).
SolveOut pcg(const Ctx& c, const Tucker& Bt, Tucker& Xout, double eps, double tol, int max_iter,
             double floor_abs, double stop_abs = 0.0) {
    fc_plan_s* p = c.p;
    Tucker& X = p->slot[1];
    Tucker& R = p->slot[2];
    Tucker& Z = p->slot[3];
    Tucker& P = p->slot[4];
    Tucker& S = p->slot[5];
    Tucker& T1 = p->slot[6];
    Tucker& T2 = p->slot[7];
    SolveOut so;
    Ctx cd = c;
    cd.clamp = true;                       // for the search directions Z and P
    const double bn = std::sqrt(tucker_norm2(c, Bt));
    X.r[0] = X.r[1] = X.r[2] = 0;
    tucker_copy(c, Bt, R);                 // R0 = B - fun(X0), X0 = 0
    apply_precond(cd, R, eps, Z, "Z0 = trunc(precond(R0))", SITE_Z);
    check_orth(c, Z, "Z0");
    tucker_copy(c, Z, P);                  // P0 = Z0
    double rz = tucker_inner(c, R, Z);
    for (int k = 0; k < max_iter; ++k) {
        had_trunc(c, p->op, P, eps, floor_abs, S, "S = trunc(fun(P))", SITE_S);
        check_orth(c, S, "S");
        const double ps = tucker_inner(c, P, S);
        if (!(ps > 0) || !std::isfinite(ps) || !std::isfinite(rz))
            throw FcError(FC_ERR_NUMERIC, "PCG breakdown: <P,S> = " + std::to_string(ps));
        const double ak = rz / ps;
        // X = trunc(X + a P)
        sum_trunc(c, {{1.0, &X}, {ak, &P}}, 0.1 * eps, 0.0, T1, "X = trunc(X + aP)", SITE_X);
        check_orth(c, T1, "X");
        std::swap(X, T1);
        // R = trunc(R - a S)
        sum_trunc(c, {{1.0, &R}, {-ak, &S}}, 0.1 * eps, floor_abs, T2, "R = trunc(R - aS)", SITE_R);
        check_orth(c, T2, "R");
        std::swap(R, T2);
        so.iterations = k + 1;
        const double rn = std::sqrt(tucker_norm2(c, R));
        so.rel_res = bn > 0 ? rn / bn : 0.0;
        FC_TRACE_PRINT("pcg%s it %d |R|/|B| %.3e ranks X %d,%d,%d R %d,%d,%d S %d,%d,%d P %d,%d,%d\n",
                       c.lowp ? "(fp32)" : "", k + 1, so.rel_res, X.r[0], X.r[1], X.r[2], R.r[0],
                       R.r[1], R.r[2], S.r[0], S.r[1], S.r[2], P.r[0], P.r[1], P.r[2]);
        if (R.empty() || so.rel_res <= tol || rn <= stop_abs) { so.converged = true; break; }
        apply_precond(cd, R, eps, Z, "Z = trunc(precond(R))", SITE_Z);
        check_orth(c, Z, "Z");
        const double rzn = tucker_inner(c, R, Z);
        const double bk = rzn / rz;
        rz = rzn;
        sum_trunc(cd, {{1.0, &Z}, {bk, &P}}, eps, 0.0, T1, "P = trunc(Z + bP)", SITE_P);
        check_orth(c, T1, "P");
        std::swap(P, T1);
        if (P.empty()) { so.converged = true; break; }
    }
    Xout = X;
    // keep slot bookkeeping consistent after swaps
    p->slot[1] = X; p->slot[2] = R; p->slot[3] = Z; p->slot[4] = P; p->slot[5] = S;
    p->slot[6] = T1; p->slot[7] = T2;
    return so;
}

// Mixed precision: outer FP64 iterative refinement on the true residual
// B - D~ (.) U (FP64 truncations), inner rank-truncated PCG on D~ C = R with the
// projection contractions on the FP32 matrix cores and a loose tolerance; the
// correction is added in FP64.  Subspace searches (whose Rayleigh-Ritz values
// square the precision), Grams, eigensolves, PCG scalars and the refinement
// residual stay FP64.  The sweeps stop on the preconditioned residual ratio
// ||D~_p (.) R|| / ||D~_p (.) B|| <= tol (an error estimate), or when it
// stagnates.
SolveOut mixed_solve(const Ctx& c0, const Tucker& Bt, Tucker& Uout, int& sweeps_out) {
    fc_plan_s* p = c0.p;
    Ctx cf = c0; cf.lowp = false;
    Ctx cl = c0; cl.lowp = true;
    const double eps = p->eps;
    Tucker& U = p->slot[8];
    Tucker& Rh = p->slot[9];
    Tucker& Un = p->slot[10];
    Tucker& S = p->slot[11];
    U.r[0] = U.r[1] = U.r[2] = 0;
    const double bn = std::sqrt(tucker_norm2(cf, Bt));
    // error estimate: || D~_p (.) R || relative to || D~_p (.) B || (D~_p ~ D~^-1)
    Tucker& Zh = p->slot[3];
    // the estimate always uses the case (B) symbol (no transforms); with case
    // (A) in the inner solves its subspaces live in other coordinates, so it
    // keeps warm starts of its own
    const int est_site = p->pc_kind == FC_PRECOND_LAPLACE ? SITE_ZE : SITE_Z;
    had_trunc(cf, p->pc, Bt, 1e-2, 0.0, Zh, "refinement: precond(B)", est_site);
    const double zbn = std::sqrt(tucker_norm2(cf, Zh));
    SolveOut total;
    int sweep = 0;
    double prev_est = 1e300;
    for (; sweep < 12; ++sweep) {
        double est;
        if (U.empty()) {
            tucker_copy(cf, Bt, Rh);
            est = 1.0;
        } else {
            had_trunc(cf, p->op, U, 0.1 * eps, 0.1 * eps * bn, S, "refinement: D~ (.) U", SITE_OS);
            sum_trunc(cf, {{1.0, &Bt}, {-1.0, &S}}, 0.1 * eps, 0.05 * eps * bn, Rh,
                      "refinement: B - D~ (.) U", SITE_OR);
            if (Rh.empty()) {
                est = 0.0;
            } else {
                // an estimate: two digits suffice
                had_trunc(cf, p->pc, Rh, 1e-2, 0.0, Zh, "refinement: precond(R)", est_site);
                est = std::sqrt(tucker_norm2(cf, Zh)) / zbn;
            }
            total.rel_res = Rh.empty() ? 0.0 : std::sqrt(tucker_norm2(cf, Rh)) / bn;
        }
        FC_TRACE_PRINT("refine sweep %d est %.3e |R|/|B| %.3e ranks U %d,%d,%d R %d,%d,%d\n", sweep,
                       est, total.rel_res, U.r[0], U.r[1], U.r[2], Rh.r[0], Rh.r[1], Rh.r[2]);
        if (est <= p->tol || Rh.empty()) { total.converged = true; break; }
        if (est > 0.5 * prev_est) {            // stagnation at the truncation floor
            total.converged = est <= 3.0 * p->tol;
            break;
        }
        prev_est = est;
        Tucker C;
        SolveOut in;
        try {
            // The correction needs absolute accuracy ~eps ||B|| only: the inner
            // tolerances (2 eps ||B|| / ||R||, clamped) are relative to ||R|| and
            // loosen as R shrinks, never below 1e-4, well above the FP32 rounding
            // of the bulk contractions.
            const double rhn = std::sqrt(tucker_norm2(cf, Rh));
            const double ratio = bn / rhn;
            const double eps_in = std::min(1e-2, std::max(1e-4, 2.0 * eps * ratio));
            const double tol_in = std::min(1e-1, std::max(1e-3, 2.0 * p->tol * ratio));
            FC_TRACE_PRINT("refine sweep %d inner eps %.2e tol %.2e\n", sweep, eps_in, tol_in);
            in = pcg(cl, Rh, C, eps_in, tol_in, p->max_iter, 0.1 * eps_in * rhn);
        } catch (const FcError& e) {
            throw FcError(e.status, e.msg + " (refinement sweep " + std::to_string(sweep) + ")");
        }
        total.iterations += in.iterations;
        if (C.empty()) break;
        sum_trunc(cf, {{1.0, &U}, {1.0, &C}}, 0.1 * eps, 0.0, Un, "refinement: U + C", SITE_OU);
        std::swap(U, Un);
    }
    sweeps_out = sweep;
    Uout = U;
    return total;
}

fc_status guard(const std::function<void()>& fn) {
    try {
        fn();
        return FC_OK;
    } catch (const FcError& e) {
        return fail(e.status, e.msg);
    } catch (const std::exception& e) {
        return fail(FC_ERR_INTERNAL, e.what());
    }
}

bool finite_pos(const double* a, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(a[i]) || !(a[i] > 0)) return false;
    return true;
}

}  // namespace

extern "C" {

const char* fc_status_string(fc_status s) {
    switch (s) {
        case FC_OK: return "ok";
        case FC_ERR_INVALID_ARG: return "invalid argument";
        case FC_ERR_OUT_OF_MEMORY: return "out of memory";
        case FC_ERR_NOT_CONVERGED: return "not converged";
        case FC_ERR_RANK_OVERFLOW: return "rank overflow";
        case FC_ERR_NUMERIC: return "numerical failure";
        case FC_ERR_HIP: return "HIP runtime error";
        case FC_ERR_INTERNAL: return "internal capacity exceeded";
    }
    return "unknown status";
}

const char* fc_last_error(void) { return g_last_error.c_str(); }

fc_status fc_host_fd_eigen(int n, const double* a_mid, double* lam, double* V) {
    if (n < 1 || !a_mid || !lam) return fail(FC_ERR_INVALID_ARG, "fc_host_fd_eigen: bad arguments");
    if (!finite_pos(a_mid, n + 1)) return fail(FC_ERR_INVALID_ARG, "coefficients must be finite and > 0");
    if (!fc::fd_eigen(n, a_mid, lam, V)) return fail(FC_ERR_NUMERIC, "QL iteration did not converge");
    return FC_OK;
}

fc_status fc_host_expsum(int kind, double p1, double p2, double p3, double s_min, double s_max,
                         int terms, double* t, double* c, double* max_rel_err) {
    if (!(s_min > 0) || !(s_max >= s_min) || terms < 1 || terms > 64 || !t || !c || !max_rel_err)
        return fail(FC_ERR_INVALID_ARG, "fc_host_expsum: bad arguments");
    std::function<double(double)> h, ref;
    if (kind == 0) {
        h = [=](double s) { return std::pow(s, -p1); };
        ref = h;
    } else if (kind == 1) {
        h = [=](double s) { return 1.0 / (p1 * std::pow(s, -p2) + p3 * std::pow(s, p2)); };
        ref = h;
    } else if (kind == 2) {
        h = [=](double s) { return p1 * std::pow(s, -p2 - 1.0) + p3 * std::pow(s, p2 - 1.0); };
        ref = h;
    } else {
        return fail(FC_ERR_INVALID_ARG, "fc_host_expsum: unknown kind");
    }
    std::vector<double> tt, cc;
    double e = 0;
    if (!fc::fit_expsum(h, ref, s_min, s_max, terms, tt, cc, e)) return fail(FC_ERR_NUMERIC, "fit failed");
    for (int k = 0; k < terms; ++k) { t[k] = tt[k]; c[k] = cc[k]; }
    *max_rel_err = e;
    return FC_OK;
}

static fc_status validate_params(const fc_setup_params* prm);
static void apply_defaults(fc_plan_s* p, const fc_setup_params* prm);
static fc_setup_params effective_params(const fc_setup_params* prm, std::vector<double>& ones);

fc_status fc_host_separable(const fc_setup_params* prm, int which, int cap, int* rank, double* w,
                            double* F, double* max_rel_err) {
    if (!prm || !rank || which < 0 || which > 2) return fail(FC_ERR_INVALID_ARG, "fc_host_separable: bad arguments");
    fc_status v = validate_params(prm);
    if (v != FC_OK) return v;
    fc_plan_s p;
    apply_defaults(&p, prm);
    std::vector<double> ones;
    const fc_setup_params q = effective_params(prm, ones);
    fc_status st = guard([&] { host_spectra_and_separables(&p, &q); });
    if (st != FC_OK) return st;
    const Separable& S = which == 0 ? p.op : which == 1 ? active_pc(&p) : p.st;
    *rank = S.Q;
    if (max_rel_err) *max_rel_err = which == 0 ? p.op_err : which == 1 ? active_pc_err(&p) : p.st_err;
    if (cap < S.Q) return fail(FC_ERR_RANK_OVERFLOW, "capacity too small");
    const int n = p.n;
    if (w) std::memcpy(w, S.w.data(), sizeof(double) * S.Q);
    if (F)
        for (int l = 0; l < 3; ++l)
            std::memcpy(F + (size_t)l * n * cap, S.F[l].data(), sizeof(double) * n * S.Q);
    return FC_OK;
}

static fc_status validate_params(const fc_setup_params* prm) {
    const int n = prm->n;
    if (n < 2 || n > 4096) return fail(FC_ERR_INVALID_ARG, "n must be in [2, 4096]");
    if (prm->dims != 0 && prm->dims != 2 && prm->dims != 3)
        return fail(FC_ERR_INVALID_ARG, "dims must be 2 or 3");
    for (int l = 0; l < (prm->dims == 2 ? 2 : 3); ++l) {
        if (!prm->a[l]) return fail(FC_ERR_INVALID_ARG, "coefficient pointer is NULL");
        if (!finite_pos(prm->a[l], n + 1))
            return fail(FC_ERR_INVALID_ARG, "coefficient samples must be finite and > 0");
    }
    if (!(prm->alpha >= 0.0 && prm->alpha <= 1.0)) return fail(FC_ERR_INVALID_ARG, "alpha must be in [0, 1]");
    if (!(prm->beta > 0.0) || !std::isfinite(prm->beta)) return fail(FC_ERR_INVALID_ARG, "beta must be > 0");
    if (!(prm->gamma > 0.0) || !std::isfinite(prm->gamma)) return fail(FC_ERR_INVALID_ARG, "gamma must be > 0");
    if (!(prm->eps > 0.0 && prm->eps < 1.0)) return fail(FC_ERR_INVALID_ARG, "eps must be in (0, 1)");
    if (prm->tol < 0 || prm->op_accuracy < 0 || prm->max_iter < 0 || prm->max_rank < 0 ||
        prm->precond_rank < 0)
        return fail(FC_ERR_INVALID_ARG, "negative option");
    if (prm->max_rank > KM) return fail(FC_ERR_INVALID_ARG, "max_rank must be <= 128");
    if (prm->precond_rank > 16) return fail(FC_ERR_INVALID_ARG, "precond_rank must be <= 16");
    if (prm->precision != FC_FP64 && prm->precision != FC_MIXED_FP32)
        return fail(FC_ERR_INVALID_ARG, "unsupported precision");
    if (prm->precond != FC_PRECOND_EIGEN && prm->precond != FC_PRECOND_LAPLACE)
        return fail(FC_ERR_INVALID_ARG, "unknown preconditioner");
    for (int l = 0; l < 3; ++l)
        if (!std::isfinite(prm->precond_b0[l]))
            return fail(FC_ERR_INVALID_ARG, "precond_b0 must be finite");
    return FC_OK;
}

static void apply_defaults(fc_plan_s* p, const fc_setup_params* prm) {
    p->n = prm->n;
    p->alpha = prm->alpha; p->beta = prm->beta; p->gamma = prm->gamma; p->eps = prm->eps;
    p->tol = prm->tol > 0 ? prm->tol : prm->eps;
    p->op_acc = prm->op_accuracy > 0 ? prm->op_accuracy : prm->eps;
    p->max_iter = prm->max_iter > 0 ? prm->max_iter : 100;
    p->rcap = prm->max_rank > 0 ? prm->max_rank : 96;
    p->pcap = 128;
    p->precond_rank = prm->precond_rank;   // 0: automatic
    p->precision = prm->precision;
    p->pc_kind = prm->precond;
    p->dims = prm->dims == 2 ? 2 : 3;
}

// The parameters the construction runs on: with d = 2 the third mode is the
// constant-coefficient Laplacian (samples all 1; `ones` keeps them alive).
static fc_setup_params effective_params(const fc_setup_params* prm, std::vector<double>& ones) {
    fc_setup_params q = *prm;
    if (prm->dims == 2) {
        ones.assign((size_t)prm->n + 1, 1.0);
        q.a[2] = ones.data();
        q.precond_b0[2] = 1.0;
    }
    return q;
}

fc_status fc_setup_ex(const fc_setup_params* prm, void* hip_stream, fc_plan* out) {
    if (!prm || !out) return fail(FC_ERR_INVALID_ARG, "fc_setup_ex: NULL argument");
    *out = nullptr;
    fc_status v = validate_params(prm);
    if (v != FC_OK) return v;
    fc_plan_s* p = new fc_plan_s();
    apply_defaults(p, prm);
    // without a caller stream the setup runs on a stream of its own: plans set
    // up on concurrent threads must not queue behind each other on the NULL
    // stream (their fits run for hundreds of milliseconds)
    hipStream_t own = nullptr;
    if (!hip_stream) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) {
            delete p;
            return fail(FC_ERR_HIP, "hipStreamCreateWithFlags failed");
        }
    }
    p->stream = own ? own : (hipStream_t)hip_stream;
    std::vector<double> ones;
    const fc_setup_params q = effective_params(prm, ones);
    fc_status st = guard([&] { setup_plan(p, &q); });
    if (own) {
        (void)hipStreamSynchronize(own);
        (void)hipStreamDestroy(own);
        p->stream = nullptr;
    }
    if (st != FC_OK) { delete p; return st; }
    *out = p;
    return FC_OK;
}

fc_status fc_setup(int n, const double* a1, const double* a2, const double* a3, double alpha,
                   double beta, double eps, fc_plan* out) {
    fc_setup_params prm;
    std::memset(&prm, 0, sizeof(prm));
    prm.n = n; prm.a[0] = a1; prm.a[1] = a2; prm.a[2] = a3;
    prm.alpha = alpha; prm.beta = beta; prm.gamma = 1.0; prm.eps = eps;
    prm.precision = FC_FP64;
    return fc_setup_ex(&prm, nullptr, out);
}

void fc_destroy(fc_plan plan) { delete plan; }

fc_status fc_plan_spectrum(fc_plan p, double* lam, double* V) {
    if (!p || !lam) return fail(FC_ERR_INVALID_ARG, "fc_plan_spectrum: NULL argument");
    const int n = p->n;
    return guard([&] {
        for (int l = 0; l < 3; ++l) {
            std::memcpy(lam + (size_t)l * n, p->lam[l].data(), sizeof(double) * n);
            if (V)
                HIPCHK(hipMemcpy(V + (size_t)l * n * n, p->V[l], sizeof(double) * n * n,
                                 hipMemcpyDeviceToHost));
        }
    });
}

fc_status fc_plan_separable(fc_plan p, int which, int cap, int* rank, double* w, double* F) {
    if (!p || !rank || which < 0 || which > 2) return fail(FC_ERR_INVALID_ARG, "fc_plan_separable: bad arguments");
    const Separable& S = which == 0 ? p->op : which == 1 ? active_pc(p) : p->st;
    *rank = S.Q;
    if (cap < S.Q) return fail(FC_ERR_RANK_OVERFLOW, "capacity too small");
    const int n = p->n;
    if (w) std::memcpy(w, S.w.data(), sizeof(double) * S.Q);
    if (F)
        return guard([&] {
            for (int l = 0; l < 3; ++l)
                HIPCHK(hipMemcpy(F + (size_t)l * n * cap, S.Fd[l], sizeof(double) * n * S.Q,
                                 hipMemcpyDeviceToHost));
        });
    return FC_OK;
}

fc_status fc_plan_tuning(fc_plan p, int* choices, double* us) {
    if (!p || !choices) return fail(FC_ERR_INVALID_ARG, "fc_plan_tuning: NULL argument");
    const Tuning& t = p->tune;
    choices[0] = t.gram_batched;
    choices[1] = t.gram_single;
    choices[2] = t.kron;
    choices[3] = t.stream_kc;
    choices[4] = t.panel_b;
    choices[5] = t.tuned ? 1 : 0;
    if (us)
        for (int i = 0; i < 10; ++i) us[i] = t.us[i];
    return FC_OK;
}

fc_status fc_mode_transform(fc_plan p, int mode, int transpose, int m, const double* X,
                            double* out, void* stream) {
    if (!p || mode < 0 || mode > 2 || m < 0 || !X || !out) return fail(FC_ERR_INVALID_ARG, "fc_mode_transform: bad arguments");
    Ctx c{p, (hipStream_t)stream, p->n};
    return guard([&] {
        KindTag tag(3);
        const double* M = transpose ? p->Vt[mode] : p->V[mode];
        gemm(c, false, false, p->n, m, p->n, 1.0, M, p->n, X, p->n, 0.0, out, p->n);
    });
}

}  // extern "C"

namespace {

// The three cross Grams G_l = A_l^T B_l (ra x rb, ld ra) of a canonical
// inner product: one launch of the Gram kernel for ranks <= 128, else the
// LDS-tiled GEMM (no split-K workspace).  Shared by fc_cp_inner and
// fc_cp_inner_noalloc, so that both give the same bits.
hipError_t cross_grams(int n, int ra, const double* const A[3], int rb, const double* const B[3],
                       double* const G[3], hipStream_t s) {
    fc::GramJobs jobs;
    for (int l = 0; l < 3; ++l) {
        fc::GemmArgs& g = jobs.g[jobs.count++];
        g.M = ra; g.N = rb; g.K = n;
        g.A = A[l]; g.lda = n; g.B = B[l]; g.ldb = n; g.C = G[l]; g.ldc = ra;
    }
    if (ra <= 128 && rb <= 128) return fc::gram_multi(true, false, jobs, s, 16, gram_staged(true));
    hipError_t e = hipSuccess;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) e = fc::gemm(true, false, jobs.g[l], s);
    return e;
}

}  // namespace

extern "C" {

fc_status fc_cp_inner(fc_plan p, int ra, const double* wa, const double* A1, const double* A2,
                      const double* A3, int rb, const double* wb, const double* B1,
                      const double* B2, const double* B3, double* out, void* stream) {
    if (!p || ra < 1 || rb < 1 || !A1 || !A2 || !A3 || !B1 || !B2 || !B3 || !out)
        return fail(FC_ERR_INVALID_ARG, "fc_cp_inner: bad arguments");
    if ((long)ra * rb > (long)p->pcap * p->pcap * p->pcap) return fail(FC_ERR_INVALID_ARG, "ranks too large");
    Ctx c{p, (hipStream_t)stream, p->n};
    const double* A[3] = {A1, A2, A3};
    const double* B[3] = {B1, B2, B3};
    return guard([&] {
        double* G[3] = {p->C, p->Cp, p->Cn1};
        HIPCHK(cross_grams(p->n, ra, A, rb, B, G, c.s));
        HIPCHK(fc::cp_inner_reduce(ra, rb, G[0], G[1], G[2], wa, wb, p->scal, c.s));
        d2h(c, out, p->scal, 1);
    });
}

}  // extern "C"

namespace {

// Scratch of fc_cp_inner_noalloc: the three cross Grams A_l^T B_l (ra x rb
// each, ra * rb <= kNoAllocPairs).  A file-scope device array, so the entry
// point needs no allocation; each GPU holds its own copy, found through
// hipGetSymbolAddress once per device (the array's name in host code is not
// a device address).
constexpr long kNoAllocPairs = 256L * 256L;
__device__ __align__(256) double scratch[3 * kNoAllocPairs];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the first call on
// that device).
fc_status noalloc_scratch(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FC_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(FC_ERR_INTERNAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(FC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                        hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return FC_OK;
}

}  // namespace

extern "C" {

fc_status fc_cp_inner_noalloc(int n, int ra, const double* wa, const double* A1, const double* A2,
                              const double* A3, int rb, const double* wb, const double* B1,
                              const double* B2, const double* B3, double* out, void* stream) {
    if (n < 1 || ra < 1 || rb < 1 || !A1 || !A2 || !A3 || !B1 || !B2 || !B3 || !out)
        return fail(FC_ERR_INVALID_ARG, "fc_cp_inner_noalloc: bad arguments");
    if ((long)ra * rb > kNoAllocPairs)
        return fail(FC_ERR_INVALID_ARG, "fc_cp_inner_noalloc: ra * rb = " +
                                            std::to_string((long)ra * rb) +
                                            " exceeds the scratch capacity of 65536 pairs");
    double* ws = nullptr;
    const fc_status st = noalloc_scratch(&ws);
    if (st != FC_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    const double* A[3] = {A1, A2, A3};
    const double* B[3] = {B1, B2, B3};
    double* G[3];
    for (int l = 0; l < 3; ++l) G[l] = ws + l * (long)ra * rb;
    hipError_t e = cross_grams(n, ra, A, rb, B, G, s);
    if (e == hipSuccess) e = fc::cp_inner_reduce(ra, rb, G[0], G[1], G[2], wa, wb, out, s);
    if (e != hipSuccess)
        return fail(FC_ERR_HIP, std::string("fc_cp_inner_noalloc: ") + hipGetErrorString(e));
    return FC_OK;
}

static fc_status canon_out(fc_plan p, const Ctx& c, const Tucker& T, double budget2, bool to_grid,
                           int cap, int* rank_out, double* w_out, double* O1, double* O2,
                           double* O3) {
    double* U[3] = {O1, O2, O3};
    const int K = tucker_to_canon_out(c, T, budget2, to_grid, cap, w_out, U);
    *rank_out = K;
    if (K > cap) return fail(FC_ERR_RANK_OVERFLOW, "result rank " + std::to_string(K) + " exceeds capacity");
    return FC_OK;
}

fc_status fc_cp_truncate(fc_plan p, int m, const double* w, const double* X1, const double* X2,
                         const double* X3, double eps, int cap, int* rank_out, double* w_out,
                         double* O1, double* O2, double* O3, void* stream) {
    if (!p || m < 1 || m > 256 || !X1 || !X2 || !X3 || !(eps > 0 && eps < 1) || cap < 0 ||
        !rank_out || !w_out || !O1 || !O2 || !O3)
        return fail(FC_ERR_INVALID_ARG, "fc_cp_truncate: bad arguments");
    Ctx c{p, (hipStream_t)stream, p->n};
    fc_status inner = FC_OK;
    fc_status st = guard([&] {
        const double* X[3] = {X1, X2, X3};
        Tucker& T = p->slot[8];
        // split the budget: half to C2T, half to T2C
        canon_to_tucker(c, m, w, X, eps / std::sqrt(2.0), T, "trunc");
        const double n2 = tucker_norm2(c, T);
        inner = canon_out(p, c, T, 0.5 * eps * eps * n2, false, cap, rank_out, w_out, O1, O2, O3);
    });
    return st != FC_OK ? st : inner;
}

fc_status fc_apply_separable(fc_plan p, int which, int m, const double* w, const double* X1,
                             const double* X2, const double* X3, double eps, int cap,
                             int* rank_out, double* w_out, double* O1, double* O2, double* O3,
                             void* stream) {
    if (!p || which < 0 || which > 2 || m < 1 || m > 256 || !X1 || !X2 || !X3 ||
        !(eps > 0 && eps < 1) || cap < 0 || !rank_out || !w_out || !O1 || !O2 || !O3)
        return fail(FC_ERR_INVALID_ARG, "fc_apply_separable: bad arguments");
    Ctx c{p, (hipStream_t)stream, p->n};
    fc_status inner = FC_OK;
    fc_status st = guard([&] {
        const double* X[3] = {X1, X2, X3};
        Tucker& T = p->slot[8];
        Tucker& O = p->slot[9];
        canon_to_tucker(c, m, w, X, 1e-3 * eps, T, "input");
        reset_warm(p);
        if (which == 1)
            apply_precond(c, T, eps / std::sqrt(2.0), O, "apply", SITE_MISC);
        else
            had_trunc(c, which == 0 ? p->op : p->st, T, eps / std::sqrt(2.0), 0.0, O, "apply",
                      SITE_MISC);
        const double n2 = tucker_norm2(c, O);
        inner = canon_out(p, c, O, 0.5 * eps * eps * n2, false, cap, rank_out, w_out, O1, O2, O3);
    });
    return st != FC_OK ? st : inner;
}

}  // extern "C"

namespace {

// Output of the optional state recovery (fc_solve_state).
struct StateOut {
    int cap = 0;
    int* rank = nullptr;
    double* w = nullptr;
    double* F[3] = {nullptr, nullptr, nullptr};
    double* J = nullptr;
};

fc_status solve_impl(fc_plan p, int rank_y, const double* w_y, const double* Y1, const double* Y2,
                     const double* Y3, int cap_u, int* rank_u, double* w_u, double* U1,
                     double* U2, double* U3, fc_info* info, void* stream, const StateOut* so_out) {
    Ctx c{p, (hipStream_t)stream, p->n};
    const int n = p->n;
    fc_status result = FC_OK;
    p->max_seen_rank = 0;
    p->worst_missed = 0;
    reset_warm(p);
    for (int i = 0; i < 16; ++i) { p->site_ms[i] = 0; p->site_calls[i] = 0; }
    const auto t_solve = std::chrono::steady_clock::now();
    fc_status st = guard([&] {
        // NaN guard on the input
        static const int zero_flag = 0;
        h2d(c, p->dflag, &zero_flag, 1);
        const double* Y[3] = {Y1, Y2, Y3};
        for (int l = 0; l < 3; ++l) HIPCHK(fc::check_finite((long)n * rank_y, Y[l], p->dflag, c.s));
        if (w_y) HIPCHK(fc::check_finite(rank_y, w_y, p->dflag, c.s));
        int flag = 0;
        d2h(c, &flag, p->dflag, 1);
        if (flag) throw FcError(FC_ERR_NUMERIC, "non-finite value in the design function");
        // entry transform Y_hat_l = V_l^T Y_l (into workspace tmp buffers)
        double* Yh[3] = {p->Yh[0], p->Yh[1], p->Yh[2]};
        {
            KindTag tag(3);
            fc::GemmArgs tr[3];
            for (int l = 0; l < 3; ++l) tr[l] = prod(n, rank_y, n, p->Vt[l], n, Y[l], n, Yh[l], n);
            gemm_group(c, false, false, tr, 3);
        }
        Tucker& B = p->slot[0];
        const double* Yc[3] = {Yh[0], Yh[1], Yh[2]};
        canon_to_tucker(c, rank_y, w_y, Yc, 1e-2 * p->eps, B, "B = C2T(Y_hat)");
        Tucker X;
        SolveOut so;
        int sweeps = 0;
        if (B.empty()) {
            so.converged = true;
        } else if (p->precision == FC_MIXED_FP32) {
            so = mixed_solve(c, B, X, sweeps);
        } else {
            const double bn = std::sqrt(tucker_norm2(c, B));
            so = pcg(c, B, X, p->eps, p->tol, p->max_iter, 0.1 * p->eps * bn);
        }
        // state y = beta A^-alpha u (eqn `State`) from the Tucker solution, and
        // the cost J = 1/2 ||y - y_Omega||^2 + gamma/2 ||u||^2 (Section 3.1,
        // M = I) from exact Tucker inner products in eigen-coordinates
        int Ks = 0;
        if (so_out) {
            Tucker& Ys = p->slot[12];
            if (X.empty()) {
                Ys.r[0] = Ys.r[1] = Ys.r[2] = 0;
            } else {
                p->warm[SITE_ST].valid = false;
                had_trunc(c, p->st, X, p->eps, 0.0, Ys, "state: trunc(beta A^-alpha u)", SITE_ST);
            }
            if (so_out->J) {
                const double yy = tucker_norm2(c, Ys), bb = tucker_norm2(c, B);
                const double yb = (Ys.empty() || B.empty()) ? 0.0 : tucker_inner(c, Ys, B);
                const double uu = tucker_norm2(c, X);
                *so_out->J = 0.5 * (yy - 2.0 * yb + bb) + 0.5 * p->gamma * uu;
            }
            const double yn2 = Ys.empty() ? 0.0 : tucker_norm2(c, Ys);
            Ks = Ys.empty() ? 0 : tucker_to_canon_out(c, Ys, 0.01 * p->eps * p->eps * yn2, true,
                                                      so_out->cap, so_out->w, so_out->F);
            *so_out->rank = Ks;
        }
        // T2C of the result and exit transform U_l = V_l (Z_l coef)
        const double xn2 = X.empty() ? 0.0 : tucker_norm2(c, X);
        double* U[3] = {U1, U2, U3};
        const int K = X.empty() ? 0 : tucker_to_canon_out(c, X, 0.01 * p->eps * p->eps * xn2, true,
                                                          cap_u, w_u, U);
        *rank_u = K;
        if (info) {
            info->iterations = so.iterations;
            info->rank_u = K;
            for (int l = 0; l < 3; ++l) info->tucker_rank[l] = X.r[l];
            info->max_tucker_rank = p->max_seen_rank;
            info->op_rank = p->op.Q;
            info->precond_rank = active_pc(p).Q;
            info->rel_residual = so.rel_res;
            info->refinements = sweeps;
            info->op_max_rel_err = p->op_err;
            info->precond_max_rel_err = active_pc_err(p);
            info->state_rank = p->st.Q;
            info->state_max_rel_err = p->st_err;
            info->subspace_miss = p->worst_missed;
        }
        if (K > cap_u) result = fail(FC_ERR_RANK_OVERFLOW, "result rank exceeds cap_u");
        else if (so_out && Ks > so_out->cap) result = fail(FC_ERR_RANK_OVERFLOW, "state rank exceeds cap_s");
        else if (!so.converged) result = fail(FC_ERR_NOT_CONVERGED, "max_iter reached");
        if (g_trace) {
            sync(c);
            const double tot = std::chrono::duration<double, std::milli>(
                                   std::chrono::steady_clock::now() - t_solve).count();
            static const char* names[NSITES] = {"Z", "S", "X", "R", "P", "misc", "ref-S", "ref-R",
                                                "ref-U", "state", "ref-Z"};
            std::string line = "[fc] solve " + std::to_string(tot) + " ms; truncations:";
            for (int i = 0; i < NSITES; ++i)
                if (p->site_calls[i])
                    line += std::string(" ") + names[i] + " " + std::to_string(p->site_calls[i]) +
                            "x " + std::to_string(p->site_ms[i]) + " ms;";
            std::fprintf(stderr, "%s\n", line.c_str());
        }
    });
    return st != FC_OK ? st : result;
}

}  // namespace

// Workers of the batched call, one pool per device and worker count: the
// threads and their non-blocking streams (default priority) live for the
// process, created by the first batched call, so a call neither starts
// threads nor creates streams.  One batched call at a time runs on a pool
// (concurrent calls queue on call_mu).  Pools are never freed: their threads
// wait on the condition variable until the process ends.
struct BatchPool {
    int dev = 0;
    int size = 0;
    std::mutex call_mu;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::function<void(int, hipStream_t)> job;
    unsigned long generation = 0;
    int pending = 0;
    int ready = 0;
    bool failed = false;   // a worker could not select the device or create its stream
};

void batch_worker(BatchPool* P, int t) {
    hipStream_t s = nullptr;
    const bool ok = hipSetDevice(P->dev) == hipSuccess &&
                    hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    unsigned long seen = 0;
    {
        std::lock_guard<std::mutex> lk(P->mu);
        if (!ok) P->failed = true;
        ++P->ready;
    }
    P->done_cv.notify_all();
    for (;;) {
        std::function<void(int, hipStream_t)> job;
        {
            std::unique_lock<std::mutex> lk(P->mu);
            P->cv.wait(lk, [&] { return P->generation != seen; });
            seen = P->generation;
            job = P->job;
        }
        if (ok && job) job(t, s);
        bool last = false;
        {
            std::lock_guard<std::mutex> lk(P->mu);
            last = --P->pending == 0;
        }
        if (last) P->done_cv.notify_all();
    }
}

BatchPool* batch_pool(int dev, int size) {
    static std::mutex m;
    static std::vector<BatchPool*> pools;
    std::lock_guard<std::mutex> lk(m);
    for (BatchPool* p : pools)
        if (p->dev == dev && p->size == size) return p;
    BatchPool* p = new BatchPool();
    p->dev = dev;
    p->size = size;
    for (int t = 0; t < size; ++t) std::thread(batch_worker, p, t).detach();
    {
        std::unique_lock<std::mutex> l2(p->mu);
        p->done_cv.wait(l2, [&] { return p->ready == size; });
    }
    pools.push_back(p);
    return p;
}

extern "C" {

fc_status fc_solve(fc_plan p, int rank_y, const double* w_y, const double* Y1, const double* Y2,
                   const double* Y3, int cap_u, int* rank_u, double* w_u, double* U1,
                   double* U2, double* U3, fc_info* info, void* stream) {
    if (!p || rank_y < 1 || rank_y > 256 || !Y1 || !Y2 || !Y3 || cap_u < 0 || !rank_u ||
        !w_u || !U1 || !U2 || !U3)
        return fail(FC_ERR_INVALID_ARG, "fc_solve: bad arguments");
    if (p->dims == 2) return fail(FC_ERR_INVALID_ARG, "fc_solve: two-dimensional plan (use fc_solve2d)");
    return solve_impl(p, rank_y, w_y, Y1, Y2, Y3, cap_u, rank_u, w_u, U1, U2, U3, info, stream,
                      nullptr);
}

fc_status fc_solve2d(fc_plan p, int rank_y, const double* w_y, const double* Y1, const double* Y2,
                     int cap_u, int* rank_u, double* w_u, double* U1, double* U2, fc_info* info,
                     void* stream) {
    if (!p || rank_y < 1 || rank_y > 256 || !Y1 || !Y2 || cap_u < 0 || !rank_u || !w_u || !U1 ||
        !U2)
        return fail(FC_ERR_INVALID_ARG, "fc_solve2d: bad arguments");
    if (p->dims != 2) return fail(FC_ERR_INVALID_ARG, "fc_solve2d: plan is not two-dimensional");
    const hipStream_t s = (hipStream_t)stream;
    const double* v = p->V[2];   // first eigenvector of the third mode (its null direction)
    fc_status st = guard([&] { HIPCHK(fc::fill_columns(p->n, rank_y, v, p->Y3d, p->n, s)); });
    if (st != FC_OK) return st;
    // the result's rank is at most min(r1, r2) <= max_rank (one core slice)
    const int cap = std::min(cap_u, 256);
    st = solve_impl(p, rank_y, w_y, Y1, Y2, p->Y3d, cap, rank_u, w_u, U1, U2, p->U3d, info, stream,
                    nullptr);
    // the written iterate (a result, or the best iterate of a solve that did
    // not converge) carries <U3[:, k], v1> = +-1 in its weights
    if (st != FC_OK && st != FC_ERR_NOT_CONVERGED) return st;
    if (*rank_u > cap) return st;
    const std::string detail = st != FC_OK ? g_last_error : std::string();
    const fc_status sc = guard([&] {
        HIPCHK(fc::scale_by_dot(p->n, *rank_u, p->U3d, p->n, v, w_u, s));
        HIPCHK(hipStreamSynchronize(s));
    });
    if (sc != FC_OK) return sc;
    if (st != FC_OK) g_last_error = detail;
    return st;
}

fc_status fc_solve_state(fc_plan p, int rank_y, const double* w_y, const double* Y1,
                         const double* Y2, const double* Y3, int cap_u, int* rank_u, double* w_u,
                         double* U1, double* U2, double* U3, int cap_s, int* rank_s, double* w_s,
                         double* S1, double* S2, double* S3, double* J, fc_info* info,
                         void* stream) {
    if (!p || rank_y < 1 || rank_y > 256 || !Y1 || !Y2 || !Y3 || cap_u < 0 || !rank_u ||
        !w_u || !U1 || !U2 || !U3 || cap_s < 0 || !rank_s || !w_s || !S1 || !S2 || !S3)
        return fail(FC_ERR_INVALID_ARG, "fc_solve_state: bad arguments");
    if (p->dims == 2) return fail(FC_ERR_INVALID_ARG, "fc_solve_state: two-dimensional plan");
    StateOut so;
    so.cap = cap_s;
    so.rank = rank_s;
    so.w = w_s;
    so.F[0] = S1; so.F[1] = S2; so.F[2] = S3;
    so.J = J;
    return solve_impl(p, rank_y, w_y, Y1, Y2, Y3, cap_u, rank_u, w_u, U1, U2, U3, info, stream,
                      &so);
}

fc_status fc_solve_batched(int count, const fc_plan* plans, const int* rank_y,
                           const double* const* w_y, const double* const* Y1,
                           const double* const* Y2, const double* const* Y3, const int* cap_u,
                           int* rank_u, double* const* w_u, double* const* U1,
                           double* const* U2, double* const* U3, fc_status* status,
                           fc_info* info, void* stream) {
    if (count < 0 || (count > 0 && (!plans || !rank_y || !Y1 || !Y2 || !Y3 || !cap_u || !rank_u ||
                                    !w_u || !U1 || !U2 || !U3 || !status)))
        return fail(FC_ERR_INVALID_ARG, "fc_solve_batched: bad arguments");
    for (int i = 0; i < count; ++i)
        if (!plans[i]) return fail(FC_ERR_INVALID_ARG, "fc_solve_batched: NULL plan");
    if (count == 0) return FC_OK;
    // Problems run concurrently: the pool's worker threads, each with its own
    // stream, take problems in order from a shared counter.  The caller's
    // stream is joined at the start (its pending work completes before any
    // solve starts); every solve synchronises its own stream before it
    // returns.
    int workers = 16;
    if (const char* env = std::getenv("FC_BATCH_STREAMS")) workers = std::max(1, std::atoi(env));
    workers = std::min(workers, 64);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FC_ERR_HIP, "hipGetDevice failed");
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return fail(FC_ERR_HIP, "hipStreamSynchronize failed");
    BatchPool* P = batch_pool(dev, workers);
    if (P->failed) return fail(FC_ERR_HIP, "fc_solve_batched: a worker stream could not be created");
    std::lock_guard<std::mutex> call(P->call_mu);
    std::atomic<int> next(0);
    std::vector<std::string> errs(count);
    for (int i = 0; i < count; ++i) status[i] = FC_ERR_INTERNAL;
    auto work = [&](int t, hipStream_t s) {
        t_no_profile = (t != 0);   // GEMM timing (when enabled) samples worker 0
        for (;;) {
            const int i = next.fetch_add(1);
            if (i >= count) break;
            std::lock_guard<std::mutex> lk(plans[i]->use_mu);
            const double* wy = w_y ? w_y[i] : nullptr;
            fc_info* inf = info ? &info[i] : nullptr;
            status[i] = plans[i]->dims == 2
                            ? fc_solve2d(plans[i], rank_y[i], wy, Y1[i], Y2[i], cap_u[i],
                                         &rank_u[i], w_u[i], U1[i], U2[i], inf, s)
                            : fc_solve(plans[i], rank_y[i], wy, Y1[i], Y2[i], Y3[i], cap_u[i],
                                       &rank_u[i], w_u[i], U1[i], U2[i], U3[i], inf, s);
            if (status[i] != FC_OK) errs[i] = g_last_error;
        }
        (void)hipStreamSynchronize(s);
        t_no_profile = false;
    };
    {
        std::lock_guard<std::mutex> lk(P->mu);
        P->job = work;
        P->pending = P->size;
        ++P->generation;
    }
    P->cv.notify_all();
    {
        std::unique_lock<std::mutex> lk(P->mu);
        P->done_cv.wait(lk, [&] { return P->pending == 0; });
        P->job = nullptr;   // it refers to this call's locals
    }
    fc_status first = FC_OK;
    for (int i = 0; i < count; ++i)
        if (status[i] != FC_OK && first == FC_OK) {
            first = status[i];
            g_last_error = "problem " + std::to_string(i) + ": " + errs[i];
        }
    return first;
}

fc_status fc_profile_gemm(int enable) {
    if (enable) {
        g_prof.on = true;
        g_prof.used = 0;
        g_prof.shapes.clear();
        for (KernelProfile& kp : k_prof) {
            kp.used = 0;
            kp.flops = kp.bytes = 0;
            kp.launches = 0;
        }
        g_prof.flops = g_prof.bytes = 0;
        g_prof.launches = 0;
    } else {
        g_prof.on = false;
    }
    return FC_OK;
}

fc_status fc_profile_kernel_read(int kind, long* launches, double* total_ms, double* flops,
                                 double* bytes) {
    if (kind < 0 || kind >= kProfKinds || !launches || !total_ms || !flops || !bytes)
        return fail(FC_ERR_INVALID_ARG, "fc_profile_kernel_read: bad arguments");
    double ms = 0;
    if (kind == 1 || kind == 2) {
        KernelProfile& kp = k_prof[kind];
        for (size_t i = 0; i + 1 < kp.used; i += 2) {
            if (hipEventSynchronize(kp.ev[i + 1]) != hipSuccess)
                return fail(FC_ERR_HIP, "hipEventSynchronize failed");
            float t = 0;
            if (hipEventElapsedTime(&t, kp.ev[i], kp.ev[i + 1]) != hipSuccess)
                return fail(FC_ERR_HIP, "hipEventElapsedTime failed");
            ms += t;
        }
        *launches = kp.launches;
        *total_ms = ms;
        *flops = kp.flops;
        *bytes = kp.bytes;
        return FC_OK;
    }
    long cnt = 0;
    double fl = 0, by = 0;
    for (size_t i = 0; i + 1 < g_prof.used && i / 2 < g_prof.shapes.size(); i += 2) {
        const GemmShape& g = g_prof.shapes[i / 2];
        if (g.kind != kind) continue;
        if (hipEventSynchronize(g_prof.ev[i + 1]) != hipSuccess)
            return fail(FC_ERR_HIP, "hipEventSynchronize failed");
        float t = 0;
        if (hipEventElapsedTime(&t, g_prof.ev[i], g_prof.ev[i + 1]) != hipSuccess)
            return fail(FC_ERR_HIP, "hipEventElapsedTime failed");
        ms += t;
        cnt += 1;
        fl += g.flops;
        by += g.bytes;
    }
    *launches = cnt;
    *total_ms = ms;
    *flops = fl;
    *bytes = by;
    return FC_OK;
}

fc_status fc_profile_gemm_read(long* launches, double* total_ms, double* flops, double* bytes) {
    if (!launches || !total_ms || !flops || !bytes) return fail(FC_ERR_INVALID_ARG, "NULL argument");
    double ms = 0;
    for (size_t i = 0; i + 1 < g_prof.used; i += 2) {
        if (hipEventSynchronize(g_prof.ev[i + 1]) != hipSuccess)
            return fail(FC_ERR_HIP, "hipEventSynchronize failed");
        float t = 0;
        if (hipEventElapsedTime(&t, g_prof.ev[i], g_prof.ev[i + 1]) != hipSuccess)
            return fail(FC_ERR_HIP, "hipEventElapsedTime failed");
        ms += t;
    }
    // diagnostic: per-launch shapes and times as CSV (environment FC_GEMMLOG = path)
    if (const char* path = std::getenv("FC_GEMMLOG")) {
        if (FILE* f = std::fopen(path, "w")) {
            std::fprintf(f, "kind,ta,tb,M,N,K,batch,inner,lowp,flops,bytes,us\n");
            for (size_t i = 0; i + 1 < g_prof.used && i / 2 < g_prof.shapes.size(); i += 2) {
                float t = 0;
                (void)hipEventElapsedTime(&t, g_prof.ev[i], g_prof.ev[i + 1]);
                const GemmShape& g = g_prof.shapes[i / 2];
                std::fprintf(f, "%d,%d,%d,%d,%d,%d,%d,%d,%d,%.6g,%.6g,%.2f\n", g.kind, g.ta, g.tb,
                             g.M, g.N, g.K, g.batch, g.inner, g.lowp, g.flops, g.bytes,
                             1000.0 * t);
            }
            std::fclose(f);
        }
    }
    *launches = g_prof.launches;
    *total_ms = ms;
    *flops = g_prof.flops;
    *bytes = g_prof.bytes;
    return FC_OK;
}

int fc_selftest_eig(int k, const double* A_host, double* evals_host, double* V_host) {
    if (k < 1 || k > 128 || !A_host || !evals_host || !V_host) return 1;
    double *A = nullptr, *ev = nullptr, *V = nullptr, *scr = nullptr;
    if (hipMalloc(&A, sizeof(double) * k * k) != hipSuccess) return 2;
    if (hipMalloc(&ev, sizeof(double) * k) != hipSuccess) return 2;
    if (hipMalloc(&V, sizeof(double) * k * k) != hipSuccess) return 2;
    if (hipMalloc(&scr, sizeof(double) * 6 * k * k) != hipSuccess) return 2;
    int rc = 0;
    if (hipMemcpy(A, A_host, sizeof(double) * k * k, hipMemcpyHostToDevice) != hipSuccess) rc = 3;
    fc::EigJobs jobs;
    jobs.count = 1;
    jobs.job[0].A = A; jobs.job[0].lda = k; jobs.job[0].k = k;
    jobs.job[0].evals = ev; jobs.job[0].V = V; jobs.job[0].ldv = k; jobs.job[0].scratch = scr;
    if (!rc && fc::sym_eig_multi(jobs, nullptr) != hipSuccess) rc = 4;
    if (!rc && hipMemcpy(evals_host, ev, sizeof(double) * k, hipMemcpyDeviceToHost) != hipSuccess) rc = 5;
    if (!rc && hipMemcpy(V_host, V, sizeof(double) * k * k, hipMemcpyDeviceToHost) != hipSuccess) rc = 5;
    (void)hipFree(A); (void)hipFree(ev); (void)hipFree(V); (void)hipFree(scr);
    return rc;
}

int fc_selftest_mfma(double* host_out) {
    double* d = nullptr;
    if (hipMalloc(&d, 512 * sizeof(double)) != hipSuccess) return 1;
    int rc = 0;
    if (fc::mfma_probe(d, nullptr) != hipSuccess) rc = 2;
    if (!rc && hipMemcpy(host_out, d, 512 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) rc = 3;
    (void)hipFree(d);
    return rc;
}

}  // extern "C"
