// Exponential-sum fits of the setup phase on the device (gfx950): the
// operator symbol f(s)/s and the state map beta s^-alpha as nonnegative
// sums (Section 3.4), the preconditioner symbol 1/f(s) as a sum of K
// exponentials with free nodes (Section 3.5, case (B); case (A) on the
// Laplacian's spectrum).  One workgroup per fit job; the candidate node
// grids and ranks of one plan are independent jobs of one launch.
#pragma once
#include <hip/hip_runtime.h>

namespace fc {

enum FitTarget {
    FIT_OPERATOR = 0,   // h(s) = g(s) - cexact, relative to g(s) = beta s^(-alpha-1) + (gamma/beta) s^(alpha-1)
    FIT_STATE = 1,      // h(s) = beta s^-alpha, relative to itself
    FIT_PRECOND = 2,    // 1/f(s), f(s) = beta s^-alpha + (gamma/beta) s^alpha, relative to itself
};

constexpr int kFitSamples = 2000;     // sample points of a nonnegative fit
constexpr int kFitMaxNodes = 256;     // node grid of a nonnegative fit, constant included
constexpr int kFitMaxK = 16;          // terms of a free-node fit
constexpr int kMaxFitJobs = 24;
constexpr int kFitThreads = 512;

struct FitJob {
    int target = 0;
    double alpha = 0, beta = 0, gamma = 0, cexact = 0;
    double smin = 0, smax = 0;
    // nonnegative fits: nodes exp(x_j), x_0 = log_tlo, x_{j+1} = x_j + hstep,
    // j < nodes; a constant term as well when with_constant
    double log_tlo = 0, hstep = 0;
    int nodes = 0, with_constant = 0;
    // free-node fits: the largest rank <= kmax whose fit has positive
    // weights and a relative error below 0.9
    int kmax = 0;
    double* work = nullptr;   // device scratch, fit_work_doubles() doubles
    double* out = nullptr;    // device results, fit_out_doubles() doubles (layout below)
};
// Results.  Nonnegative fit: out[0..N) the coefficients of the nodes and of
// the constant (N = nodes + with_constant; zero where not used), out[N] the
// maximum relative error of the sum on a dense grid of [smin, smax] (20001
// log-spaced points), out[N + 1] for the operator the gate max |D~(s)/f(s) - 1|
// on the same grid (D~(s) = s (cexact + constant + sum)), out[N + 2] = 1 when
// the fit ran, out[N + 3 + j] the node values (j < nodes).  Free-node fit: out[0..K) nodes ascending, out[K..2K) weights,
// out[2 kFitMaxK] the maximum relative error (20001 points), out[2 kFitMaxK + 1]
// the rank K found (0: none).
struct FitJobs {
    int count = 0;
    FitJob job[kMaxFitJobs];
};
long fit_work_doubles(const FitJob& j);
long fit_out_doubles(const FitJob& j);
hipError_t fit_run(const FitJobs& jobs, hipStream_t s);

// Separable factors from exponential terms: for term q and mode l,
// F_l[i, q] = e_q(lam_l[i]) * (l == lmode[q] ? lam_l[i] : 1) with
// e_q(x) = exp(-t[q] x) (t[q] >= 0) or 1 (t[q] < 0), and D_l = cbrt(w[q]) F_l,
// D2_l = D_l^2 (all n x Q, column-major); lam holds the three spectra (3 n).
hipError_t expsum_factors(int n, int Q, const double* lam, const double* w, const double* t,
                          const int* lmode, double* const F[3], double* const D[3],
                          double* const D2[3], hipStream_t s);

}  // namespace fc
