// Exponential-sum fits of the setup phase on the device (see fit.h).
//
// Each job is one workgroup of kFitThreads threads.  The algorithms are the
// library's host fits, step for step, with the loops over samples and
// columns spread over the workgroup:
//  * nonnegative fits (operator f(s)/s, state map beta s^-alpha; Section
//    3.4): nodes on a geometric grid, weighted least squares with
//    nonnegative coefficients by the Lawson-Hanson active-set method
//    (Householder QR of the passive columns), ten rounds of Lawson
//    reweighting towards equal relative error, the best round kept;
//  * free-node fits (preconditioner 1/f, Section 3.5): Levenberg-Marquardt
//    on the variable-projection functional (Golub-Pereyra, Kaufman's
//    Jacobian) in log-nodes, three start grids, three Lawson rounds.
// Every decision (pivot, step acceptance, stop) is taken from values that
// all threads read after a barrier or from workgroup reductions, so the
// control flow is uniform; every loop has a fixed bound.
#include "fit.h"

#include <algorithm>
#include <cmath>

namespace fc {
namespace {

constexpr int T = kFitThreads;
constexpr int NW = T / 64;

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wmax(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
// Workgroup sum / maximum; every thread receives the same value.
__device__ double bsum(double v, double* red) {
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w];
    return s;
}
__device__ double bmax(double v, double* red) {
    v = wmax(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < NW; ++w) s = fmax(s, red[w]);
    return s;
}

// ---- targets ---------------------------------------------------------------
__device__ inline double f_symbol(const FitJob& J, double s) {
    return J.beta * pow(s, -J.alpha) + (J.gamma / J.beta) * pow(s, J.alpha);
}
__device__ inline double g_symbol(const FitJob& J, double s) {
    return J.beta * pow(s, -J.alpha - 1.0) + (J.gamma / J.beta) * pow(s, J.alpha - 1.0);
}
__device__ inline double target_h(const FitJob& J, double s) {
    if (J.target == FIT_OPERATOR) return g_symbol(J, s) - J.cexact;
    if (J.target == FIT_STATE) return J.beta * pow(s, -J.alpha);
    return 1.0 / f_symbol(J, s);
}
__device__ inline double target_ref(const FitJob& J, double s) {
    if (J.target == FIT_OPERATOR) return g_symbol(J, s);
    if (J.target == FIT_STATE) return J.beta * pow(s, -J.alpha);
    return 1.0 / f_symbol(J, s);
}

// ---- Householder least squares on a column-major M x K block --------------
// Factor Qm in place (reflectors below the diagonal with unit leading
// entry implied, R on and above it, scalars in tau).  False when a column
// vanishes or R is numerically singular (a diagonal entry below 1e-18 of the
// largest).  Starts with a barrier; uniform.
__device__ bool house_factor(double* Qm, int M, int K, double* tau, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double rmax = 0.0;
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        double* col = Qm + (long)j * M;
        double part = 0.0;
        for (int i = j + tid; i < M; i += T) part += col[i] * col[i];
        const double nrm = sqrt(bsum(part, red));
        if (nrm == 0.0) return false;
        const double cj = col[j];
        const double alpha = cj > 0 ? -nrm : nrm;
        const double v0 = cj - alpha;
        const double tj = -v0 / alpha;
        rmax = fmax(rmax, fabs(alpha));
        for (int i = j + 1 + tid; i < M; i += T) col[i] /= v0;
        __syncthreads();
        if (tid == 0) { tau[j] = tj; col[j] = alpha; }
        // the later columns, one wavefront each: c -= tau v (v^T c)
        for (int jj = j + 1 + wv; jj < K; jj += NW) {
            double* cc = Qm + (long)jj * M;
            double s = 0.0;
            #pragma unroll 4
            for (int i = j + 1 + lane; i < M; i += 64) s += col[i] * cc[i];
            s = (wsum(s) + cc[j]) * tj;
            if (lane == 0) cc[j] -= s;
            #pragma unroll 4
            for (int i = j + 1 + lane; i < M; i += 64) cc[i] -= s * col[i];
        }
        __syncthreads();
    }
    for (int j = 0; j < K; ++j)
        if (fabs(Qm[(long)j * M + j]) < 1e-18 * rmax) return false;
    return true;
}

// x = R^-1 (Q^T y)[0..K) for a block factored by house_factor; y (length M)
// is overwritten by Q^T y, ys (K, LDS) is scratch, x (K) is written.
__device__ void house_solve(const double* Qm, int M, int K, const double* tau, double* y,
                            double* x, double* ys, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        const double* col = Qm + (long)j * M;
        double part = (tid == 0) ? y[j] : 0.0;
        for (int i = j + 1 + tid; i < M; i += T) part += col[i] * y[i];
        const double s = bsum(part, red) * tau[j];
        if (tid == 0) y[j] -= s;
        for (int i = j + 1 + tid; i < M; i += T) y[i] -= s * col[i];
        __syncthreads();
    }
    for (int k = tid; k < K; k += T) ys[k] = y[k];
    __syncthreads();
    // back substitution by the first wavefront, column by column
    if (wv == 0) {
        for (int j = K - 1; j >= 0; --j) {
            const double xj = ys[j] / Qm[(long)j * M + j];
            if (lane == 0) x[j] = xj;
            for (int i = lane; i < j; i += 64) ys[i] -= Qm[(long)j * M + i] * xj;
        }
    }
    __syncthreads();
}

// ---- nonnegative fits --------------------------------------------------------
struct NonnegShared {
    int passive[kFitMaxNodes];
    int plist[kFitMaxNodes];
    double x[kFitMaxNodes], w[kFitMaxNodes], z[kFitMaxNodes], tau[kFitMaxNodes],
        ys[kFitMaxNodes];
};

// Householder reflectors j0 .. j1-1 of the block Qm (column-major, ld M)
// applied to the vector v (length M, LDS) by the first wavefront: v <- H v.
__device__ void reflect_lds(const double* Qm, int M, int j0, int j1, const double* tau, double* v) {
    const int lane = threadIdx.x & 63;
    for (int j = j0; j < j1; ++j) {
        const double* col = Qm + (long)j * M;
        double sp = 0.0;
        #pragma unroll 4
        for (int i = j + 1 + lane; i < M; i += 64) sp += col[i] * v[i];
        const double sj = (wsum(sp) + v[j]) * tau[j];
        if (lane == 0) v[j] -= sj;
        #pragma unroll 4
        for (int i = j + 1 + lane; i < M; i += 64) v[i] -= sj * col[i];
    }
}

// Lawson-Hanson: min ||A x - b|| over x >= 0 (A column-major M x N in global
// scratch; Qm, M x N, the Householder factors of the passive columns in the
// order they entered; r length M; col and qb, length M each, in LDS).  The
// factors are updated as columns enter (the new column is reduced by the
// existing reflectors and gets one of its own; Q^T b follows) and rebuilt
// when columns leave.  A column that is numerically dependent on the passive
// set ends the iteration: the host formulation would select it again from an
// unchanged state and fail again until its iteration limit.
__device__ void nnls(int M, int N, const double* A, const double* b, double* r, double* Qm,
                     double* col, double* qb, NonnegShared& sh, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __syncthreads();
    for (int j = tid; j < N; j += T) { sh.x[j] = 0.0; sh.passive[j] = 0; }
    double am = 0.0;
    for (int i = tid; i < M; i += T) { r[i] = b[i]; qb[i] = b[i]; }
    for (long e = tid; e < (long)M * N; e += T) am = fmax(am, fabs(A[e]));
    const double anorm = bmax(am, red);
    const double tol = 1e-13 * anorm * (double)(M > N ? M : N);
    auto grad = [&]() {   // w = A^T r
        __syncthreads();
        for (int j = wv; j < N; j += NW) {
            const double* a = A + (long)j * M;
            double s = 0.0;
            #pragma unroll 4
            for (int i = lane; i < M; i += 64) s += a[i] * r[i];
            s = wsum(s);
            if (lane == 0) sh.w[j] = s;
        }
        __syncthreads();
    };
    // rank test over the diagonal of R (uniform)
    auto rank_ok = [&](int K) {
        double rmax = 0.0;
        for (int j = 0; j < K; ++j) rmax = fmax(rmax, fabs(Qm[(long)j * M + j]));
        for (int j = 0; j < K; ++j)
            if (fabs(Qm[(long)j * M + j]) < 1e-18 * rmax) return false;
        return true;
    };
    int K = 0;
    grad();
    for (int outer = 0; outer < 3 * N; ++outer) {
        int jmax = -1;
        double best = tol;
        for (int j = 0; j < N; ++j)
            if (!sh.passive[j] && sh.w[j] > best) { best = sh.w[j]; jmax = j; }
        if (jmax < 0) break;
        // append column jmax: reduce it by the K reflectors, then its own
        for (int i = tid; i < M; i += T) col[i] = A[(long)jmax * M + i];
        __syncthreads();
        if (wv == 0) reflect_lds(Qm, M, 0, K, sh.tau, col);
        __syncthreads();
        double part = 0.0;
        for (int i = K + tid; i < M; i += T) part += col[i] * col[i];
        const double nrm = sqrt(bsum(part, red));
        bool ok = nrm != 0.0;
        if (ok) {
            const double ck = col[K];
            const double alpha = ck > 0 ? -nrm : nrm;
            const double v0 = ck - alpha;
            double* dst = Qm + (long)K * M;
            for (int i = tid; i < M; i += T)
                dst[i] = (i < K) ? col[i] : (i == K) ? alpha : col[i] / v0;
            if (tid == 0) sh.tau[K] = -v0 / alpha;
            __syncthreads();
            ok = rank_ok(K + 1);
        }
        __syncthreads();
        if (!ok) break;
        if (tid == 0) { sh.passive[jmax] = 1; sh.plist[K] = jmax; }
        ++K;
        // Q^T b for the new reflector
        if (wv == 0) reflect_lds(Qm, M, K - 1, K, sh.tau, qb);
        __syncthreads();
        bool stop = false;
        for (int inner = 0; inner < 3 * N; ++inner) {
            // z = R^-1 (Q^T b)[0..K), first wavefront, column by column
            for (int k = tid; k < K; k += T) sh.ys[k] = qb[k];
            __syncthreads();
            if (wv == 0)
                for (int j = K - 1; j >= 0; --j) {
                    const double zj = sh.ys[j] / Qm[(long)j * M + j];
                    if (lane == 0) sh.z[j] = zj;
                    for (int i = lane; i < j; i += 64) sh.ys[i] -= Qm[(long)j * M + i] * zj;
                }
            __syncthreads();
            bool allpos = true;
            for (int k = 0; k < K; ++k) allpos = allpos && sh.z[k] > 0.0;
            if (allpos) {
                for (int k = tid; k < K; k += T) sh.x[sh.plist[k]] = sh.z[k];
                __syncthreads();
                break;
            }
            double alpha = 1.0;
            for (int k = 0; k < K; ++k)
                if (sh.z[k] <= 0.0) {
                    const double xk = sh.x[sh.plist[k]];
                    alpha = fmin(alpha, xk / (xk - sh.z[k]));
                }
            __syncthreads();
            for (int k = tid; k < K; k += T) {
                const int j = sh.plist[k];
                double xk = sh.x[j];
                xk += alpha * (sh.z[k] - xk);
                if (xk <= 1e-300) { xk = 0.0; sh.passive[j] = 0; }
                sh.x[j] = xk;
            }
            __syncthreads();
            // the columns that left: keep the others in order and refactor
            int K2 = 0;
            for (int k = 0; k < K; ++k) {
                const int j = sh.plist[k];
                if (sh.passive[j]) { if (tid == 0) sh.plist[K2] = j; ++K2; }
            }
            __syncthreads();
            if (K2 == K) continue;   // nothing left the set: same factors
            K = K2;
            for (long e = tid; e < (long)M * K; e += T) {
                const int k = (int)(e / M), i = (int)(e % M);
                Qm[e] = A[(long)sh.plist[k] * M + i];
            }
            if (!house_factor(Qm, M, K, sh.tau, red)) {
                // a dependent column: the newest one leaves the passive set
                __syncthreads();
                if (tid == 0) { sh.passive[jmax] = 0; sh.w[jmax] = 0.0; }
                __syncthreads();
                stop = true;
                break;
            }
            for (int i = tid; i < M; i += T) qb[i] = b[i];
            __syncthreads();
            if (wv == 0) reflect_lds(Qm, M, 0, K, sh.tau, qb);
            __syncthreads();
        }
        if (stop) {
            // rebuild the passive list and factors without jmax for the next round
            int K2 = 0;
            for (int j = 0; j < N; ++j)
                if (sh.passive[j]) { if (tid == 0) sh.plist[K2] = j; ++K2; }
            __syncthreads();
            K = K2;
            for (long e = tid; e < (long)M * K; e += T) {
                const int k = (int)(e / M), i = (int)(e % M);
                Qm[e] = A[(long)sh.plist[k] * M + i];
            }
            const bool fok = house_factor(Qm, M, K, sh.tau, red);
            for (int i = tid; i < M; i += T) qb[i] = b[i];
            __syncthreads();
            if (!fok) break;
            if (wv == 0) reflect_lds(Qm, M, 0, K, sh.tau, qb);
            __syncthreads();
        }
        // r = b - A x (the terms with x_j = 0 subtract an exact zero)
        for (int i = tid; i < M; i += T) {
            double ri = b[i];
#pragma unroll 4
            for (int j = 0; j < N; ++j) ri -= A[(long)j * M + i] * sh.x[j];
            r[i] = ri;
        }
        grad();
    }
}

__device__ inline double nn_basis(const double* t, int N0, int j, double s) {
    return j < N0 ? exp(-t[j] * s) : 1.0;
}

__device__ void fit_nonneg(const FitJob& J, double* lds, NonnegShared& sh, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int M = kFitSamples, N0 = J.nodes, N = N0 + (J.with_constant ? 1 : 0);
    double* W = J.work;
    double* s = W;
    double* hv = s + M;
    double* rf = hv + M;
    double* wl = rf + M;
    double* b = wl + M;
    double* r = b + M;
    double* e = r + M;
    double* t = e + M;
    double* coef = t + kFitMaxNodes;
    double* best = coef + kFitMaxNodes;
    double* cs = best + kFitMaxNodes;
    double* A = cs + kFitMaxNodes;
    double* Qm = A + (long)M * N;
    double* out = J.out;
    if (tid == 0) {
        double x = J.log_tlo;
        for (int j = 0; j < N0; ++j) { t[j] = exp(x); x += J.hstep; }
    }
    const double la = log(J.smin), lb = log(fmax(J.smax, J.smin * (1 + 1e-9)));
    for (int i = tid; i < M; i += T) {
        const double si = exp(la + (lb - la) * (double)i / (M - 1));
        s[i] = si;
        hv[i] = target_h(J, si);
        rf[i] = target_ref(J, si);
        wl[i] = 1.0;
    }
    __syncthreads();
    double best_err = 1e300;
    bool have_best = false;
    for (int round = 0; round < 10; ++round) {
        // weighted design, columns scaled to unit length
        for (int j = wv; j < N; j += NW) {
            double* a = A + (long)j * M;
            double nrm = 0.0;
            for (int i = lane; i < M; i += 64) {
                const double v = wl[i] * nn_basis(t, N0, j, s[i]) / rf[i];
                a[i] = v;
                nrm += v * v;
            }
            nrm = sqrt(wsum(nrm));
            const double c = nrm > 0 ? nrm : 1.0;
            for (int i = lane; i < M; i += 64) a[i] /= c;
            if (lane == 0) cs[j] = c;
        }
        for (int i = tid; i < M; i += T) b[i] = wl[i] * hv[i] / rf[i];
        __syncthreads();
        nnls(M, N, A, b, r, Qm, lds, lds + M, sh, red);
        for (int j = tid; j < N; j += T) coef[j] = sh.x[j] / cs[j];
        __syncthreads();
        double em = 0.0;
        for (int i = tid; i < M; i += T) {
            double v = 0.0;
            for (int j = 0; j < N; ++j) v += coef[j] * nn_basis(t, N0, j, s[i]);
            const double ei = fabs(v - hv[i]) / rf[i];
            e[i] = ei;
            em = fmax(em, ei);
        }
        const double emax = bmax(em, red);
        if (emax < best_err) {
            best_err = emax;
            have_best = true;
            for (int j = tid; j < N; j += T) best[j] = coef[j];
        }
        if (!(emax > 0)) break;
        double wm = 0.0;
        for (int i = tid; i < M; i += T) {
            wl[i] *= sqrt(fmax(e[i] / emax, 1e-3));
            wm = fmax(wm, wl[i]);
        }
        wm = bmax(wm, red);
        for (int i = tid; i < M; i += T) wl[i] /= wm;
        __syncthreads();
    }
    const double* fin = have_best ? best : coef;
    __syncthreads();
    // the positive node terms and the constant
    for (int j = tid; j < N; j += T) out[j] = (j < N0) ? (fin[j] > 0 ? fin[j] : 0.0) : fin[j];
    const double c0 = J.with_constant ? fin[N - 1] : 0.0;
    const double c0tot = J.cexact + c0;
    const int G = 20000;
    double em = 0.0, gm = 0.0;
    for (int i = tid; i <= G; i += T) {
        const double si = exp(la + (lb - la) * (double)i / G);
        double v = c0, v2 = c0tot * si;
        for (int j = 0; j < N0; ++j)
            if (fin[j] > 0) {
                const double ex = exp(-t[j] * si);
                v += fin[j] * ex;
                v2 += si * fin[j] * ex;
            }
        em = fmax(em, fabs(v - target_h(J, si)) / target_ref(J, si));
        if (J.target == FIT_OPERATOR) gm = fmax(gm, fabs(v2 / f_symbol(J, si) - 1.0));
    }
    const double err = bmax(em, red);
    const double gate = bmax(gm, red);
    for (int j = tid; j < N0; j += T) out[N + 3 + j] = t[j];
    if (tid == 0) {
        out[N] = err;
        out[N + 1] = gate;
        out[N + 2] = isfinite(err) ? 1.0 : 0.0;
    }
}

// ---- free-node fits ----------------------------------------------------------
struct FreeShared {
    double x[kFitMaxK], c[kFitMaxK], xn[kFitMaxK], cn[kFitMaxK], cd[kFitMaxK];
    double bx[kFitMaxK], bc[kFitMaxK], tauA[kFitMaxK], tauB[kFitMaxK], ys[kFitMaxK];
    double JtJ[kFitMaxK * kFitMaxK], Jtr[kFitMaxK], L[kFitMaxK * kFitMaxK];
    double zt[kFitMaxK], dxt[kFitMaxK];
    double step;
    int ok;
};

struct FreeCtx {
    const FitJob* J;
    int M, K;
    double la, lb;
    double *s, *h, *rf, *wl, *y;   // global, length M
};

// residual of the variable-projection functional at log-nodes xv: the
// linear weights c by least squares (factor kept in Qm / tau), r = W (E c - h)
__device__ bool vp_eval(const FreeCtx& F, const double* xv, double* Qm, double* tau, double* c,
                        double* r, FreeShared& sh, double* red) {
    const int tid = threadIdx.x;
    const int M = F.M, K = F.K;
    for (long e = tid; e < (long)M * K; e += T) {
        const int k = (int)(e / M), i = (int)(e % M);
        const double w = F.wl[i] / F.rf[i];
        Qm[e] = w * exp(-exp(xv[k]) * F.s[i]);
    }
    for (int i = tid; i < M; i += T) F.y[i] = (F.wl[i] / F.rf[i]) * F.h[i];
    if (!house_factor(Qm, M, K, tau, red)) return false;
    house_solve(Qm, M, K, tau, F.y, c, sh.ys, red);
    for (int i = tid; i < M; i += T) {
        const double w = F.wl[i] / F.rf[i];
        double v = 0.0;
        for (int k = 0; k < K; ++k) v += c[k] * exp(-exp(xv[k]) * F.s[i]);
        r[i] = w * (v - F.h[i]);
    }
    __syncthreads();
    return true;
}

__device__ double norm_of(const double* r, int M, double* red) {
    double p = 0.0;
    for (int i = threadIdx.x; i < M; i += T) p += r[i] * r[i];
    return sqrt(bsum(p, red));
}

// Levenberg-Marquardt on the variable-projection functional (x, c in LDS,
// updated in place); QA, QB the two M x K factor buffers, rA, rB residuals.
__device__ bool vp_lm(const FreeCtx& F, int maxit, double* QA, double* QB, double* rA, double* rB,
                      FreeShared& sh, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int M = F.M, K = F.K;
    double* Qa = QA; double* Qb = QB;
    double* ta = sh.tauA; double* tb = sh.tauB;
    double* ra = rA; double* rb = rB;
    if (!vp_eval(F, sh.x, Qa, ta, sh.c, ra, sh, red)) return false;
    double f = norm_of(ra, M, red);
    double mu = 1e-3;
    const int npairs = K * (K + 1) / 2;
    for (int it = 0; it < maxit; ++it) {
        // Kaufman's Jacobian: column k = -P_perp (t_k s W exp(-t_k s) c_k), one wavefront each
        for (int k = wv; k < K; k += NW) {
            double* col = Qb + (long)k * M;
            const double tk = exp(sh.x[k]);
            for (int i = lane; i < M; i += 64) {
                const double w = F.wl[i] / F.rf[i];
                col[i] = -tk * F.s[i] * w * exp(-tk * F.s[i]) * sh.c[k];
            }
            for (int j = 0; j < K; ++j) {           // Q^T
                const double* q = Qa + (long)j * M;
                double sp = 0.0;
                for (int i = j + 1 + lane; i < M; i += 64) sp += q[i] * col[i];
                const double sj = (wsum(sp) + col[j]) * ta[j];
                if (lane == 0) col[j] -= sj;
                for (int i = j + 1 + lane; i < M; i += 64) col[i] -= sj * q[i];
            }
            for (int i = lane; i < K; i += 64) col[i] = 0.0;
            for (int j = K - 1; j >= 0; --j) {      // Q
                const double* q = Qa + (long)j * M;
                double sp = 0.0;
                for (int i = j + 1 + lane; i < M; i += 64) sp += q[i] * col[i];
                const double sj = (wsum(sp) + col[j]) * ta[j];
                if (lane == 0) col[j] -= sj;
                for (int i = j + 1 + lane; i < M; i += 64) col[i] -= sj * q[i];
            }
        }
        __syncthreads();
        for (int item = wv; item < npairs + K; item += NW) {
            double sp = 0.0;
            if (item < npairs) {
                int a = 0;
                while ((a + 1) * (a + 2) / 2 <= item) ++a;
                const int bb = item - a * (a + 1) / 2;
                const double* ca = Qb + (long)a * M;
                const double* cb = Qb + (long)bb * M;
                for (int i = lane; i < M; i += 64) sp += ca[i] * cb[i];
                sp = wsum(sp);
                if (lane == 0) { sh.JtJ[a * K + bb] = sp; sh.JtJ[bb * K + a] = sp; }
            } else {
                const int a = item - npairs;
                const double* ca = Qb + (long)a * M;
                for (int i = lane; i < M; i += 64) sp += ca[i] * ra[i];
                sp = wsum(sp);
                if (lane == 0) sh.Jtr[a] = sp;
            }
        }
        __syncthreads();
        bool improved = false;
        for (int tries = 0; tries < 12 && !improved; ++tries) {
            __syncthreads();
            if (tid == 0) {
                // (JtJ + mu diag(JtJ)) dx = -Jtr by Cholesky
                double* L = sh.L;
                for (int a = 0; a < K * K; ++a) L[a] = sh.JtJ[a];
                for (int a = 0; a < K; ++a) { L[a * K + a] *= (1.0 + mu); L[a * K + a] += 1e-300; }
                int ok = 1;
                for (int j = 0; j < K && ok; ++j) {
                    double d = L[j * K + j];
                    for (int k = 0; k < j; ++k) d -= L[j * K + k] * L[j * K + k];
                    if (!(d > 0)) { ok = 0; break; }
                    d = sqrt(d);
                    L[j * K + j] = d;
                    for (int i = j + 1; i < K; ++i) {
                        double v = L[i * K + j];
                        for (int k = 0; k < j; ++k) v -= L[i * K + k] * L[j * K + k];
                        L[i * K + j] = v / d;
                    }
                }
                if (ok) {
                    double* z = sh.zt;
                    double* dx = sh.dxt;
                    for (int i = 0; i < K; ++i) {
                        double v = -sh.Jtr[i];
                        for (int k = 0; k < i; ++k) v -= L[i * K + k] * z[k];
                        z[i] = v / L[i * K + i];
                    }
                    for (int i = K - 1; i >= 0; --i) {
                        double v = z[i];
                        for (int k = i + 1; k < K; ++k) v -= L[k * K + i] * dx[k];
                        dx[i] = v / L[i * K + i];
                    }
                    double step = 0.0;
                    for (int k = 0; k < K; ++k) {
                        const double d = fmax(-1.0, fmin(1.0, dx[k]));
                        sh.xn[k] = sh.x[k] + d;
                        step = fmax(step, fabs(d));
                    }
                    sh.step = step;
                }
                sh.ok = ok;
            }
            __syncthreads();
            if (!sh.ok) { mu *= 10; continue; }
            const double step = sh.step;
            if (vp_eval(F, sh.xn, Qb, tb, sh.cn, rb, sh, red)) {
                const double fn = norm_of(rb, M, red);
                if (fn < f) {
                    const double rel = (f - fn) / f;
                    __syncthreads();
                    for (int k = tid; k < K; k += T) { sh.x[k] = sh.xn[k]; sh.c[k] = sh.cn[k]; }
                    __syncthreads();
                    double* q = Qa; Qa = Qb; Qb = q;
                    double* tt = ta; ta = tb; tb = tt;
                    double* rr = ra; ra = rb; rb = rr;
                    f = fn;
                    mu = fmax(mu / 3.0, 1e-12);
                    improved = true;
                    if (rel < 1e-12 && step < 1e-9) return true;
                    break;
                }
            }
            mu *= 4.0;
        }
        if (!improved) return true;
    }
    return true;
}

// max relative error of sum_k c_k exp(-exp(xv_k) s) on grid + 1 log-spaced points
__device__ double grid_err(const FreeCtx& F, const double* xv, const double* c, int grid,
                           bool nodes_are_logs, double* red) {
    double em = 0.0;
    for (int i = threadIdx.x; i <= grid; i += T) {
        const double si = exp(F.la + (F.lb - F.la) * (double)i / grid);
        double v = 0.0;
        for (int k = 0; k < F.K; ++k) v += c[k] * exp(-(nodes_are_logs ? exp(xv[k]) : xv[k]) * si);
        em = fmax(em, fabs(v - target_h(*F.J, si)) / target_ref(*F.J, si));
    }
    return bmax(em, red);
}

// One free-node fit of rank K; on success sh.bx holds the nodes (ascending,
// as nodes, not logs), sh.bc the weights, and the error is returned.
__device__ bool fit_free_rank(const FitJob& J, int K, double* lds, FreeShared& sh, double* red,
                              double& err_out) {
    const int tid = threadIdx.x;
    FreeCtx F;
    F.J = &J;
    F.K = K;
    F.M = 30 * K > 300 ? 30 * K : 300;
    const int M = F.M;
    double smax = J.smax;
    if (smax < J.smin * (1.0 + 1e-12)) smax = J.smin * (1.0 + 1e-9);
    F.la = log(J.smin);
    F.lb = log(smax);
    double* W = J.work;
    F.s = W; F.h = W + M; F.rf = W + 2 * M; F.wl = W + 3 * M; F.y = W + 4 * M;
    double* rA = W + 5 * M;
    double* rB = W + 6 * M;
    double* QA = lds;
    double* QB = lds + (long)M * K;
    for (int i = tid; i < M; i += T) {
        const double si = exp(F.la + (F.lb - F.la) * (double)i / (M - 1));
        F.s[i] = si;
        F.h[i] = target_h(J, si);
        F.rf[i] = target_ref(J, si);
        F.wl[i] = 1.0;
    }
    __syncthreads();
    bool started = false;
    const double fasts[3] = {30.0, 3.0, 1.0};
    for (int fi = 0; fi < 3 && !started; ++fi) {
        __syncthreads();
        if (tid == 0) {
            const double x0 = log(0.5 / smax) - 2.0, x1 = log(fasts[fi] / J.smin);
            for (int k = 0; k < K; ++k)
                sh.x[k] = K == 1 ? 0.5 * (x0 + x1) : x0 + (x1 - x0) * (double)k / (K - 1);
        }
        __syncthreads();
        started = vp_lm(F, 150, QA, QB, rA, rB, sh, red);
    }
    if (!started) return false;
    __syncthreads();
    for (int k = tid; k < K; k += T) { sh.bx[k] = sh.x[k]; sh.bc[k] = sh.c[k]; }
    __syncthreads();
    double best = grid_err(F, sh.x, sh.c, 4000, true, red);
    for (int round = 0; round < 3; ++round) {
        // residual of the current nodes under the current weights
        if (!vp_eval(F, sh.x, QB, sh.tauB, sh.cd, rB, sh, red)) break;
        double rm = 0.0;
        for (int i = tid; i < M; i += T) rm = fmax(rm, fabs(rB[i]) / F.wl[i]);
        const double rmax = bmax(rm, red);
        if (!(rmax > 0)) break;
        double wm = 0.0;
        for (int i = tid; i < M; i += T) {
            F.wl[i] *= sqrt(fmax(fabs(rB[i]) / F.wl[i] / rmax, 1e-3));
            wm = fmax(wm, F.wl[i]);
        }
        wm = bmax(wm, red);
        for (int i = tid; i < M; i += T) F.wl[i] /= wm;
        __syncthreads();
        if (!vp_lm(F, 80, QA, QB, rA, rB, sh, red)) break;
        const double e = grid_err(F, sh.x, sh.c, 4000, true, red);
        if (e < best) {
            best = e;
            __syncthreads();
            for (int k = tid; k < K; k += T) { sh.bx[k] = sh.x[k]; sh.bc[k] = sh.c[k]; }
            __syncthreads();
        }
    }
    __syncthreads();
    if (tid == 0) {
        // sort by node, then nodes from their logs
        for (int a = 1; a < K; ++a) {
            const double xa = sh.bx[a], ca = sh.bc[a];
            int b = a - 1;
            while (b >= 0 && sh.bx[b] > xa) { sh.bx[b + 1] = sh.bx[b]; sh.bc[b + 1] = sh.bc[b]; --b; }
            sh.bx[b + 1] = xa;
            sh.bc[b + 1] = ca;
        }
        for (int k = 0; k < K; ++k) sh.bx[k] = exp(sh.bx[k]);
    }
    __syncthreads();
    err_out = grid_err(F, sh.bx, sh.bc, 20000, false, red);
    return isfinite(err_out);
}

__device__ void fit_free(const FitJob& J, double* lds, FreeShared& sh, double* red) {
    const int tid = threadIdx.x;
    double* out = J.out;
    int found = 0;
    double err = 0.0;
    for (int K = J.kmax; K >= 1 && !found; --K) {
        double e = 0.0;
        if (!fit_free_rank(J, K, lds, sh, red, e)) continue;
        bool pos = true;
        for (int k = 0; k < K; ++k) pos = pos && sh.bc[k] > 0;
        if (pos && e < 0.9) {
            found = K;
            err = e;
        }
    }
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < found; ++k) { out[k] = sh.bx[k]; out[found + k] = sh.bc[k]; }
        out[2 * kFitMaxK] = err;
        out[2 * kFitMaxK + 1] = (double)found;
    }
}

// One launch per kind (nonnegative, free-node): each kernel keeps only its
// own path's registers.  Blocks whose job is of the other kind return.
__global__ __launch_bounds__(kFitThreads) void fit_nonneg_kernel(FitJobs jobs) {
    extern __shared__ double fit_lds[];
    __shared__ NonnegShared nsh;
    __shared__ double red[NW];
    const FitJob& J = jobs.job[blockIdx.x];
    if (J.target == FIT_PRECOND) return;
    fit_nonneg(J, fit_lds, nsh, red);
}

__global__ __launch_bounds__(kFitThreads) void fit_free_kernel(FitJobs jobs) {
    extern __shared__ double fit_lds[];
    __shared__ FreeShared fsh;
    __shared__ double red[NW];
    const FitJob& J = jobs.job[blockIdx.x];
    if (J.target != FIT_PRECOND) return;
    fit_free(J, fit_lds, fsh, red);
}

int free_rows(int K) { return 30 * K > 300 ? 30 * K : 300; }

struct FactorPtrs {
    double* p[3];
};

__global__ void expsum_factors_kernel(int n, int Q, const double* lam, const double* w,
                                      const double* t, const int* lm, FactorPtrs F, FactorPtrs D,
                                      FactorPtrs D2) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (idx >= (long)n * Q) return;
    const int i = (int)(idx % n), q = (int)(idx / n);
    const double x = lam[(long)l * n + i];
    double v = t[q] >= 0 ? exp(-t[q] * x) : 1.0;
    if (lm[q] == l) v *= x;
    const double d = cbrt(w[q]) * v;
    F.p[l][idx] = v;
    D.p[l][idx] = d;
    D2.p[l][idx] = d * d;
}

}  // namespace

long fit_work_doubles(const FitJob& j) {
    if (j.target == FIT_PRECOND) return 7L * free_rows(j.kmax);
    const long N = j.nodes + (j.with_constant ? 1 : 0);
    return 7L * kFitSamples + 4L * kFitMaxNodes + 2L * kFitSamples * N;
}

long fit_out_doubles(const FitJob& j) {
    if (j.target == FIT_PRECOND) return 2L * kFitMaxK + 2;
    return 2L * j.nodes + (j.with_constant ? 1 : 0) + 3;
}

hipError_t fit_run(const FitJobs& jobs, hipStream_t s) {
    if (jobs.count <= 0) return hipSuccess;
    if (jobs.count > kMaxFitJobs) return hipErrorInvalidValue;
    size_t lds_free = 0;
    bool any_nonneg = false, any_free = false;
    for (int k = 0; k < jobs.count; ++k) {
        const FitJob& j = jobs.job[k];
        if (j.target == FIT_PRECOND) {
            if (j.kmax < 1 || j.kmax > kFitMaxK) return hipErrorInvalidValue;
            lds_free = std::max(lds_free, sizeof(double) * 2 * (size_t)free_rows(j.kmax) * j.kmax);
            any_free = true;
        } else {
            if (j.nodes < 1 || j.nodes + (j.with_constant ? 1 : 0) > kFitMaxNodes)
                return hipErrorInvalidValue;
            any_nonneg = true;
        }
        if (!j.work || !j.out) return hipErrorInvalidValue;
    }
    static hipError_t attr = hipFuncSetAttribute((const void*)fit_free_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)(sizeof(double) * 2 * 480 * kFitMaxK));
    if (attr != hipSuccess) return attr;
    if (any_nonneg)
        hipLaunchKernelGGL(fit_nonneg_kernel, dim3(jobs.count), dim3(kFitThreads),
                           sizeof(double) * 2 * (size_t)kFitSamples, s, jobs);
    if (any_free)
        hipLaunchKernelGGL(fit_free_kernel, dim3(jobs.count), dim3(kFitThreads), lds_free, s, jobs);
    return hipGetLastError();
}

hipError_t expsum_factors(int n, int Q, const double* lam, const double* w, const double* t,
                          const int* lmode, double* const F[3], double* const D[3],
                          double* const D2[3], hipStream_t s) {
    if (n <= 0 || Q <= 0) return hipSuccess;
    FactorPtrs f, d, d2;
    for (int l = 0; l < 3; ++l) { f.p[l] = F[l]; d.p[l] = D[l]; d2.p[l] = D2[l]; }
    const long total = (long)n * Q;
    hipLaunchKernelGGL(expsum_factors_kernel, dim3((unsigned)((total + 255) / 256), 3), dim3(256),
                       0, s, n, Q, lam, w, t, lmode, f, d, d2);
    return hipGetLastError();
}

}  // namespace fc
