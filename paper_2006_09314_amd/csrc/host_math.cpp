// Host-side numerics of the setup phase: the 1D finite-difference
// Sturm-Liouville matrices and their eigenpairs (paper Sections 3.2-3.3), and
// the exponential sums that give the operator and the preconditioner a low
// Kronecker rank in the eigenbasis (Sections 3.4-3.5).
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>

namespace fc {

// ---------------------------------------------------------------------------
// Tridiagonal matrix of -d/dx a(x) d/dx on n interior nodes, h = 1/(n+1),
// coefficient at the midpoints a_{i+1/2}, i = 0..n (conservative FD scheme).
void fd_tridiag(int n, const double* a_mid, double* diag, double* off) {
    const double h2inv = double(n + 1) * double(n + 1);
    for (int i = 0; i < n; ++i) diag[i] = (a_mid[i] + a_mid[i + 1]) * h2inv;
    for (int i = 0; i + 1 < n; ++i) off[i] = -a_mid[i + 1] * h2inv;
}

// Symmetric tridiagonal eigensolver: implicit QL iteration with a Wilkinson
// shift, accumulating the plane rotations into Z (column-major n x n,
// initialised to the identity).  On exit d holds the eigenvalues in ascending
// order and Z the matching orthonormal eigenvectors (columns), each with its
// entry of largest magnitude positive.
bool tridiag_eigen(int n, std::vector<double>& d, std::vector<double> e, double* Z) {
    const double eps = std::numeric_limits<double>::epsilon();
    e.resize(n, 0.0);
    if (Z) {
        std::memset(Z, 0, sizeof(double) * size_t(n) * n);
        for (int i = 0; i < n; ++i) Z[size_t(i) * n + i] = 1.0;
    }
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) return false;
            // Wilkinson-type shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                double f = s * e[i];
                double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                if (Z) {
                    double* zi = Z + size_t(i) * n;
                    double* zj = Z + size_t(i + 1) * n;
                    for (int k = 0; k < n; ++k) {
                        const double t = zj[k];
                        zj[k] = s * zi[k] + c * t;
                        zi[k] = c * zi[k] - s * t;
                    }
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // sort ascending (selection sort on indices, then permute)
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    std::vector<double> ds(n);
    for (int i = 0; i < n; ++i) ds[i] = d[idx[i]];
    if (Z) {
        std::vector<double> Zs(size_t(n) * n);
        for (int i = 0; i < n; ++i) {
            const double* src = Z + size_t(idx[i]) * n;
            double* dst = Zs.data() + size_t(i) * n;
            int kmax = 0;
            for (int k = 1; k < n; ++k)
                if (std::fabs(src[k]) > std::fabs(src[kmax])) kmax = k;
            const double sg = src[kmax] < 0 ? -1.0 : 1.0;
            for (int k = 0; k < n; ++k) dst[k] = sg * src[k];
        }
        std::memcpy(Z, Zs.data(), sizeof(double) * size_t(n) * n);
    }
    d = ds;
    return true;
}

bool fd_eigen(int n, const double* a_mid, double* lam, double* V) {
    std::vector<double> d(n), e(std::max(n - 1, 1));
    fd_tridiag(n, a_mid, d.data(), e.data());
    if (!tridiag_eigen(n, d, e, V)) return false;
    std::copy(d.begin(), d.end(), lam);
    return true;
}

// ---------------------------------------------------------------------------
// Exponential sums  h(s) ~ sum_k c_k exp(-t_k s)  on [s_min, s_max], measured
// in the relative sense against ref(s).
//
// For the completely monotone targets of this method the Laplace-transform
// representation (Section 3.4) guarantees positive weights; its sinc
// (trapezoidal) discretisation needs many terms, so the nodes are instead
// optimised directly: variable projection (the weights solve a linear least
// squares problem for given nodes), Levenberg-Marquardt on log t_k with the
// Kaufman Jacobian, followed by Lawson reweighting towards the uniform
// (minimax) relative error.

namespace {

// Householder QR least squares: solves min ||A x - b|| for A (M x K,
// column-major, overwritten), returns x (K) and the Householder data for
// later projections.  Returns false if A is numerically rank deficient.
struct HouseQR {
    int M = 0, K = 0;
    std::vector<double> A;      // reflectors below the diagonal, R above
    std::vector<double> tau;
    bool factor(int m, int k, const std::vector<double>& a) {
        M = m; K = k; A = a; tau.assign(k, 0.0);
        double rmax = 0.0;
        for (int j = 0; j < K; ++j) {
            double* col = &A[size_t(j) * M];
            double nrm = 0.0;
            for (int i = j; i < M; ++i) nrm += col[i] * col[i];
            nrm = std::sqrt(nrm);
            if (nrm == 0.0) return false;
            const double alpha = col[j] > 0 ? -nrm : nrm;
            const double v0 = col[j] - alpha;
            for (int i = j + 1; i < M; ++i) col[i] /= v0;
            tau[j] = (alpha - col[j]) / alpha;   // = -v0/alpha
            tau[j] = -v0 / alpha;
            col[j] = alpha;
            for (int jj = j + 1; jj < K; ++jj) {
                double* cj = &A[size_t(jj) * M];
                double s = cj[j];
                for (int i = j + 1; i < M; ++i) s += col[i] * cj[i];
                s *= tau[j];
                cj[j] -= s;
                for (int i = j + 1; i < M; ++i) cj[i] -= s * col[i];
            }
            rmax = std::max(rmax, std::fabs(alpha));
        }
        for (int j = 0; j < K; ++j)
            if (std::fabs(A[size_t(j) * M + j]) < 1e-18 * rmax) return false;
        return true;
    }
    // y <- Q^T y
    void qt(std::vector<double>& y) const {
        for (int j = 0; j < K; ++j) {
            const double* col = &A[size_t(j) * M];
            double s = y[j];
            for (int i = j + 1; i < M; ++i) s += col[i] * y[i];
            s *= tau[j];
            y[j] -= s;
            for (int i = j + 1; i < M; ++i) y[i] -= s * col[i];
        }
    }
    // y <- Q y
    void q(std::vector<double>& y) const {
        for (int j = K - 1; j >= 0; --j) {
            const double* col = &A[size_t(j) * M];
            double s = y[j];
            for (int i = j + 1; i < M; ++i) s += col[i] * y[i];
            s *= tau[j];
            y[j] -= s;
            for (int i = j + 1; i < M; ++i) y[i] -= s * col[i];
        }
    }
    // solve R x = (Q^T y)[0:K]
    void solve(std::vector<double> y, std::vector<double>& x) const {
        qt(y);
        x.assign(K, 0.0);
        for (int j = K - 1; j >= 0; --j) {
            double s = y[j];
            for (int jj = j + 1; jj < K; ++jj) s -= A[size_t(jj) * M + j] * x[jj];
            x[j] = s / A[size_t(j) * M + j];
        }
    }
    // orthogonal complement projection: y <- (I - Q_K Q_K^T) y
    void perp(std::vector<double>& y) const {
        qt(y);
        for (int j = 0; j < K; ++j) y[j] = 0.0;
        q(y);
    }
};

struct FitProblem {
    std::vector<double> s, h, ref, wl;   // samples, target part, reference, Lawson weights
};

// residual for nodes x = log t; returns false on a rank-deficient design
bool vp_eval(const FitProblem& P, const std::vector<double>& x, std::vector<double>& c,
             std::vector<double>& r, HouseQR* qr_out) {
    const int M = int(P.s.size()), K = int(x.size());
    std::vector<double> E(size_t(M) * K);
    std::vector<double> y(M);
    for (int i = 0; i < M; ++i) {
        const double w = P.wl[i] / P.ref[i];
        y[i] = w * P.h[i];
        for (int k = 0; k < K; ++k) E[size_t(k) * M + i] = w * std::exp(-std::exp(x[k]) * P.s[i]);
    }
    HouseQR qr;
    if (!qr.factor(M, K, E)) return false;
    qr.solve(y, c);
    r.assign(M, 0.0);
    for (int i = 0; i < M; ++i) {
        const double w = P.wl[i] / P.ref[i];
        double v = 0.0;
        for (int k = 0; k < K; ++k) v += c[k] * std::exp(-std::exp(x[k]) * P.s[i]);
        r[i] = w * (v - P.h[i]);
    }
    if (qr_out) *qr_out = std::move(qr);
    return true;
}

double nrm2(const std::vector<double>& v) {
    double s = 0.0;
    for (double a : v) s += a * a;
    return std::sqrt(s);
}

// Levenberg-Marquardt on the variable-projection functional.
bool vp_lm(const FitProblem& P, std::vector<double>& x, std::vector<double>& c, int maxit) {
    const int M = int(P.s.size()), K = int(x.size());
    std::vector<double> r, cn, rn;
    HouseQR qr;
    if (!vp_eval(P, x, c, r, &qr)) return false;
    double f = nrm2(r);
    double mu = 1e-3;
    for (int it = 0; it < maxit; ++it) {
        // Kaufman Jacobian J_k = -P_perp (t_k s E_k c_k)
        std::vector<double> J(size_t(M) * K);
        for (int k = 0; k < K; ++k) {
            std::vector<double> v(M);
            const double t = std::exp(x[k]);
            for (int i = 0; i < M; ++i) {
                const double w = P.wl[i] / P.ref[i];
                v[i] = -t * P.s[i] * w * std::exp(-t * P.s[i]) * c[k];
            }
            qr.perp(v);
            std::copy(v.begin(), v.end(), J.begin() + size_t(k) * M);
        }
        std::vector<double> JtJ(size_t(K) * K), Jtr(K);
        for (int a = 0; a < K; ++a) {
            for (int b = 0; b <= a; ++b) {
                double s = 0.0;
                for (int i = 0; i < M; ++i) s += J[size_t(a) * M + i] * J[size_t(b) * M + i];
                JtJ[size_t(a) * K + b] = JtJ[size_t(b) * K + a] = s;
            }
            double s = 0.0;
            for (int i = 0; i < M; ++i) s += J[size_t(a) * M + i] * r[i];
            Jtr[a] = s;
        }
        bool improved = false;
        for (int tries = 0; tries < 12 && !improved; ++tries) {
            // (JtJ + mu diag) dx = -Jtr, Cholesky
            std::vector<double> L(JtJ);
            for (int a = 0; a < K; ++a) L[size_t(a) * K + a] *= (1.0 + mu);
            for (int a = 0; a < K; ++a) L[size_t(a) * K + a] += 1e-300;
            bool ok = true;
            for (int j = 0; j < K && ok; ++j) {
                double s = L[size_t(j) * K + j];
                for (int k = 0; k < j; ++k) s -= L[size_t(j) * K + k] * L[size_t(j) * K + k];
                if (!(s > 0)) { ok = false; break; }
                s = std::sqrt(s);
                L[size_t(j) * K + j] = s;
                for (int i = j + 1; i < K; ++i) {
                    double v = L[size_t(i) * K + j];
                    for (int k = 0; k < j; ++k) v -= L[size_t(i) * K + k] * L[size_t(j) * K + k];
                    L[size_t(i) * K + j] = v / s;
                }
            }
            if (!ok) { mu *= 10; continue; }
            std::vector<double> z(K), dx(K);
            for (int i = 0; i < K; ++i) {
                double v = -Jtr[i];
                for (int k = 0; k < i; ++k) v -= L[size_t(i) * K + k] * z[k];
                z[i] = v / L[size_t(i) * K + i];
            }
            for (int i = K - 1; i >= 0; --i) {
                double v = z[i];
                for (int k = i + 1; k < K; ++k) v -= L[size_t(k) * K + i] * dx[k];
                dx[i] = v / L[size_t(i) * K + i];
            }
            std::vector<double> xn(x);
            double step = 0.0;
            for (int k = 0; k < K; ++k) {
                double d = std::max(-1.0, std::min(1.0, dx[k]));
                xn[k] += d;
                step = std::max(step, std::fabs(d));
            }
            HouseQR qrn;
            if (vp_eval(P, xn, cn, rn, &qrn)) {
                const double fn = nrm2(rn);
                if (fn < f) {
                    const double rel = (f - fn) / f;
                    x = xn; c = cn; r = rn; qr = std::move(qrn); f = fn;
                    mu = std::max(mu / 3.0, 1e-12);
                    improved = true;
                    if (rel < 1e-12 && step < 1e-9) return true;
                    break;
                }
            }
            mu *= 4.0;
        }
        if (!improved) return true;   // converged (no further decrease)
    }
    return true;
}

}  // namespace

double expsum_max_rel_err(const std::function<double(double)>& h,
                          const std::function<double(double)>& ref, double s_min, double s_max,
                          const double* t, const double* c, int K, int grid) {
    double emax = 0.0;
    const double la = std::log(s_min), lb = std::log(s_max);
    for (int i = 0; i <= grid; ++i) {
        const double s = std::exp(la + (lb - la) * double(i) / grid);
        double v = 0.0;
        for (int k = 0; k < K; ++k) v += c[k] * std::exp(-t[k] * s);
        emax = std::max(emax, std::fabs(v - h(s)) / ref(s));
    }
    return emax;
}

bool fit_expsum(const std::function<double(double)>& h, const std::function<double(double)>& ref,
                double s_min, double s_max, int K, std::vector<double>& t, std::vector<double>& c,
                double& max_rel_err) {
    if (!(s_min > 0) || !(s_max >= s_min) || K < 1) return false;
    if (s_max < s_min * (1.0 + 1e-12)) s_max = s_min * (1.0 + 1e-9);
    FitProblem P;
    const int M = std::max(300, 30 * K);
    const double la = std::log(s_min), lb = std::log(s_max);
    for (int i = 0; i < M; ++i) {
        const double s = std::exp(la + (lb - la) * double(i) / (M - 1));
        P.s.push_back(s);
        P.h.push_back(h(s));
        P.ref.push_back(ref(s));
        P.wl.push_back(1.0);
    }
    std::vector<double> x(K);
    // initial nodes: geometric between the scales of the interval ends.  The
    // fastest node starts at 30/s_min; on wide intervals its column can fall
    // below the rank test of the weighted design (it is ~exp(-30) at s_min
    // against columns of size ~s_max), and then a slower start is taken.
    std::vector<double> cc;
    bool started = false;
    for (double fast : {30.0, 3.0, 1.0}) {
        const double x0 = std::log(0.5 / s_max) - 2.0, x1 = std::log(fast / s_min);
        for (int k = 0; k < K; ++k)
            x[k] = K == 1 ? 0.5 * (x0 + x1) : x0 + (x1 - x0) * double(k) / (K - 1);
        if (vp_lm(P, x, cc, 150)) { started = true; break; }
    }
    if (!started) return false;
    std::vector<double> bx = x, bc = cc;
    std::vector<double> tt(K);
    for (int k = 0; k < K; ++k) tt[k] = std::exp(x[k]);
    double best = expsum_max_rel_err(h, ref, s_min, s_max, tt.data(), cc.data(), K, 4000);
    // Lawson reweighting towards equal-ripple relative error
    for (int round = 0; round < 3; ++round) {
        std::vector<double> r, cdummy;
        if (!vp_eval(P, x, cdummy, r, nullptr)) break;
        double rmax = 0.0;
        for (int i = 0; i < M; ++i) rmax = std::max(rmax, std::fabs(r[i]) / P.wl[i]);
        if (!(rmax > 0)) break;
        for (int i = 0; i < M; ++i) {
            P.wl[i] *= std::sqrt(std::max(std::fabs(r[i]) / P.wl[i] / rmax, 1e-3));
        }
        double wmax = *std::max_element(P.wl.begin(), P.wl.end());
        for (double& w : P.wl) w /= wmax;
        if (!vp_lm(P, x, cc, 80)) break;
        for (int k = 0; k < K; ++k) tt[k] = std::exp(x[k]);
        const double e = expsum_max_rel_err(h, ref, s_min, s_max, tt.data(), cc.data(), K, 4000);
        if (e < best) { best = e; bx = x; bc = cc; }
    }
    // sort by node
    std::vector<int> idx(K);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return bx[a] < bx[b]; });
    t.resize(K); c.resize(K);
    for (int k = 0; k < K; ++k) { t[k] = std::exp(bx[idx[k]]); c[k] = bc[idx[k]]; }
    max_rel_err = expsum_max_rel_err(h, ref, s_min, s_max, t.data(), c.data(), K, 20000);
    return std::isfinite(max_rel_err);
}

// ---------------------------------------------------------------------------
// Non-negative least squares (Lawson-Hanson active set): min ||A x - b||,
// x >= 0, A column-major M x N.
static bool nnls(int M, int N, const std::vector<double>& A, const std::vector<double>& b,
                 std::vector<double>& x) {
    x.assign(N, 0.0);
    std::vector<char> passive(N, 0);
    std::vector<double> r(b), w(N);
    double anorm = 0.0;
    for (double v : A) anorm = std::max(anorm, std::fabs(v));
    const double tol = 1e-13 * anorm * std::max(M, N);
    auto grad = [&]() {
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int i = 0; i < M; ++i) s += A[size_t(j) * M + i] * r[i];
            w[j] = s;
        }
    };
    auto residual = [&]() {
        r = b;
        for (int j = 0; j < N; ++j)
            if (x[j] != 0.0)
                for (int i = 0; i < M; ++i) r[i] -= A[size_t(j) * M + i] * x[j];
    };
    grad();
    for (int outer = 0; outer < 3 * N; ++outer) {
        int jmax = -1;
        double wmax = tol;
        for (int j = 0; j < N; ++j)
            if (!passive[j] && w[j] > wmax) { wmax = w[j]; jmax = j; }
        if (jmax < 0) break;
        passive[jmax] = 1;
        for (int inner = 0; inner < 3 * N; ++inner) {
            std::vector<int> P;
            for (int j = 0; j < N; ++j)
                if (passive[j]) P.push_back(j);
            std::vector<double> Ap(size_t(M) * P.size());
            for (size_t k = 0; k < P.size(); ++k)
                std::copy(A.begin() + size_t(P[k]) * M, A.begin() + size_t(P[k] + 1) * M,
                          Ap.begin() + k * M);
            HouseQR qr;
            std::vector<double> z;
            if (!qr.factor(M, int(P.size()), Ap)) {
                // dependent column: drop the newest one
                passive[jmax] = 0;
                w[jmax] = 0.0;
                break;
            }
            qr.solve(b, z);
            bool allpos = true;
            for (double v : z) allpos = allpos && v > 0.0;
            if (allpos) {
                for (size_t k = 0; k < P.size(); ++k) x[P[k]] = z[k];
                break;
            }
            double alpha = 1.0;
            for (size_t k = 0; k < P.size(); ++k)
                if (z[k] <= 0.0) {
                    const double xk = x[P[k]];
                    alpha = std::min(alpha, xk / (xk - z[k]));
                }
            for (size_t k = 0; k < P.size(); ++k) {
                x[P[k]] += alpha * (z[k] - x[P[k]]);
                if (x[P[k]] <= 1e-300) { x[P[k]] = 0.0; passive[P[k]] = 0; }
            }
        }
        residual();
        grad();
    }
    return true;
}

bool fit_expsum_nnls(const std::function<double(double)>& h,
                     const std::function<double(double)>& ref, double s_min, double s_max,
                     double t_lo, double t_hi, double hstep, bool with_constant,
                     std::vector<double>& t, std::vector<double>& c, double& c0,
                     double& max_rel_err) {
    if (!(s_min > 0) || !(s_max >= s_min) || !(t_lo > 0) || !(t_hi > t_lo) || !(hstep > 0))
        return false;
    std::vector<double> nodes;
    for (double x = std::log(t_lo); x <= std::log(t_hi) + 1e-12; x += hstep) nodes.push_back(std::exp(x));
    const int N = int(nodes.size()) + (with_constant ? 1 : 0);
    const int M = 2000;
    std::vector<double> s(M), hv(M), rf(M);
    const double la = std::log(s_min), lb = std::log(std::max(s_max, s_min * (1 + 1e-9)));
    for (int i = 0; i < M; ++i) {
        s[i] = std::exp(la + (lb - la) * double(i) / (M - 1));
        hv[i] = h(s[i]);
        rf[i] = ref(s[i]);
    }
    std::vector<double> wl(M, 1.0), coef, colscale(N);
    std::vector<double> A(size_t(M) * N), b(M);
    // Lawson reweighting rounds; the round with the smallest maximum
    // relative error on the sample grid is kept (the iteration need not be
    // monotone on a nearly dependent exponential basis)
    std::vector<double> best;
    double best_err = 1e300;
    for (int round = 0; round < 10; ++round) {
        for (int j = 0; j < N; ++j) {
            double nrm = 0.0;
            for (int i = 0; i < M; ++i) {
                const double basis = (j < int(nodes.size())) ? std::exp(-nodes[j] * s[i]) : 1.0;
                const double v = wl[i] * basis / rf[i];
                A[size_t(j) * M + i] = v;
                nrm += v * v;
            }
            nrm = std::sqrt(nrm);
            colscale[j] = nrm > 0 ? nrm : 1.0;
            for (int i = 0; i < M; ++i) A[size_t(j) * M + i] /= colscale[j];
        }
        for (int i = 0; i < M; ++i) b[i] = wl[i] * hv[i] / rf[i];
        std::vector<double> x;
        nnls(M, N, A, b, x);
        coef.assign(N, 0.0);
        for (int j = 0; j < N; ++j) coef[j] = x[j] / colscale[j];
        // Lawson reweighting towards a uniform relative error
        std::vector<double> e(M);
        double emax = 0.0;
        for (int i = 0; i < M; ++i) {
            double v = 0.0;
            for (int j = 0; j < N; ++j)
                v += coef[j] * ((j < int(nodes.size())) ? std::exp(-nodes[j] * s[i]) : 1.0);
            e[i] = std::fabs(v - hv[i]) / rf[i];
            emax = std::max(emax, e[i]);
        }
        if (emax < best_err) { best_err = emax; best = coef; }
        if (!(emax > 0)) break;
        for (int i = 0; i < M; ++i) wl[i] *= std::sqrt(std::max(e[i] / emax, 1e-3));
        const double wm = *std::max_element(wl.begin(), wl.end());
        for (double& v : wl) v /= wm;
    }
    if (!best.empty()) coef = best;
    t.clear(); c.clear(); c0 = 0.0;
    for (int j = 0; j < int(nodes.size()); ++j)
        if (coef[j] > 0) { t.push_back(nodes[j]); c.push_back(coef[j]); }
    if (with_constant) c0 = coef[N - 1];
    // accuracy on a dense grid
    double emax = 0.0;
    const int G = 20000;
    for (int i = 0; i <= G; ++i) {
        const double ss = std::exp(la + (lb - la) * double(i) / G);
        double v = c0;
        for (size_t k = 0; k < t.size(); ++k) v += c[k] * std::exp(-t[k] * ss);
        emax = std::max(emax, std::fabs(v - h(ss)) / ref(ss));
    }
    max_rel_err = emax;
    return std::isfinite(emax);
}

}  // namespace fc
