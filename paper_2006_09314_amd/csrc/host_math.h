// Host numerics of the setup phase (see host_math.cpp).
#pragma once
#include <functional>
#include <vector>

namespace fc {

void fd_tridiag(int n, const double* a_mid, double* diag, double* off);
bool tridiag_eigen(int n, std::vector<double>& d, std::vector<double> e, double* Z);
bool fd_eigen(int n, const double* a_mid, double* lam, double* V);

double expsum_max_rel_err(const std::function<double(double)>& h,
                          const std::function<double(double)>& ref, double s_min, double s_max,
                          const double* t, const double* c, int K, int grid);

bool fit_expsum(const std::function<double(double)>& h, const std::function<double(double)>& ref,
                double s_min, double s_max, int K, std::vector<double>& t, std::vector<double>& c,
                double& max_rel_err);

// Positive exponential sum on the fixed nodes exp(log t_lo + k hstep) <= t_hi
// (plus a constant term if requested) by non-negative least squares on the
// relative error with Lawson reweighting; zero-weight nodes are dropped.
bool fit_expsum_nnls(const std::function<double(double)>& h,
                     const std::function<double(double)>& ref, double s_min, double s_max,
                     double t_lo, double t_hi, double hstep, bool with_constant,
                     std::vector<double>& t, std::vector<double>& c, double& c0,
                     double& max_rel_err);

}  // namespace fc
