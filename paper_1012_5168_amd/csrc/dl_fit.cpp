// dl_fit.cpp -- the flavour-singlet combination and the ratio fit of
// Section 3 (Eqs. 3 and 4): C_eta'(t) = C_pi(t) - 2 D(t), and
//     D(t) / C_pi(t) = A - B g_m(t) / g_mpi(t),  g_m(t) = e^{-m t} + e^{-m (T - t)},
// fitted over [tmin, tmax] with the pion mass given.  Host computation on a
// few dozen numbers: no device work.
//
// The fit is a variable projection: for a fixed m the model is linear in
// (A, B), so the weighted least squares for (A, B) has a closed form and
// chi^2 becomes a function of m alone; it is scanned on a logarithmic grid
// over [1e-3, 10] and the best grid point refined by golden-section search.
// Weights are 1 / var(R(t)) from a jackknife over configurations (unit
// weights for a single configuration); errors are jackknife errors of the
// fitted parameters, each jackknife sample refitted with the same weights.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dl_internal.hpp"

namespace dl {

namespace {

struct Fit {
    double A, B, m, chi2;
};

// g_m(t) / g_mpi(t), each cosh-like sum factored so that no term overflows
double shape(double m, double mpi, int t, int T)
{
    const double a = std::exp(-m * t) + std::exp(-m * (T - t));
    const double b = std::exp(-mpi * t) + std::exp(-mpi * (T - t));
    return a / b;
}

// weighted linear least squares of y = A - B g at fixed m; returns chi^2
double linear_ab(const std::vector<double> &y, const std::vector<double> &w, double m, double mpi, int tmin, int T,
                 double &A, double &B)
{
    double S = 0, Sg = 0, Sgg = 0, Sy = 0, Sgy = 0;
    std::vector<double> g(y.size());
    for (size_t k = 0; k < y.size(); ++k) {
        g[k] = shape(m, mpi, tmin + (int)k, T);
        S += w[k];
        Sg += w[k] * g[k];
        Sgg += w[k] * g[k] * g[k];
        Sy += w[k] * y[k];
        Sgy += w[k] * g[k] * y[k];
    }
    const double det = S * Sgg - Sg * Sg;
    if (!(std::fabs(det) > 1e-300 * std::max(1.0, S * Sgg))) {
        A = Sy / S;
        B = 0.0;
    } else {
        A = (Sgg * Sy - Sg * Sgy) / det;
        B = -(S * Sgy - Sg * Sy) / det;
    }
    double chi2 = 0;
    for (size_t k = 0; k < y.size(); ++k) {
        const double r = y[k] - (A - B * g[k]);
        chi2 += w[k] * r * r;
    }
    return chi2;
}

Fit fit_ratio(const std::vector<double> &y, const std::vector<double> &w, double mpi, int tmin, int T)
{
    const int NG = 400;
    const double lo = std::log(1e-3), hi = std::log(10.0);
    auto chi2_at = [&](double m) {
        double A, B;
        return linear_ab(y, w, m, mpi, tmin, T, A, B);
    };
    int kb = 0;
    double cb = INFINITY;
    std::vector<double> grid(NG);
    for (int k = 0; k < NG; ++k) {
        grid[k] = std::exp(lo + (hi - lo) * k / (NG - 1));
        const double c = chi2_at(grid[k]);
        if (c < cb) {
            cb = c;
            kb = k;
        }
    }
    double a = grid[std::max(kb - 1, 0)], b = grid[std::min(kb + 1, NG - 1)];
    const double phi = 0.5 * (std::sqrt(5.0) - 1.0);
    double x1 = b - phi * (b - a), x2 = a + phi * (b - a);
    double f1 = chi2_at(x1), f2 = chi2_at(x2);
    for (int it = 0; it < 200 && (b - a) > 1e-14 * b; ++it) {
        if (f1 < f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - phi * (b - a);
            f1 = chi2_at(x1);
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + phi * (b - a);
            f2 = chi2_at(x2);
        }
    }
    Fit f;
    f.m = 0.5 * (a + b);
    f.chi2 = linear_ab(y, w, f.m, mpi, tmin, T, f.A, f.B);
    if (cb < f.chi2) {  // the refinement can only improve on the grid; keep the grid point otherwise
        f.m = grid[kb];
        f.chi2 = linear_ab(y, w, f.m, mpi, tmin, T, f.A, f.B);
    }
    return f;
}

// R(t) over [tmin, tmax] from the configuration sums, leaving out `skip` (-1: none)
std::vector<double> ratio(const double *d, const double *c, int ncfg, int T, int tmin, int tmax, int skip)
{
    std::vector<double> r;
    for (int t = tmin; t <= tmax; ++t) {
        double sd = 0, sc = 0;
        for (int n = 0; n < ncfg; ++n) {
            if (n == skip) continue;
            sd += d[(size_t)n * T + t];
            sc += c[(size_t)n * T + t];
        }
        DL_REQUIRE(sc != 0.0 && std::isfinite(sc) && std::isfinite(sd), "dl_eta_prime_fit: C_pi must be finite and "
                                                                        "nonzero in the fit range");
        r.push_back(sd / sc);
    }
    return r;
}

}  // namespace

void eta_prime_fit(const double *d, const double *c, int ncfg, int T, double m_pi, int tmin, int tmax, double *c_eta,
                   double *params, double *errors, double *chi2)
{
    DL_REQUIRE(d && c && c_eta && params && errors && chi2, "dl_eta_prime_fit: null pointer");
    DL_REQUIRE(ncfg >= 1 && ncfg <= (1 << 20), "dl_eta_prime_fit: ncfg must be in [1, 2^20]");
    DL_REQUIRE(T >= 4 && T <= 65535, "dl_eta_prime_fit: T must be in [4, 65535]");
    DL_REQUIRE(tmin >= 0 && tmax < T && tmax - tmin + 1 >= 4,
               "dl_eta_prime_fit: need 0 <= tmin, tmax < T and at least 4 points for 3 parameters");
    DL_REQUIRE(m_pi > 0 && std::isfinite(m_pi), "dl_eta_prime_fit: m_pi must be positive");
    for (int t = 0; t < T; ++t) {
        double sd = 0, sc = 0;
        for (int n = 0; n < ncfg; ++n) {
            sd += d[(size_t)n * T + t];
            sc += c[(size_t)n * T + t];
        }
        c_eta[t] = (sc - 2.0 * sd) / ncfg;
    }
    const std::vector<double> y = ratio(d, c, ncfg, T, tmin, tmax, -1);
    const size_t np = y.size();
    std::vector<double> w(np, 1.0);
    std::vector<std::vector<double>> jk;
    if (ncfg >= 2) {
        for (int k = 0; k < ncfg; ++k) jk.push_back(ratio(d, c, ncfg, T, tmin, tmax, k));
        bool all_positive = true;
        std::vector<double> var(np, 0.0);
        for (size_t i = 0; i < np; ++i) {
            double mean = 0;
            for (int k = 0; k < ncfg; ++k) mean += jk[k][i];
            mean /= ncfg;
            for (int k = 0; k < ncfg; ++k) var[i] += (jk[k][i] - mean) * (jk[k][i] - mean);
            var[i] *= (double)(ncfg - 1) / ncfg;
            all_positive = all_positive && var[i] > 0;
        }
        if (all_positive)
            for (size_t i = 0; i < np; ++i) w[i] = 1.0 / var[i];
    }
    const Fit f = fit_ratio(y, w, m_pi, tmin, T);
    params[0] = f.A;
    params[1] = f.B;
    params[2] = f.m;
    *chi2 = f.chi2;
    errors[0] = errors[1] = errors[2] = 0.0;
    if (ncfg >= 2) {
        std::vector<Fit> fk;
        for (int k = 0; k < ncfg; ++k) fk.push_back(fit_ratio(jk[k], w, m_pi, tmin, T));
        double mean[3] = {0, 0, 0};
        for (const Fit &x : fk) {
            mean[0] += x.A;
            mean[1] += x.B;
            mean[2] += x.m;
        }
        for (double &v : mean) v /= ncfg;
        double var[3] = {0, 0, 0};
        for (const Fit &x : fk) {
            var[0] += (x.A - mean[0]) * (x.A - mean[0]);
            var[1] += (x.B - mean[1]) * (x.B - mean[1]);
            var[2] += (x.m - mean[2]) * (x.m - mean[2]);
        }
        for (int i = 0; i < 3; ++i) errors[i] = std::sqrt(var[i] * (double)(ncfg - 1) / ncfg);
    }
}

}  // namespace dl
