// Host-side parameter selection and tables (FP64).
//
// Paper passages implemented here:
//  * PSWF psi_0^c and its use as splitting kernel chi = psi/int_0^1 psi and as
//    window phi(x) = psi^{c1}(2x/(P h)) (Methods, PSWF section, eq. pswf).
//  * c from psi_0^c(1) = eps; P from Table 2; n from the Fourier truncation
//    rule (eq. pswfparameters) and rc = kappa c h / pi.
//  * c1 by minimising the aliasing estimate E_A (eq. errorformula).
//  * Influence function p_m = h^6 S^(2 pi m/L) / (L^3 phi^(2 pi m/L)^2) with
//    S^(k) = chi^(rc k)/k^2 (eqs. hS, pk), factored into a radial table over
//    |m|^2 and a per-axis table of 1/phi^_1^2.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>

namespace esp {

static constexpr double kPi = 3.14159265358979323846;

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Solve (T - s I) v = b for symmetric tridiagonal T (diag d, off e) by
// Gaussian elimination with partial pivoting.
static void tridiag_solve(const std::vector<double>& d, const std::vector<double>& e, double s,
                          std::vector<double>& b) {
    const int n = (int)d.size();
    std::vector<double> dl(n > 1 ? n - 1 : 0), dd(n), du(n > 1 ? n - 1 : 0), du2(n > 2 ? n - 2 : 0, 0.0);
    for (int i = 0; i < n; ++i) dd[i] = d[i] - s;
    for (int i = 0; i + 1 < n; ++i) dl[i] = du[i] = e[i];
    const double tiny = 1e-300;
    for (int i = 0; i + 1 < n; ++i) {
        if (std::fabs(dd[i]) >= std::fabs(dl[i])) {
            if (dd[i] == 0.0) dd[i] = tiny;
            double f = dl[i] / dd[i];
            dd[i + 1] -= f * du[i];
            b[i + 1] -= f * b[i];
            if (i + 2 < n) du2[i] = 0.0;
        } else {
            double f = dd[i] / dl[i];
            dd[i] = dl[i];
            double t = dd[i + 1];
            dd[i + 1] = du[i] - f * t;
            du[i] = t;
            if (i + 2 < n) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du2[i];
            }
            std::swap(b[i], b[i + 1]);
            b[i + 1] -= f * b[i];
        }
    }
    if (dd[n - 1] == 0.0) dd[n - 1] = tiny;
    b[n - 1] /= dd[n - 1];
    if (n > 1) b[n - 2] = (b[n - 2] - du[n - 2] * b[n - 1]) / (dd[n - 2] == 0.0 ? tiny : dd[n - 2]);
    for (int i = n - 3; i >= 0; --i)
        b[i] = (b[i] - du[i] * b[i + 1] - du2[i] * b[i + 2]) / (dd[i] == 0.0 ? tiny : dd[i]);
}

Prolate::Prolate(double c) : c_(c) {
    const int K = (int)(c + 40.0);  // even Legendre degrees 0, 2, ..., 2(K-1)
    std::vector<double> d(K), e(K - 1);
    for (int i = 0; i < K; ++i) {
        const double k = 2.0 * i;
        double t = (k + 1) * (k + 1) / ((2 * k + 1) * (2 * k + 3));
        if (i > 0) t += k * k / ((2 * k + 1) * (2 * k - 1));
        d[i] = k * (k + 1) + c * c * t;
        if (i + 1 < K)
            e[i] = c * c * (k + 1) * (k + 2) / ((2 * k + 1) * (2 * k + 3)) *
                   std::sqrt((2 * k + 1) / (2 * k + 5));
    }
    // smallest eigenvalue by bisection on the Sturm count
    auto count_below = [&](double x) {
        int cnt = 0;
        double q = d[0] - x;
        if (q < 0) ++cnt;
        for (int i = 1; i < K; ++i) {
            if (q == 0.0) q = 1e-300;
            q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    double lo = d[0] - std::fabs(e[0]) - 1.0, hi = d[0] + std::fabs(e[0]) + 1.0;
    for (int i = 1; i < K; ++i) {
        const double r = std::fabs(e[i - 1]) + (i + 1 < K ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= 1) hi = mid; else lo = mid;
    }
    const double lam = 0.5 * (lo + hi);
    // inverse iteration
    std::vector<double> v(K, 1.0);
    for (int it = 0; it < 4; ++it) {
        tridiag_solve(d, e, lam, v);
        double nrm = 0.0;
        for (double t : v) nrm += t * t;
        nrm = std::sqrt(nrm);
        for (double& t : v) t /= nrm;
    }
    if (v[0] < 0) for (double& t : v) t = -t;
    a_.resize(K);
    for (int i = 0; i < K; ++i) a_[i] = v[i] * std::sqrt(2.0 * i + 0.5);
    std::vector<double> w;
    gauss_legendre(256, qx_, w);
    qw_psi_.resize(qx_.size());
    for (size_t q = 0; q < qx_.size(); ++q) qw_psi_[q] = w[q] * (*this)(qx_[q]);
}

double Prolate::operator()(double x) const {
    // sum_i a_i P_{2i}(x) with the Legendre three-term recurrence
    double p0 = 1.0, p1 = x, s = a_[0];
    const int deg = 2 * ((int)a_.size() - 1);
    for (int k = 1; k < deg; ++k) {
        const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
        if ((k + 1) % 2 == 0) s += a_[(k + 1) / 2] * p1;
    }
    return s;
}

double Prolate::deriv(double x) const {
    double p0 = 1.0, p1 = x, dp0 = 0.0, dp1 = 1.0, s = 0.0;
    const int deg = 2 * ((int)a_.size() - 1);
    for (int k = 1; k < deg; ++k) {
        const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        const double dp2 = ((2.0 * k + 1.0) * (p1 + x * dp1) - k * dp0) / (k + 1.0);
        p0 = p1; p1 = p2; dp0 = dp1; dp1 = dp2;
        if ((k + 1) % 2 == 0) s += a_[(k + 1) / 2] * dp1;
    }
    return s;
}

double Prolate::integral(double x) const {
    // int_0^x P_0 = x; int_0^x P_k = (P_{k+1}(x) - P_{k-1}(x))/(2k+1) for even k >= 2
    const int deg = 2 * ((int)a_.size() - 1) + 1;
    std::vector<double> P(deg + 1);
    P[0] = 1.0;
    P[1] = x;
    for (int k = 1; k < deg; ++k) P[k + 1] = ((2.0 * k + 1.0) * x * P[k] - k * P[k - 1]) / (k + 1.0);
    double s = a_[0] * x;
    for (size_t i = 1; i < a_.size(); ++i) {
        const int k = 2 * (int)i;
        s += a_[i] * (P[k + 1] - P[k - 1]) / (2.0 * k + 1.0);
    }
    return s;
}

double Prolate::ft(double w) const {
    double s = 0.0;
    for (size_t q = 0; q < qx_.size(); ++q) s += qw_psi_[q] * std::cos(w * qx_[q]);
    return s;
}

static double c_for_tolerance_uncached(double eps);

double c_for_tolerance(double eps) {
    static std::mutex mu;
    static std::map<double, double> cache;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(eps);
        if (it != cache.end()) return it->second;
    }
    const double c = c_for_tolerance_uncached(eps);
    std::lock_guard<std::mutex> g(mu);
    cache[eps] = c;
    return c;
}

static double c_for_tolerance_uncached(double eps) {
    // psi_0^c(1) decreases monotonically in c; bisection on log psi(1)
    double lo = std::max(0.5, std::log(1.0 / eps) - 3.0), hi = std::log(1.0 / eps) + 10.0;
    const double target = std::log(eps);
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double v = Prolate(mid)(1.0);
        if (v > 0 && std::log(v) > target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

int order_for_tol(double tol) {
    // Table 2: P_esp = 5, 5, 6, 7, 8 at eps = 1e-3, 5e-4, 1e-4, 5e-5, 1e-5
    static const double eps[5] = {1e-5, 5e-5, 1e-4, 5e-4, 1e-3};
    static const int P[5] = {8, 7, 6, 5, 5};
    if (tol >= 1e-3) return 5;
    if (tol < 1e-5) {
        const int p = 8 + (int)std::ceil(3.0 * std::log10(1e-5 / tol) - 1e-9);
        return std::min(p, 12);
    }
    int best = 0;
    for (int i = 0; i < 5; ++i)
        if (eps[i] <= tol * (1 + 1e-12)) best = i;
    return P[best];
}

bool is_smooth(int n) {
    if (n < 2 || n % 2) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

int grid_size(double L, double h_max) {
    int n = std::max(8, (int)std::ceil(L / h_max - 1e-12));
    while (!is_smooth(n)) ++n;
    return n;
}

// c1-independent factor of E_A: a(m_x) = sum_{m_y, m_z} |chi^(2 pi rc |m|/L)| / |m|^2
// for m_x = -n/2 .. n/2-1 (only the x factor of the window ratio depends on c1).
static std::vector<double> aliasing_weights(int n, double L, const Prolate& chi, double rc) {
    const double I1 = chi.integral(1.0);
    const int h2 = n / 2;
    std::vector<double> chat(3 * h2 * h2 + 1, 0.0);
    for (int m2 = 1; m2 <= 3 * h2 * h2; ++m2)
        chat[m2] = std::fabs(0.5 * chi.ft(2 * kPi * rc * std::sqrt((double)m2) / L) / I1) / m2;
    // a(m_x) depends on |m_x| only: sum over (m_y, m_z) once per |m_x|
    std::vector<double> byabs(h2 + 1, 0.0);
    for (int ax_ = 0; ax_ <= h2; ++ax_)
        for (int my = -h2; my < h2; ++my)
            for (int mz = -h2; mz < h2; ++mz) byabs[ax_] += chat[ax_ * ax_ + my * my + mz * mz];
    std::vector<double> ax(n);
    for (int mx = -h2; mx < h2; ++mx) ax[mx + h2] = byabs[mx < 0 ? -mx : mx];
    return ax;
}

static double aliasing_from_weights(const std::vector<double>& ax, int n, double L, double c1, int P) {
    const double h = L / n;
    const int h2 = n / 2;
    Prolate win(c1);
    double s = 0.0;
    for (int mx = -h2; mx < h2; ++mx) {
        const double a = win.ft(2 * kPi * (mx + n) / L * P * h / 2);
        const double b = win.ft(2 * kPi * mx / L * P * h / 2);
        s += ax[mx + h2] * std::fabs(a / b);
    }
    return 6.0 * s;
}

double aliasing_error(int n, double L, const Prolate& chi, double rc, double c1, int P) {
    // E_A = 6 sum_{m in I\0} | chi^(2 pi rc|m|/L)/|m|^2 * phi^(k + 2 pi (n,0,0)/L)/phi^(k) |
    return aliasing_from_weights(aliasing_weights(n, L, chi, rc), n, L, c1, P);
}

// Memoised per-c quantities: psi(0) / int_0^1 psi (for S(0)).
static double chi0_over_I1(double c) {
    static std::mutex mu;
    static std::map<double, double> cache;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(c);
        if (it != cache.end()) return it->second;
    }
    Prolate chi(c);
    const double v = chi(0.0) / chi.integral(1.0);
    std::lock_guard<std::mutex> g(mu);
    cache[c] = v;
    return v;
}

// Classical method (Methods, classical fast Ewald methods, eq. cem): Gaussian
// splitting kernel chi(t) = 2 sqrt(alpha/pi) exp(-alpha t^2) (t = r/rc; its
// transform chi^(w) = exp(-w^2/(4 alpha)), classical Ewald with
// beta = sqrt(alpha)/rc) and the cardinal B-spline of order P as window,
// phi^_1(xi) = h (sin(xi h/2)/(xi h/2))^P.
static double gauss_chi(double alpha, double t) { return 2.0 * std::sqrt(alpha / kPi) * std::exp(-alpha * t * t); }

// Centred cardinal B-spline of order P (support [-P/2, P/2]) by the
// Cox-de Boor recursion M_k(x) = (x M_{k-1}(x) + (k - x) M_{k-1}(x - 1))/(k - 1).
static double bspline(int P, double x) {
    x += 0.5 * P;
    if (x <= 0.0 || x >= P) return 0.0;
    double M[16];
    for (int j = 0; j < P; ++j) M[j] = (x >= j && x < j + 1) ? 1.0 : 0.0;  // M_1(x - j)
    for (int k = 2; k <= P; ++k)
        for (int j = 0; j + k <= P; ++j) {
            const double xj = x - j;
            M[j] = (xj * M[j] + (k - xj) * M[j + 1]) / (k - 1);
        }
    return M[0];
}

static double sinc(double x) { return std::fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : std::sin(x) / x; }

// Parameters of the classical method: alpha = log(1/eps) and
// n_f = 2 ceil(alpha L/(pi rc)) (eq. cemparameters), rounded up to a grid size
// with FFT kernels; P = 5 (the default of common MD codes); rc the ESP cutoff
// at the same tolerance unless given.
static esp_status resolve_classical(double L, double Lmax, double Lmin, double tol, esp_params r, esp_params* out,
                                    std::string& msg) {
    if (r.c <= 0) r.c = std::log(1.0 / tol);
    if (r.P <= 0) r.P = 5;
    if (r.P < 4 || r.P > 12) { msg = "window width P must lie in [4, 12]"; return ESP_E_UNSUPPORTED; }
    if (r.h_max <= 0) r.h_max = 1.25;
    if (r.kappa <= 0) r.kappa = 1.2;
    if (r.rc <= 0) {
        const int n_esp = grid_size(Lmax, r.h_max);
        r.rc = r.kappa * c_for_tolerance(tol) / kPi * (Lmax / n_esp);
    }
    if (r.nf <= 0) {
        int n = 2 * (int)std::ceil(r.c * Lmax / (kPi * r.rc) - 1e-12);
        while (n <= 144 && !is_smooth(n)) n += 2;
        r.nf = std::max(n, 8);
    }
    if (!is_smooth(r.nf) || r.nf < 8 || r.nf > 144) {
        msg = "grid size must be even, of the form 2^a 3^b, within [8, 144]";
        return ESP_E_UNSUPPORTED;
    }
    if (r.nf < r.P) { msg = "grid size must be at least P"; return ESP_E_UNSUPPORTED; }
    r.h = L / r.nf;
    const double rho = std::round(r.rc / r.h * 1e12) / 1e12;
    if (r.precision == 0) r.precision = 32;
    if (r.precision != 32 && r.precision != 64) { msg = "precision must be 32 or 64"; return ESP_E_INVALID; }
    if (r.tile != 0 && (r.tile < 8 || r.tile > 16)) { msg = "tile must lie in [8, 16]"; return ESP_E_UNSUPPORTED; }
    if (r.fft_passes != 0 && r.fft_passes != 1) { msg = "fft_passes must be 0 or 1"; return ESP_E_INVALID; }
    if (r.force_method != 0 && r.force_method != 1) { msg = "force_method must be 0 or 1"; return ESP_E_INVALID; }
    if (r.local != 0 && r.local != 1) { msg = "local must be 0 or 1"; return ESP_E_INVALID; }
    if (r.local && r.rc > 0.5 * Lmin * (1 + 1e-12)) {
        msg = "the local part needs rc <= L/2 (nearest images only)";
        return ESP_E_UNSUPPORTED;
    }
    (void)rho;
    r.c1 = 0.0;                       // the window is the B-spline: no shape parameter
    r.degree = std::max(4, r.P - 1);  // exact piecewise polynomial
    r.s0 = gauss_chi(r.c, 0.0) / (4.0 * kPi * r.rc);
    *out = r;
    return ESP_OK;
}

esp_status resolve_params(double L, int64_t N, double tol, const esp_params* req, esp_params* out,
                          std::string& msg) {
    esp_params r{};
    if (req) r = *req;
    if (!(L > 0) || !std::isfinite(L)) { msg = "box side must be positive and finite"; return ESP_E_INVALID; }
    if (N < 1) { msg = "N must be >= 1"; return ESP_E_INVALID; }
    if (!(tol >= 1e-8 && tol <= 1e-2)) { msg = "tol must lie in [1e-8, 1e-2]"; return ESP_E_INVALID; }
    r.L = L;
    r.tol = tol;
    if (r.method != 0 && r.method != 1) { msg = "method must be 0 (ESP) or 1 (classical)"; return ESP_E_INVALID; }
    if (r.deterministic != 0 && r.deterministic != 1) { msg = "deterministic must be 0 or 1"; return ESP_E_INVALID; }
    if (r.deterministic == 1 && r.precision == 64) {
        msg = "FP64 plans are not bitwise reproducible (the spread adds with FP64 LDS atomics)";
        return ESP_E_UNSUPPORTED;
    }
    // FP32 plans sum the spread in fixed point and everything else in a fixed
    // order; FP64 plans add the spread with floating-point LDS atomics
    r.deterministic = r.precision == 64 ? 0 : 1;
    if (r.Ly < 0 || r.Lz < 0) { msg = "box sides must be positive"; return ESP_E_INVALID; }
    if (r.Ly == 0) r.Ly = L;
    if (r.Lz == 0) r.Lz = L;
    if (!(std::isfinite(r.Ly) && std::isfinite(r.Lz))) { msg = "box sides must be finite"; return ESP_E_INVALID; }
    if (!(std::isfinite(r.xy) && std::isfinite(r.xz) && std::isfinite(r.yz))) {
        msg = "cell tilts must be finite";
        return ESP_E_INVALID;
    }
    // the longest lattice vector sets the grid and the cutoff (the resolved
    // modes |m_d| <= n/2 then hold the sphere |k| <= pi n / Lmax); nearest
    // images need rc at most half the smallest lattice-plane spacing
    const Cell cell = cell_of(r);
    const double Lmax = cell.amax, Lmin = cell.dmin;
    if (r.method == 1) return resolve_classical(L, Lmax, Lmin, tol, r, out, msg);
    if (r.c <= 0) r.c = c_for_tolerance(tol);
    if (r.P <= 0) r.P = order_for_tol(tol);
    if (r.P < 4 || r.P > 12) { msg = "window width P must lie in [4, 12]"; return ESP_E_UNSUPPORTED; }
    if (r.h_max <= 0) r.h_max = 1.25;
    if (r.kappa <= 0) r.kappa = 1.2;
    if (r.nf <= 0) r.nf = grid_size(Lmax, r.h_max);
    if (!is_smooth(r.nf) || r.nf < 8 || r.nf > 144) {
        msg = "grid size must be even, of the form 2^a 3^b, within [8, 144]";
        return ESP_E_UNSUPPORTED;
    }
    if (r.nf < r.P) { msg = "grid size must be at least P"; return ESP_E_UNSUPPORTED; }
    r.h = L / r.nf;
    // rho = rc/h keys every L-independent cache; exact under the default rule
    // (along the coarsest axis, which the window's aliasing is chosen for)
    double rho;
    if (r.rc <= 0) {
        rho = r.kappa * r.c / kPi;
        r.rc = rho * Lmax / r.nf;
    } else {
        rho = std::round(r.rc / (Lmax / r.nf) * 1e12) / 1e12;
    }
    if (r.precision == 0) r.precision = 32;
    if (r.precision != 32 && r.precision != 64) { msg = "precision must be 32 or 64"; return ESP_E_INVALID; }
    if (r.tile != 0 && (r.tile < 8 || r.tile > 16)) { msg = "tile must lie in [8, 16]"; return ESP_E_UNSUPPORTED; }
    if (r.fft_passes != 0 && r.fft_passes != 1) { msg = "fft_passes must be 0 or 1"; return ESP_E_INVALID; }
    if (r.force_method != 0 && r.force_method != 1) { msg = "force_method must be 0 or 1"; return ESP_E_INVALID; }
    if (r.local != 0 && r.local != 1) { msg = "local must be 0 or 1"; return ESP_E_INVALID; }
    if (r.local && r.rc > 0.5 * Lmin * (1 + 1e-12)) {
        msg = tilted(r) ? "the local part needs rc <= half the smallest lattice-plane spacing"
                        : "the local part needs rc <= L/2 (nearest images only)";
        return ESP_E_UNSUPPORTED;
    }
    if (r.c1 <= 0) {
        // E_A depends on L only through rc/h; memoise per (n, P, c, rc/h).
        // Evaluated in the reference box L = n (h = 1, rc = rho).
        static std::mutex mu;
        static std::map<std::tuple<int, int, double, double>, double> cache;
        const auto key = std::make_tuple(r.nf, r.P, r.c, rho);
        bool hit = false;
        {
            std::lock_guard<std::mutex> g(mu);
            auto it = cache.find(key);
            if (it != cache.end()) { r.c1 = it->second; hit = true; }
        }
        if (!hit) {
            Prolate chi(r.c);
            const std::vector<double> ax = aliasing_weights(r.nf, (double)r.nf, chi, rho);
            double best = std::numeric_limits<double>::infinity(), bc1 = r.c;
            for (int i = 0; i <= 50; ++i) {
                const double c1 = r.c * (0.9 + 0.5 * i / 50.0);
                const double ea = aliasing_from_weights(ax, r.nf, (double)r.nf, c1, r.P);
                if (ea < best) { best = ea; bc1 = c1; }
            }
            r.c1 = bc1;
            std::lock_guard<std::mutex> g(mu);
            cache[key] = bc1;
        }
    }
    r.s0 = chi0_over_I1(r.c) / (4.0 * kPi * r.rc);
    if (r.degree != 0 && (r.degree < 4 || r.degree > 16)) { msg = "degree must lie in [4, 16]"; return ESP_E_UNSUPPORTED; }
    if (r.degree == 0) {
        // smallest adequate degree; memoised per (c1, P, tol)
        static std::mutex mu;
        static std::map<std::tuple<double, int, double>, int> cache;
        const auto key = std::make_tuple(r.c1, r.P, r.tol);
        int d = 0;
        {
            std::lock_guard<std::mutex> g(mu);
            auto it = cache.find(key);
            if (it != cache.end()) d = it->second;
        }
        if (d) {
            r.degree = d;
        } else {
            std::vector<double> coef;
            window_polynomials(r, coef);
            std::lock_guard<std::mutex> g(mu);
            cache[key] = r.degree;
        }
    }
    *out = r;
    return ESP_OK;
}

// Chebyshev interpolation of f on [-1/2, 1/2] at degree d, returned as
// monomial coefficients in y.
template <class F>
static std::vector<double> cheb_fit(F f, int d) {
    const int m = d + 1;
    std::vector<double> fv(m), s(m);
    for (int i = 0; i < m; ++i) {
        s[i] = std::cos(kPi * (i + 0.5) / m);
        fv[i] = f(0.5 * s[i]);
    }
    std::vector<double> ck(m, 0.0);
    for (int k = 0; k < m; ++k) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += fv[i] * std::cos(k * kPi * (i + 0.5) / m);
        ck[k] = acc * 2.0 / m;
    }
    ck[0] *= 0.5;
    // sum ck T_k(s) -> monomials in s, T_{k+1} = 2 s T_k - T_{k-1}
    std::vector<double> mono(m, 0.0), Tkm1(m, 0.0), Tk(m, 0.0), Tkp1(m, 0.0);
    Tkm1[0] = 1.0;
    mono[0] += ck[0];
    if (m > 1) {
        Tk[1] = 1.0;
        mono[1] += ck[1];
    }
    for (int k = 1; k + 1 < m; ++k) {
        std::fill(Tkp1.begin(), Tkp1.end(), 0.0);
        for (int j = 0; j + 1 < m; ++j) Tkp1[j + 1] += 2.0 * Tk[j];
        for (int j = 0; j < m; ++j) Tkp1[j] -= Tkm1[j];
        for (int j = 0; j < m; ++j) mono[j] += ck[k + 1] * Tkp1[j];
        Tkm1 = Tk;
        Tk = Tkp1;
    }
    // s = 2y
    double sc = 1.0;
    for (int j = 0; j < m; ++j, sc *= 2.0) mono[j] *= sc;
    return mono;
}

void window_polynomials(esp_params& p, std::vector<double>& coef) {
    if (p.method == 1) {
        // B-spline: weight of point l0 + j is B_P(y + 1/2 + P/2 - 1 - j), a
        // polynomial of degree P - 1 in y on [-1/2, 1/2)
        const int P = p.P, d = std::max(4, P - 1);
        coef.assign((size_t)P * (d + 1), 0.0);
        for (int j = 0; j < P; ++j) {
            const std::vector<double> a = cheb_fit([&](double y) { return bspline(P, y + 0.5 + 0.5 * P - 1.0 - j); }, d);
            for (int m = 0; m <= d; ++m) coef[(size_t)j * (d + 1) + m] = a[m];
        }
        p.degree = d;
        return;
    }
    Prolate win(p.c1);
    const int P = p.P;
    const double peak = win(0.0);
    auto piece = [&](int j) {
        // weight of point l0 + j as a function of y = z - 1/2, z = frac(u - P/2):
        // psi(2 (u - l0 - j)/P) with u - l0 = P/2 - 1 + z
        return [&win, j, P](double y) { return win(2.0 * (y + 0.5 + 0.5 * P - 1.0 - j) / P); };
    };
    auto eval = [](const std::vector<double>& a, double y) {
        double s = 0.0;
        for (int m = (int)a.size() - 1; m >= 0; --m) s = s * y + a[m];
        return s;
    };
    int d0 = p.degree, d1 = p.degree;
    if (p.degree == 0) { d0 = 4; d1 = 16; }
    for (int d = d0; d <= d1; ++d) {
        coef.assign((size_t)P * (d + 1), 0.0);
        double err = 0.0;
        for (int j = 0; j < P; ++j) {
            auto f = piece(j);
            std::vector<double> a = cheb_fit(f, d);
            for (int m = 0; m <= d; ++m) coef[(size_t)j * (d + 1) + m] = a[m];
            for (int t = 0; t <= 64; ++t) {
                const double y = -0.5 + t / 64.0;
                err = std::max(err, std::fabs(eval(a, y) - f(y)));
            }
        }
        if (p.degree != 0 || err <= 0.05 * p.tol * peak || d == d1) {
            p.degree = d;
            return;
        }
    }
}

void influence_tables(const esp_params& p, std::vector<double>& TS, std::vector<double>& Tphi) {
    if (p.method == 1) {
        const int n = p.nf, h2 = n / 2, P = p.P;
        const double L = p.L, h = p.h, pref = std::pow(h, 6) / (L * L * L);
        TS.assign(3 * h2 * h2 + 1, 0.0);
        for (int m2 = 1; m2 <= 3 * h2 * h2; ++m2) {
            const double k = 2 * kPi * std::sqrt((double)m2) / L, w = p.rc * k;
            TS[m2] = pref * std::exp(-w * w / (4.0 * p.c)) / (k * k);
        }
        Tphi.assign(h2 + 1, 0.0);
        for (int m = 0; m <= h2; ++m) {
            const double ph = h * std::pow(sinc(kPi * m / n), P);  // xi h / 2 = pi m / n
            Tphi[m] = 1.0 / (ph * ph);
        }
        return;
    }
    Prolate chi(p.c), win(p.c1);
    const int n = p.nf, h2 = n / 2, P = p.P;
    const double L = p.L, h = p.h, I1 = chi.integral(1.0);
    TS.assign(3 * h2 * h2 + 1, 0.0);
    const double pref = std::pow(h, 6) / (L * L * L);
    for (int m2 = 1; m2 <= 3 * h2 * h2; ++m2) {
        const double k = 2 * kPi * std::sqrt((double)m2) / L;
        const double chat = 0.5 * chi.ft(p.rc * k) / I1;
        TS[m2] = pref * chat / (k * k);
    }
    Tphi.assign(h2 + 1, 0.0);
    for (int m = 0; m <= h2; ++m) {
        const double xi = 2 * kPi * m / L;
        const double ph = 0.5 * P * h * win.ft(xi * P * h / 2);
        Tphi[m] = 1.0 / (ph * ph);
    }
}

void local_kernel(const esp_params& p, const double* r, int64_t n, double* Lr, double* dLr) {
    if (p.method == 1) {
        for (int64_t i = 0; i < n; ++i) {
            const double t = r[i] / p.rc;
            if (t >= 1.0) {
                Lr[i] = 0.0;
                dLr[i] = 0.0;
                continue;
            }
            const double Gc = std::erfc(std::sqrt(p.c) * t);
            Lr[i] = Gc / (4 * kPi * r[i]);
            dLr[i] = -Gc / (4 * kPi * r[i] * r[i]) - gauss_chi(p.c, t) / (p.rc * 4 * kPi * r[i]);
        }
        return;
    }
    Prolate chi(p.c);
    const double I1 = chi.integral(1.0);
    for (int64_t i = 0; i < n; ++i) {
        const double t = r[i] / p.rc;
        if (t >= 1.0) {
            Lr[i] = 0.0;
            dLr[i] = 0.0;
            continue;
        }
        const double G = chi.integral(t) / I1;
        const double ch = chi(t) / I1;
        Lr[i] = (1.0 - G) / (4 * kPi * r[i]);
        dLr[i] = -(1.0 - G) / (4 * kPi * r[i] * r[i]) - ch / (p.rc * 4 * kPi * r[i]);
    }
}

// Local part in grid units (h = 1, rc = rho), for the device's short-range
// pass: L(r) = 1/(4 pi r) - s(r) for r < rho, with s(r) = G(r/rho)/(4 pi r)
// the smooth part of the split (eq. kernelsplitting), G(t) = int_0^t chi.
// With t = r/rho, substituting u = t v in the integrals gives
//   s(r)    = (1/(4 pi rho))     int_0^1 chi(t v) dv,
//   s'(r)/r = (1/(4 pi rho^3 t)) int_0^1 v chi'(t v) dv,
// smooth functions of x = t^2 without cancellation at small t. Each is fitted
// by Chebyshev interpolation on kLocalPieces equal intervals of x, at the
// smallest degree (kLocalMinDegree .. kLocalMaxDegree) whose error stays
// below 1e-12 of the function's largest value. Memoised per (c, rho).
void local_polynomials(int method, double c, double rho, int& degree, std::vector<double>& A,
                       std::vector<double>& B) {
    static std::mutex mu;
    static std::map<std::tuple<int, double, double>, std::tuple<int, std::vector<double>, std::vector<double>>> cache;
    const auto key = std::make_tuple(method, c, rho);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            std::tie(degree, A, B) = it->second;
            return;
        }
    }
    // chi and chi' of the split on [0, 1]: PSWF psi/int_0^1 psi, or Gaussian
    Prolate psi(method == 1 ? 1.0 : c);
    const double I1 = method == 1 ? 1.0 : psi.integral(1.0);
    auto chi = [&](double t) { return method == 1 ? gauss_chi(c, t) : psi(t) / I1; };
    auto dchi = [&](double t) { return method == 1 ? -2.0 * c * t * gauss_chi(c, t) : psi.deriv(t) / I1; };
    std::vector<double> gx, gw;
    gauss_legendre(40, gx, gw);
    auto sfun = [&](double x) {
        const double t = std::sqrt(std::max(x, 0.0));
        double a = 0.0;
        for (size_t i = 0; i < gx.size(); ++i) a += 0.5 * gw[i] * chi(t * 0.5 * (gx[i] + 1.0));
        return a / (4.0 * kPi * rho);
    };
    auto bfun = [&](double x) {
        const double t = std::sqrt(x);
        double a = 0.0;
        for (size_t i = 0; i < gx.size(); ++i) {
            const double v = 0.5 * (gx[i] + 1.0);
            a += 0.5 * gw[i] * v * dchi(t * v);
        }
        return a / (4.0 * kPi * rho * rho * rho * t);
    };
    const int K = kLocalPieces, nchk = 257;
    std::vector<double> chk_x, chk_s, chk_b;
    double ms = 0.0, mb = 0.0;
    for (int k = 0; k < K; ++k)
        for (int i = 0; i < nchk; ++i) {
            const double x = (k + (i + 0.5) / nchk) / K;
            chk_x.push_back(x);
            chk_s.push_back(sfun(x));
            chk_b.push_back(bfun(x));
            ms = std::max(ms, std::fabs(chk_s.back()));
            mb = std::max(mb, std::fabs(chk_b.back()));
        }
    auto eval = [](const double* a, int d, double y) {
        double v = 0.0;
        for (int m = d; m >= 0; --m) v = v * y + a[m];
        return v;
    };
    int d = kLocalMinDegree;
    for (;; ++d) {
        A.assign((size_t)K * (d + 1), 0.0);
        B.assign((size_t)K * (d + 1), 0.0);
        for (int k = 0; k < K; ++k) {
            const std::vector<double> a = cheb_fit([&](double y) { return sfun((k + 0.5 + y) / K); }, d);
            const std::vector<double> b = cheb_fit([&](double y) { return bfun((k + 0.5 + y) / K); }, d);
            std::copy(a.begin(), a.end(), A.begin() + (size_t)k * (d + 1));
            std::copy(b.begin(), b.end(), B.begin() + (size_t)k * (d + 1));
        }
        double es = 0.0, eb = 0.0;
        for (size_t i = 0; i < chk_x.size(); ++i) {
            const int k = std::min((int)(chk_x[i] * K), K - 1);
            const double y = chk_x[i] * K - k - 0.5;
            es = std::max(es, std::fabs(eval(&A[(size_t)k * (d + 1)], d, y) - chk_s[i]));
            eb = std::max(eb, std::fabs(eval(&B[(size_t)k * (d + 1)], d, y) - chk_b[i]));
        }
        if ((es <= 1e-12 * ms && eb <= 1e-12 * mb) || d == kLocalMaxDegree) break;
    }
    degree = d;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = std::make_tuple(d, A, B);
}

double grid_rho(const esp_params& p) {
    if (p.method == 1) return std::round(p.rc / p.h * 1e12) / 1e12;
    double rho = p.kappa * p.c / kPi;  // the default rule's exact rc/h
    if (std::fabs(rho * p.h - p.rc) > 1e-12 * p.rc) rho = std::round(p.rc / p.h * 1e12) / 1e12;
    return rho;
}

Cell cell_of(const esp_params& p) {
    Cell c;
    const double Lx = p.L, Ly = p.Ly, Lz = p.Lz;
    c.i00 = 1.0 / Lx;
    c.i11 = 1.0 / Ly;
    c.i22 = 1.0 / Lz;
    c.ixy = -p.xy / (Lx * Ly);
    c.iyz = -p.yz / (Ly * Lz);
    c.ixz = (p.xy * p.yz - p.xz * Ly) / (Lx * Ly * Lz);
    c.amax = std::max(Lx, std::max(std::hypot(p.xy, Ly), std::hypot(std::hypot(p.xz, p.yz), Lz)));
    // plane spacing of family d: 1 / |row d of H^-1|
    const double ry = p.yz / Lz, rx1 = p.xy / Ly, rx2 = (p.xy * p.yz - p.xz * Ly) / (Ly * Lz);
    c.dmin = std::min(Lz, std::min(Ly / std::sqrt(1.0 + ry * ry), Lx / std::sqrt(1.0 + rx1 * rx1 + rx2 * rx2)));
    return c;
}

void box_influence(const esp_params& p, const ClassTables& ct, std::vector<double>& out) {
    // p_m = S^(|k|)/V Tphi[|m_x|] Tphi[|m_y|] Tphi[|m_z|]: the window's transform
    // in grid units is the same on every axis (Tphi of the class, h = 1), so the
    // spacings cancel against the h^6 of eq. pk. k = 2 pi H^-T m; in an
    // orthorhombic box k_d = 2 pi m_d/L_d.
    const int n = p.nf, hs = n / 2 + 1;
    const double box[3] = {p.L, p.Ly, p.Lz}, V = box[0] * box[1] * box[2];
    const Cell cell = cell_of(p);
    const bool tilt = tilted(p);
    Prolate chi(p.method == 1 ? 1.0 : p.c);
    const double I1 = p.method == 1 ? 1.0 : chi.integral(1.0);
    auto chat = [&](double k2) {
        const double w = p.rc * std::sqrt(k2);
        return p.method == 1 ? std::exp(-w * w / (4.0 * p.c)) : 0.5 * chi.ft(w) / I1;
    };
    // a tilted cell's p depends on the signs of m; an index at the Nyquist
    // frequency n/2 stands for both signs, and p there is the mean over them,
    // which keeps p(-m) = p(m) on the index grid (a real inverse transform)
    auto p_tilted = [&](int mx, int my, int mz) {
        const int fx = std::abs(mx) == n / 2 ? 2 : 1, fy = std::abs(my) == n / 2 ? 2 : 1,
                  fz = std::abs(mz) == n / 2 ? 2 : 1;
        double acc = 0.0;
        for (int a = 0; a < fx; ++a)
            for (int b = 0; b < fy; ++b)
                for (int c = 0; c < fz; ++c) {
                    const double ax = a ? -mx : mx, by = b ? -my : my, cz = c ? -mz : mz;
                    const double kx = 2 * kPi * (ax * cell.i00), ky = 2 * kPi * (ax * cell.ixy + by * cell.i11),
                                 kz = 2 * kPi * (ax * cell.ixz + by * cell.iyz + cz * cell.i22);
                    acc += chat(kx * kx + ky * ky + kz * kz) / (kx * kx + ky * ky + kz * kz);
                }
        return acc / (fx * fy * fz);
    };
    out.assign((size_t)n * n * hs, 0.0);
    for (int x = 0; x < n; ++x) {
        const int mx = x <= n / 2 ? x : x - n;
        for (int y = 0; y < n; ++y) {
            const int my = y <= n / 2 ? y : y - n;
            for (int z = 0; z < hs; ++z) {
                if (mx == 0 && my == 0 && z == 0) continue;
                double s;
                if (tilt) {
                    s = p_tilted(mx, my, z);
                } else {
                    const double kx = 2 * kPi * mx / box[0], ky = 2 * kPi * my / box[1], kz = 2 * kPi * z / box[2];
                    const double k2 = kx * kx + ky * ky + kz * kz;
                    s = chat(k2) / k2;
                }
                out[((size_t)x * n + y) * hs + z] =
                    s / V * ct.Tphi[std::abs(mx)] * ct.Tphi[std::abs(my)] * ct.Tphi[z];
            }
        }
    }
}

std::shared_ptr<const ClassTables> class_tables(const esp_params& p) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, double, double, double>, std::shared_ptr<const ClassTables>> cache;
    const double rho = grid_rho(p);
    const auto key = std::make_tuple(p.method, p.nf, p.P, p.degree, p.c, p.c1, rho);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    auto t = std::make_shared<ClassTables>();
    t->n = p.nf;
    t->P = p.P;
    t->degree = p.degree;
    t->c = p.c;
    t->c1 = p.c1;
    t->rho = rho;
    esp_params ref = p;                 // the reference box L = n
    ref.L = p.nf;
    ref.h = 1.0;
    ref.rc = rho;
    influence_tables(ref, t->TS, t->Tphi);
    window_polynomials(ref, t->poly);
    for (int k = 0; k < p.nf; ++k) {
        const double a = 2.0 * kPi * k / p.nf;
        t->tw.push_back(std::cos(a));
        t->tw.push_back(std::sin(a));
    }
    if (p.method == 1) {
        t->s0_ref = gauss_chi(p.c, 0.0) / (4.0 * kPi * rho);
    } else {
        Prolate chi(p.c);
        t->s0_ref = chi(0.0) / (chi.integral(1.0) * 4.0 * kPi * rho);
    }
    local_polynomials(p.method, p.c, rho, t->ldeg, t->lA, t->lB);
    double wm = 0.0;
    for (int j = 0; j < p.P; ++j)
        for (int s = 0; s <= 64; ++s) {
            const double y = -0.5 + s / 64.0;
            double v = 0.0;
            for (int m = p.degree; m >= 0; --m) v = v * y + t->poly[(size_t)j * (p.degree + 1) + m];
            wm = std::max(wm, std::fabs(v));
        }
    wm *= 1.001;
    t->wmax3 = wm * wm * wm;
    std::lock_guard<std::mutex> g(mu);
    auto& slot = cache[key];
    if (!slot) slot = t;
    return slot;
}

}  // namespace esp
