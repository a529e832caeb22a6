// Host-side (FP64) parameter selection and table generation for the ESP
// long-range pipeline. No device code here.
#pragma once
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "esp.h"

namespace esp {

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// psi_0^c, L2-normalised on [-1, 1], psi(0) > 0: eigenvector of the prolate
// differential operator -(d/dx)(1-x^2)(d/dx) + c^2 x^2 with the smallest
// eigenvalue, expanded in the orthonormal even Legendre functions
// (Slepian & Pollak 1961). Eigenvalue by Sturm-sequence bisection, vector by
// inverse iteration on the tridiagonal matrix.
class Prolate {
  public:
    explicit Prolate(double c);
    double c() const { return c_; }
    double operator()(double x) const;     // psi(x), |x| <= 1
    double deriv(double x) const;          // psi'(x)
    double integral(double x) const;       // int_0^x psi
    double ft(double w) const;             // int_{-1}^{1} psi(t) cos(w t) dt
  private:
    double c_;
    std::vector<double> a_;                // psi = sum_k a_k P_{2k}(x)
    std::vector<double> qx_, qw_psi_;      // quadrature nodes, w * psi(nodes)
};

double c_for_tolerance(double eps);
int order_for_tol(double tol);
bool is_smooth(int n);
int grid_size(double L, double h_max);
double aliasing_error(int n, double L, const Prolate& chi, double rc, double c1, int P);

struct Resolved {
    esp_params p;                // fully resolved parameters
    std::vector<double> poly;    // P * (degree + 1)
    std::vector<double> TS;      // 3 (n/2)^2 + 1
    std::vector<double> Tphi;    // n/2 + 1
};

// Resolve parameters; returns ESP_OK or an error with msg filled in.
esp_status resolve_params(double L, int64_t N, double tol, const esp_params* req,
                          esp_params* out, std::string& msg);
// Window polynomials for resolved params (fits degree if p.degree == 0 and
// writes it back).
void window_polynomials(esp_params& p, std::vector<double>& coef);
void influence_tables(const esp_params& p, std::vector<double>& TS, std::vector<double>& Tphi);
void local_kernel(const esp_params& p, const double* r, int64_t n, double* Lr, double* dLr);
// Polynomials of the local part for the device (grid units), in
// y = K x - k - 1/2 on pieces [k/K, (k+1)/K) of x = r^2/rho^2 (K =
// kLocalPieces: one piece, so a pair's coefficients are the same for every
// lane). A approximates the smooth part s(r), so that L(r) = 1/(4 pi r) - A,
// and B approximates s'(r)/r.
constexpr int kLocalPieces = 1;
constexpr int kLocalMinDegree = 8;
constexpr int kLocalMaxDegree = 16;
void local_polynomials(int method, double c, double rho, int& degree, std::vector<double>& A,
                       std::vector<double>& B);

// Tables of one parameter class. With rc proportional to h (the default
// rule), the influence tables, window polynomials and c1 depend on
// (n, P, degree, c, c1, rc/h) only; a box of side L then needs just the
// scalars pscale = n/L (p ~ 1/L), s0 = s0_ref n/L and 1/L. Tables are made for
// the reference box L = n (h = 1) and cached process-wide.
struct ClassTables {
    int n, P, degree;
    double c, c1, rho;            // rho = rc/h
    std::vector<double> TS, Tphi, poly, tw;  // tw interleaved (cos, sin)
    double s0_ref;                // S(0) for L = n
    double wmax3;                 // cube of the window polynomials' peak
    int ldeg;                     // local-part polynomials (local_polynomials)
    std::vector<double> lA, lB;
};
// rc/h of resolved params as the table classes key it.
double grid_rho(const esp_params& p);
std::shared_ptr<const ClassTables> class_tables(const esp_params& p);
// Influence table of a non-cubic box over the half spectrum, (x, ky, kz) in
// the grid's order: n x n x (n/2 + 1) doubles.
void box_influence(const esp_params& p, const ClassTables& ct, std::vector<double>& out);

// The cell H = [[L, xy, xz], [0, Ly, yz], [0, 0, Lz]] of resolved params: its
// inverse (upper triangular), the longest lattice vector and the smallest
// distance between lattice planes (exactly the sides' max and min when the
// tilts are 0).
struct Cell {
    double i00, ixy, ixz, i11, iyz, i22;
    double amax, dmin;
};
Cell cell_of(const esp_params& p);
inline bool tilted(const esp_params& p) { return p.xy != 0.0 || p.xz != 0.0 || p.yz != 0.0; }

}  // namespace esp
