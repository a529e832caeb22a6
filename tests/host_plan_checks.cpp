// Host planning code under AddressSanitizer and UndefinedBehaviorSanitizer:
// parameter resolution, table classes, influence tables and local-part
// polynomials for cubic, orthorhombic and triclinic cells and both methods,
// plus rejected requests. Built and run by tests/test_host_sanitizers.py.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "plan.hpp"

namespace {

int failures = 0;

void check(bool ok, const char* what) {
    if (!ok) {
        std::printf("FAIL %s\n", what);
        ++failures;
    }
}

void run_case(double L, double Ly, double Lz, double xy, double xz, double yz, int method, int local, double tol,
              bool expect_ok) {
    esp_params req{};
    req.Ly = Ly;
    req.Lz = Lz;
    req.xy = xy;
    req.xz = xz;
    req.yz = yz;
    req.method = method;
    req.local = local;
    esp_params p{};
    std::string msg;
    const esp_status st = esp::resolve_params(L, 3000, tol, &req, &p, msg);
    if (!expect_ok) {
        check(st != ESP_OK && !msg.empty(), "rejected request has a status and a message");
        return;
    }
    check(st == ESP_OK, msg.c_str());
    if (st != ESP_OK) return;
    std::vector<double> coef;
    esp_params w = p;
    esp::window_polynomials(w, coef);
    check(coef.size() == (size_t)w.P * (w.degree + 1), "window polynomial size");
    auto ct = esp::class_tables(p);
    check(ct && ct->TS.size() == (size_t)(3 * (p.nf / 2) * (p.nf / 2) + 1), "radial table size");
    if (p.Ly != p.L || p.Lz != p.L || esp::tilted(p)) {
        std::vector<double> t;
        esp::box_influence(p, *ct, t);
        bool finite = t.size() == (size_t)p.nf * p.nf * (p.nf / 2 + 1);
        for (double v : t) finite = finite && std::isfinite(v);
        check(finite, "box influence table finite");
    }
    std::vector<double> r = {0.5 * p.rc, 0.9 * p.rc, 1.5 * p.rc}, Lr(3), dLr(3);
    esp::local_kernel(p, r.data(), 3, Lr.data(), dLr.data());
    check(std::isfinite(Lr[0]) && Lr[2] == 0.0, "local kernel inside and beyond rc");
}

}  // namespace

int main() {
    for (double tol : {1e-3, 1e-4, 1e-5}) {
        run_case(31.0, 0, 0, 0, 0, 0, 0, 1, tol, true);
        run_case(18.0, 21.0, 24.0, 0, 0, 0, 0, 1, tol, true);
        run_case(30.0, 28.0, 26.0, 6.0, -4.0, 5.0, 0, 1, tol, true);
        run_case(31.0, 0, 0, 0, 0, 0, 1, 1, tol, true);
    }
    run_case(20.0, 18.0, 16.0, 14.0, 0.0, -11.0, 0, 0, 1e-4, true);
    run_case(14.0, 14.0, 14.0, 13.0, 0.0, 0.0, 0, 1, 1e-4, false);  // rc beyond half a plane spacing
    run_case(16.0, 15.0, 14.0, 1.0, 0.0, 0.0, 1, 1, 1e-4, true);    // classical method in a tilted cell
    run_case(10.0, -1.0, 10.0, 0, 0, 0, 0, 0, 1e-4, false);         // negative side
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
