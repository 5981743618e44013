// Host float64 thermodynamics: bulk chemical potential and pressure of the two
// free energies, their critical temperature, and the Maxwell construction.
//   vdW (Eq. 30): E_f = rho R T ln[rho/(1 - b rho)] - a rho^2, T_c = 8a/(27 R b)
//   CS          : E_f = rho R T [ln rho + (4h - 3h^2)/(1-h)^2] - a rho^2, h = b rho/4;
//                 T_c from dp/drho = d2p/drho2 = 0 (solved numerically).
// Coexistence: equal mu_EOS and p_EOS on the gas and liquid branches; the
// pressure is bisected between the spinodal pressures and each branch density
// is bracketed on its own monotone branch of p_EOS.

#include "host_thermo.hpp"

#include <cmath>
#include <vector>

namespace lbm {
namespace host {

double mu_eos(int kind, double a, double b, double R, double T, double rho) {
    if (kind == 0) {
        const double br = 1.0 - b * rho;
        return R * T * (std::log(rho / br) + 1.0 / br) - 2.0 * a * rho;
    }
    const double h = 0.25 * b * rho, om = 1.0 - h;
    return R * T * (std::log(rho) + 1.0 + h * (8.0 - 9.0 * h + 3.0 * h * h) / (om * om * om)) - 2.0 * a * rho;
}

double p_eos(int kind, double a, double b, double R, double T, double rho) {
    if (kind == 0) return rho * R * T / (1.0 - b * rho) - a * rho * rho;
    const double h = 0.25 * b * rho, om = 1.0 - h;
    return rho * R * T * (1.0 + h + h * h - h * h * h) / (om * om * om) - a * rho * rho;
}

static double dp_eos(int kind, double a, double b, double R, double T, double rho) {
    if (kind == 0) {
        const double br = 1.0 - b * rho;
        return R * T / (br * br) - 2.0 * a * rho;
    }
    const double h = 0.25 * b * rho, om = 1.0 - h;
    const double num = 1.0 + 4.0 * h + 4.0 * h * h - 4.0 * h * h * h + h * h * h * h;
    return R * T * num / (om * om * om * om) - 2.0 * a * rho;
}

double rho_limit(int kind, double b) { return kind == 0 ? 1.0 / b : 4.0 / b; }

template <class F>
static double bisect(F f, double lo, double hi, int iters = 200) {
    double flo = f(lo);
    for (int i = 0; i < iters; ++i) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double fm = f(mid);
        if ((fm < 0) == (flo < 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

double critical_temperature(int kind, double a, double b, double R) {
    if (kind == 0) return 8.0 * a / (27.0 * R * b);
    // hard-sphere part g(h) = h Z(h): g' = n(h)/(1-h)^4, g'' = [n'(h)(1-h) + 4 n(h)]/(1-h)^5
    auto g1 = [](double h) {
        const double om = 1.0 - h;
        return (1.0 + 4.0 * h + 4.0 * h * h - 4.0 * h * h * h + h * h * h * h) / (om * om * om * om);
    };
    auto g2 = [](double h) {
        const double om = 1.0 - h;
        const double n = 1.0 + 4.0 * h + 4.0 * h * h - 4.0 * h * h * h + h * h * h * h;
        const double dn = 4.0 + 8.0 * h - 12.0 * h * h + 4.0 * h * h * h;
        return (dn * om + 4.0 * n) / (om * om * om * om * om);
    };
    const double hc = bisect([&](double h) { return g1(h) - h * g2(h); }, 0.05, 0.3);
    // dp/drho = R T g'(h) - 2 a rho = 0 at rho = 4 h / b
    return 8.0 * a * hc / (b * R * g1(hc));
}

int maxwell(int kind, double a, double b, double R, double T_over_Tc, double* rho_g, double* rho_l, double* mu_sat,
            double* p_sat) {
    if (!(a > 0) || !(b > 0) || !(R > 0) || !(T_over_Tc > 0)) return -1;
    const double T = T_over_Tc * critical_temperature(kind, a, b, R);
    const double rmax = rho_limit(kind, b);
    // spinodals: sign changes of dp/drho on a fine grid, refined by bisection
    const int G = 4000;
    std::vector<double> roots;
    double prev_r = rmax * 0.5 / G, prev = dp_eos(kind, a, b, R, T, prev_r);
    for (int i = 1; i < G; ++i) {
        const double r = rmax * (i + 0.5) / G;
        const double v = dp_eos(kind, a, b, R, T, r);
        if ((v < 0) != (prev < 0)) roots.push_back(bisect([&](double x) { return dp_eos(kind, a, b, R, T, x); },
                                                          prev_r, r));
        prev = v;
        prev_r = r;
    }
    if (roots.size() != 2) return -2;
    const double s1 = roots[0], s2 = roots[1];
    const double p_hi = p_eos(kind, a, b, R, T, s1);
    const double p_lo = std::fmax(p_eos(kind, a, b, R, T, s2), 0.0);
    auto gas = [&](double P) {
        return bisect([&](double x) { return p_eos(kind, a, b, R, T, x) - P; }, 1e-300, s1);
    };
    auto liq = [&](double P) {
        return bisect([&](double x) { return p_eos(kind, a, b, R, T, x) - P; }, s2, rmax * (1.0 - 1e-15));
    };
    const double eps = (p_hi - p_lo) * 1e-12;
    const double P = bisect(
        [&](double Pv) {
            return mu_eos(kind, a, b, R, T, liq(Pv)) - mu_eos(kind, a, b, R, T, gas(Pv));
        },
        p_lo + eps, p_hi - eps);
    const double rg = gas(P), rl = liq(P);
    if (rho_g) *rho_g = rg;
    if (rho_l) *rho_l = rl;
    if (mu_sat) *mu_sat = mu_eos(kind, a, b, R, T, rg);
    if (p_sat) *p_sat = P;
    return 0;
}

}  // namespace host
}  // namespace lbm
