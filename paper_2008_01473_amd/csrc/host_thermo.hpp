#pragma once

namespace lbm {
namespace host {

double mu_eos(int kind, double a, double b, double R, double T, double rho);
double p_eos(int kind, double a, double b, double R, double T, double rho);
double rho_limit(int kind, double b);
double critical_temperature(int kind, double a, double b, double R);
// 0 on success, -1 bad arguments, -2 no coexistence at this temperature
int maxwell(int kind, double a, double b, double R, double T_over_Tc, double* rho_g, double* rho_l, double* mu_sat,
            double* p_sat);

}  // namespace host
}  // namespace lbm
