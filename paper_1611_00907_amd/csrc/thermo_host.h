// Host FP64 thermodynamics (Sec. III) and contact angle (Sec. V) of the library.
#pragma once

namespace cplbm {

namespace thermo {

constexpr int EOS_VDW = 0, EOS_CS = 1, EOS_PR = 2, EOS_RKS = 3, EOS_RK = 4;

struct Fluid {
    int eos;
    double a, b, R;
    double T, alpha;
    double Tc, rho_c;
};

double rho_pole(int eos, double b);
void critical_point(int eos, double a, double b, double R, double* Tc, double* rho_c, double* p_c);
double alpha_of(int eos, double T, double Tc, double omega);
Fluid make_fluid(int eos, double a, double b, double R, double Tr, double omega);
double p0(const Fluid& f, double rho);
double dp0(const Fluid& f, double rho);
double mu_b(const Fluid& f, double rho);
// Spinodal densities: dp0/drho < 0 for lo < rho < hi; false at or above Tc.
bool spinodal(const Fluid& f, double* lo, double* hi);
bool coexistence(const Fluid& f, double* rho_g, double* rho_l, double* p_sat, double* mu_sat);
int contact_angle(const double* rho, int nx, int ny, int base_row, double surface_y, double rho_mid,
                  double* theta, double* L, double* H);

}  // namespace thermo
}  // namespace cplbm
