// Host FP64 thermodynamics of Sec. III and the contact-angle measurement of Sec. V.
//
// p0 = T g(rho) - alpha h(rho): g is the repulsive part per unit temperature and h
// the attractive part; analytic derivatives give the spinodal and the Newton
// Jacobians (d mu_b / d rho = p0'(rho) / rho follows from Eq 3).
#include "thermo_host.h"

#include <cmath>
#include <vector>

namespace cplbm {
namespace thermo {
namespace {

const double SQ2 = 1.4142135623730950488;

// Repulsive pressure per unit temperature and its derivative.
void g_of(int eos, double b, double R, double rho, double* g, double* dg) {
    if (eos == EOS_CS) {
        const double q = b * rho / 4.0, om = 1.0 - q;
        *g = R * rho * (1.0 + q + q * q - q * q * q) / (om * om * om);
        *dg = R * (1.0 + 4.0 * q + 4.0 * q * q - 4.0 * q * q * q + q * q * q * q) / (om * om * om * om);
    } else {
        const double om = 1.0 - b * rho;
        *g = R * rho / om;
        *dg = R / (om * om);
    }
}

// Attractive pressure per unit a*alpha and its derivative.
void h_of(int eos, double b, double rho, double* h, double* dh) {
    switch (eos) {
    case EOS_VDW:
    case EOS_CS:
        *h = rho * rho;
        *dh = 2.0 * rho;
        break;
    case EOS_PR: {
        const double d = 1.0 + 2.0 * b * rho - b * b * rho * rho;
        *h = rho * rho / d;
        *dh = 2.0 * rho * (1.0 + b * rho) / (d * d);
        break;
    }
    default: {  // RK, RKS
        const double d = 1.0 + b * rho;
        *h = rho * rho / d;
        *dh = rho * (2.0 + b * rho) / (d * d);
    }
    }
}

// Spinodal temperature: T at which dp0/drho = 0 at this density (alpha = 1 for
// the Soave forms at Tc; alpha = T^-1/2 for RK).
double t_spinodal(int eos, double a, double b, double R, double rho) {
    double g, dg, h, dh;
    g_of(eos, b, R, rho, &g, &dg);
    h_of(eos, b, rho, &h, &dh);
    const double ratio = a * dh / dg;
    return eos == EOS_RK ? std::pow(ratio, 2.0 / 3.0) : ratio;
}

}  // namespace

double rho_pole(int eos, double b) { return eos == EOS_CS ? 4.0 / b : 1.0 / b; }

void critical_point(int eos, double a, double b, double R, double* Tc, double* rho_c, double* p_c) {
    // Golden-section search for the maximum of the spinodal temperature.
    double lo = 1e-6 * rho_pole(eos, b), hi = 0.999 * rho_pole(eos, b);
    const double gr = 0.6180339887498949;
    double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    double f1 = t_spinodal(eos, a, b, R, x1), f2 = t_spinodal(eos, a, b, R, x2);
    for (int it = 0; it < 200 && (hi - lo) > 1e-15 * hi; ++it) {
        if (f1 < f2) {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + gr * (hi - lo);
            f2 = t_spinodal(eos, a, b, R, x2);
        } else {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - gr * (hi - lo);
            f1 = t_spinodal(eos, a, b, R, x1);
        }
    }
    const double rc = 0.5 * (lo + hi);
    const double T = t_spinodal(eos, a, b, R, rc);
    double g, dg, h, dh;
    g_of(eos, b, R, rc, &g, &dg);
    h_of(eos, b, rc, &h, &dh);
    const double al = eos == EOS_RK ? 1.0 / std::sqrt(T) : 1.0;
    *Tc = T;
    *rho_c = rc;
    *p_c = T * g - a * al * h;
}

double alpha_of(int eos, double T, double Tc, double omega) {
    switch (eos) {
    case EOS_RK: return 1.0 / std::sqrt(T);
    case EOS_RKS: {
        const double m = 0.480 + 1.574 * omega - 0.176 * omega * omega;
        const double s = 1.0 + m * (1.0 - std::sqrt(T / Tc));
        return s * s;
    }
    case EOS_PR: {
        const double m = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
        const double s = 1.0 + m * (1.0 - std::sqrt(T / Tc));
        return s * s;
    }
    default: return 1.0;
    }
}

Fluid make_fluid(int eos, double a, double b, double R, double Tr, double omega) {
    Fluid f;
    double Tc, rc, pc;
    critical_point(eos, a, b, R, &Tc, &rc, &pc);
    f.eos = eos;
    f.a = a;
    f.b = b;
    f.R = R;
    f.Tc = Tc;
    f.rho_c = rc;
    f.T = Tr * Tc;
    f.alpha = alpha_of(eos, f.T, Tc, omega);
    return f;
}

double p0(const Fluid& f, double rho) {
    double g, dg, h, dh;
    g_of(f.eos, f.b, f.R, rho, &g, &dg);
    h_of(f.eos, f.b, rho, &h, &dh);
    return f.T * g - f.a * f.alpha * h;
}

double dp0(const Fluid& f, double rho) {
    double g, dg, h, dh;
    g_of(f.eos, f.b, f.R, rho, &g, &dg);
    h_of(f.eos, f.b, rho, &h, &dh);
    return f.T * dg - f.a * f.alpha * dh;
}

double mu_b(const Fluid& f, double rho) {
    const double RT = f.R * f.T, aa = f.a * f.alpha, b = f.b;
    switch (f.eos) {
    case EOS_VDW: return RT * (std::log(rho / (1.0 - b * rho)) + 1.0 / (1.0 - b * rho)) - 2.0 * f.a * rho;
    case EOS_CS: {
        const double q = b * rho / 4.0, om = 1.0 - q;
        return RT * ((3.0 - q) / (om * om * om) + std::log(rho) + 1.0) - 2.0 * f.a * rho;
    }
    case EOS_PR:
        return RT * std::log(rho / (1.0 - b * rho)) -
               aa / (2.0 * SQ2 * b) * std::log((SQ2 - 1.0 + b * rho) / (SQ2 + 1.0 - b * rho)) +
               RT / (1.0 - b * rho) - aa * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    default:
        return RT * std::log(rho / (1.0 - b * rho)) + RT / (1.0 - b * rho) - aa / b * std::log(1.0 + b * rho) -
               aa * rho / (1.0 + b * rho);
    }
}

namespace {
// Root of dp0 on [lo, hi] where it changes sign (bisection).
double bisect_dp0(const Fluid& f, double lo, double hi) {
    double flo = dp0(f, lo);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double fm = dp0(f, mid);
        if ((fm > 0) == (flo > 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
        if (hi - lo <= 1e-16 * hi) break;
    }
    return 0.5 * (lo + hi);
}

// Density on a stable branch [lo, hi] (p0 increasing there) where p0 = p; log-space bisection.
double branch_rho(const Fluid& f, double p, double lo, double hi) {
    double l = std::log(lo), h = std::log(hi);
    for (int it = 0; it < 300; ++it) {
        const double m = 0.5 * (l + h);
        const double v = p0(f, std::exp(m)) - p;
        if (v < 0) l = m;
        else h = m;
        if (h - l < 1e-16) break;
    }
    return std::exp(0.5 * (l + h));
}
}  // namespace

bool spinodal(const Fluid& f, double* lo, double* hi) {
    if (!(f.T < f.Tc)) return false;
    const double pole = rho_pole(f.eos, f.b);
    // dp0 > 0 on the gas side, < 0 between, > 0 on the liquid side; a scan finds the
    // two sign changes (rho_c of alpha = 1 can differ from the spinodal centre for
    // PR/RKS away from Tc), bisection refines them
    const int n = 4000;
    std::vector<double> xs(n), ds(n);
    for (int i = 0; i < n; ++i) {
        xs[i] = pole * (1e-6 + (0.9999 - 1e-6) * i / (n - 1));
        ds[i] = dp0(f, xs[i]);
    }
    int first = -1, last = -1;
    for (int i = 0; i + 1 < n; ++i)
        if ((ds[i] > 0) != (ds[i + 1] > 0)) {
            if (first < 0) first = i;
            last = i;
        }
    if (first < 0 || first == last) return false;
    *lo = bisect_dp0(f, xs[first], xs[first + 1]);
    *hi = bisect_dp0(f, xs[last], xs[last + 1]);
    return true;
}

bool coexistence(const Fluid& f, double* rho_g, double* rho_l, double* p_sat, double* mu_sat) {
    double s1, s2;
    if (!spinodal(f, &s1, &s2)) return false;
    const double pole = rho_pole(f.eos, f.b);
    const double pmax = p0(f, s1), pmin = p0(f, s2);
    double plo = pmin > 0 ? pmin : 0.0, phi = pmax;
    auto dmu = [&](double p, double* rg, double* rl) {
        *rg = branch_rho(f, p, 1e-300, s1);
        *rl = branch_rho(f, p, s2, pole * (1.0 - 1e-15));
        return mu_b(f, *rl) - mu_b(f, *rg);
    };
    double rg = 0, rl = 0;
    // mu_l - mu_g falls with p (Gibbs-Duhem), positive at plo, negative at phi
    double a = plo + 1e-14 * (phi - plo), b = phi - 1e-14 * (phi - plo);
    for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (a + b);
        if (dmu(m, &rg, &rl) > 0) a = m;
        else b = m;
        if (b - a <= 1e-16 * b) break;
    }
    dmu(0.5 * (a + b), &rg, &rl);
    // Newton polish on (rho_g, rho_l): d mu_b/d rho = p0'/rho
    for (int it = 0; it < 4; ++it) {
        const double F1 = mu_b(f, rl) - mu_b(f, rg), F2 = p0(f, rl) - p0(f, rg);
        const double dpg = dp0(f, rg), dpl = dp0(f, rl);
        const double J11 = -dpg / rg, J12 = dpl / rl, J21 = -dpg, J22 = dpl;
        const double det = J11 * J22 - J12 * J21;
        if (det == 0.0) break;
        const double dg = (-F1 * J22 + F2 * J12) / det;
        const double dl = (-F2 * J11 + F1 * J21) / det;
        rg += dg;
        rl += dl;
    }
    *rho_g = rg;
    *rho_l = rl;
    *p_sat = p0(f, rg);
    *mu_sat = mu_b(f, rg);
    return true;
}

// Sec. V: base width L on base_row and height H on the drop axis, then
// R = (4H^2 + L^2)/(8H) and theta = atan2(L/2, R - H).
int contact_angle(const double* rho, int nx, int ny, int base_row, double surface_y, double rho_mid,
                  double* theta, double* Lout, double* Hout) {
    if (!rho || nx < 3 || ny < 3 || base_row < 0 || base_row >= ny) return -1;
    // centre of the excess mass above the base
    double sum = 0.0, sx = 0.0;
    for (int y = base_row; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const double e = rho[(size_t)y * nx + x] - rho_mid;
            if (e > 0) {
                sum += e;
                sx += e * x;
            }
        }
    if (!(sum > 0)) return -2;
    const int xc = ((int)std::lround(sx / sum) % nx + nx) % nx;
    auto at = [&](int x, int y) { return rho[(size_t)y * nx + ((x % nx) + nx) % nx]; };
    auto cross = [&](double x_in, double r_in, double x_out, double r_out) {
        return x_in + (rho_mid - r_in) / (r_out - r_in) * (x_out - x_in);
    };
    // height: first liquid node at or above the base on the axis, then the top of that run
    int y = base_row;
    while (y < ny && !(at(xc, y) > rho_mid)) ++y;
    if (y >= ny) return -2;
    while (y + 1 < ny && at(xc, y + 1) > rho_mid) ++y;
    const double ytop = (y + 1 < ny) ? cross(y, at(xc, y), y + 1, at(xc, y + 1)) : double(y);
    const double H = ytop - surface_y;
    double L = 0.0, th = 180.0;
    if (at(xc, base_row) > rho_mid) {
        int xl = xc, xr = xc, guard = 0;
        while (at(xl - 1, base_row) > rho_mid && guard++ < nx) --xl;
        guard = 0;
        while (at(xr + 1, base_row) > rho_mid && guard++ < nx) ++xr;
        const double xL = cross(xl, at(xl, base_row), xl - 1, at(xl - 1, base_row));
        const double xR = cross(xr, at(xr, base_row), xr + 1, at(xr + 1, base_row));
        L = xR - xL;
        const double R = (4.0 * H * H + L * L) / (8.0 * H);
        th = std::atan2(0.5 * L, R - H) * 180.0 / 3.14159265358979323846;
    }
    if (theta) *theta = th;
    if (Lout) *Lout = L;
    if (Hout) *Hout = H;
    return 0;
}

}  // namespace thermo
}  // namespace cplbm
